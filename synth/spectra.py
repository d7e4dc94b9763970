"""Seeded synthetic time series, spectra and request streams.

Recipe (the paper names no data set; its searches run on de-dispersed
time series of radio observations, so white Gaussian noise with injected
accelerated/jerked tones stands in for them):

1. ``N`` float32 samples of N(0, 1) noise from ``numpy.random.Generator(PCG64(seed))``.
2. Add each injected tone ``a * cos(2 pi (r0 u + z0 u^2/2 + w0 u^3/6) + phi0)``
   with ``u = j / N`` (computed in float64, then the sum is rounded to float32
   once: the time series is float32).
3. Real FFT in float64 of the float32 samples; keep bins ``0 .. N/2 - 1``
   (the Nyquist bin is dropped), set bin 0 (DC) to zero.
4. Scale by ``1 / sqrt(mean_{k >= 1} |X_k|^2)`` (unit mean power).
5. Round once to complex64.

Seeds: the 2^15-bin single search uses 191101, the 2^22-bin search 191102, the
256-spectrum batch 191103 and the request stream 191105; spectrum ``i`` of a
batch uses ``seed * 1000 + i``.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Tone:
    """An injected tone, parameterised at the start of the observation.

    ``r0``, ``z0``, ``w0`` are the frequency (bins), fdot (bins) and fddot (bins)
    at ``u = 0`` times the observation length to the power 1, 2 and 3.
    """

    amp: float
    r0: float
    z0: float
    w0: float
    phi0: float = 0.0


@dataclass(frozen=True)
class SearchConfig:
    """One benchmark/parity configuration."""

    name: str
    n_samples: int
    seed: int
    zmax: float
    wmax: float
    dz: float
    dw: float
    tones: tuple = field(default_factory=tuple)

    @property
    def n_bins(self) -> int:
        return self.n_samples // 2


def time_series(n_samples: int, seed: int, tones=()) -> np.ndarray:
    """Float32 N(0,1) noise plus the given tones (steps 1-2 of the recipe)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal(n_samples)  # float64
    if tones:
        u = np.arange(n_samples, dtype=np.float64) / n_samples
        for tone in tones:
            cyc = tone.r0 * u + tone.z0 * u * u / 2.0 + tone.w0 * u * u * u / 6.0
            cyc = cyc - np.floor(cyc)
            x = x + tone.amp * np.cos(2.0 * np.pi * cyc + tone.phi0)
    return x.astype(np.float32)


def spectrum_from_series(x: np.ndarray) -> np.ndarray:
    """Unit-mean-power complex64 spectrum of a float32 series (steps 3-5)."""
    x = np.asarray(x)
    n = x.shape[0]
    if n < 4 or n % 2:
        raise ValueError("series length must be even and >= 4")
    spec = np.fft.rfft(x.astype(np.float64))[: n // 2]
    spec[0] = 0.0
    mean_pow = np.mean(spec.real[1:] ** 2 + spec.imag[1:] ** 2)
    spec = spec / math.sqrt(mean_pow)
    return spec.astype(np.complex64)


def time_series_device(n_samples: int, seed: int, tones=(), device="cuda"):
    """``time_series``'s recipe generated on a device with torch, for batches too large to
    build on the host: N(0, 1) float32 noise from torch's generator seeded with ``seed`` (a
    different stream from numpy's), each tone added in float64, the sum rounded once to float32."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    x = torch.randn(n_samples, device=device, generator=g, dtype=torch.float32)
    if tones:
        u = torch.arange(n_samples, device=device, dtype=torch.float64) / n_samples
        acc = x.double()
        for t in tones:
            ph = 2.0 * math.pi * (t.r0 * u + t.z0 * u * u / 2.0 + t.w0 * u * u * u / 6.0) + t.phi0
            acc += t.amp * torch.cos(ph)
        x = acc.float()
    return x.contiguous()


def make_spectrum(cfg: SearchConfig) -> np.ndarray:
    return spectrum_from_series(time_series(cfg.n_samples, cfg.seed, cfg.tones))


def draw_tones(rng: np.random.Generator, n_bins: int, zmax: float, wmax: float,
               count: int, amp_lo: float = 0.01, amp_hi: float = 0.05) -> tuple:
    """Tones whose observation-average frequency and fdot fall inside the grid.

    The mid-observation frequency is uniform on ``[0.05 n, 0.95 n]``, the
    mid-observation fdot uniform on ``[-0.9, 0.9] zmax``, fddot uniform on
    ``[-0.9, 0.9] wmax``, the amplitude uniform on ``[amp_lo, amp_hi]`` and the
    phase uniform on ``[0, 2 pi)``. The tone is then written down by its
    start-of-observation values (a tone's fdot drifts by ``w0`` over the
    observation and its frequency by ``z0 + w0/2``).
    """
    out = []
    for _ in range(count):
        r_mid = rng.uniform(0.05 * n_bins, 0.95 * n_bins)
        z_mid = rng.uniform(-0.9, 0.9) * zmax
        w0 = rng.uniform(-0.9, 0.9) * wmax
        amp = rng.uniform(amp_lo, amp_hi)
        phi0 = rng.uniform(0.0, 2.0 * np.pi)
        z0 = z_mid - w0 / 2.0
        r0 = r_mid - z0 / 2.0 - w0 / 6.0
        out.append(Tone(amp=amp, r0=r0, z0=z0, w0=w0, phi0=phi0))
    return tuple(out)


def _config2_tones() -> tuple:
    rng = np.random.Generator(np.random.PCG64(191102 + 7))
    return draw_tones(rng, 2 ** 22, 200.0, 600.0, 4)


CONFIGS = {
    # One spectrum, small grid: 2^16 samples, one tone at r0=8000.3, z0=6, w0=20.
    "bins2e15_z20_w60": SearchConfig("bins2e15_z20_w60", 2 ** 16, 191101, 20.0, 60.0, 2.0, 20.0,
                       (Tone(0.05, 8000.3, 6.0, 20.0, 0.0),)),
    # One realistic search: 2^23 samples, four seeded tones, 201 x 61 templates.
    "bins2e22_z200_w600": SearchConfig("bins2e22_z200_w600", 2 ** 23, 191102, 200.0, 600.0, 2.0, 20.0, _config2_tones()),
}


def batch_spectra_specs(count: int = 256, seed: int = 191103, zmax: float = 100.0,
                        wmax: float = 300.0, lengths=(2 ** 20, 2 ** 21, 2 ** 22),
                        tone_fraction: float = 0.1) -> list:
    """Specs (n_samples, seed, tones) of a batch of uneven de-dispersion-trial spectra."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        n_bins = int(lengths[int(rng.integers(0, len(lengths)))])
        has_tone = bool(rng.random() < tone_fraction)
        tones = draw_tones(rng, n_bins, zmax, wmax, 1) if has_tone else ()
        out.append((2 * n_bins, seed * 1000 + i, tones))
    return out


def serving_requests(count: int, rate_hz: float, seed: int = 191105,
                     exp_lo: int = 18, exp_hi: int = 23, zmax_lo: int = 50,
                     zmax_hi: int = 300, tone_prob: float = 0.5,
                     split_prob: float = 0.5) -> list:
    """A Poisson request stream: dicts with arrival time, spectrum spec and grid.

    Spectrum length ``2^e`` bins with ``e`` uniform on ``{exp_lo..exp_hi}``;
    ``zmax`` an even integer uniform on ``[zmax_lo, zmax_hi]``, ``wmax = 3 zmax``,
    ``dz = 2``, ``dw = 20``; a tone with probability ``tone_prob``; the
    split-BF16 path with probability ``split_prob``, otherwise FP32.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate_hz) if rate_hz > 0 else 0.0
        e = int(rng.integers(exp_lo, exp_hi + 1))
        n_bins = 2 ** e
        zmax = float(2 * int(rng.integers(zmax_lo // 2, zmax_hi // 2 + 1)))
        wmax = 3.0 * zmax
        tones = draw_tones(rng, n_bins, zmax, wmax, 1) if rng.random() < tone_prob else ()
        split = bool(rng.random() < split_prob)
        out.append({
            "arrival_s": t, "n_samples": 2 * n_bins, "seed": seed * 1000 + i,
            "tones": tones, "zmax": zmax, "wmax": wmax, "dz": 2.0, "dw": 20.0,
            "split_bf16": split,
        })
    return out
