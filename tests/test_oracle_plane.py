"""Pins of the oracle's direct correlation and power plane.

Special cases that reduce to textbook results (integer-r identity, Fourier
interpolation), the matched-filter energy identity, brute-force time-domain
demodulation on a tiny input, shift invariance and noise statistics.
"""

import numpy as np
import pytest

import synth
from oracle.grid import Grid, half_width
from oracle.metrics import peak_index
from oracle.plane import correlate_row, oracle_plane
from oracle.response import template_response, template_taps


def _noise_spectrum(n, seed):
    rng = np.random.default_rng(seed)
    return ((rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2)).astype(np.complex64)


def test_integer_r_zero_template_is_bin_power():
    """At zbar = w = 0 and integer r the template is a delta: P = |X[k0]|^2."""
    x = _noise_spectrum(300, 3)
    g = Grid(0.0, 0.0, 2.0, 20.0)
    plane = oracle_plane(x, g)
    want = np.abs(x.astype(np.complex128)) ** 2
    assert np.max(np.abs(plane[0, 0::2] - want)) < 1e-12 * want.max()


def test_half_bin_zero_template_is_fourier_interpolation():
    """At zbar = w = 0 and r = k0 + 1/2 the output is truncated sinc interpolation."""
    x = _noise_spectrum(200, 4).astype(np.complex128)
    h = half_width(0.0, 0.0)
    g = Grid(0.0, 0.0, 2.0, 20.0)
    plane = oracle_plane(x, g)
    n = x.shape[0]
    for k0 in (0, 5, 77, 150, n - 1):
        acc = 0j
        for k in range(k0 - h + 1, k0 + h + 1):
            if 0 <= k < n:
                q = k0 + 0.5 - k
                acc += x[k] * np.conj(np.exp(1j * np.pi * q) * np.sin(np.pi * q) / (np.pi * q))
        assert abs(plane[0, 2 * k0 + 1] - abs(acc) ** 2) < 1e-12


@pytest.mark.parametrize("zb,w", [(16.0, 20.0), (-8.0, -40.0), (0.0, 60.0)])
def test_matched_filter_energy(zb, w):
    """A spectrum shaped exactly like a template gives P = (sum |taps|^2)^2 at its own (r, z, w)."""
    n = 400
    k0 = 211
    rbar = k0 + 0.5
    x = template_response(rbar - np.arange(n), zb, w)
    g = Grid(20.0, 60.0, 2.0, 20.0)
    t = next(t for t in range(g.n_templates) if g.params(t)[:2] == (zb, w))
    h = g.params(t)[2]
    row = oracle_plane(x, g, templates=[t])[0]
    energy = np.sum(np.abs(template_taps(zb, w, h, 1)) ** 2)
    assert abs(row[2 * k0 + 1] - energy ** 2) < 1e-12
    assert int(np.argmax(row)) == 2 * k0 + 1


def test_tiny_brute_force_demodulation_peak():
    """On a tiny input the plane agrees with time-domain demodulation and peaks at the injected tone.

    Brute force: for each trial (rbar, zbar, w) multiply the time series by the
    conjugate trial tone and sum. The frequency-domain correlation over 2h bins
    is the same quantity up to the template's truncated tails.
    """
    n_t = 4096
    r0, z0, w0 = 700.3, 3.0, 20.0         # rbar = 705.13, zbar = 13, w = 20
    u = np.arange(n_t) / n_t
    cyc = r0 * u + z0 * u * u / 2 + w0 * u ** 3 / 6
    rng = np.random.default_rng(9)
    x_t = 0.3 * np.exp(2j * np.pi * cyc) + (rng.standard_normal(n_t) + 1j * rng.standard_normal(n_t)) * 0.05
    spec = np.fft.fft(x_t) / n_t
    g = Grid(20.0, 40.0, 2.0, 20.0)
    plane = oracle_plane(spec, g, p_lo=1380, p_hi=1440)
    t_pk, p_pk = peak_index(plane)
    zb, w, _ = g.params(t_pk)
    assert (zb, w) == (14.0, 20.0) or (zb, w) == (12.0, 20.0)
    assert abs((1380 + p_pk) / 2 - 705.13) <= 0.5
    # brute-force demodulation at every (template, r) of the window
    for t in (t_pk, t_pk - 1, 5):
        zb, w, _ = g.params(t)
        for p in range(1380, 1440, 7):
            rb = p / 2
            r0t, z0t = rb - zb / 2 + w / 12, zb - w / 2
            ph = r0t * u + z0t * u * u / 2 + w * u ** 3 / 6
            demod = np.sum(x_t * np.exp(-2j * np.pi * ph)) / n_t
            bf = abs(demod) ** 2
            got = plane[t, p - 1380]
            assert abs(got - bf) <= 0.03 * max(bf, 1e-3) + 2e-3 * 0.09


def test_shift_invariance():
    x = _noise_spectrum(500, 6)
    g = Grid(4.0, 20.0, 2.0, 20.0)
    a = oracle_plane(x, g, templates=[0, 7, 14])
    xs = np.concatenate([[0], x[:-1]]).astype(np.complex64)
    b = oracle_plane(xs, g, templates=[0, 7, 14])
    # away from both ends, shifting by one bin shifts the plane by two points
    assert np.max(np.abs(b[:, 102:900] - a[:, 100:898])) < 1e-12


def test_noise_mean_power_is_captured_energy():
    x = _noise_spectrum(20000, 8)
    g = Grid(20.0, 60.0, 2.0, 20.0)
    for t in (0, 70, 146):
        zb, w, h = g.params(t)
        row = oracle_plane(x, g, templates=[t])[0][200:-200]
        energy = np.sum(np.abs(template_taps(zb, w, h, 0)) ** 2)
        assert abs(row[0::2].mean() - energy) < 0.05
        # |Y|^2 of complex Gaussian noise is exponential: variance = mean^2
        assert abs(row[0::2].std() / row[0::2].mean() - 1.0) < 0.08


def test_correlate_row_edges_and_subrange():
    x = _noise_spectrum(64, 10)
    h = half_width(0.0, 20.0)
    taps = template_taps(0.0, 20.0, h, 1)
    full = correlate_row(x, taps, h, 0, 64)
    part = correlate_row(x, taps, h, 10, 30)
    assert np.array_equal(full[10:30], part)
    # beyond the spectrum the window is zero-extended: output at the last bin
    # only sees bins up to n-1
    k0 = 63
    acc = sum(x[k] * taps[k - (k0 - h + 1)] for k in range(k0 - h + 1, 64))
    assert abs(full[k0] - acc) < 1e-12


def test_small_search_peak_at_injected_tone(small_spectrum):
    """The 2^15-bin config puts its peak where the tone's average (r, z, w) lies.

    Tone start values (r0, z0, w0) = (8000.3, 6, 20): rbar = 8006.633 (nearest
    half-bin r = 8006.5, p = 16013), zbar = 16 (i = 18), w = 20 (j = 4), so
    t = 4 * 21 + 18 = 102.
    """
    cfg = synth.CONFIGS["bins2e15_z20_w60"]
    g = Grid(cfg.zmax, cfg.wmax, cfg.dz, cfg.dw)
    plane = oracle_plane(small_spectrum, g, p_lo=15990, p_hi=16040)
    t, p = peak_index(plane)
    assert (t, 15990 + p) == (102, 16013)
    # a^2 N / 4 times captured energy, plus noise
    assert 30.0 < plane[t, p] < 55.0
