"""GPU spectrum preparation (FP64 on the device) against the oracle's recipe.

Both sides compute in FP64 and round once to complex64, by different FFT
algorithms, so bins may differ by the last bit: per component the difference
must stay within 2^-22 of max(1, |X[k]|) and almost every bin must be equal.
"""

import numpy as np
import pytest

import paper_1911_01353_amd as J
import synth
from oracle.spectrum import prepare_spectrum

from gpu_helpers import build_bank, device

pytestmark = pytest.mark.gpu


def _gpu_spectrum(x):
    import torch
    dev = device()
    xs = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)
    out, _ws = J.prepare_spectrum(xs)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _compare(got, want):
    g = got.view(np.float32).astype(np.float64)
    w = want.view(np.float32).astype(np.float64)
    mag = np.repeat(np.maximum(1.0, np.abs(want.astype(np.complex128))), 2)
    assert np.all(np.abs(g - w) <= 2.0 ** -22 * mag)
    assert np.mean(g != w) < 1e-3


@pytest.mark.parametrize("log_n", [2, 3, 4, 5, 6, 10, 13, 16, 19])
def test_noise_series(log_n):
    n = 1 << log_n
    x = synth.time_series(n, 1000 + log_n)
    _compare(_gpu_spectrum(x), prepare_spectrum(x))


def test_full_size_series_with_tones():
    cfg = synth.CONFIGS["bins2e22_z200_w600"]
    x = synth.time_series(cfg.n_samples, cfg.seed, cfg.tones)
    got = _gpu_spectrum(x)
    assert got.shape == (cfg.n_bins,)
    _compare(got, prepare_spectrum(x))


def test_constant_series_gives_zeros():
    assert np.all(_gpu_spectrum(np.full(1024, 1.5, dtype=np.float32)) == 0)


def test_prepared_spectrum_feeds_the_search():
    """Time series -> spectrum -> plane, all on the device: the tone of the 2^15-bin search."""
    import torch
    dev = device()
    cfg = synth.CONFIGS["bins2e15_z20_w60"]
    x = torch.from_numpy(synth.time_series(cfg.n_samples, cfg.seed, cfg.tones)).to(dev)
    spec, _ws = J.prepare_spectrum(x)
    n = cfg.n_bins
    plan = J.Plan(n, cfg.zmax, cfg.wmax, cfg.dz, cfg.dw, path="fft")
    bank = build_bank(plan)
    T = plan.info()["n_templates"]
    plane = torch.empty((T, 2 * n), dtype=torch.float32, device=dev)
    plan.search(bank, spec, plane, 0, T)
    torch.cuda.synchronize()
    flat = int(torch.argmax(plane).item())
    assert divmod(flat, 2 * n) == (102, 16013)
