"""GPU tests of the MFMA path across the width groups whose plane launches use the four-wave
kernel (48, 64 and 80 taps) and their neighbours (32 and 96 taps, one-wave kernels): whole
planes against the FP64 oracle, and the one-wave peak-key kernel against the planes."""

import numpy as np
import pytest

import paper_1911_01353_amd as J
from oracle import Grid, error_summary, oracle_plane, peak_index

from gpu_helpers import build_bank, device, gpu_plane

pytestmark = pytest.mark.gpu

ZMAX, WMAX = 40.0, 120.0  # 41 x 13 = 533 templates, groups of 32 ... 96 taps


def _spec(n, seed):
    rng = np.random.default_rng(seed)
    x = ((rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2)).astype(np.complex64)
    x[n // 3] += 8.0
    return x


@pytest.fixture(scope="module")
def ragged_case():
    n = 9001
    spec = _spec(n, 61)
    return spec, oracle_plane(spec, Grid(ZMAX, WMAX, 2.0, 20.0))


@pytest.mark.parametrize("path,tol", [("split_bf16", 1e-4), ("fp16", 1e-2)])
def test_all_groups_against_oracle(ragged_case, path, tol):
    """Every row of a 533-template plane over a ragged 9001-bin spectrum (several windows per
    workgroup, a partial last window, member ranges not filling the last block of 8)."""
    device()
    spec, ora = ragged_case
    n = spec.shape[0]
    plan = J.Plan(n, ZMAX, WMAX, 2.0, 20.0, path=path)
    taps = sorted({g["taps"] for g in plan.groups()})
    assert {48, 64, 80}.issubset(taps) and max(taps) >= 96
    got = gpu_plane(plan, build_bank(plan), spec)
    assert not np.isnan(got).any()
    s = error_summary(got, ora)
    print(f"[mfma groups] {path}: max {s['max']:.2e}, rms {s['rms']:.2e}", flush=True)
    assert s["max"] <= tol
    assert peak_index(got) == peak_index(ora)
    plan.close()


def test_peak_keys_equal_plane_row_maxima():
    """search_peaks (one-wave kernels with peak keys) equals the row argmax of the plane written
    by the four-wave kernels, bit for bit, on the 48-96-tap groups of a 2^18-bin spectrum."""
    import torch
    dev = device()
    n = 1 << 18
    spec_np = _spec(n, 62)
    plan = J.Plan(n, ZMAX, WMAX, 2.0, 20.0, path="split_bf16")
    bank = build_bank(plan)
    plane = gpu_plane(plan, bank, spec_np)
    spec = torch.from_numpy(spec_np).to(dev)
    pk = J.peaks_numpy(plan.search_peaks(bank, spec))
    idx = np.argmax(plane, axis=1)
    assert np.array_equal(pk["power"].view(np.uint32), plane[np.arange(plane.shape[0]), idx].view(np.uint32))
    assert np.array_equal(pk["p"].astype(np.int64), idx)
    plan.close()
