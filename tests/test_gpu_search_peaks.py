"""Per-row peaks without a plane (jerk_search_peaks) against the row maximum and its index in the
plane that jerk_search writes for the same plan and spectrum: power bit-equal, index equal (the
lowest index among equal powers on both sides), on every path, for a ragged spectrum length, a
template slab, and inside a replayed graph."""

import numpy as np
import pytest

import paper_1911_01353_amd as J

from gpu_helpers import build_bank, device, gpu_plane

pytestmark = pytest.mark.gpu


def _spectrum(n, seed):
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2)
    x[n // 3] += 8.0
    return x.astype(np.complex64)


def _row_peaks(plane):
    idx = np.argmax(plane, axis=1)  # first index of the largest value
    return plane[np.arange(plane.shape[0]), idx], idx


@pytest.mark.parametrize("path", ["fft", "split_bf16", "fp16", "auto"])
def test_peaks_equal_plane_row_maxima(path):
    import torch
    dev = device()
    n = 20011
    plan = J.Plan(n, 20.0, 60.0, 2.0, 20.0, path=path)
    bank = build_bank(plan)
    spec_np = _spectrum(n, 3)
    T = plan.info()["n_templates"]
    plane = gpu_plane(plan, bank, spec_np)
    wp, wi = _row_peaks(plane)
    spec = torch.from_numpy(spec_np).to(dev)
    for t0, t1 in ((0, T), (13, 101)):
        out = plan.search_peaks(bank, spec, t0, t1)
        torch.cuda.synchronize()
        got = J.peaks_numpy(out, t1 - t0)
        assert np.array_equal(got["power"].view(np.uint32), wp[t0:t1].view(np.uint32)), path
        assert np.array_equal(got["p"].astype(np.int64), wi[t0:t1]), path
    plan.close()


@pytest.mark.parametrize("kind", ["zeros", "constant"])
@pytest.mark.parametrize("path", ["fft", "split_bf16"])
def test_peaks_ties_go_to_the_lowest_index(kind, path):
    """Spectra whose planes hold many exactly equal powers: all zero (every point of every row
    ties, so each row's peak is index 0) and constant (equal segment inputs give bit-equal
    powers at the same offset of different segments). The reduction over lanes, columns and
    segments must keep the first of equal powers, as the argmax of the plane does."""
    import torch
    dev = device()
    n = 20011
    plan = J.Plan(n, 20.0, 60.0, 2.0, 20.0, path=path)
    bank = build_bank(plan)
    spec_np = np.zeros(n, np.complex64) if kind == "zeros" else np.full(n, 1 - 0.5j, np.complex64)
    T = plan.info()["n_templates"]
    plane = gpu_plane(plan, bank, spec_np)
    wp, wi = _row_peaks(plane)
    if kind == "zeros":
        assert not wp.any() and not wi.any()
    else:
        # ties do occur: some row holds its maximum at more than one index
        assert any(np.count_nonzero(plane[r] == wp[r]) > 1 for r in range(T))
    got = J.peaks_numpy(plan.search_peaks(bank, torch.from_numpy(spec_np).to(dev)), T)
    torch.cuda.synchronize()
    assert np.array_equal(got["power"].view(np.uint32), wp.view(np.uint32))
    assert np.array_equal(got["p"].astype(np.int64), wi)
    plan.close()


FFT_VARIANTS = [(512, 8), (1024, 8), (1024, 16), (2048, 8), (2048, 16), (4096, 8), (4096, 16)]


@pytest.mark.parametrize("seg,ept", FFT_VARIANTS)
def test_peaks_every_fft_variant(seg, ept):
    """The peak-key epilogue of every FFT kernel variant (segment length, elements per thread)
    against the row maxima of the plane the same variant writes: 8 and 16 templates per block
    (member ranges that leave the last block part-filled), a noise spectrum with a tone and a
    constant one (bit-equal powers at equal segment offsets), over a ragged 20011-bin length
    whose last segment is cut short."""
    import torch
    dev = device()
    n = 20011
    plan = J.Plan(n, 20.0, 60.0, 2.0, 20.0, path="fft")
    T = plan.info()["n_templates"]
    for tpb in (8, 16):
        for g in range(len(plan.groups())):
            plan.set_group(g, seg, tpb, "fft", ept)
        bank = build_bank(plan)
        for spec_np in (_spectrum(n, 7), np.full(n, 0.75 + 0.25j, np.complex64)):
            plane = gpu_plane(plan, bank, spec_np)
            wp, wi = _row_peaks(plane)
            got = J.peaks_numpy(plan.search_peaks(bank, torch.from_numpy(spec_np).to(dev)), T)
            torch.cuda.synchronize()
            assert np.array_equal(got["power"].view(np.uint32), wp.view(np.uint32)), (seg, ept, tpb)
            assert np.array_equal(got["p"].astype(np.int64), wi), (seg, ept, tpb)
    plan.close()


def test_peaks_graph_replays():
    import torch
    dev = device()
    n = 8192
    plan = J.Plan(n, 20.0, 60.0, 2.0, 20.0, path="auto")
    bank = build_bank(plan)
    T = plan.info()["n_templates"]
    a, b = _spectrum(n, 4), _spectrum(n, 5)
    spec = torch.from_numpy(a).to(dev)
    out = torch.empty((T, 2), dtype=torch.int32, device=dev)
    ws = torch.empty(8 * T, dtype=torch.uint8, device=dev)
    want = {}
    for key, x in (("a", a), ("b", b)):
        spec.copy_(torch.from_numpy(x).to(dev))
        plan.search_peaks(bank, spec, out=out, ws=ws)
        torch.cuda.synchronize()
        want[key] = J.peaks_numpy(out).copy()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.search_peaks(bank, spec, out=out, ws=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.search_peaks(bank, spec, out=out, ws=ws)
    for rep, key in enumerate(("a", "b", "a", "b")):
        spec.copy_(torch.from_numpy(a if key == "a" else b).to(dev))
        out.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(J.peaks_numpy(out), want[key]), rep
    plan.close()
