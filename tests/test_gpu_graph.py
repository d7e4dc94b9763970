"""jerk_search inside a captured graph: every replay equals the eager plane bit for bit.

The search path enqueues kernels only (no memset, allocation or synchronisation), so
a caller may capture it. The graph is replayed several times with eager library work
and synchronisations in between, and each replay is checked.
"""

import numpy as np
import pytest

import paper_1911_01353_amd as J
import synth

from gpu_helpers import build_bank, device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("path", ["fft", "split_bf16", "fp16"])
def test_graph_replays_match_eager(path, small_spectrum):
    import torch
    dev = device()
    cfg = synth.CONFIGS["bins2e15_z20_w60"]
    n = small_spectrum.shape[0]
    plan = J.Plan(n, cfg.zmax, cfg.wmax, cfg.dz, cfg.dw, path=path)
    bank = build_bank(plan)
    T = plan.info()["n_templates"]
    spec = torch.from_numpy(small_spectrum).to(dev)
    eager = torch.empty((T, 2 * n), dtype=torch.float32, device=dev)
    plan.search(bank, spec, eager, 0, T)
    torch.cuda.synchronize()
    want = eager.cpu().numpy()
    out = torch.full((T, 2 * n), float("nan"), dtype=torch.float32, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.search(bank, spec, out, 0, T)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.search(bank, spec, out, 0, T)
    other = torch.empty_like(eager)
    for rep in range(3):
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint32), want.view(np.uint32)), (path, rep)
        plan.search(bank, spec, other, 0, T)  # eager work between replays
        torch.cuda.synchronize()
    plan.close()


def test_search_candidates_graph_replays_match_eager(small_spectrum):
    """The search with fused candidate selection captured once and replayed with a new spectrum
    copied into the captured buffer before each replay, eager work in between: every replay's
    candidates and row statistics equal the eager call's for that spectrum."""
    import torch
    dev = device()
    cfg = synth.CONFIGS["bins2e15_z20_w60"]
    n = small_spectrum.shape[0]
    plan = J.Plan(n, cfg.zmax, cfg.wmax, cfg.dz, cfg.dw, path="fft")
    bank = build_bank(plan)
    T = plan.info()["n_templates"]
    k = 3.0
    pre = 0.9 * (1 + k)
    rng = np.random.default_rng(5)
    other_np = ((rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2)).astype(np.complex64)
    spectra = [small_spectrum, other_np]
    spec = torch.from_numpy(small_spectrum).to(dev)
    ws = torch.empty(plan.search_candidates_workspace_bytes(n, pre), dtype=torch.uint8, device=dev)
    out = torch.zeros((1 << 20, 4), dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    stats = torch.empty((T, 2), dtype=torch.float64, device=dev)

    def eager(x):
        spec.copy_(torch.from_numpy(x).to(dev))
        count.zero_()
        plan.search_candidates(bank, spec, k, pre, out, count, stats=stats, ws=ws)
        torch.cuda.synchronize()
        return J.candidates_numpy(out, count), stats.cpu().numpy().copy()

    want = [eager(x) for x in spectra]
    assert len(want[0][0]) > 100
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.search_candidates(bank, spec, k, pre, out, count, stats=stats, ws=ws)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.search_candidates(bank, spec, k, pre, out, count, stats=stats, ws=ws)
    plane = torch.empty((T, 2 * n), dtype=torch.float32, device=dev)
    for rep in range(4):
        i = rep % 2
        spec.copy_(torch.from_numpy(spectra[i]).to(dev))
        out.zero_()
        count.zero_()
        stats.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = J.candidates_numpy(out, count)
        assert np.array_equal(got, want[i][0]), rep
        assert np.array_equal(stats.cpu().numpy(), want[i][1]), rep
        plan.search(bank, spec, plane, 0, T)  # eager work between replays
        torch.cuda.synchronize()
    plan.close()
