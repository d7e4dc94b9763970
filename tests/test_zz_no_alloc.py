"""GPU test of jerk_search_peaks_noalloc (no device allocation, library-owned key workspace)
against jerk_search_peaks (caller workspace) on the same inputs, bit for bit."""

import numpy as np
import pytest

import paper_1911_01353_amd as J

from gpu_helpers import build_bank, device

pytestmark = pytest.mark.gpu


def _spec(n, seed):
    rng = np.random.default_rng(seed)
    x = ((rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2)).astype(np.complex64)
    x[n // 3] += 10.0
    return x


@pytest.mark.parametrize("path", ["fft", "split_bf16"])
def test_noalloc_equals_search_peaks_on_two_calls(path):
    """Two calls in a row, the second with a smaller spectrum and template range: the no-allocation
    entry point's peaks equal jerk_search_peaks's bit for bit each time, so the shared array is
    cleared between calls and nothing of the first call leaks into the second."""
    import torch
    dev = device()
    cases = [(1 << 17, 40.0, 120.0, 0, None, 51), (30001, 20.0, 60.0, 17, 130, 52)]
    for n, zm, wm, t0, t1, seed in cases:
        plan = J.Plan(n, zm, wm, 2.0, 20.0, path=path)
        bank = build_bank(plan)
        T = plan.info()["n_templates"]
        t1 = T if t1 is None else t1
        spec = torch.from_numpy(_spec(n, seed)).to(dev)
        want = plan.search_peaks(bank, spec, t0, t1)
        got = torch.full((t1 - t0, 2), -1, dtype=torch.int32, device=dev)
        plan.search_peaks_noalloc(bank, spec, got, t0, t1)
        torch.cuda.synchronize()
        print(f"[noalloc] {path} n={n} rows [{t0}, {t1})", flush=True)
        assert np.array_equal(got.cpu().numpy(), want[: t1 - t0].cpu().numpy())
        plan.close()


def test_noalloc_rejects_more_rows_than_its_array():
    import torch
    dev = device()
    plan = J.Plan(1 << 12, 400.0, 1200.0, 2.0, 20.0, path="fft")   # 401 x 121 = 48521 templates
    T = plan.info()["n_templates"]
    assert T > J.NOALLOC_MAX_ROWS
    spec = torch.zeros(1 << 12, dtype=torch.complex64, device=dev)
    out = torch.empty((T, 2), dtype=torch.int32, device=dev)
    with pytest.raises(J.JerkError) as ei:
        # rejected before anything is queued (the bank is never read)
        plan.search_peaks_noalloc(torch.empty(256, dtype=torch.uint8, device=dev), spec, out, 0, T)
    assert ei.value.status == J.JERK_EINVAL and "NOALLOC_MAX_ROWS" in str(ei.value)
    plan.close()


def test_noalloc_in_a_captured_graph():
    """Captured once and replayed with a new spectrum copied into the captured buffer before each
    replay, eager library work in between: every replay's peaks equal jerk_search_peaks's."""
    import torch
    dev = device()
    n = 20000
    plan = J.Plan(n, 20.0, 60.0, 2.0, 20.0, path="fft")
    bank = build_bank(plan)
    T = plan.info()["n_templates"]
    spec = torch.from_numpy(_spec(n, 70)).to(dev)
    out = torch.empty((T, 2), dtype=torch.int32, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.search_peaks_noalloc(bank, spec, out)  # first call on the device: the array's address
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.search_peaks_noalloc(bank, spec, out)
    for rep in range(3):
        new = torch.from_numpy(_spec(n, 71 + rep)).to(dev)
        spec.copy_(new)
        out.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        want = plan.search_peaks(bank, new)  # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want[:T].cpu().numpy()), rep
    plan.close()
