"""GPU tests of the batched persistent launch, its hipGraph replay and the peak reduction."""

import numpy as np
import pytest

import paper_1911_01353_amd as J
from oracle import Grid, error_summary, oracle_plane

from gpu_helpers import build_bank, device, gpu_plane

pytestmark = pytest.mark.gpu

LENGTHS = [1 << 14, 3000, 1 << 15, 1, 777, 20000]


def _spectra(lengths, seed):
    rng = np.random.default_rng(seed)
    out = []
    for n in lengths:
        x = ((rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2)).astype(np.complex64)
        out.append(x)
    return out


def _row_peaks(plane):
    """Host peak of each row: largest FP32 power, lowest index on ties."""
    idx = np.argmax(plane, axis=1)
    return plane[np.arange(plane.shape[0]), idx], idx


def _run_batch(plan, bank, specs_np, graph, t_begin, t_end, with_keys=True, ws=None, flat=False):
    import torch
    dev = device()
    rows = t_end - t_begin
    specs = [torch.from_numpy(s).to(dev) for s in specs_np]
    planes = [torch.full((rows, 2 * s.shape[0] + 4), float("nan"), dtype=torch.float32, device=dev) for s in specs_np]
    keys = [torch.zeros((rows, plan.keys_per_row(s.shape[0]) + 3), dtype=torch.int64, device=dev) if with_keys
            else None for s in specs_np]
    if ws is None:
        ws = torch.empty(plan.batch_workspace_bytes(len(specs)), dtype=torch.uint8, device=dev)
    plan.batch_search(bank, list(zip(specs, planes, keys)), ws, t_begin, t_end, graph=graph, flat=flat)
    torch.cuda.synchronize()
    out = []
    for s, pl, k in zip(specs_np, planes, keys):
        pk = None
        if k is not None:
            red = torch.empty((rows, 2), dtype=torch.int32, device=dev)
            J.peaks_reduce(k, plan.keys_per_row(s.shape[0]), red)
            torch.cuda.synchronize()
            r = red.cpu().numpy()
            pk = (r[:, 0].view(np.float32).copy(), r[:, 1].view(np.uint32).astype(np.int64))
        out.append((pl.cpu().numpy()[:, : 2 * s.shape[0]], pk))
    return out


@pytest.fixture(scope="module")
def plan_bank():
    device()
    plan = J.Plan(1 << 15, 20.0, 60.0, 2.0, 20.0, path="fft", seg_len=1024)
    return plan, build_bank(plan)


@pytest.mark.parametrize("flat", [False, True])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_single_searches(plan_bank, graph, flat):
    plan, bank = plan_bank
    specs = _spectra(LENGTHS, 11)
    T = plan.info()["n_templates"]
    res = _run_batch(plan, bank, specs, graph, 0, T, flat=flat)
    for s, (pl, (pw, pp)) in zip(specs, res):
        ref = gpu_plane(plan, bank, s)
        assert not np.isnan(pl).any()
        assert np.array_equal(pl.view(np.uint32), ref.view(np.uint32)), s.shape
        hp, hi = _row_peaks(ref)
        assert np.array_equal(pw, hp) and np.array_equal(pp, hi)


def test_batch_template_slab_and_oracle(plan_bank):
    plan, bank = plan_bank
    specs = _spectra([5000, 1234], 12)
    res = _run_batch(plan, bank, specs, False, 40, 90)
    grid = Grid(20.0, 60.0, 2.0, 20.0)
    for s, (pl, _) in zip(specs, res):
        ora = oracle_plane(s, grid, templates=range(40, 90))
        assert error_summary(pl, ora)["max"] <= 1e-4


@pytest.mark.parametrize("flat", [False, True])
def test_graph_replays_match_eager(plan_bank, flat):
    """Replays of captured graphs with new job tables, with eager work in between (the persistent
    launch keeps one graph; the flat launch captures again when the tile count changes)."""
    import torch
    plan, bank = plan_bank
    T = plan.info()["n_templates"]
    dev = device()
    rng_lengths = [[4096, 999, 30000], [17, 8192], [30000, 4096, 999, 5, 12345]]
    ws = torch.empty(plan.batch_workspace_bytes(8), dtype=torch.uint8, device=dev)  # one graph for all replays
    for k, lengths in enumerate(rng_lengths):
        specs = _spectra(lengths, 100 + k)
        # unrelated eager work on the same stream between replays
        junk = torch.randn(1 << 20, device=dev)
        _ = (junk * 2).sum().item()
        got = _run_batch(plan, bank, specs, True, 0, T, ws=ws, flat=flat)
        want = _run_batch(plan, bank, specs, False, 0, T)
        for (a, pa), (b, pb) in zip(got, want):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
            assert np.array_equal(pa[0], pb[0]) and np.array_equal(pa[1], pb[1])


@pytest.mark.parametrize("flat", [False, True])
def test_reused_key_buffers_hold_no_stale_keys(plan_bank, flat):
    """One key buffer per item, reused over graph replays with other spectra and never cleared by the
    caller: the rows' tail keys (past a narrow group's segment count) are rewritten, so the peaks
    equal each plane's row argmax. The buffers start filled with the largest possible key."""
    import torch
    plan, bank = plan_bank
    T = plan.info()["n_templates"]
    dev = device()
    n = 30000
    ws = torch.empty(plan.batch_workspace_bytes(2), dtype=torch.uint8, device=dev)
    kpr = plan.keys_per_row(n)
    keys = [torch.full((T, kpr + 5), -1, dtype=torch.int64, device=dev) for _ in range(2)]
    for rep in range(3):
        specs_np = _spectra([n, n], 300 + rep)
        specs = [torch.from_numpy(x).to(dev) for x in specs_np]
        planes = [torch.empty((T, 2 * n), dtype=torch.float32, device=dev) for _ in specs]
        plan.batch_search(bank, list(zip(specs, planes, keys)), ws, 0, T, graph=True, flat=flat)
        torch.cuda.synchronize()
        for pl, k in zip(planes, keys):
            red = torch.empty((T, 2), dtype=torch.int32, device=dev)
            J.peaks_reduce(k, kpr, red)
            torch.cuda.synchronize()
            r = red.cpu().numpy()
            hp, hi = _row_peaks(pl.cpu().numpy())
            assert np.array_equal(r[:, 0].view(np.float32), hp) and np.array_equal(r[:, 1].astype(np.int64), hi)
            tail = k[:, kpr:].cpu().numpy()
            assert not tail.any(), "keys past jerk_batch_keys_per_row are not cleared"


def test_batch_rejects_mixed_paths():
    device()
    plan = J.Plan(4096, 20.0, 60.0, 2.0, 20.0, path="auto")
    bank = build_bank(plan)
    import torch
    ws = torch.empty(plan.batch_workspace_bytes(1), dtype=torch.uint8, device="cuda")
    spec = torch.zeros(4096, dtype=torch.complex64, device="cuda")
    plane = torch.zeros((147, 8192), dtype=torch.float32, device="cuda")
    with pytest.raises(J.JerkError) as ei:
        plan.batch_search(bank, [(spec, plane, None)], ws)
    assert ei.value.status == J.JERK_EINVAL


def test_stream_check_reports_finished_work():
    import torch
    import synth
    dev = device()
    cfg = synth.CONFIGS["bins2e15_z20_w60"]
    spec = torch.from_numpy(synth.make_spectrum(cfg)).to(dev)
    n = spec.shape[0]
    plan = J.Plan(n, cfg.zmax, cfg.wmax, cfg.dz, cfg.dw, path="fft")
    bank = plan.new_bank()
    plan.build_templates(bank)
    T = plan.info()["n_templates"]
    plane = torch.empty((T, 2 * n), dtype=torch.float32, device=dev)
    plan.search(bank, spec, plane, 0, T)
    assert J.stream_check() in (J.JERK_OK, J.JERK_EPENDING)
    torch.cuda.synchronize()
    assert J.stream_check() == J.JERK_OK
    plan.close()


@pytest.mark.parametrize("flat", [False, True])
def test_batch_full_size_matches_single_searches(flat):
    """At the batched workload's sizes (spectra of 2^20, 2^21 + 4321 and 2^22 bins; zmax 100,
    wmax 300, 3131 templates) the batched launch writes the same bits as single searches, on the
    narrowest and the widest 16-template slabs, and its fused row peaks are the planes' argmax."""
    import torch
    dev = device()
    lengths = [1 << 20, (1 << 21) + 4321, 1 << 22]
    plan = J.Plan(1 << 22, 100.0, 300.0, 2.0, 20.0, path="fft")
    bank = build_bank(plan)
    T = plan.info()["n_templates"]
    specs_np = _spectra(lengths, 1911)
    ws = torch.empty(plan.batch_workspace_bytes(len(specs_np)), dtype=torch.uint8, device=dev)
    specs = [torch.from_numpy(s).to(dev) for s in specs_np]
    for t0, t1 in ((0, 16), (T - 16, T)):
        rows = t1 - t0
        planes = [torch.full((rows, 2 * s.shape[0]), float("nan"), dtype=torch.float32, device=dev) for s in specs]
        keys = [torch.zeros((rows, plan.keys_per_row(s.shape[0])), dtype=torch.int64, device=dev) for s in specs]
        plan.batch_search(bank, list(zip(specs, planes, keys)), ws, t0, t1, graph=True, flat=flat)
        torch.cuda.synchronize()
        for s, pl, k in zip(specs, planes, keys):
            n = s.shape[0]
            ref = torch.full((rows, 2 * n), float("nan"), dtype=torch.float32, device=dev)
            plan.search(bank, s, ref, t0, t1)
            torch.cuda.synchronize()
            print(f"[full-size batch] flat={flat} rows [{t0}, {t1}) nbins {n}", flush=True)
            assert torch.equal(pl.view(torch.int32), ref.view(torch.int32)), (n, t0)
            red = torch.empty((rows, 2), dtype=torch.int32, device=dev)
            J.peaks_reduce(k, plan.keys_per_row(n), red)
            torch.cuda.synchronize()
            r = red.cpu().numpy()
            hp, hi = _row_peaks(ref.cpu().numpy())
            assert np.array_equal(r[:, 0].view(np.float32), hp) and np.array_equal(r[:, 1].view(np.uint32).astype(np.int64), hi), n
            del ref
        del planes, keys
    plan.close()
