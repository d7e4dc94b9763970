"""GPU parity of the search with fused candidate selection (no plane written).

Against the library's own two-step path (plane from the search, then row
statistics and the peak finder, both pinned to the oracle in
test_gpu_candidates.py) on the same spectrum: the (t, p) sets must be equal
except for points whose power lies within 1e-9 sigma of their row's threshold,
powers bit-equal (both sides run the same FFT arithmetic), row statistics within
1e-12 relative. Against the FP64 oracle plane directly: every disagreement must
sit at a decision the plane's 1e-4 relative error can flip (threshold or a
neighbour comparison). The speculative level and the staging size only change
the cost, never the result: every test runs several of them, including a level
above every threshold (the exact pass recomputes every row) and a single staging
slot per tile (tiles spill into the shared pool until it is full, then rows are
recomputed).
"""

import numpy as np
import pytest

import paper_1911_01353_amd as J
import synth
from paper_1911_01353_amd import _lib
from oracle import Grid, oracle_plane
from oracle.candidates import find_candidates, row_statistics

from gpu_helpers import build_bank, device

pytestmark = pytest.mark.gpu

VARIANTS = [(512, 8), (1024, 16), (1024, 8), (2048, 16), (2048, 8), (4096, 16), (4096, 8)]


def _spectrum(n, seed, tone=None):
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2)
    if tone is not None:
        k0, amp = tone
        x[k0] += amp
    return x.astype(np.complex64)


def _fused(plan, bank, spec_np, k, pre, staged=0, t_begin=0, t_end=None, capacity=None):
    import torch
    dev = device()
    if t_end is None:
        t_end = plan.info()["n_templates"]
    spec = torch.from_numpy(spec_np).to(dev)
    rows = t_end - t_begin
    cap = capacity if capacity is not None else max(64, rows * spec_np.shape[0])
    out = torch.zeros((cap, 4), dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    stats = torch.full((max(rows, 1), 2), float("nan"), dtype=torch.float64, device=dev)
    plan.search_candidates(bank, spec, k, pre, out, count, t_begin, t_end, staged=staged, stats=stats)
    torch.cuda.synchronize()
    return stats.cpu().numpy()[:rows], J.candidates_numpy(out, count), int(count.item())


def _two_step(plan, bank, spec_np, k, t_begin=0, t_end=None):
    """Plane, then statistics and candidates, all on the GPU."""
    import torch
    dev = device()
    if t_end is None:
        t_end = plan.info()["n_templates"]
    n = spec_np.shape[0]
    spec = torch.from_numpy(spec_np).to(dev)
    plane = torch.empty((t_end - t_begin, 2 * n), dtype=torch.float32, device=dev)
    plan.search(bank, spec, plane, t_begin, t_end)
    stats = torch.empty((t_end - t_begin, 2), dtype=torch.float64, device=dev)
    J.plane_stats(plane, stats)
    out = torch.zeros((max(64, plane.numel() // 2), 4), dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    J.find_candidates(plane, stats, k, out, count, t_base=t_begin)
    torch.cuda.synchronize()
    return plane.cpu().numpy(), stats.cpu().numpy(), J.candidates_numpy(out, count)


def _same(got, want, plane, stats, k, t_begin=0):
    g = {(int(r["t"]), int(r["p"])): r for r in got}
    w = {(int(r["t"]), int(r["p"])): r for r in want}
    assert len(g) == len(got), "a candidate was stored twice"
    for t, p in set(g) ^ set(w):
        i = t - t_begin
        thr = stats[i, 0] + k * stats[i, 1]
        assert abs(float(plane[i, p]) - thr) <= 1e-9 * stats[i, 1], ("candidate mismatch", t, p)
    for key in set(g) & set(w):
        assert g[key]["power"] == w[key]["power"], key
        assert abs(float(g[key]["sigma"]) - float(w[key]["sigma"])) <= 1e-6 * max(1.0, abs(float(w[key]["sigma"])))


def _levels(k):
    """(speculative level, staging slots per tile): a good guess, one near the typical threshold
    (part of the rows flagged), far too low, above every threshold (every row recomputed), and
    one slot per tile (most tiles spill into the pool, which then fills: those rows recomputed)."""
    return [(0.9 * (1.0 + k), 0), (1.0 + k, 0), (0.5, 0), (1e9, 0), (0.9 * (1.0 + k), 1)]


@pytest.fixture(scope="module")
def fft_plan():
    device()
    plan = J.Plan(1 << 15, 20.0, 60.0, 2.0, 20.0, path="fft")
    return plan, build_bank(plan)


@pytest.mark.parametrize("k", [1.0, 4.0])
def test_matches_two_step_path(fft_plan, k):
    plan, bank = fft_plan
    spec = _spectrum(1 << 15, 5, tone=(9000, 12.0))
    plane, stats, want = _two_step(plan, bank, spec, k)
    for pre, staged in _levels(k):
        st, got, count = _fused(plan, bank, spec, k, pre, staged)
        assert count == len(got)
        scale = np.maximum(np.abs(stats), 1e-30)
        assert np.all(np.abs(st - stats) <= 1e-12 * scale), pre
        _same(got, want, plane, stats, k)
    assert len(want) > 100


@pytest.mark.parametrize("seg,ept", VARIANTS)
def test_every_fft_variant(seg, ept):
    """Single- and multi-wave workgroups (64 to 512 threads): lane, wave and column neighbours."""
    device()
    n = 20011
    plan = J.Plan(n, 20.0, 60.0, 2.0, 20.0, path="fft")
    for g in range(plan.info()["n_groups"]):
        plan.set_group(g, seg, 4, "fft", ept)
    bank = build_bank(plan)
    spec = _spectrum(n, seg + ept)
    k = 1.5
    plane, stats, want = _two_step(plan, bank, spec, k)
    for pre, staged in [(0.9 * (1 + k), 0), (1e9, 0), (0.9 * (1 + k), 1)]:
        st, got, _ = _fused(plan, bank, spec, k, pre, staged)
        assert np.all(np.abs(st - stats) <= 1e-12 * np.maximum(np.abs(stats), 1e-30))
        _same(got, want, plane, stats, k)


@pytest.mark.parametrize("n", [1, 2, 7, 449, 450, 481, 482, 963, 3000])
def test_short_and_ragged_spectra(n):
    """Lengths below one segment, exactly one or two segments, and a last segment of a single lag
    (U = 512 - K + 1 is 481 for the 32-tap group and 449 for the 64-tap group)."""
    device()
    plan = J.Plan(max(n, 1), 20.0, 60.0, 2.0, 20.0, path="fft", seg_len=512)
    bank = build_bank(plan)
    spec = _spectrum(n, 100 + n)
    for k in (0.0, 1.0):
        plane, stats, want = _two_step(plan, bank, spec, k)
        for pre, staged in _levels(k):
            st, got, _ = _fused(plan, bank, spec, k, pre, staged)
            _same(got, want, plane, stats, k)


def test_template_slab_and_empty_range(fft_plan):
    plan, bank = fft_plan
    spec = _spectrum(1 << 15, 8)
    k = 2.0
    plane, stats, want = _two_step(plan, bank, spec, k, 40, 97)
    st, got, _ = _fused(plan, bank, spec, k, 0.9 * (1 + k), 0, 40, 97)
    assert got["t"].min() >= 40 and got["t"].max() < 97
    _same(got, want, plane, stats, k, t_begin=40)
    _, got0, c0 = _fused(plan, bank, spec, k, 3.0, 0, 50, 50)
    assert c0 == 0 and len(got0) == 0


def test_oracle_parity_and_injected_signal():
    """Against the FP64 oracle plane of the 2^15-bin workload's spectrum (147 templates),
    on a window of bins around the injected signal."""
    device()
    cfg = synth.CONFIGS["bins2e15_z20_w60"]
    spec = synth.make_spectrum(cfg)
    lo, hi = 7700, 8300                 # bins; the signal sits at r = 8006.5
    sub = np.ascontiguousarray(spec[lo:hi])
    plan = J.Plan(sub.shape[0], cfg.zmax, cfg.wmax, cfg.dz, cfg.dw, path="fft")
    bank = build_bank(plan)
    k = 2.0
    st, got, _ = _fused(plan, bank, sub, k, 0.9 * (1 + k))
    grid = Grid(cfg.zmax, cfg.wmax, cfg.dz, cfg.dw)
    ora = oracle_plane(sub, grid)
    ora32 = ora.astype(np.float32)
    ost = row_statistics(ora32)
    assert np.all(np.abs(st[:, 0] - ost[:, 0]) <= 1e-4 * ost[:, 0])
    assert np.all(np.abs(st[:, 1] - ost[:, 1]) <= 1e-4 * ost[:, 1])
    want = find_candidates(ora32, k)
    g = {(int(r["t"]), int(r["p"])) for r in got}
    w = {(int(r["t"]), int(r["p"])) for r in want}
    n_r = ora.shape[1]
    for t, p in g ^ w:
        row = ora[t]
        tol = 2e-4 * max(float(row[p]), ost[t, 0])
        thr = ost[t, 0] + k * ost[t, 1]
        near = abs(row[p] - thr) <= tol + 1e-4 * ost[t, 1] * k
        near |= p > 0 and abs(row[p] - row[p - 1]) <= tol
        near |= p + 1 < n_r and abs(row[p] - row[p + 1]) <= tol
        assert near, ("candidate disagrees with the oracle away from any boundary", t, p)
    assert len(g ^ w) <= max(2, len(w) // 50)
    # the injected signal: template 102, p = 2 (8006.5 - lo)
    best = got[np.argmax(got["power"])]
    assert (int(best["t"]), int(best["p"])) == (102, 2 * (8006 - lo) + 1)


def test_capacity_overflow_counts_everything(fft_plan):
    plan, bank = fft_plan
    spec = _spectrum(1 << 15, 9)
    k = 1.0
    _, full, full_count = _fused(plan, bank, spec, k, 1.8)
    _, part, count = _fused(plan, bank, spec, k, 1.8, capacity=100)
    assert full_count == len(full) > 100
    assert count == len(full) and len(part) == 100
    keys = {(int(r["t"]), int(r["p"])) for r in full}
    assert {(int(r["t"]), int(r["p"])) for r in part} <= keys


@pytest.mark.parametrize("path", ["split_bf16", "fp16", "auto"])
def test_mfma_groups_through_plane_slabs(path):
    """Groups on an MFMA path go through plane slabs; the result equals the two-step path."""
    device()
    n = 20000
    plan = J.Plan(n, 20.0, 60.0, 2.0, 20.0, path=path)
    bank = build_bank(plan)
    spec = _spectrum(n, 77, tone=(5000, 10.0))
    k = 2.0
    plane, stats, want = _two_step(plan, bank, spec, k)
    for pre in (0.9 * (1 + k), 1e9):
        st, got, _ = _fused(plan, bank, spec, k, pre)
        assert np.all(np.abs(st - stats) <= 1e-12 * np.maximum(np.abs(stats), 1e-30))
        _same(got, want, plane, stats, k)
    st, got, _ = _fused(plan, bank, spec, k, 0.9 * (1 + k), 0, 30, 101)
    _same(got, want[(want["t"] >= 30) & (want["t"] < 101)], plane[30:101], stats[30:101], k, t_begin=30)


def test_mixed_fft_and_mfma_groups():
    """A plan whose groups are split between the FFT and the split-BF16 paths."""
    device()
    n = 30011
    plan = J.Plan(n, 20.0, 60.0, 2.0, 20.0, path="fft")
    for g in range(plan.info()["n_groups"]):
        gi = plan.group(g)
        plan.set_group(g, gi["seg_len"], gi["templates_per_block"], "split_bf16" if g % 2 else "fft",
                       gi["fft_ept"])
    bank = build_bank(plan)
    spec = _spectrum(n, 78)
    k = 1.5
    plane, stats, want = _two_step(plan, bank, spec, k)
    st, got, _ = _fused(plan, bank, spec, k, 0.9 * (1 + k))
    _same(got, want, plane, stats, k)


def test_short_workspace():
    import torch
    dev = device()
    plan = J.Plan(4096, 20.0, 60.0, 2.0, 20.0, path="fft")
    bank = build_bank(plan)
    spec = torch.zeros(4096, dtype=torch.complex64, device=dev)
    out = torch.zeros((16, 4), dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(16, dtype=torch.uint8, device=dev)
    with pytest.raises(J.JerkError) as ei:
        plan.search_candidates(bank, spec, 2.0, 2.7, out, count, ws=ws)
    assert ei.value.status == J.JERK_ENOMEM


@pytest.mark.parametrize("path", ["fft", "auto"])
def test_full_size_sampled_rows(path):
    """The 2^22-bin search (12261 templates, zmax 200, wmax 600) with fused selection in the bench's
    configuration (autotuned plan, k = 6, speculative level 6.3), checked on whole rows: two
    corners, the centre, the templates nearest two injected tones and (AUTO: on the split-BF16
    path, through plane slabs whose last one is partial) rows of the 48- and 64-tap groups. Each
    row's candidates and statistics against the library's two-step path on that row (exact bar)
    and against the FP64 oracle's row (every disagreement at a decision within the plane's error)."""
    import torch
    dev = device()
    cfg = synth.CONFIGS["bins2e22_z200_w600"]
    spec_np = synth.make_spectrum(cfg)
    n = spec_np.shape[0]
    spec = torch.from_numpy(spec_np).to(dev)
    plan = J.Plan(n, cfg.zmax, cfg.wmax, cfg.dz, cfg.dw, path=path)
    plan.autotune(spec)
    bank = build_bank(plan)
    T = plan.info()["n_templates"]
    k, pre = 6.0, 6.3
    out = torch.zeros((1 << 27, 4), dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    stats = torch.empty((T, 2), dtype=torch.float64, device=dev)
    plan.search_candidates(bank, spec, k, pre, out, count, stats=stats)
    torch.cuda.synchronize()
    total = int(count.item())
    assert 0 < total <= out.shape[0]
    grid = Grid(cfg.zmax, cfg.wmax, cfg.dz, cfg.dw)
    n_z, J_w = grid.n_z, int(cfg.wmax // cfg.dw)
    tone_rows = []
    for tone in cfg.tones[:2]:
        zb, w = tone.z0 + tone.w0 / 2, tone.w0
        i = int(round((zb + cfg.zmax) / cfg.dz))
        j = int(round(w / cfg.dw)) + J_w
        tone_rows.append(j * n_z + i)
    rows = [0, T - 1, T // 2] + tone_rows + [J_w * n_z + 105, J_w * n_z + 115]  # zbar 10, 30 at w 0: 42, 62 taps
    sel = out[:total][torch.isin(out[:total, 0], torch.tensor(rows, dtype=torch.int32, device=dev))]
    got_all = np.sort(sel.cpu().numpy().view(J.CANDIDATE_DTYPE).reshape(-1), order=["t", "p"])
    st_all = stats.cpu().numpy()
    plane_row = torch.empty((1, 2 * n), dtype=torch.float32, device=dev)
    row_stats = torch.empty((1, 2), dtype=torch.float64, device=dev)
    ws = torch.empty(max(1, J.stats_workspace_bytes(1, 2 * n)), dtype=torch.uint8, device=dev)
    for t in rows:
        got = got_all[got_all["t"] == t]
        # two-step path on this row
        plan.search(bank, spec, plane_row, t, t + 1)
        J.plane_stats(plane_row, row_stats, ws=ws)
        o2 = torch.zeros((1 << 20, 4), dtype=torch.int32, device=dev)
        c2 = torch.zeros(1, dtype=torch.int64, device=dev)
        J.find_candidates(plane_row, row_stats, k, o2, c2, t_base=t)
        torch.cuda.synchronize()
        want2 = J.candidates_numpy(o2, c2)
        gp = plane_row.cpu().numpy()
        gs = row_stats.cpu().numpy()
        assert np.all(np.abs(st_all[t] - gs[0]) <= 1e-12 * np.abs(gs[0])), t
        _same(got, want2, gp, gs, k, t_begin=t)
        # FP64 oracle row
        ora = oracle_plane(spec_np, grid, templates=[t])[0]
        ost = row_statistics(ora.astype(np.float32)[None, :])[0]
        assert np.all(np.abs(st_all[t] - ost) <= 1e-4 * ost), (t, st_all[t], ost)
        want = find_candidates(ora.astype(np.float32)[None, :], k, row_template=[t])
        g = {int(r["p"]) for r in got}
        w = {int(r["p"]) for r in want}
        thr = ost[0] + k * ost[1]
        for p in g ^ w:
            tol = 2e-4 * max(float(ora[p]), ost[0])
            near = abs(ora[p] - thr) <= tol + 1e-4 * k * ost[1]
            near |= p > 0 and abs(ora[p] - ora[p - 1]) <= tol
            near |= p + 1 < ora.shape[0] and abs(ora[p] - ora[p + 1]) <= tol
            assert near, ("candidate disagrees with the oracle away from any boundary", t, p)
        assert len(g ^ w) <= max(2, len(w) // 100), (t, len(g ^ w), len(w))
        if t in tone_rows:
            best = got[np.argmax(got["power"])]
            assert int(best["p"]) == int(np.argmax(ora)), (t, int(best["p"]), int(np.argmax(ora)))
    plan.close()


def test_zero_spectrum_and_negative_k(fft_plan):
    """A zero spectrum: every row constant 0 (sigma 0), every row flagged (threshold 0 below the
    level) and recomputed, no candidates. A negative k puts the threshold below the mean: most
    peaks are candidates, the staging slots overflow into the pool; still the two-step result."""
    import torch
    plan, bank = fft_plan
    n = 1 << 15
    zero = np.zeros(n, dtype=np.complex64)
    st, got, count = _fused(plan, bank, zero, 3.0, 0.9 * 4.0)
    assert count == 0 and len(got) == 0
    assert np.all(st == 0.0)
    spec = _spectrum(n, 21)
    k = -0.5
    plane, stats, want = _two_step(plan, bank, spec, k)
    for pre, staged in [(0.2, 0), (2.0, 0)]:
        st, got, _ = _fused(plan, bank, spec, k, pre, staged)
        _same(got, want, plane, stats, k)
    assert len(want) > plane.size // 8


def test_batch_equals_single_searches():
    """Spectra of different lengths through one batched call (one shared workspace) give, per
    spectrum, the candidates and statistics of the single-spectrum call."""
    import torch
    dev = device()
    plan = J.Plan(1 << 15, 20.0, 60.0, 2.0, 20.0, path="auto")
    bank = build_bank(plan)
    T = plan.info()["n_templates"]
    lengths = [30011, 1 << 15, 777, 12345]
    k = 2.0
    items, want = [], []
    for i, n in enumerate(lengths):
        x = _spectrum(n, 300 + i, tone=(n // 2, 9.0))
        st, got, c = _fused(plan, bank, x, k, 0.9 * (1 + k))
        want.append((st, got, c))
        spec = torch.from_numpy(x).to(dev)
        out = torch.zeros((max(64, T * n), 4), dtype=torch.int32, device=dev)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        stats = torch.empty((T, 2), dtype=torch.float64, device=dev)
        items.append((spec, out, cnt, stats))
    plan.batch_search_candidates(bank, items, k)
    torch.cuda.synchronize()
    for (spec, out, cnt, stats), (st, got, c) in zip(items, want):
        assert int(cnt.item()) == c
        assert np.array_equal(J.candidates_numpy(out, cnt), got)
        assert np.array_equal(stats.cpu().numpy(), st)


def test_batch_full_size_equals_single_searches():
    """At the batched workload's sizes (2^20, 2^21 + 4321 and 2^22 bins; zmax 100, wmax 300) the
    batched call's candidates and statistics equal the single-spectrum call's, on the narrowest and
    the widest 16-template slabs (k = 4: some 10^5 candidates per spectrum and slab)."""
    import torch
    dev = device()
    plan = J.Plan(1 << 22, 100.0, 300.0, 2.0, 20.0, path="fft")
    bank = build_bank(plan)
    T = plan.info()["n_templates"]
    lengths = [1 << 20, (1 << 21) + 4321, 1 << 22]
    k = 4.0
    specs_np = [_spectrum(n, 400 + i) for i, n in enumerate(lengths)]
    for t0, t1 in ((0, 16), (T - 16, T)):
        rows = t1 - t0
        items, want = [], []
        for x in specs_np:
            n = x.shape[0]
            cap = rows * 2 * n // 50
            want.append(_fused(plan, bank, x, k, 0.9 * (1 + k), t_begin=t0, t_end=t1, capacity=cap))
            items.append((torch.from_numpy(x).to(dev), torch.zeros((cap, 4), dtype=torch.int32, device=dev),
                          torch.zeros(1, dtype=torch.int64, device=dev),
                          torch.empty((rows, 2), dtype=torch.float64, device=dev)))
        plan.batch_search_candidates(bank, items, k, t_begin=t0, t_end=t1)
        torch.cuda.synchronize()
        for (spec, out, cnt, stats), (st, got, c) in zip(items, want):
            print(f"[full-size batch candidates] rows [{t0}, {t1}) nbins {spec.shape[0]}: {c} candidates",
                  flush=True)
            assert 0 < c <= out.shape[0]
            assert int(cnt.item()) == c
            assert np.array_equal(J.candidates_numpy(out, cnt), got)
            assert np.array_equal(stats.cpu().numpy(), st)
        del items
    plan.close()
