"""GPU parity of candidate selection (row statistics, threshold, peaks) against the oracle.

Both sides read the same FP32 plane. Statistics: mean and sigma within 1e-12
relative (FP64 sums of FP32 values in different orders). Candidates: the (t, p)
sets must be equal except for points whose power lies within 1e-9 sigma of the
threshold (there the two FP64 thresholds may fall on either side), powers
bit-equal, significance within FP32 rounding.
"""

import numpy as np
import pytest

import paper_1911_01353_amd as J
import synth
from oracle.candidates import find_candidates, row_statistics

from gpu_helpers import build_bank, device

pytestmark = pytest.mark.gpu


def _run(plane_np, k, ld=None, capacity=None, row_template=None, t_base=0, pad_value=1e30):
    import torch
    dev = device()
    rows, n_r = plane_np.shape
    ld = ld or n_r
    buf = torch.full((rows, ld), pad_value, dtype=torch.float32, device=dev)
    buf[:, :n_r] = torch.from_numpy(np.ascontiguousarray(plane_np, dtype=np.float32)).to(dev)
    stats = torch.full((rows, 2), float("nan"), dtype=torch.float64, device=dev)
    J.plane_stats(buf, stats, n_r=n_r)
    cap = capacity if capacity is not None else max(16, rows * n_r // 2)
    out = torch.zeros((cap, 4), dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    rt = None if row_template is None else torch.tensor(row_template, dtype=torch.int32, device=dev)
    J.find_candidates(buf, stats, k, out, count, n_r=n_r, row_template=rt, t_base=t_base)
    torch.cuda.synchronize()
    return stats.cpu().numpy(), J.candidates_numpy(out, count), int(count.item())


def _check_stats(got, plane):
    want = row_statistics(plane)
    scale = np.maximum(np.abs(want[:, 0]), 1e-30)
    assert np.all(np.abs(got[:, 0] - want[:, 0]) <= 1e-12 * scale)
    assert np.all(np.abs(got[:, 1] - want[:, 1]) <= 1e-12 * np.maximum(want[:, 1], 1e-30))


def _check_candidates(got, plane, k, row_template=None):
    rows = plane.shape[0]
    tmpl = np.arange(rows) if row_template is None else np.asarray(row_template)
    row_of = {int(t): i for i, t in enumerate(tmpl)}
    want = find_candidates(plane, k, row_template=tmpl)
    st = row_statistics(plane)
    g = {(int(r["t"]), int(r["p"])): r for r in got}
    w = {(int(r["t"]), int(r["p"])): r for r in want}
    assert len(g) == len(got), "a candidate was stored twice"
    for t, p in set(g) ^ set(w):
        i = row_of[t]
        thr = st[i, 0] + k * st[i, 1]
        assert abs(float(plane[i, p]) - thr) <= 1e-9 * st[i, 1], ("candidate mismatch", t, p)
    for key in set(g) & set(w):
        assert g[key]["power"] == w[key]["power"]
        assert abs(float(g[key]["sigma"]) - w[key]["sigma"]) <= 1e-6 * max(1.0, abs(w[key]["sigma"]))
    return len(w)


def _noise_plane(rows, n_r, seed):
    rng = np.random.default_rng(seed)
    return rng.exponential(1.0, size=(rows, n_r)).astype(np.float32)


@pytest.mark.parametrize("n_r,ld", [(1, 1), (2, 8), (1023, 1023), (1025, 1100), (5037, 5040), (70001, 70001)])
def test_ragged_rows_and_padding(n_r, ld):
    plane = _noise_plane(5, n_r, n_r)
    if n_r >= 8:
        plane[1, 3:7] = 40.0           # plateau: one candidate at its left end
        plane[2, 0] = 50.0             # peak at the first point
        plane[3, n_r - 1] = 50.0       # peak at the last point
    for k in (0.0, 2.5):
        stats, got, count = _run(plane, k, ld=ld)
        _check_stats(stats, plane)
        _check_candidates(got, plane, k)
        assert count == len(got)
    if n_r >= 8:
        keys = {(int(r["t"]), int(r["p"])) for r in got}
        assert {(1, 3), (2, 0), (3, n_r - 1)} <= keys and (1, 4) not in keys


def test_constant_and_spike_rows():
    n = 4096
    plane = np.full((3, n), 0.75, dtype=np.float32)
    plane[1] = 0.0
    plane[1, 1234] = 7.0
    plane[2, :] = np.float32(1e-3) * np.arange(n, dtype=np.float32) % 5
    stats, got, _ = _run(plane, 1.0)
    assert stats[0, 0] == np.float32(0.75) and stats[0, 1] == 0.0
    assert abs(stats[1, 1] - 7.0 * np.sqrt(n - 1) / n) <= 1e-13 * 7.0
    assert not np.any(got["t"] == 0)
    assert [(int(r["t"]), int(r["p"])) for r in got if r["t"] == 1] == [(1, 1234)]
    _check_candidates(got, plane, 1.0)


def test_many_rows_and_template_mapping():
    rows = 70000                        # more rows than one grid dimension holds
    plane = _noise_plane(rows, 16, 11)
    tmpl = (np.arange(rows) * 7 + 3) % 100003
    stats, got, _ = _run(plane, 2.0, row_template=tmpl)
    _check_stats(stats, plane)
    _check_candidates(got, plane, 2.0, row_template=tmpl)
    stats2, got2, _ = _run(plane[:50], 2.0, t_base=1000)
    _check_candidates(got2, plane[:50], 2.0, row_template=np.arange(1000, 1050))


def test_capacity_overflow_and_accumulation():
    import torch
    dev = device()
    plane = _noise_plane(4, 20000, 5)
    want = find_candidates(plane, 0.5)
    buf = torch.from_numpy(plane).to(dev)
    stats = torch.empty((4, 2), dtype=torch.float64, device=dev)
    J.plane_stats(buf, stats)
    cap = 100
    out = torch.zeros((cap, 4), dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    J.find_candidates(buf[:2], stats[:2], 0.5, out, count)
    J.find_candidates(buf[2:], stats[2:], 0.5, out, count, t_base=2)
    torch.cuda.synchronize()
    assert abs(int(count.item()) - len(want)) <= 2 and len(want) > cap
    got = J.candidates_numpy(out, count)
    assert len(got) == cap
    wk = {(int(r["t"]), int(r["p"])) for r in want}
    st = row_statistics(plane)
    for r in got:
        t, p = int(r["t"]), int(r["p"])
        assert (t, p) in wk or abs(float(plane[t, p]) - (st[t, 0] + 0.5 * st[t, 1])) <= 1e-9 * st[t, 1]


def test_search_plane_2e15_bins_finds_the_tone(small_spectrum):
    """Candidates of the GPU's own plane of the 2^15-bin search; the tone is among them."""
    import torch
    dev = device()
    cfg = synth.CONFIGS["bins2e15_z20_w60"]
    n = small_spectrum.shape[0]
    plan = J.Plan(n, cfg.zmax, cfg.wmax, cfg.dz, cfg.dw, path="fft")
    bank = build_bank(plan)
    T = plan.info()["n_templates"]
    plane = torch.empty((T, 2 * n), dtype=torch.float32, device=dev)
    plan.search(bank, torch.from_numpy(small_spectrum).to(dev), plane, 0, T)
    torch.cuda.synchronize()
    host = plane.cpu().numpy()
    stats, got, _ = _run(host, 6.0)
    _check_stats(stats, host)
    _check_candidates(got, host, 6.0)
    best = got[np.argmax(got["power"])]
    assert (int(best["t"]), int(best["p"])) == (102, 16013)
    assert best["sigma"] > 20


def test_full_size_slab_2e22_bins():
    """A 32-row member slab of the 2^22-bin search: statistics and candidates of sampled rows."""
    import torch
    dev = device()
    cfg = synth.CONFIGS["bins2e22_z200_w600"]
    spec = synth.make_spectrum(cfg)
    n = spec.shape[0]
    plan = J.Plan(n, cfg.zmax, cfg.wmax, cfg.dz, cfg.dw, path="fft")
    bank = build_bank(plan)
    g = len(plan.groups()) // 2
    gi = plan.group(g)
    m = min(32, gi["n_members"])
    members = plan.members()[gi["first_member"]: gi["first_member"] + m]
    slab = torch.empty((m, 2 * n), dtype=torch.float32, device=dev)
    plan.search_members(bank, torch.from_numpy(spec).to(dev), slab, g, 0, m)
    stats = torch.empty((m, 2), dtype=torch.float64, device=dev)
    J.plane_stats(slab, stats)
    out = torch.zeros((1 << 20, 4), dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    J.find_candidates(slab, stats, 5.0, out, count,
                      row_template=torch.tensor(members, dtype=torch.int32, device=dev))
    torch.cuda.synchronize()
    assert int(count.item()) <= out.shape[0]
    got = J.candidates_numpy(out, count)
    st = stats.cpu().numpy()
    for i in (0, m // 2, m - 1):
        row = slab[i: i + 1].cpu().numpy()
        _check_stats(st[i: i + 1], row)
        sub = got[got["t"] == members[i]]
        _check_candidates(sub, row, 5.0, row_template=[members[i]])
