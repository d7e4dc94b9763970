"""GPU tests of the serving loop: results alone equal results in a mix, and equal jerk_search."""

import numpy as np
import pytest

import paper_1911_01353_amd as J
from oracle import Grid, oracle_plane

from gpu_helpers import build_bank, device, gpu_plane

pytestmark = pytest.mark.gpu


def _spec(n, seed, tone_bin=None):
    rng = np.random.default_rng(seed)
    x = ((rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2)).astype(np.complex64)
    if tone_bin is not None:
        x[tone_bin] += 12.0
    return x


def _row_peaks(plane):
    idx = np.argmax(plane, axis=1)
    return plane[np.arange(plane.shape[0]), idx], idx


REQS = [  # (nbins, zmax, wmax, path, seed)
    (1 << 16, 20.0, 60.0, "fft", 1),
    (1 << 17, 30.0, 90.0, "fft", 2),
    (1 << 15, 20.0, 60.0, "split_bf16", 3),
    (100000, 40.0, 120.0, "fft", 4),
]


@pytest.fixture(scope="module")
def server():
    import torch
    device()
    arena = torch.empty(4 << 30, dtype=torch.uint8, device="cuda")
    srv = J.Server(arena, max_active=3, queue_capacity=32, tiles_per_launch=4096)
    yield srv
    srv.close()


def _submit(srv, specs, idx, top_k=0):
    out = []
    for i in idx:
        n, zm, wm, path, _ = REQS[i]
        T = Grid(zm, wm, 2.0, 20.0).n_templates
        out.append(srv.submit(specs[i], zm, wm, path=path, n_templates=T, top_k=top_k))
    return out


def _top_from_peaks(power, p, k):
    order = sorted(range(power.shape[0]), key=lambda t: (-float(power[t]), t))[:k]
    return [(t, int(p[t]), float(power[t])) for t in order]


def test_results_alone_equal_results_in_mix(server):
    import torch
    specs = [torch.from_numpy(_spec(n, seed, tone_bin=n // 3)).cuda() for n, _, _, _, seed in REQS]
    alone = []
    for i in range(len(REQS)):
        (t,) = _submit(server, specs, [i])
        r = server.wait(t, 120.0)
        assert r is not None and r["status"] == J.JERK_OK
        alone.append(r)
    # all at once, twice over, in an interleaved order: admission is held until every request
    # is queued, so the first three are admitted together and the rest as slots free up
    order = [0, 1, 2, 3, 2, 0, 3, 1]
    st0 = server.stats()
    server.inject_failure(3, 1)
    tickets = _submit(server, specs, order, top_k=8)
    server.inject_failure(3, 0)
    mixed = [server.wait(t, 120.0) for t in tickets]
    st1 = server.stats()
    # the requests' work overlapped on the device: launches carried units of several requests,
    # and pairs of requests were in flight together (each started before the other finished)
    assert st1["shared_launches"] > st0["shared_launches"], (st0, st1)
    assert st1["max_in_flight"] >= 2
    overlap = sum(1 for a in mixed for b in mixed if a is not b and a["t_first_launch"] < b["t_done"]
                  and b["t_first_launch"] < a["t_done"])
    print(f"[serve mix] shared launches {st1['shared_launches'] - st0['shared_launches']} of "
          f"{st1['launches'] - st0['launches']}, overlapping pairs {overlap // 2}", flush=True)
    assert overlap > 0
    for i, r in zip(order, mixed):
        want = _top_from_peaks(r["peaks_power"], r["peaks_p"], 8)
        assert r["top_count"] == 8
        assert [(int(e["t"]), int(e["p"]), float(e["power"])) for e in r["top"]] == want
        assert (int(r["top"][0]["t"]), int(r["top"][0]["p"])) == (r["best_t"], r["best_p"])
        assert r["status"] == J.JERK_OK
        a = alone[i]
        assert np.array_equal(r["peaks_power"].view(np.uint32), a["peaks_power"].view(np.uint32))
        assert np.array_equal(r["peaks_p"], a["peaks_p"])
        assert (r["best_t"], r["best_p"], r["best_power"]) == (a["best_t"], a["best_p"], a["best_power"])
        assert r["t_submit"] <= r["t_admit"] <= r["t_first_launch"] <= r["t_done"]
    st = server.stats()
    assert st["failed"] == 0 and st["completed"] >= len(REQS) + len(order)


@pytest.mark.parametrize("i", [0, 2])
def test_results_equal_search_plane_peaks(server, i):
    import torch
    n, zm, wm, path, seed = REQS[i]
    spec_np = _spec(n, seed, tone_bin=n // 3)
    spec = torch.from_numpy(spec_np).cuda()
    (t,) = _submit(server, [spec if k == i else None for k in range(len(REQS))], [i])
    r = server.wait(t, 120.0)
    plan = J.Plan(n, zm, wm, 2.0, 20.0, path=path)
    plane = gpu_plane(plan, build_bank(plan), spec_np)
    hp, hi = _row_peaks(plane)
    assert np.array_equal(r["peaks_power"], hp) and np.array_equal(r["peaks_p"], hi)
    # and against the FP64 oracle around the injected bin
    grid = Grid(zm, wm, 2.0, 20.0)
    p0 = 2 * (n // 3) - 100
    ora = oracle_plane(spec_np, grid, p_lo=p0, p_hi=p0 + 200)
    t_or, p_or = divmod(int(np.argmax(ora)), ora.shape[1])
    assert (r["best_t"], r["best_p"]) == (t_or, p0 + p_or)
    assert abs(r["best_power"] - ora.max()) <= 1e-4 * ora.max()


def test_plane_mode_writes_the_plane(server):
    import torch
    n, zm, wm = 20000, 20.0, 60.0
    spec_np = _spec(n, 9)
    spec = torch.from_numpy(spec_np).cuda()
    T = Grid(zm, wm, 2.0, 20.0).n_templates
    plane = torch.full((T, 2 * n), float("nan"), dtype=torch.float32, device="cuda")
    t = server.submit(spec, zm, wm, path="fft", plane=plane, n_templates=T)
    assert server.wait(t, 60.0)["status"] == J.JERK_OK
    p = J.Plan(n, zm, wm, 2.0, 20.0, path="fft")
    ref = gpu_plane(p, build_bank(p), spec_np)
    assert np.array_equal(plane.cpu().numpy().view(np.uint32), ref.view(np.uint32))


def test_injected_failure_spares_other_requests(server):
    import torch
    specs = [torch.from_numpy(_spec(n, seed)).cuda() for n, _, _, _, seed in REQS]
    server.inject_failure(3, 1)       # hold admission so the failing launch is the next one
    tickets = _submit(server, specs, [0, 1])
    server.inject_failure(1, 1)
    server.inject_failure(3, 0)
    res = [server.wait(t, 120.0) for t in tickets]
    assert any(r["status"] == J.JERK_EHIP for r in res)
    server.inject_failure(1, 0)
    (t,) = _submit(server, specs, [3])
    assert server.wait(t, 120.0)["status"] == J.JERK_OK


def test_full_size_request_equals_search_peaks(server):
    """A 2^22-bin request (zmax 100, wmax 300: 3131 templates, 2.6e10 points, the large end of the
    served mix) returns the per-row peaks of jerk_search_peaks with the same plan, bit for bit, and
    its best point is the largest of them."""
    import torch
    n, zm, wm = 1 << 22, 100.0, 300.0
    spec_np = _spec(n, 5, tone_bin=n // 3)
    spec = torch.from_numpy(spec_np).cuda()
    T = Grid(zm, wm, 2.0, 20.0).n_templates
    t = server.submit(spec, zm, wm, path="fft", n_templates=T)
    r = server.wait(t, 300.0)
    assert r is not None and r["status"] == J.JERK_OK
    plan = J.Plan(n, zm, wm, 2.0, 20.0, path="fft")
    bank = build_bank(plan)
    pk = J.peaks_numpy(plan.search_peaks(bank, spec))
    print(f"[full-size request] {T} rows, best {r['best_power']:.2f} at ({r['best_t']}, {r['best_p']})", flush=True)
    assert np.array_equal(r["peaks_power"].view(np.uint32), pk["power"].view(np.uint32))
    assert np.array_equal(r["peaks_p"], pk["p"])
    assert r["best_power"] == pk["power"].max()
    assert pk["power"][r["best_t"]] == r["best_power"] and pk["p"][r["best_t"]] == r["best_p"]
    plan.close()
