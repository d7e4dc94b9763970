"""Host-side tests of the serving scheduler (dry-run mode: no device calls, tiles finish at once)."""

import pytest

import paper_1911_01353_amd as J

FAKE_ARENA = 0x10000000     # never dereferenced in dry-run mode
FAKE_SPEC = 0x20000000


def _server(arena_gb=8.0, **kw):
    return J.Server(FAKE_ARENA, int(arena_gb * (1 << 30)), dry_run=True, **kw)


def test_all_requests_complete_and_banks_are_cached():
    s = _server(max_active=2, queue_capacity=8)
    tickets = [s.submit(FAKE_SPEC, 20, 60, nbins=1 << 18, n_templates=147) for _ in range(5)]
    res = [s.wait(t, 10.0) for t in tickets]
    assert all(r is not None and r["status"] == J.JERK_OK for r in res)
    for r in res:
        assert r["t_submit"] <= r["t_admit"] <= r["t_first_launch"] <= r["t_done"]
        assert r["points"] == 147 * 2 * (1 << 18)
    st = s.stats()
    assert st["completed"] == 5 and st["bank_builds"] == 1 and st["failed"] == 0
    s.close()


def test_queue_full_returns_eagain():
    s = _server(max_active=1, queue_capacity=3)
    s.inject_failure(3, 1)  # hold admission
    tickets = [s.submit(FAKE_SPEC, 20, 60, nbins=4096) for _ in range(3)]
    with pytest.raises(J.JerkError) as ei:
        s.submit(FAKE_SPEC, 20, 60, nbins=4096)
    assert ei.value.status == J.JERK_EAGAIN
    assert s.poll(tickets[0]) is None
    s.inject_failure(3, 0)
    assert all(s.wait(t, 10.0)["status"] == J.JERK_OK for t in tickets)
    s.close()


def test_request_larger_than_arena_is_rejected():
    s = _server(arena_gb=0.05)
    with pytest.raises(J.JerkError) as ei:
        s.submit(FAKE_SPEC, 300, 900, nbins=1 << 23)   # ~0.9 GB template bank
    assert ei.value.status == J.JERK_ENOMEM
    with pytest.raises(J.JerkError) as ei:
        s.submit(FAKE_SPEC, 20, 60, nbins=0)
    assert ei.value.status == J.JERK_EINVAL
    s.close()


def test_admission_waits_for_memory_and_evicts_unused_banks():
    # room for one 200/600 bank at a time: the second grid must wait and evict the first
    p = J.Plan(1 << 20, 200, 600, path="fft")
    bank = p.info()["bank_bytes"]
    s = _server(arena_gb=(bank * 1.5) / (1 << 30), max_active=2)
    a = s.submit(FAKE_SPEC, 200, 600, nbins=1 << 20)
    b = s.submit(FAKE_SPEC, 200, 580, nbins=1 << 20)
    ra, rb = s.wait(a, 10.0), s.wait(b, 10.0)
    assert ra["status"] == rb["status"] == J.JERK_OK
    assert rb["t_admit"] >= ra["t_done"]
    st = s.stats()
    assert st["bank_builds"] == 2 and st["bank_evictions"] == 1
    s.close()


def test_injected_launch_failure_fails_only_its_requests():
    s = _server(max_active=1, queue_capacity=8)
    s.inject_failure(1, 1)      # the next launch fails
    tickets = [s.submit(FAKE_SPEC, 20, 60, nbins=1 << 16) for _ in range(3)]
    res = [s.wait(t, 10.0) for t in tickets]
    assert res[0]["status"] == J.JERK_EHIP
    assert [r["status"] for r in res[1:]] == [J.JERK_OK, J.JERK_OK]
    st = s.stats()
    assert st["failed"] == 1 and st["completed"] == 2
    s.close()


def test_injected_bank_build_failure():
    s = _server(max_active=2)
    s.inject_failure(2, 1)
    bad = s.submit(FAKE_SPEC, 20, 60, nbins=1 << 16)
    assert s.wait(bad, 10.0)["status"] == J.JERK_EHIP
    good = s.submit(FAKE_SPEC, 22, 66, nbins=1 << 16)
    assert s.wait(good, 10.0)["status"] == J.JERK_OK
    # the failed bank is not cached: the same grid builds again and succeeds
    again = s.submit(FAKE_SPEC, 20, 60, nbins=1 << 16)
    assert s.wait(again, 10.0)["status"] == J.JERK_OK
    assert s.stats()["bank_builds"] == 3
    s.close()


def test_bad_descriptors():
    with pytest.raises(J.JerkError):
        J.Server(FAKE_ARENA, 1 << 30, max_active=0, dry_run=True)
    with pytest.raises(J.JerkError):
        J.Server(FAKE_ARENA + 3, 1 << 30, dry_run=True)
    with pytest.raises(J.JerkError):
        J.Server(FAKE_ARENA, 1024, dry_run=True)


def test_requests_in_flight_together_share_launches():
    s = _server(max_active=3, queue_capacity=8)
    s.inject_failure(3, 1)      # hold admission until all three are queued
    tickets = [s.submit(FAKE_SPEC, 20, 60, nbins=1 << 18) for _ in range(3)]
    s.inject_failure(3, 0)
    assert all(s.wait(t, 10.0)["status"] == J.JERK_OK for t in tickets)
    st = s.stats()
    assert st["shared_launches"] >= 1 and st["max_in_flight"] >= 2
    s.close()


def test_top_k_has_k_distinct_templates_in_order():
    s = _server(max_active=1)
    t = s.submit(FAKE_SPEC, 20, 60, nbins=1 << 16, top_k=5)
    r = s.wait(t, 10.0)
    assert r["status"] == J.JERK_OK and r["top_count"] == 5
    # dry run: every row peak has power 0, so ties go to the lowest templates
    assert list(r["top"]["t"]) == [0, 1, 2, 3, 4]
    with pytest.raises(J.JerkError):
        s.submit(FAKE_SPEC, 20, 60, nbins=1 << 16, top_k=-1)
    s.close()


def test_device_error_in_completion_query_fails_in_flight_requests_and_server_recovers():
    """A completion query that reports a device error (as a sticky fault would) ends every request
    with work in flight with EHIP, releases the launch slots and leaves the server running."""
    s = _server(max_active=2, queue_capacity=8)
    s.inject_failure(3, 1)
    s.inject_failure(4, 1 << 30)    # every completion query fails until disarmed
    bad = [s.submit(FAKE_SPEC, 20, 60, nbins=1 << 16) for _ in range(3)]
    s.inject_failure(3, 0)
    res = [s.wait(t, 10.0) for t in bad]
    assert all(r is not None and r["status"] == J.JERK_EHIP for r in res)
    s.inject_failure(4, 0)
    good = s.submit(FAKE_SPEC, 20, 60, nbins=1 << 16)
    r = s.wait(good, 10.0)
    assert r is not None and r["status"] == J.JERK_OK
    st = s.stats()
    assert st["failed"] == 3 and st["completed"] == 1 and st["active"] == 0
    s.close()
