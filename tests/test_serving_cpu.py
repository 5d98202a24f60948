"""Scheduler of the request loop on the CPU, with a fake executor and a fake
clock: continuous batching, admission by device footprint, rejection and
time-out paths, failure isolation, latency percentiles."""
import numpy as np
import pytest

from paper_2506_18150_amd.serving import FakeClock, FakeExecutor, Request, Server

MB = 1 << 20


def mk(n_groups=3, cost=lambda g, b: 0.010 + 0.002 * b, streams=2, budget=1 << 40, max_batch=8, **kw):
    clock = FakeClock()
    ex = FakeExecutor(clock, cost, n_streams=streams, unit_bytes=MB, ws_bytes=lambda g, b: b * MB, **kw)
    return clock, ex, Server(ex, clock, n_groups, budget, max_batch=max_batch)


def req(rid, t, groups):
    return Request(rid=rid, arrival=t, units=[(g, f"ct{rid}_{g}") for g in groups])


def test_all_requests_complete_with_their_results():
    clock, ex, srv = mk()
    reqs = [req(i, 0.001 * i, [i % 3, (i + 1) % 3]) for i in range(20)]
    rep = srv.run(reqs)
    assert rep["completed"] == 20 and rep["rejected"] == 0
    for r in reqs:
        assert set(r.results) == {g for g, _ in r.units}
        for g, payload in r.units:
            assert r.results[g] == ("result", r.rid, g, payload)
        assert r.done_at >= r.arrival


def test_units_of_different_requests_share_batches_and_streams_overlap():
    clock, ex, srv = mk(n_groups=1, streams=2)
    reqs = [req(i, 0.0, [0]) for i in range(16)]
    srv.run(reqs)
    sizes = [b for (_, _, b, _) in ex.launches]
    assert max(sizes) > 1                        # continuous batching across requests
    starts = {}
    for stream, _, _, start in ex.launches:
        starts.setdefault(start, set()).add(stream)
    assert any(len(v) == 2 for v in starts.values())   # both streams busy at once


def test_late_arrivals_join_while_others_run():
    clock, ex, srv = mk(n_groups=1, streams=1, cost=lambda g, b: 0.05)
    reqs = [req(0, 0.0, [0])] + [req(i, 0.01 + 0.001 * i, [0]) for i in range(1, 6)]
    srv.run(reqs)
    # request 0 runs alone; the five later arrivals are admitted during it and go together
    assert [b for (_, _, b, _) in ex.launches] == [1, 5]


def test_admission_by_footprint():
    # capacity for exactly two single-unit requests in flight (2 MB each)
    streams, max_batch = 1, 4
    ws = max_batch * MB
    clock, ex, srv = mk(n_groups=1, streams=streams, max_batch=max_batch, budget=ws + 4 * MB,
                        cost=lambda g, b: 0.1)
    reqs = [req(i, 0.0, [0]) for i in range(3)]
    srv.run(reqs)
    r0, r1, r2 = reqs
    assert r0.admitted_at == 0.0 and r1.admitted_at == 0.0
    assert r2.admitted_at >= min(r0.done_at, r1.done_at)
    assert all(r.done_at is not None for r in reqs)


def test_oversized_request_rejected_at_once():
    clock, ex, srv = mk(n_groups=3, streams=1, max_batch=1, budget=1 * MB + 3 * MB)
    big = req(0, 0.0, [0, 1, 2])                 # needs 6 MB > 3 MB of capacity
    small = req(1, 0.0, [1])
    rep = srv.run([big, small])
    assert big.rejected and not small.rejected
    assert rep["completed"] == 1 and rep["rejected"] == 1


def test_waiting_requests_time_out():
    clock = FakeClock()
    ex = FakeExecutor(clock, lambda g, b: 1.0, n_streams=1, unit_bytes=MB, ws_bytes=lambda g, b: MB)
    srv = Server(ex, clock, 1, hbm_budget=MB + 2 * MB, max_batch=1, admit_timeout=0.5)
    reqs = [req(i, 0.0, [0]) for i in range(3)]
    rep = srv.run(reqs)
    assert rep["completed"] == 1 and rep["rejected"] == 2


def test_failed_batch_fails_only_its_requests():
    fails = {"n": 0}

    def fail(g, b):
        if g == 1 and fails["n"] == 0:
            fails["n"] += 1
            return True
        return False

    clock, ex, srv = mk(n_groups=2, streams=1, fail=fail)
    reqs = [req(0, 0.0, [1]), req(1, 0.0, [0]), req(2, 0.5, [1])]
    rep = srv.run(reqs)
    assert reqs[0].rejected and not reqs[1].rejected and not reqs[2].rejected
    assert rep["failed_batches"] == 1 and rep["completed"] == 2
    assert srv.in_flight == 0


def test_latency_percentiles_with_known_costs():
    # one stream, batch 1, each unit 10 ms, arrivals every 20 ms: no queueing
    clock, ex, srv = mk(n_groups=1, streams=1, max_batch=1, cost=lambda g, b: 0.010)
    reqs = [req(i, 0.020 * i, [0]) for i in range(50)]
    rep = srv.run(reqs)
    assert rep["p50_ms"] == pytest.approx(10.0) and rep["p99_ms"] == pytest.approx(10.0)
    # arrivals every 5 ms: queueing builds up and p99 grows past p50
    clock, ex, srv = mk(n_groups=1, streams=1, max_batch=1, cost=lambda g, b: 0.010)
    rep = srv.run([req(i, 0.005 * i, [0]) for i in range(50)])
    assert rep["p99_ms"] > rep["p50_ms"] > 10.0
    lat = np.array([r.latency for r in srv.completed]) * 1e3
    assert rep["p99_ms"] == pytest.approx(np.percentile(lat, 99))


def test_deadline_cancels_queued_units_and_frees_bytes():
    # one stream, batches of 1, 0.1 s each: request 0 runs first; request 1
    # (deadline 0.05 s) is still queued when its deadline passes and is
    # cancelled without running; request 2 (no deadline) completes
    clock, ex, srv = mk(n_groups=1, streams=1, max_batch=1, cost=lambda g, b: 0.1)
    r0, r1, r2 = req(0, 0.0, [0]), req(1, 0.0, [0]), req(2, 0.0, [0])
    r1.deadline = 0.05
    rep = srv.run([r0, r1, r2])
    assert rep["completed"] == 2 and rep["expired"] == 1 and rep["rejected"] == 0
    assert r1.cancelled == "deadline" and r1.done_at is None and not r1.results
    assert [b for (_, _, b, _) in ex.launches] == [1, 1]     # r1 never launched
    assert srv.in_flight == 0 and not ex.resident           # every admitted byte released
    assert r2.done_at == pytest.approx(0.2)


def test_deadline_while_running_drops_the_result():
    # the request's only unit is already on the device when the deadline
    # passes: it finishes, its result is discarded, the request is expired
    clock, ex, srv = mk(n_groups=1, streams=1, cost=lambda g, b: 0.1)
    r = req(0, 0.0, [0])
    r.deadline = 0.05
    rep = srv.run([r])
    assert rep["completed"] == 0 and rep["expired"] == 1
    assert r.done_at is None and not r.results
    assert srv.in_flight == 0 and not ex.resident


def test_client_cancellation_and_waiting_request_expiry():
    # capacity for one request in flight: request 1 waits for admission; it is
    # cancelled by the client, request 2 expires while waiting
    streams, max_batch = 1, 1
    clock, ex, srv = mk(n_groups=1, streams=streams, max_batch=max_batch, budget=MB + 2 * MB,
                        cost=lambda g, b: 0.1)
    r0, r1, r2 = req(0, 0.0, [0]), req(1, 0.0, [0]), req(2, 0.0, [0])
    r2.deadline = 0.05
    for r in (r0, r1, r2):
        r.remaining = 0
        srv.submit(r)
    srv.step()
    assert r0.admitted_at is not None and r1.admitted_at is None
    assert srv.cancel(1) and not srv.cancel(1)
    clock.sleep_until(0.06)
    srv.step()
    assert r1.cancelled == "client" and r2.cancelled == "deadline"
    while not srv.idle():
        clock.sleep_until(ex.next_done_time() or clock.now() + 0.01)
        srv.step()
    rep = srv.report()
    assert rep["completed"] == 1 and rep["cancelled"] == 1 and rep["expired"] == 1
    assert srv.in_flight == 0 and not ex.resident


def test_admitted_requests_are_resident_until_done():
    clock, ex, srv = mk(n_groups=2, streams=1, cost=lambda g, b: 0.01)
    seen = []
    orig = ex.launch

    def launch(stream, group, units):
        seen.append({u.req.rid for u in units} <= ex.resident)
        return orig(stream, group, units)
    ex.launch = launch
    srv.run([req(i, 0.0, [0, 1]) for i in range(6)])
    assert seen and all(seen) and not ex.resident


def test_mixed_group_batches_take_the_oldest_units_of_any_group():
    clock = FakeClock()
    ex = FakeExecutor(clock, lambda g, b: 0.05, n_streams=1, unit_bytes=MB, ws_bytes=lambda g, b: b * MB)
    srv = Server(ex, clock, 3, 1 << 40, max_batch=4, mix_groups=True)
    reqs = [req(0, 0.0, [0])] + [req(i, 0.01 * i, [i % 3]) for i in range(1, 9)]
    rep = srv.run(reqs)
    assert rep["completed"] == 9
    groups_per_launch = [g for (_, g, _, _) in ex.launches]
    sizes = [b for (_, _, b, _) in ex.launches]
    assert sizes[0] == 1 and max(sizes) == 4            # the first runs alone, later ones fill a batch
    assert -1 in groups_per_launch or len(set(groups_per_launch)) > 1
    for r in reqs:
        assert set(r.results) == {g for g, _ in r.units}
