"""Scheduling logic of the continuous-batching server, on the CPU with a
simulated executor (no GPU)."""
import types

import pytest

from paper_2205_14330_amd.serving import Request, Server, SimulatedExecutor, latency_stats


class Cam:
    def __init__(self, w, h):
        self.width, self.height = w, h


def _req(i, t, w=256, h=256, scene=0):
    return Request(i, scene, Cam(w, h), t)


def _drive(server, reqs, dt=1e-4, t_end=10.0):
    """Feeds requests at their arrival times and steps the server on a manual clock."""
    t, i = 0.0, 0
    reqs = sorted(reqs, key=lambda r: r.arrival)
    while t < t_end:
        while i < len(reqs) and reqs[i].arrival <= t:
            server.submit(reqs[i])
            i += 1
        server.step(t)
        if i == len(reqs) and server.idle():
            break
        t += dt
    return server.finished


def test_all_requests_complete_fifo_and_bounded_batches():
    ex = SimulatedExecutor(n_slots=2, fixed=0.001, per_pixel=2e-9)
    srv = Server(ex, hbm_budget=1 << 40, max_views=8)
    reqs = [_req(i, 0.0001 * i) for i in range(100)]
    done = _drive(srv, reqs)
    assert len(done) == 100 and all(r.error is None for r in done)
    assert all(r.latency >= 0 for r in done)
    assert max(srv.batches) <= 8
    order = [rid for _, rids in ex.launched for rid in rids]
    assert order == sorted(order)                    # FIFO admission


def test_requests_arriving_during_a_batch_join_the_next_one():
    ex = SimulatedExecutor(n_slots=1, fixed=0.01, per_pixel=0.0)
    srv = Server(ex, hbm_budget=1 << 40, max_views=64)
    reqs = [_req(0, 0.0)] + [_req(i, 0.001 * i) for i in range(1, 6)]
    _drive(srv, reqs)
    assert srv.batches[0] == 1 and srv.batches[1] == 5
    assert len(ex.launched) == 2


def test_two_slots_overlap():
    ex = SimulatedExecutor(n_slots=2, fixed=0.01, per_pixel=0.0)
    srv = Server(ex, hbm_budget=1 << 40, max_views=1)
    _drive(srv, [_req(0, 0.0), _req(1, 0.0005)])
    t0, t1 = ex.launched[0][0], ex.launched[1][0]
    assert t1 - t0 < 0.005                           # second batch started while the first ran


def test_admission_respects_the_memory_budget():
    ex = SimulatedExecutor(n_slots=4, fixed=0.005, per_pixel=0.0, bytes_per_pixel=16)
    one = 16 * 256 * 256
    srv = Server(ex, hbm_budget=3 * one, max_views=64)
    reqs = [_req(i, 0.0) for i in range(20)]
    done = _drive(srv, reqs)
    assert len(done) == 20
    assert srv.peak_in_use <= 3 * one
    assert max(srv.batches) <= 3


def test_oversized_request_runs_alone_instead_of_deadlocking():
    ex = SimulatedExecutor(n_slots=2, fixed=0.001, per_pixel=0.0, bytes_per_pixel=16)
    srv = Server(ex, hbm_budget=1000, max_views=4)
    done = _drive(srv, [_req(0, 0.0, 512, 512), _req(1, 0.0)])
    assert len(done) == 2 and all(r.error is None for r in done)


def test_failed_launch_frees_the_slot_and_memory_and_others_complete():
    ex = SimulatedExecutor(n_slots=1, fixed=0.001, per_pixel=0.0, fail_scene=7)
    srv = Server(ex, hbm_budget=1 << 40, max_views=1)
    reqs = [_req(0, 0.0), _req(1, 0.0, scene=7), _req(2, 0.0)]
    done = _drive(srv, reqs)
    byid = {r.rid: r for r in done}
    assert byid[1].error and byid[0].error is None and byid[2].error is None
    assert srv.in_use == 0 and not srv.inflight


def test_latency_stats():
    reqs = [_req(i, 0.0) for i in range(10)]
    for i, r in enumerate(reqs):
        r.done = 0.001 * (i + 1)
    st = latency_stats(reqs, wall=1.0)
    assert st["requests"] == 10 and st["failed"] == 0
    assert abs(st["p50_ms"] - 5.5) < 1e-9 and st["max_ms"] == pytest.approx(10.0)
    assert st["served_mpix_s"] == pytest.approx(10 * 256 * 256 / 1e6)
