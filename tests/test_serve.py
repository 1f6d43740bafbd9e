"""Host logic of the continuous-batching server, on a fake engine (CPU)."""
import dataclasses

import numpy as np
import pytest

from paper_1403_4238_amd.serve import FakeClock, FakeEngine, Server, summarize


@dataclasses.dataclass
class J:
    name: str
    arrival_s: float
    iters: int
    nbytes: int
    bad: bool = False


def _server(jobs, budget, capacity, G=1, step_cost=0.001, **kw):
    clock = FakeClock()
    eng = FakeEngine(lambda j: j.iters, lambda j: j.nbytes, clock=clock, step_cost_s=step_cost,
                     fail_on=lambda j: j.bad)
    srv = Server(eng, budget, capacity, G, clock=clock, sleep=clock.sleep, **kw)
    return srv, eng, srv.run(jobs)


def test_all_jobs_complete_with_exact_latency():
    # One job at a time, 1 ms per step, G = 1: a job of n iterations that
    # starts at once finishes n ms after it arrives.
    jobs = [J("a", 0.0, 5, 10), J("b", 0.100, 3, 10)]
    srv, eng, recs = _server(jobs, budget=100, capacity=4)
    assert [r.status for r in recs] == ["done", "done"]
    assert recs[0].latency_s == pytest.approx(0.005)
    assert recs[1].latency_s == pytest.approx(0.003)
    assert eng.released == 2


def test_admission_by_memory_budget():
    jobs = [J(f"j{i}", 0.0, 10, 40) for i in range(6)]
    srv, eng, recs = _server(jobs, budget=100, capacity=8)
    assert all(r.status == "done" for r in recs)
    assert eng.max_live == 2            # 2 x 40 bytes fit in 100, a third does not
    assert srv.peak_used <= 100


def test_admission_by_slots():
    jobs = [J(f"j{i}", 0.0, 4, 1) for i in range(7)]
    srv, eng, recs = _server(jobs, budget=1 << 30, capacity=3)
    assert eng.max_live == 3 and all(r.status == "done" for r in recs)


def test_continuous_batching_admits_while_others_run():
    # A long job is running; a short job arriving later is admitted next to it
    # and finishes first.
    jobs = [J("long", 0.0, 200, 10), J("short", 0.010, 5, 10)]
    srv, eng, recs = _server(jobs, budget=100, capacity=2)
    long, short = recs
    assert short.admit_s < long.done_s
    assert short.done_s < long.done_s
    assert eng.max_live == 2


def test_fifo_order_under_memory_pressure():
    # A big job at the head of the queue is not overtaken by smaller ones.
    jobs = [J("a", 0.0, 50, 60), J("big", 0.001, 5, 80), J("small", 0.002, 5, 10)]
    srv, eng, recs = _server(jobs, budget=100, capacity=4)
    a, big, small = recs
    assert big.admit_s >= a.done_s - 1e-12
    assert small.admit_s >= big.admit_s


def test_rejects_jobs_larger_than_the_budget_and_isolates_failures():
    jobs = [J("ok1", 0.0, 3, 10), J("huge", 0.0, 3, 1000), J("bad", 0.0, 3, 10, bad=True), J("ok2", 0.0, 3, 10)]
    srv, eng, recs = _server(jobs, budget=100, capacity=4)
    assert [r.status for r in recs] == ["done", "rejected", "failed", "done"]
    s = summarize(recs)
    assert s["completed"] == 2 and s["rejected"] == 1 and s["failed"] == 1
    assert srv.used == 0


def test_percentiles_and_throughput():
    rng = np.random.default_rng(0)
    t, jobs = 0.0, []
    for i in range(200):
        t += float(rng.exponential(0.01))
        jobs.append(J(f"j{i}", t, int(rng.integers(1, 30)), int(rng.integers(1, 20))))
    srv, eng, recs = _server(jobs, budget=60, capacity=8, G=2, step_cost=0.0005)
    s = summarize(recs)
    lat = np.array([r.latency_s for r in recs])
    assert s["completed"] == 200
    assert s["p50_latency_ms"] == pytest.approx(1000 * np.percentile(lat, 50), rel=1e-6, abs=1e-3)
    assert s["p99_latency_ms"] == pytest.approx(1000 * np.percentile(lat, 99), rel=1e-6, abs=1e-3)
    assert s["p99_latency_ms"] >= s["p50_latency_ms"] > 0
    assert s["jobs_per_s"] == pytest.approx(200 / s["span_s"], rel=1e-3)
    assert srv.peak_used <= 60 and eng.max_live <= 8
    # every job needed exactly its scripted iterations
    assert all(r.iterations == j.iters for r, j in zip(recs, jobs))


def test_idle_gaps_are_waited_out():
    jobs = [J("a", 0.0, 2, 1), J("b", 5.0, 2, 1)]
    srv, eng, recs = _server(jobs, budget=10, capacity=2)
    assert recs[1].admit_s >= 5.0
    assert recs[1].latency_s == pytest.approx(0.002)


def test_bad_configuration():
    with pytest.raises(ValueError):
        Server(FakeEngine(lambda j: 1, lambda j: 1), budget_bytes=0, capacity=1)
    with pytest.raises(ValueError):
        Server(FakeEngine(lambda j: 1, lambda j: 1), budget_bytes=10, capacity=0)


def test_async_admission_matches_sync():
    # Contexts prepared on worker threads join between steps: every job
    # completes with its scripted iterations, the limits hold, and an invalid
    # job fails alone, as with admission on the loop.
    rng = np.random.default_rng(1)
    t, jobs = 0.0, []
    for i in range(60):
        t += float(rng.exponential(0.005))
        jobs.append(J(f"j{i}", t, int(rng.integers(1, 40)), int(rng.integers(1, 20)), bad=(i == 7)))
    out = {}
    for workers in (0, 2):
        srv, eng, recs = _server(jobs, budget=50, capacity=6, G=3, workers=workers)
        assert [r.status for r in recs].count("failed") == 1 and recs[7].status == "failed"
        assert all(r.status == "done" for k, r in enumerate(recs) if k != 7)
        assert all(r.iterations == j.iters for k, (r, j) in enumerate(zip(recs, jobs)) if k != 7)
        assert srv.peak_used <= 50 and eng.max_live <= 6 and srv.used == 0
        out[workers] = [r.iterations for r in recs]
    assert out[0] == out[2]


def test_async_admission_counts_preparing_jobs_against_the_limits():
    jobs = [J(f"j{i}", 0.0, 5, 30) for i in range(5)]
    srv, eng, recs = _server(jobs, budget=100, capacity=4, workers=3)
    assert all(r.status == "done" for r in recs)
    assert eng.max_live <= 3          # 3 x 30 bytes fit in 100, a fourth does not
    assert srv.peak_used <= 100


def _room_server(jobs, limit, workers=0, capacity=8):
    # room: the running jobs' "tiles" (J.nbytes here) plus the new job's fit
    # under `limit`; every attach is recorded with the tiles then running
    clock = FakeClock()
    attached = []
    eng = FakeEngine(lambda j: j.iters, lambda j: 1, clock=clock, step_cost_s=0.001,
                     room=lambda running, j: sum(r.nbytes for r in running) + j.nbytes <= limit)
    attach = eng.attach

    def spy(job):
        attached.append((job.name, sum(st[0].nbytes for st in eng.live.values())))
        return attach(job)
    eng.attach = spy
    srv = Server(eng, 1 << 30, capacity, 1, clock=clock, sleep=clock.sleep, workers=workers)
    return attached, srv.run(jobs)


def test_attach_waits_for_room_in_arrival_order():
    # tiles 6, 3, 5, 2 under a limit of 10: "c" (5) does not fit beside "a"
    # and "b" (9), so it waits for room and "d", which would fit, waits
    # behind it; a job larger than the limit starts alone.  (Synchronous
    # preparation, so the attach times are exact.)
    jobs = [J("a", 0.0, 20, 6), J("b", 0.0, 30, 3), J("c", 0.0, 10, 5), J("d", 0.0, 5, 2),
            J("e", 0.001, 5, 12)]
    attached, recs = _room_server(jobs, 10, 0)
    assert all(r.status == "done" for r in recs)
    assert [a[0] for a in attached] == ["a", "b", "c", "d", "e"]
    limits = dict(attached)
    assert limits["a"] == 0 and limits["b"] == 6
    assert limits["c"] + 5 <= 10 and limits["d"] + 2 <= 10
    assert limits["e"] == 0          # too large for any room: runs once the batch is empty
    assert recs[2].admit_s >= recs[0].done_s - 1e-12   # "c" started only after "a" left


def test_room_never_exceeded_with_several_running():
    rng = np.random.default_rng(3)
    jobs = [J(f"j{i}", float(i) * 0.002, int(rng.integers(1, 40)), int(rng.integers(1, 9))) for i in range(40)]
    attached, recs = _room_server(jobs, 12, workers=1)
    assert all(r.status == "done" for r in recs)
    assert [a[0] for a in attached] == [j.name for j in jobs]   # arrival order
    for (name, running), j in zip(attached, jobs):
        assert running == 0 or running + j.nbytes <= 12, name
