"""Serving on the GPU: jobs arriving while others run share batch steps, and
each job's result is exactly its result alone (and the oracle's)."""
import numpy as np
import pytest

import oracle
from paper_1403_4238_amd import synth

from _util import assert_logs_equal

pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_1403_4238_amd.binding")
serve = pytest.importorskip("paper_1403_4238_amd.serve")


def _jobs(n=10, rate=400.0, seed=9):
    rng = np.random.default_rng(seed)
    t, jobs = 0.0, []
    for i in range(n):
        t += float(rng.exponential(1.0 / rate))
        W, H = int(rng.integers(40, 140)), int(rng.integers(40, 110))
        r = int(rng.choice([3, 4, 5]))
        rgb = rng.integers(0, 256, size=(H, W, 3)).astype(np.uint8)
        mask = np.zeros((H, W), np.uint8)
        y0, x0 = int(rng.integers(r + 2, H // 2)), int(rng.integers(r + 2, W // 2))
        mask[y0:y0 + H // 5, x0:x0 + W // 6] = 1
        jobs.append(synth.Job(f"s{i}-{W}x{H}-r{r}", rgb, mask, r, arrival_s=t))
    return jobs


@pytest.mark.parametrize("capacity,budget_jobs,workers,path,form,tpg", [(4, 3, 0, "simt", "persistent", 0),
                                                                        (16, 16, 0, "mfma", "persistent", 0),
                                                                        (4, 3, 2, "mfma", "persistent", 1),
                                                                        (6, 6, 1, "mfma", "graph", 0)])
def test_served_results_equal_alone_and_oracle(capacity, budget_jobs, workers, path, form, tpg):
    jobs = _jobs()
    eng = serve.GpuEngine(capacity=capacity, graph_iters=6, autotune=False, path=path, form=form,
                          tiles_per_group=tpg)
    budget = budget_jobs * max(eng.footprint(j) for j in jobs)
    srv = serve.Server(eng, budget, capacity, graph_iters=6, workers=workers)
    recs = srv.run(jobs)
    assert all(r.status == "done" for r in recs), [(r.name, r.status, r.error) for r in recs]
    assert srv.peak_active <= capacity and srv.peak_used <= budget
    s = serve.summarize(recs)
    assert s["completed"] == len(jobs) and s["p99_latency_ms"] >= s["p50_latency_ms"]
    for j, r in zip(jobs, recs):
        o = oracle.Oracle(j.rgb, j.mask, j.patch_radius)
        want = o.run()
        assert_logs_equal(r.result["log"], want, j.name)
        assert (r.result["image"] == o.read()[0]).all(), j.name
        alone = B.Inpainter(j.rgb, j.mask, j.patch_radius)
        _, n, log = alone.run(log_cap=len(want))
        assert_logs_equal(log, r.result["log"], j.name + " alone")
    if capacity == 4:
        assert srv.peak_active >= 2      # jobs did overlap on the device


def test_batch_room_counts_resident_tiles():
    # A 1080p 9x9 image has 510 MFMA search tiles: alone it keeps every tile
    # resident, a second one beside it does not (unless two tiles may share
    # a search work-group).
    hd = synth.hd()
    small = synth.small()
    batch = B.Batch(capacity=4, graph_iters=8, form="persistent")
    a = B.Inpainter(hd.rgb, hd.mask, hd.patch_radius, path=B.PATH_MFMA)
    b = B.Inpainter(hd.rgb, hd.mask, hd.patch_radius, path=B.PATH_MFMA)
    c = B.Inpainter(small.rgb, small.mask, small.patch_radius, path=B.PATH_MFMA)
    assert batch.room(a) and batch.room(c)
    batch.attach(a)
    batch.step(1)
    assert not batch.room(b)
    assert batch.room(b, tiles_per_group=2)
    with pytest.raises(B.InpaintError):
        batch.room(a)   # already attached
    with pytest.raises(B.InpaintError):
        batch.room(b, tiles_per_group=0)
    for x in (a, b, c):
        x.close()
    batch.close()


def test_invalid_job_is_isolated():
    jobs = _jobs(4)
    bad = synth.Job("bad", jobs[0].rgb, np.zeros_like(jobs[0].mask), 3, arrival_s=jobs[1].arrival_s)
    jobs.insert(2, bad)
    eng = serve.GpuEngine(capacity=4, graph_iters=4, autotune=False)
    srv = serve.Server(eng, 1 << 32, 4, graph_iters=4)
    recs = srv.run(jobs)
    assert [r.status for r in recs].count("failed") == 1 and recs[2].status == "failed"
    assert all(r.status == "done" for k, r in enumerate(recs) if k != 2)


def test_serving_workload_full_size():
    # The seeded serving workload at its stated size: 128 Poisson arrivals
    # (20 jobs/s), images 256x256 .. 2048x1536, holes 1-10% in 1-3 blobs,
    # patches 7/9/11, full search, 16 slots under a 4 GiB workspace budget.
    # The first 16 jobs equal their stored oracle results; every served job
    # equals the same job run alone.
    import hashlib
    from _util import assert_matches_golden, load_golden, log_sha256
    jobs = synth.serving()
    golds = [load_golden(f"serve{i:02d}") for i in range(16)]
    assert all(g is not None for g in golds), "stored oracle results missing"
    eng = serve.GpuEngine(capacity=16, graph_iters=16, autotune=True)
    srv = serve.Server(eng, 4 << 30, 16, graph_iters=16, workers=1)
    recs = srv.run(jobs)
    assert all(r.status == "done" for r in recs), [(r.name, r.status, r.error) for r in recs if r.status != "done"]
    assert srv.peak_active >= 2 and srv.peak_used <= 4 << 30
    s = serve.summarize(recs)
    assert s["completed"] == len(jobs) and s["p99_latency_ms"] >= s["p50_latency_ms"] > 0
    for j, g, r in zip(jobs, golds, recs):
        assert g["input_sha256"] == j.sha256(), j.name
        assert_matches_golden(g, r.result["log"], r.result["image"], j.name)
    for j, r in zip(jobs, recs):
        alone = B.Inpainter(j.rgb, j.mask, j.patch_radius, log_capacity=int(j.mask.sum()), form="persistent",
                            iters_per_check=256, path=B.PATH_MFMA if j.patch_radius <= 6 else B.PATH_SIMT)
        st, n, log = alone.run(log_cap=int(j.mask.sum()))
        assert st == B.DONE and n == len(r.result["log"]), j.name
        assert log_sha256(log) == log_sha256(r.result["log"]), j.name + ": log differs from the job alone"
        assert hashlib.sha256(alone.read_image().tobytes()).digest() == \
            hashlib.sha256(r.result["image"].tobytes()).digest(), j.name + ": image differs from the job alone"
        alone.close()
