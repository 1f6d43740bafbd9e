"""The batched persistent form (many images per iteration, hipGraph replay,
autotuned tiles) gives each image exactly its single-image result."""
import os

import numpy as np
import pytest

import oracle
from paper_1403_4238_amd import synth

from _util import assert_logs_equal

pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_1403_4238_amd.binding")


def _mixed_jobs():
    jobs = []
    for seed, (W, H, r) in enumerate([(64, 48, 2), (90, 70, 4), (50, 61, 3), (128, 40, 4), (33, 33, 1),
                                      (77, 90, 4)]):
        rng = np.random.default_rng(200 + seed)
        rgb = rng.integers(0, 256, size=(H, W, 3)).astype(np.uint8)
        mask = np.zeros((H, W), np.uint8)
        mask[H // 3:H // 3 + H // 5, W // 4:W // 4 + W // 5] = 1
        if seed % 2:
            mask[0:3, 0:W // 3] = 1   # a second blob on the border
        jobs.append(synth.Job(f"mix{seed}", rgb, mask, r))
    jobs.append(synth.small())
    return jobs


def _oracle_result(job):
    o = oracle.Oracle(job.rgb, job.mask, job.patch_radius)
    log = o.run()
    return log, o.read()[0]


@pytest.mark.parametrize("G,autotune,form,path", [(4, False, "graph", "simt"), (7, True, "graph", "simt"),
                                                   (5, False, "persistent", "simt"),
                                                   (6, False, "persistent", "mfma")])
def test_batch_equals_alone(tmp_path, G, autotune, form, path):
    jobs = _mixed_jobs()
    cache = str(tmp_path / "tune.json")
    batch = B.Batch(capacity=len(jobs) + 2, graph_iters=G, autotune=autotune, tune_cache=cache, form=form)
    pid = B.PATH_MFMA if path == "mfma" else B.PATH_SIMT
    ctxs = [B.Inpainter(j.rgb, j.mask, j.patch_radius, path=pid) for j in jobs]
    for c in ctxs:
        batch.attach(c)
    steps = 0
    while batch.step() > 0:
        steps += 1
        assert steps < 10_000
    assert batch.last_form() == form
    for j, c in zip(jobs, ctxs):
        want_log, want_img = _oracle_result(j)
        got = c.read_log(0, len(want_log))
        assert_logs_equal(got, want_log, j.name)
        assert c.remaining() == 0
        assert (c.read_image() == want_img).all(), j.name
    if autotune and form == "graph":
        assert os.path.exists(cache)
        # a second batch picks its choices from the cache and still agrees
        b2 = B.Batch(capacity=2, graph_iters=G, autotune=True, tune_cache=cache)
        c2 = B.Inpainter(jobs[1].rgb, jobs[1].mask, jobs[1].patch_radius)
        b2.attach(c2)
        while b2.step() > 0:
            pass
        want_log, _ = _oracle_result(jobs[1])
        assert_logs_equal(c2.read_log(0, len(want_log)), want_log, "cached tune")


@pytest.mark.parametrize("form", ["graph", "persistent"])
def test_attach_detach_mid_run(form):
    jobs = _mixed_jobs()
    batch = B.Batch(capacity=4, graph_iters=3, autotune=False, form=form)
    ctxs = [B.Inpainter(j.rgb, j.mask, j.patch_radius) for j in jobs]
    batch.attach(ctxs[0])
    batch.attach(ctxs[1])
    batch.step()
    batch.attach(ctxs[2])            # joins while the others are mid-run
    batch.step()
    batch.detach(ctxs[1])            # leaves unfinished ...
    batch.attach(ctxs[3])            # ... and its slot is reused
    batch.step()
    with pytest.raises(B.InpaintError):
        batch.attach(ctxs[0])        # already attached
    batch.attach(ctxs[4])
    with pytest.raises(B.InpaintError):
        batch.attach(ctxs[5])        # full
    while batch.step() > 0:
        pass
    ctxs[1].run()                    # the detached job finishes on its own
    for i in range(5):
        want_log, want_img = _oracle_result(jobs[i])
        assert_logs_equal(ctxs[i].read_log(0, len(want_log)), want_log, jobs[i].name)
        assert (ctxs[i].read_image() == want_img).all()


def test_batch_of_vga_sized_images_prefix():
    # Two 640x480 images in one batch for a few replays: every logged
    # iteration equals the oracle's (the oracle runs the same prefix).
    a = synth.vga()
    b = synth.Job("vga-shift", np.ascontiguousarray(a.rgb[::-1]), np.ascontiguousarray(a.mask[:, ::-1]), 4)
    batch = B.Batch(capacity=2, graph_iters=5, autotune=False)
    ctxs = [B.Inpainter(j.rgb, j.mask, 4) for j in (a, b)]
    for c in ctxs:
        batch.attach(c)
    batch.step()
    batch.step()
    for j, c in zip((a, b), ctxs):
        o = oracle.Oracle(j.rgb, j.mask, 4)
        want = o.run(max_iters=10)
        assert_logs_equal(c.read_log(0, 10), want, j.name)


@pytest.mark.parametrize("form,path", [("persistent", "mfma"), ("persistent", "simt"), ("graph", "simt"),
                                       ("auto", "mfma")])
def test_batch_of_64_full_size_matches_stored_oracle(tmp_path, form, path):
    # The seeded 64-image batch (320x240 .. 1280x720, 1-3 blobs covering
    # 2-10%, 9x9 patch, full search), run to the end with 16 iterations per
    # step: in the batched persistent form (one persistent dispatch per
    # step advances every image) on either search path, and in the graph
    # form with the autotuner on; and as the bench runs it, AUTO with 64
    # iterations per step (graph form, then persistent once the running
    # tiles fit four per search group).  Every image's whole fill log and
    # final image equal its stored oracle result.
    from _util import assert_matches_golden, load_golden
    jobs = synth.batch()
    golds = [load_golden(f"batch{i:02d}") for i in range(len(jobs))]
    assert all(g is not None for g in golds), "stored oracle results missing"
    for j, g in zip(jobs, golds):
        assert g["input_sha256"] == j.sha256(), j.name
    batch = B.Batch(capacity=len(jobs), graph_iters=64 if form == "auto" else 16, autotune=True,
                    tune_cache=str(tmp_path / "tune.json"), form=form)
    pid = B.PATH_MFMA if path == "mfma" else B.PATH_SIMT
    ctxs = [B.Inpainter(j.rgb, j.mask, j.patch_radius, path=pid) for j in jobs]
    for c in ctxs:
        batch.attach(c)
    steps = 0
    while batch.step() > 0:
        steps += 1
        assert steps < 2000
    assert batch.last_form() == (form if form != "auto" else "persistent")
    for j, g, c in zip(jobs, golds, ctxs):
        assert c.remaining() == 0, j.name
        assert_matches_golden(g, c.read_log(0, g["iterations"]), c.read_image(), j.name)


def test_mixed_radii_beyond_resident_tiles_match_stored_oracle():
    # Serving jobs 1, 2, 3 and 8 (7x7, 11x11, 9x9, 9x9 patches; about 1040
    # int8-MFMA search tiles, twice the co-resident search work-groups) in
    # the batched persistent form: every step is one mixed-radius dispatch
    # whose search groups each hold tiles of one radius and restage them per
    # iteration.  Every job's fill log and final image equal its stored
    # oracle result.
    from _util import assert_matches_golden, load_golden
    jobs = synth.serving()
    pick = [1, 2, 3, 8]
    assert sorted({jobs[i].patch_radius for i in pick}) == [3, 4, 5]
    golds = [load_golden(f"serve{i:02d}") for i in pick]
    assert all(g is not None for g in golds), "stored oracle results missing"
    batch = B.Batch(capacity=len(pick), graph_iters=32, autotune=False, form="persistent")
    ctxs = [B.Inpainter(jobs[i].rgb, jobs[i].mask, jobs[i].patch_radius, path=B.PATH_MFMA,
                        log_capacity=int(jobs[i].mask.sum())) for i in pick]
    for c in ctxs:
        batch.attach(c)
    steps = 0
    while batch.step() > 0:
        steps += 1
        assert steps < 1000
    assert batch.last_form() == "persistent"
    for i, g, c in zip(pick, golds, ctxs):
        assert g["input_sha256"] == jobs[i].sha256(), jobs[i].name
        it, _ = c.progress()
        assert_matches_golden(g, c.read_log(0, it), c.read_image(), jobs[i].name)
        c.close()
    batch.close()


def test_persistent_batch_with_mixed_and_per_radius_dispatches():
    # MFMA contexts of radius 2 and 5 share the mixed-radius dispatch; a
    # radius-6 MFMA context and a radius-7 context (SIMT: past the MFMA
    # form's radii) get a dispatch each.  Every image equals the oracle.
    jobs = []
    for seed, (W, H, r) in enumerate([(70, 60, 2), (96, 80, 5), (110, 90, 6), (120, 100, 7)]):
        rng = np.random.default_rng(400 + seed)
        rgb = rng.integers(0, 256, size=(H, W, 3)).astype(np.uint8)
        mask = np.zeros((H, W), np.uint8)
        mask[H // 3:H // 3 + H // 6, W // 3:W // 3 + W // 6] = 1
        jobs.append(synth.Job(f"pr{seed}-r{r}", rgb, mask, r))
    batch = B.Batch(capacity=len(jobs), graph_iters=8, autotune=False, form="persistent")
    ctxs = [B.Inpainter(j.rgb, j.mask, j.patch_radius, path=B.PATH_MFMA if j.patch_radius <= 6 else B.PATH_SIMT)
            for j in jobs]
    for c in ctxs:
        batch.attach(c)
    steps = 0
    while batch.step() > 0:
        steps += 1
        assert steps < 10_000
    assert batch.last_form() == "persistent"
    for j, c in zip(jobs, ctxs):
        want_log, want_img = _oracle_result(j)
        assert_logs_equal(c.read_log(0, len(want_log)), want_log, j.name)
        assert (c.read_image() == want_img).all(), j.name
