"""The persistent fill form (one cooperative dispatch runs many iterations)
against the CPU oracle and the other forms, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_1403_4238_amd import synth

from _util import assert_logs_equal, assert_matches_golden, load_golden

pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_1403_4238_amd.binding")


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    B.lib()


def _full(job, n=32, **kw):
    o = oracle.Oracle(job.rgb, job.mask, job.patch_radius, job.search_mode, job.alpha, rect=job.rect)
    g = B.Inpainter(job.rgb, job.mask, job.patch_radius, job.search_mode, job.alpha, rect=job.rect,
                    form="persistent", iters_per_check=n, **kw)
    want = o.run()
    st, cnt, got = g.run(log_cap=len(want) + 8)
    assert st == B.DONE and cnt == len(want)
    assert_logs_equal(got, want, job.name)
    rgb_o, _, hole_o, conf_o = o.read()
    hole_g, conf_g = g.read_state()
    assert (g.read_image() == rgb_o).all(), f"{job.name}: final image differs"
    assert (hole_g == hole_o).all() and hole_g.sum() == 0
    assert (conf_g.view(np.int64) == conf_o.view(np.int64)).all(), f"{job.name}: confidence differs"
    return g


@pytest.mark.parametrize("n", [1, 5, 64])
def test_small_job_matches_oracle(n):
    g = _full(synth.small(), n)
    assert g.run_form() == "persistent"


def test_equals_plain_form_and_partial_runs():
    job = synth.small()
    plain = B.Inpainter(job.rgb, job.mask, 4, form="plain")
    _, n1, want = plain.run(log_cap=100)
    g = B.Inpainter(job.rgb, job.mask, 4, form="persistent", iters_per_check=7)
    recs = [g.step(), g.step()]
    st, n, more = g.run(max_iters=9, log_cap=16)
    assert st == B.OK and n == 9
    st, n2, rest = g.run(log_cap=100)
    assert st == B.DONE and 2 + n + n2 == n1
    got = np.concatenate([np.array(recs, dtype=B.STEP_DTYPE), more, rest])
    assert_logs_equal(got, want, "step+persistent")
    assert (plain.read_image() == g.read_image()).all()
    assert g.run()[0] == B.DONE


@pytest.mark.parametrize("seed,W,H,r", [(21, 90, 70, 1), (22, 120, 80, 2), (23, 150, 96, 3), (24, 130, 100, 5),
                                        (25, 160, 120, 8), (26, 97, 61, 4)])
def test_random_jobs_all_radii(seed, W, H, r):
    rng = np.random.default_rng(seed)
    rgb = rng.integers(0, 256, size=(H, W, 3)).astype(np.uint8)
    rgb[:, : W // 2] //= 4   # some structure: a darker half
    mask = np.zeros((H, W), np.uint8)
    mask[H // 3:H // 3 + max(H // 5, 2), W // 3:W // 3 + max(W // 6, 2)] = 1
    mask[0:max(H // 9, 1), W - max(W // 8, 2):] = 1
    g = _full(synth.Job(f"persist{seed}", rgb, mask, r), n=16)
    assert g.run_form() in ("persistent", "stream")


def test_window_and_rect_searches():
    job = synth.small()
    _full(synth.Job("small-win", job.rgb, job.mask, 4, synth.SEARCH_ALPHA, (1, 2)))
    _full(synth.Job("small-rect", job.rgb, job.mask, 3, synth.SEARCH_RECT, (0, 1), (5, 3, 100, 70)))


def test_timing_counts_dispatches():
    job = synth.small()
    g = B.Inpainter(job.rgb, job.mask, 4, form="persistent", iters_per_check=8)
    g.profile_search(True)
    st, n, log = g.run(log_cap=100)
    ms, cnt = g.search_time()
    assert st == B.DONE and cnt == (n + 7) // 8 and ms > 0.0
    assert_logs_equal(log, oracle.Oracle(job.rgb, job.mask, 4).run(), "timed persistent")


@pytest.mark.parametrize("n", [1, 6, 64])
def test_mfma_small_job_matches_oracle(n):
    g = _full(synth.small(), n, path=B.PATH_MFMA)
    assert g.run_form() == "persistent"


@pytest.mark.parametrize("seed,W,H,r", [(31, 90, 70, 1), (32, 150, 96, 3), (33, 130, 100, 5), (34, 140, 90, 6),
                                        (35, 97, 61, 4)])
def test_mfma_random_jobs(seed, W, H, r):
    rng = np.random.default_rng(seed)
    rgb = rng.integers(0, 256, size=(H, W, 3)).astype(np.uint8)
    rgb[H // 2:, :] = 255 - rgb[H // 2:, :] // 3   # saturated lower half
    mask = np.zeros((H, W), np.uint8)
    mask[H // 3:H // 3 + max(H // 5, 2), W // 3:W // 3 + max(W // 6, 2)] = 1
    mask[0:max(H // 9, 1), W - max(W // 8, 2):] = 1
    _full(synth.Job(f"mfmapersist{seed}", rgb, mask, r), n=16, path=B.PATH_MFMA)


def test_mfma_then_plain_steps_use_fresh_fragments():
    # A persistent dispatch leaves the staged target's MFMA operands for the
    # one-search-per-launch kernels: mixing the forms stays exact.
    job = synth.small()
    want = oracle.Oracle(job.rgb, job.mask, 4).run()
    g = B.Inpainter(job.rgb, job.mask, 4, form="persistent", iters_per_check=5, path=B.PATH_MFMA)
    st, n1, a = g.run(max_iters=11, log_cap=16)
    recs = [g.step() for _ in range(3)]
    st, n2, b = g.run(log_cap=len(want))
    got = np.concatenate([a, np.array(recs, dtype=B.STEP_DTYPE), b])
    assert_logs_equal(got, want, "mfma persistent + steps")


@pytest.mark.parametrize("key,path", [("hd9", "simt"), ("hd13w", "simt"), ("hd9", "mfma"), ("hd13w", "mfma")])
def test_hd_full_run_matches_stored_oracle(key, path):
    gold = load_golden(key)
    if gold is None:
        pytest.skip(f"stored oracle result for {key} not generated")
    job = synth.hd(patch=int(key[2:].rstrip("w")), window=key.endswith("w"))
    assert job.sha256() == gold["input_sha256"]
    g = B.Inpainter(job.rgb, job.mask, job.patch_radius, job.search_mode, job.alpha, form="persistent",
                    iters_per_check=32, path=B.PATH_MFMA if path == "mfma" else B.PATH_SIMT)
    st, n, log = g.run(log_cap=gold["iterations"] + 8)
    assert st == B.DONE
    assert_matches_golden(gold, log, g.read_image(), f"{key} persistent {path}")
    if key == "hd9":
        assert g.run_form() == "persistent"


@pytest.mark.parametrize("dispatch_iters", [1024, 4096])
def test_hd_long_dispatches_match_stored_oracle(dispatch_iters):
    # The 1080p removal in the launch configuration the benchmark times:
    # 1024 iterations per persistent dispatch (4 dispatches, the last one
    # partial), and the whole removal in one dispatch.
    gold = load_golden("hd9")
    if gold is None:
        pytest.skip("stored oracle result for hd9 not generated")
    job = synth.hd(patch=9)
    assert job.sha256() == gold["input_sha256"]
    g = B.Inpainter(job.rgb, job.mask, job.patch_radius, form="persistent", iters_per_check=dispatch_iters,
                    path=B.PATH_MFMA)
    assert g.run_form() == "persistent"
    st, n, log = g.run(log_cap=gold["iterations"] + 8)
    assert st == B.DONE and n == gold["iterations"]
    assert_matches_golden(gold, log, g.read_image(), f"hd9 persistent mfma, {dispatch_iters} per dispatch")


@pytest.mark.parametrize("path", ["mfma", "simt"])
def test_persistent_above_coresident_tiles_matches_stored_oracle(path):
    # 1992x1221, 7x7 patch: more search tiles (640 MFMA / 1248 SIMT) than
    # work-groups that can be co-resident with one tile each, so the
    # persistent form spreads the tiles over the batched dispatch's search
    # groups (several tiles per group) instead of falling back to the stream
    # form.  The whole removal equals the stored oracle result.
    from _util import assert_matches_golden, load_golden
    job = synth.serving()[0]
    gold = load_golden("serve00")
    assert gold is not None and gold["input_sha256"] == job.sha256()
    g = B.Inpainter(job.rgb, job.mask, job.patch_radius, form="persistent", iters_per_check=64,
                    path=B.PATH_MFMA if path == "mfma" else B.PATH_SIMT)
    assert g.run_form() == "persistent"
    st, n, log = g.run(log_cap=gold["iterations"] + 8)
    assert st == B.DONE
    assert_matches_golden(gold, log, g.read_image(), f"{job.name} {path}")
