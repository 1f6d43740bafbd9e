"""Parity of the candidate-domain variants (current source policy,
INTERSECT scoring) between the HIP path and the CPU oracle.  Fill logs,
final images, hole maps and confidences must be bit-exact."""
import numpy as np
import pytest

import oracle
from paper_1403_4238_amd import synth

from _util import assert_logs_equal

pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_1403_4238_amd.binding")

MODES = [(B.SOURCE_CURRENT, B.SCORE_WHOLE), (B.SOURCE_ORIGINAL, B.SCORE_INTERSECT),
         (B.SOURCE_CURRENT, B.SCORE_INTERSECT)]
MODE_IDS = ["current", "intersect", "current+intersect"]


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    B.lib()


def _pair(job, policy, scoring, **kw):
    o = oracle.Oracle(job.rgb, job.mask, job.patch_radius, job.search_mode, job.alpha, rect=job.rect,
                      source_policy=policy, scoring=scoring)
    g = B.Inpainter(job.rgb, job.mask, job.patch_radius, job.search_mode, job.alpha, rect=job.rect,
                    source_policy=policy, scoring=scoring, **kw)
    return o, g


def _full_run(job, policy, scoring, label, **kw):
    o, g = _pair(job, policy, scoring, **kw)
    want = o.run()
    st, n, got = g.run(log_cap=len(want) + 8)
    assert st == B.DONE and n == len(want), (label, n, len(want))
    assert_logs_equal(got, want, label)
    rgb_o, _, hole_o, conf_o = o.read()
    hole_g, conf_g = g.read_state()
    assert (g.read_image() == rgb_o).all(), f"{label}: final image differs"
    assert (hole_g == hole_o).all() and hole_g.sum() == 0
    assert (conf_g.view(np.int64) == conf_o.view(np.int64)).all(), f"{label}: confidence differs"
    g.close()
    return got


def _random_job(seed, W, H, r, levels=256):
    rng = np.random.default_rng(seed)
    rgb = rng.integers(0, levels, size=(H, W, 3)).astype(np.uint8)
    if levels < 256:
        rgb = (rgb * (255 // (levels - 1))).astype(np.uint8)
    mask = np.zeros((H, W), np.uint8)
    mask[H // 3:H // 3 + max(H // 4, 2), W // 3:W // 3 + max(W // 5, 2)] = 1
    mask[0:max(H // 8, 1), W - max(W // 7, 2):] = 1   # touches the border
    return synth.Job(f"dom{seed}", rgb, mask, r)


@pytest.mark.parametrize("policy,scoring", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("seed,W,H,r", [(31, 24, 20, 1), (32, 40, 31, 2), (33, 67, 45, 4), (34, 90, 70, 8),
                                        (35, 33, 70, 6)])
def test_random_images_full_run(policy, scoring, seed, W, H, r):
    job = _random_job(seed, W, H, r)
    _full_run(job, policy, scoring, f"{job.name} {policy}/{scoring}")


@pytest.mark.parametrize("policy,scoring", MODES, ids=MODE_IDS)
def test_few_levels_many_ties(policy, scoring):
    job = _random_job(36, 48, 40, 2, levels=3)
    _full_run(job, policy, scoring, f"ties {policy}/{scoring}")


@pytest.mark.parametrize("policy,scoring", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("path,form,tile_rows", [(B.PATH_SIMT, "stream", 4), (B.PATH_SIMT, "graph", 16),
                                                 (B.PATH_SIMT_DIRECT, "stream", 8), (B.PATH_SIMT, "plain", 8)])
def test_small_workload_paths_and_forms(policy, scoring, path, form, tile_rows):
    job = synth.small()
    _full_run(job, policy, scoring, f"small {policy}/{scoring}", path=path, form=form, tile_rows=tile_rows,
              iters_per_check=5)


@pytest.mark.parametrize("policy,scoring", MODES, ids=MODE_IDS)
def test_alpha_window(policy, scoring):
    job = synth.small()
    job.search_mode, job.alpha = synth.SEARCH_ALPHA, (1, 2)
    _full_run(job, policy, scoring, f"small-win {policy}/{scoring}", form="stream", iters_per_check=8)


@pytest.mark.parametrize("policy,scoring", MODES, ids=MODE_IDS)
def test_persistent_request_runs_stream_form(policy, scoring):
    job = synth.small()
    o, g = _pair(job, policy, scoring, form="persistent")
    assert g.run_form() == "stream"
    g.close()
    _full_run(job, policy, scoring, "persistent request", form="persistent")


@pytest.mark.parametrize("policy,scoring", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("r", [1, 3, 5, 8])
def test_find_exemplar_after_some_iterations(policy, scoring, r):
    # After a few fills (sources added under the CURRENT policy), queries of
    # every radius must agree with the oracle in the same state.
    job = synth.small()
    o, g = _pair(job, policy, scoring)
    o.run(max_iters=6)
    g.run(max_iters=6, log_cap=8)
    rng = np.random.default_rng(300 + r)
    front = o.front()
    targets = [(int(i % job.width), int(i // job.width)) for i in front[:: max(len(front) // 5, 1)]]
    targets += [(int(rng.integers(0, job.width)), int(rng.integers(0, job.height))) for _ in range(3)]
    for (x, y) in targets:
        for rect in [(0, 0, job.width, job.height), (30, 20, 100, 80)]:
            try:
                want = o.find_exemplar(x, y, r, rect)[:2]
            except oracle.OracleError as e:
                assert e.status == oracle.NO_CANDIDATE
                with pytest.raises(B.InpaintError):
                    g.find_exemplar(x, y, r, rect)
                continue
            assert g.find_exemplar(x, y, r, rect) == want, (r, x, y, rect)


@pytest.mark.parametrize("policy,scoring", MODES, ids=MODE_IDS)
def test_vga_prefix(policy, scoring):
    job = synth.vga()
    o, g = _pair(job, policy, scoring, form="stream", iters_per_check=16)
    want = o.run(max_iters=24)
    _, n, got = g.run(max_iters=24, log_cap=32)
    assert n == 24
    assert_logs_equal(got, want, f"vga prefix {policy}/{scoring}")


def test_mfma_path_and_batch_reject_other_domains():
    job = synth.small()
    for policy, scoring in MODES:
        with pytest.raises(B.InpaintError) as e:
            B.Inpainter(job.rgb, job.mask, 4, path=B.PATH_MFMA, source_policy=policy, scoring=scoring)
        assert e.value.status == B.INVALID_ARGUMENT
    g = B.Inpainter(job.rgb, job.mask, 4, scoring=B.SCORE_INTERSECT)
    b = B.Batch(capacity=2)
    with pytest.raises(B.InpaintError):
        b.attach(g)
    b.close()
    g.close()
