"""Resume and iterative editing through the C ABI (inpaint_import_state),
checked bit-exact against the CPU oracle: continuing from a checkpoint must
give exactly the rest of the uninterrupted removal."""
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


def _case(seed, W, H):
    rng = np.random.default_rng(seed)
    rgb = rng.integers(0, 256, size=(H, W, 3)).astype(np.uint8)
    mask = np.zeros((H, W), np.uint8)
    mask[H // 4:H // 4 + H // 3, W // 3:W // 3 + W // 3] = 1
    mask[H - 2:, :3] = 1
    return rgb, mask


def _check_tail(g, o_full, want_tail, label):
    st, n, got = g.run(log_cap=len(want_tail) + 8)
    assert st == B.DONE and n == len(want_tail), (label, n, len(want_tail))
    assert_logs_equal(got, want_tail, label)
    rgb_o, _, hole_o, conf_o = o_full.read()
    hole_g, conf_g = g.read_state()
    assert (g.read_image() == rgb_o).all(), f"{label}: final image differs"
    assert (hole_g == hole_o).all()
    assert (conf_g.view(np.int64) == conf_o.view(np.int64)).all(), f"{label}: confidence differs"


MODES = [(B.SOURCE_ORIGINAL, B.SCORE_WHOLE), (B.SOURCE_CURRENT, B.SCORE_WHOLE),
         (B.SOURCE_ORIGINAL, B.SCORE_INTERSECT), (B.SOURCE_CURRENT, B.SCORE_INTERSECT)]


@pytest.mark.parametrize("policy,scoring", MODES, ids=["default", "current", "intersect", "both"])
@pytest.mark.parametrize("cut", [1, 9])
def test_gpu_checkpoint_resumes_in_a_fresh_context(policy, scoring, cut):
    rgb, mask = _case(11, 48, 40)
    r = 2
    o_full = oracle.Oracle(rgb, mask, r, source_policy=policy, scoring=scoring)
    want = o_full.run()
    g1 = B.Inpainter(rgb, mask, r, source_policy=policy, scoring=scoring)
    g1.run(max_iters=cut, log_cap=cut + 4)
    ck = g1.export_state()
    assert ck[3] == cut
    g1.close()
    # a new job from the checkpoint image and the original mask
    g2 = B.Inpainter(ck[0], mask, r, source_policy=policy, scoring=scoring, log_capacity=len(want) + 8)
    g2.import_state(*ck)
    assert g2.progress() == (cut, int(ck[1].sum()))
    _check_tail(g2, o_full, want[cut:], f"resume {policy}/{scoring} at {cut}")


@pytest.mark.parametrize("form,path", [("persistent", B.PATH_MFMA), ("persistent", B.PATH_SIMT),
                                       ("graph", B.PATH_SIMT), ("stream", B.PATH_SIMT_DIRECT)])
def test_resume_in_every_form(form, path):
    job = synth.small()
    o_full = oracle.Oracle(job.rgb, job.mask, 4)
    want = o_full.run()
    g1 = B.Inpainter(job.rgb, job.mask, 4, form=form, path=path, iters_per_check=4)
    g1.run(max_iters=6, log_cap=8)
    ck = g1.export_state()
    g2 = B.Inpainter(ck[0], job.mask, 4, form=form, path=path, iters_per_check=4)
    g2.import_state(*ck)
    _check_tail(g2, o_full, want[6:], f"resume {form}")


def test_oracle_checkpoint_imports_on_the_gpu():
    rgb, mask = _case(12, 56, 44)
    o_full = oracle.Oracle(rgb, mask, 3)
    want = o_full.run()
    o_part = oracle.Oracle(rgb, mask, 3)
    o_part.run(max_iters=5)
    g = B.Inpainter(rgb, mask, 3, form="persistent", path=B.PATH_MFMA)
    g.import_state(*o_part.export_state())
    _check_tail(g, o_full, want[5:], "oracle checkpoint")


def test_rewind_to_an_earlier_checkpoint():
    job = synth.small()
    o_full = oracle.Oracle(job.rgb, job.mask, 4)
    want = o_full.run()
    g = B.Inpainter(job.rgb, job.mask, 4, form="stream", path=B.PATH_SIMT, iters_per_check=3)
    g.run(max_iters=4, log_cap=8)
    ck = g.export_state()
    g.run(max_iters=7, log_cap=8)          # go further, then back
    g.import_state(*ck)
    _check_tail(g, o_full, want[4:], "rewind")


def test_invalid_checkpoints_are_rejected_and_change_nothing():
    job = synth.small()
    o_full = oracle.Oracle(job.rgb, job.mask, 4)
    want = o_full.run()
    g = B.Inpainter(job.rgb, job.mask, 4, form="persistent", path=B.PATH_MFMA)
    g.run(max_iters=3, log_cap=4)
    rgb, hole, conf, it = g.export_state()
    bad_hole = hole.copy()
    bad_hole[0, 0] = 1
    assert job.mask[0, 0] == 0
    filled = tuple(np.argwhere((job.mask == 1) & (hole == 0))[0])
    bad_conf = conf.copy()
    bad_conf[filled] = np.nan
    for args in [(rgb, bad_hole, conf, it), (rgb, hole, bad_conf, it), (rgb, hole, conf, -1)]:
        with pytest.raises(B.InpaintError) as e:
            g.import_state(*args)
        assert e.value.status == B.INVALID_ARGUMENT
    _check_tail(g, o_full, want[3:], "after rejected imports")


def test_vga_resumed_half_way_matches_the_stored_oracle():
    gold = load_golden("vga")
    if gold is None:
        pytest.skip("stored oracle result for the 640x480 workload not generated")
    job = synth.vga()
    g1 = B.Inpainter(job.rgb, job.mask, 4, form="persistent", path=B.PATH_MFMA, iters_per_check=64)
    st, n1, log1 = g1.run(max_iters=300, log_cap=300)
    assert n1 == 300
    ck = g1.export_state()
    g1.close()
    g2 = B.Inpainter(ck[0], job.mask, 4, form="persistent", path=B.PATH_MFMA, iters_per_check=64)
    g2.import_state(*ck)
    st, n2, log2 = g2.run(log_cap=gold["iterations"])
    assert st == B.DONE
    assert_matches_golden(gold, np.concatenate([log1, log2]), g2.read_image(), "vga resumed at 300")


def test_iterative_editing_second_removal_on_the_output():
    job = synth.small()
    o1 = oracle.Oracle(job.rgb, job.mask, 4)
    o1.run()
    g1 = B.Inpainter(job.rgb, job.mask, 4, form="persistent", path=B.PATH_MFMA)
    g1.run()
    out = g1.read_image()
    assert (out == o1.read()[0]).all()
    mask2 = np.zeros_like(job.mask)
    mask2[10:22, 90:110] = 1
    o2 = oracle.Oracle(out, mask2, 4)
    want = o2.run()
    g2 = B.Inpainter(out, mask2, 4, form="persistent", path=B.PATH_MFMA)
    _check_tail(g2, o2, want, "second removal")
