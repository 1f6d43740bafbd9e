"""Pins for the oracle's resume (iterative editing): continuing from an
exported checkpoint must give exactly the rest of the uninterrupted run, in
every candidate-domain mode.  Invalid checkpoints are rejected and leave the
state untouched."""
import numpy as np
import pytest

import oracle as O

MODES = [(O.SOURCE_ORIGINAL, O.SCORE_WHOLE), (O.SOURCE_CURRENT, O.SCORE_WHOLE),
         (O.SOURCE_ORIGINAL, O.SCORE_INTERSECT), (O.SOURCE_CURRENT, O.SCORE_INTERSECT)]


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build()


def _case(seed, W, H):
    rng = np.random.default_rng(seed)
    rgb = rng.integers(0, 256, size=(H, W, 3)).astype(np.uint8)
    mask = np.zeros((H, W), np.uint8)
    mask[H // 4:H // 4 + H // 3, W // 3:W // 3 + W // 3] = 1
    mask[H - 2:, :3] = 1
    return rgb, mask


def _state(o):
    rgb, gray, hole, conf = o.read()
    return rgb, gray, hole, conf.view(np.int64), o.remaining(), o.iterations()


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("policy,scoring", MODES)
@pytest.mark.parametrize("seed,W,H,r,cut", [(1, 30, 24, 2, 1), (2, 30, 24, 2, 7), (3, 26, 30, 1, 15),
                                            (4, 40, 28, 3, 4)])
def test_resume_equals_uninterrupted(policy, scoring, seed, W, H, r, cut):
    rgb, mask = _case(seed, W, H)
    full = O.Oracle(rgb, mask, r, source_policy=policy, scoring=scoring)
    log_full = full.run()
    assert len(log_full) > cut
    part = O.Oracle(rgb, mask, r, source_policy=policy, scoring=scoring)
    part.run(max_iters=cut)
    ck_rgb, ck_hole, ck_conf, ck_iter = part.export_state()
    assert ck_iter == cut
    # a fresh job of the same removal, created from the checkpoint image
    res = O.Oracle(ck_rgb, mask, r, source_policy=policy, scoring=scoring)
    res.import_state(ck_rgb, ck_hole, ck_conf, ck_iter)
    assert _same(_state(res), _state(part))
    log_res = res.run()
    assert log_res.tobytes() == log_full[cut:].tobytes()
    assert _same(_state(res), _state(full))


def test_importing_the_initial_state_changes_nothing():
    rgb, mask = _case(5, 28, 22)
    o = O.Oracle(rgb, mask, 2)
    before = _state(o)
    o.import_state(*o.export_state())
    assert _same(_state(o), before)


def test_invalid_checkpoints_are_rejected_and_change_nothing():
    rgb, mask = _case(6, 28, 22)
    o = O.Oracle(rgb, mask, 2)
    o.run(max_iters=3)
    ck_rgb, ck_hole, ck_conf, it = o.export_state()
    before = _state(o)
    bad_hole = ck_hole.copy()
    bad_hole[0, 0] = 1                      # outside the original hole
    assert mask[0, 0] == 0
    filled = np.argwhere((mask == 1) & (ck_hole == 0))[0]
    bad_conf = ck_conf.copy()
    bad_conf[tuple(filled)] = 1.5           # out of [0, 1] on a filled pixel
    nan_conf = ck_conf.copy()
    nan_conf[tuple(filled)] = np.nan
    for args in [(ck_rgb, bad_hole, ck_conf, it), (ck_rgb, ck_hole, bad_conf, it),
                 (ck_rgb, ck_hole, nan_conf, it), (ck_rgb, ck_hole, ck_conf, -1)]:
        with pytest.raises(O.OracleError):
            o.import_state(*args)
        assert _same(_state(o), before)


def test_checkpoint_values_outside_the_original_hole_are_ignored():
    rgb, mask = _case(7, 28, 22)
    full = O.Oracle(rgb, mask, 2)
    log_full = full.run()
    part = O.Oracle(rgb, mask, 2)
    part.run(max_iters=5)
    ck_rgb, ck_hole, ck_conf, it = part.export_state()
    noisy = ck_rgb.copy()
    noisy[mask == 0] ^= 0x5A                # the source region is the job's own
    res = O.Oracle(rgb, mask, 2)
    res.import_state(noisy, ck_hole, ck_conf, it)
    assert res.run().tobytes() == log_full[5:].tobytes()


def test_iterative_editing_second_removal_on_the_output():
    # Remove one object, then a second one from the result: the second job
    # sees the first one's output as its source image.
    rgb, mask = _case(8, 32, 26)
    first = O.Oracle(rgb, mask, 2)
    first.run()
    out = first.read()[0]
    mask2 = np.zeros_like(mask)
    mask2[2:6, 20:27] = 1
    second = O.Oracle(out, mask2, 2)
    log2 = second.run()
    assert second.remaining() == 0 and len(log2) >= 1
    final = second.read()[0]
    assert (final[mask2 == 0] == out[mask2 == 0]).all()   # only the new hole changes
