"""Pins for the oracle's candidate-domain variants (source policy CURRENT,
INTERSECT scoring), checked against definitions written out again here in
numpy, independently of oracle.c.

Selection (priority, argmax) is the pinned default code and is taken from the
oracle.  What each variant changes is checked step by step by brute force:
- the candidate set;
- the SSD domain of Eq. 4;
- which hole pixels the copy fills.
"""
import numpy as np
import pytest

import oracle as O

MODES = [(O.SOURCE_ORIGINAL, O.SCORE_WHOLE), (O.SOURCE_CURRENT, O.SCORE_WHOLE),
         (O.SOURCE_ORIGINAL, O.SCORE_INTERSECT), (O.SOURCE_CURRENT, O.SCORE_INTERSECT)]


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build()


def source_map(hole, hole0, policy):
    """Phi as a boolean map: the original or the current known region."""
    return ~(hole if policy == O.SOURCE_CURRENT else hole0).astype(bool)


def brute_search(rgb, hole, hole0, p, r, rect, policy, scoring):
    """(index, ssd) of the lexicographic (ssd, index) minimum, by definition."""
    H, W, _ = rgb.shape
    phi = source_map(hole, hole0, policy)
    known = ~hole.astype(bool)
    px, py = p % W, p // W
    img = rgb.astype(np.int64)
    best = None
    for cy in range(max(rect[1], 0), min(rect[3], H)):
        for cx in range(max(rect[0], 0), min(rect[2], W)):
            if scoring == O.SCORE_INTERSECT:
                if not phi[cy, cx]:
                    continue
            else:
                if cx - r < 0 or cy - r < 0 or cx + r >= W or cy + r >= H:
                    continue
                if not phi[cy - r:cy + r + 1, cx - r:cx + r + 1].all():
                    continue
            d = 0
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    tx, ty, sx, sy = px + dx, py + dy, cx + dx, cy + dy
                    if not (0 <= tx < W and 0 <= ty < H) or not known[ty, tx]:
                        continue
                    if not (0 <= sx < W and 0 <= sy < H) or not phi[sy, sx]:
                        continue   # only reachable under INTERSECT scoring
                    d += int(((img[ty, tx] - img[sy, sx]) ** 2).sum())
            if best is None or d < best[1]:
                best = (cy * W + cx, d)
    return best


def brute_copy(rgb, hole, hole0, p, q, r, policy, scoring):
    """Image and hole map after copying source centre q into target p."""
    H, W, _ = rgb.shape
    phi = source_map(hole, hole0, policy)
    out, h = rgb.copy(), hole.copy()
    px, py, qx, qy = p % W, p // W, q % W, q // W
    n = 0
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            x, y, sx, sy = px + dx, py + dy, qx + dx, qy + dy
            if not (0 <= x < W and 0 <= y < H) or not hole[y, x]:
                continue
            if scoring == O.SCORE_INTERSECT and not (0 <= sx < W and 0 <= sy < H and phi[sy, sx]):
                continue
            out[y, x] = rgb[sy, sx]   # sources read from the state before the copy
            h[y, x] = 0
            n += 1
    return out, h, n


def _case(seed, W, H):
    rng = np.random.default_rng(seed)
    # few levels so that ties and exact matches occur
    rgb = (rng.integers(0, 4, size=(H, W, 3)) * 60).astype(np.uint8)
    mask = np.zeros((H, W), np.uint8)
    mask[H // 3:H // 3 + H // 3, W // 3:W // 3 + W // 4 + 1] = 1
    mask[H - 3:, W - 4:] = 1   # a second hole touching the border
    return rgb, mask


@pytest.mark.parametrize("policy,scoring", MODES)
@pytest.mark.parametrize("seed,W,H,r", [(1, 20, 16, 1), (2, 22, 18, 2), (3, 17, 21, 1)])
def test_each_step_matches_the_definition(policy, scoring, seed, W, H, r):
    rgb, mask = _case(seed, W, H)
    o = O.Oracle(rgb, mask, r, source_policy=policy, scoring=scoring)
    hole0 = mask.astype(np.uint8)
    rect = o.rect()
    steps = 0
    while True:
        cur, _, hole, _ = o.read()
        sel = o.select()
        if sel is None:
            assert hole.sum() == 0
            break
        p = sel[0]
        want_q, want_d = brute_search(cur, hole, hole0, p, r, rect, policy, scoring)
        rec = o.step()
        assert (rec["source_index"], rec["ssd"]) == (want_q, want_d), (steps, p)
        img2, hole2, n = brute_copy(cur, hole, hole0, p, want_q, r, policy, scoring)
        rgb_o, _, hole_o, _ = o.read()
        assert rec["n_filled"] == n >= 1
        assert (rgb_o == img2).all() and (hole_o == hole2).all(), steps
        steps += 1
        assert steps <= mask.sum()


def test_current_policy_equals_original_on_the_first_step():
    rgb, mask = _case(4, 24, 18)
    a = O.Oracle(rgb, mask, 2).step()
    b = O.Oracle(rgb, mask, 2, source_policy=O.SOURCE_CURRENT).step()
    assert a.tobytes() == b.tobytes()


def _run_log(rgb, mask, r, policy, scoring):
    o = O.Oracle(rgb, mask, r, source_policy=policy, scoring=scoring)
    return o, o.run()


def test_current_policy_uses_filled_pixels_as_sources():
    # A periodic texture with a large hole: once part of the hole is filled,
    # windows that contain filled pixels become candidates; at least one chosen
    # source window must contain originally-unknown pixels.
    rng = np.random.default_rng(5)
    tile = rng.integers(0, 256, size=(3, 4, 3), dtype=np.uint8)
    rgb = np.tile(tile, (10, 8, 1))[:28, :30]
    mask = np.zeros((28, 30), np.uint8)
    mask[6:22, 5:25] = 1
    r = 2
    _, log = _run_log(rgb, mask, r, O.SOURCE_CURRENT, O.SCORE_WHOLE)
    W = 30
    uses_filled = 0
    for q in log["source_index"]:
        qx, qy = q % W, q // W
        uses_filled += bool(mask[qy - r:qy + r + 1, qx - r:qx + r + 1].any())
    assert uses_filled > 0
    # ... which the original policy never does
    _, log0 = _run_log(rgb, mask, r, O.SOURCE_ORIGINAL, O.SCORE_WHOLE)
    for q in log0["source_index"]:
        qx, qy = q % W, q // W
        assert not mask[qy - r:qy + r + 1, qx - r:qx + r + 1].any()


def test_intersect_scoring_takes_overlapping_candidates_and_partial_copies():
    rgb, mask = _case(6, 26, 20)
    r = 2
    o, log = _run_log(rgb, mask, r, O.SOURCE_ORIGINAL, O.SCORE_INTERSECT)
    W, H = 26, 20
    overlapping = 0
    for q in log["source_index"]:
        qx, qy = q % W, q // W
        assert not mask[qy, qx]                       # the centre is a source pixel
        win = np.zeros((H + 2 * r, W + 2 * r), bool)  # out-of-image counts as non-source
        win[r:r + H, r:r + W] = mask == 0
        overlapping += not win[qy:qy + 2 * r + 1, qx:qx + 2 * r + 1].all()
    assert overlapping > 0
    # some iteration leaves hole pixels of its target patch for later
    assert len(log) > O.Oracle(rgb, mask, r).run().shape[0]
    assert o.remaining() == 0


def test_intersect_ssd_is_zero_when_the_known_sets_do_not_meet():
    # The target's only known pixels are the column left of it.  Under
    # INTERSECT scoring the corner centre (0, 0) is a candidate; its left
    # column lies outside the image, so its Eq. 4 sum is empty (SSD 0), and
    # it has the lowest index.
    W, H, r = 12, 9, 1
    rgb = np.full((H, W, 3), 200, np.uint8)
    rgb[:, :4] = 10
    mask = np.zeros((H, W), np.uint8)
    mask[:, 4:8] = 1
    o = O.Oracle(rgb, mask, r, scoring=O.SCORE_INTERSECT)
    # target (4, 4): known offsets dx = -1 (column 3, value 10)
    q, d, k = o.find_exemplar(4, 4, r, (0, 0, W, H))
    assert (q, d, k) == (0, 0, 3)
    # a centre right of the hole, whose left column is hole, also scores 0
    assert o.find_exemplar(4, 4, r, (8, 0, W, H))[:2] == (8, 0)
    # under the default scoring every full window must lie in the known
    # region: the dark strip matches exactly at the lowest centre (1, 1)
    assert O.Oracle(rgb, mask, r).find_exemplar(4, 4, r, (0, 0, W, H))[:2] == (1 * W + 1, 0)


def test_modes_are_validated():
    rgb, mask = _case(7, 16, 16)
    for bad in [dict(source_policy=2), dict(source_policy=-1), dict(scoring=2)]:
        with pytest.raises(O.OracleError):
            O.Oracle(rgb, mask, 1, **bad)
