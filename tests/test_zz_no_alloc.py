"""The allocation-free query (inpaint_find_exemplar_static, scratch in a
static device array) returns exactly what inpaint_find_exemplar (scratch in
the context's workspace) returns, call after call, including a second call
on a smaller input."""
import numpy as np
import pytest

import oracle
from paper_1403_4238_amd import synth

pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_1403_4238_amd.binding")


def _targets(job, o, n_front, seed):
    rng = np.random.default_rng(seed)
    front = o.front()
    t = [(int(i % job.width), int(i // job.width)) for i in front[:: max(len(front) // n_front, 1)]]
    t += [(int(rng.integers(0, job.width)), int(rng.integers(0, job.height))) for _ in range(3)]
    return t + [(0, 0), (job.width - 1, job.height - 1)]


@pytest.mark.parametrize("path", ["mfma", "simt"])
def test_static_query_equals_workspace_query(path):
    pid = B.PATH_MFMA if path == "mfma" else B.PATH_SIMT
    # first a 640x480 job, then (second call, smaller input) the 128x96 one
    for job, rects in ((synth.vga(), [None, (100, 80, 400, 300)]), (synth.small(), [None, (10, 7, 60, 41)])):
        o = oracle.Oracle(job.rgb, job.mask, job.patch_radius)
        g = B.Inpainter(job.rgb, job.mask, job.patch_radius, path=pid)
        for r in (job.patch_radius, 2, 6):
            for rect in rects:
                for (x, y) in _targets(job, o, 4, r):
                    try:
                        want = g.find_exemplar(x, y, r, rect)
                    except B.InpaintError as e:
                        assert e.status == B.NO_CANDIDATE
                        with pytest.raises(B.InpaintError) as ge:
                            g.find_exemplar_static(x, y, r, rect)
                        assert ge.value.status == B.NO_CANDIDATE
                        continue
                    assert g.find_exemplar_static(x, y, r, rect) == want, (job.name, path, r, rect, x, y)
        # and against the oracle for the job's own radius
        for (x, y) in _targets(job, o, 3, 7)[:3]:
            assert g.find_exemplar_static(x, y) == o.find_exemplar(x, y)[:2]
        g.close()


def test_static_query_rejects_bad_arguments():
    job = synth.small()
    g = B.Inpainter(job.rgb, job.mask, job.patch_radius)
    for args in [(-1, 0, 4, None), (0, 0, 0, None), (0, 0, 9, None), (5, 5, 4, (10, 10, 5, 20))]:
        with pytest.raises(B.InpaintError) as e:
            g.find_exemplar_static(*args)
        assert e.value.status == B.INVALID_ARGUMENT
    with pytest.raises(B.InpaintError) as e:
        g.find_exemplar_static(60, 40, 4, (0, 0, 3, 3))
    assert e.value.status == B.NO_CANDIDATE
    g.close()
