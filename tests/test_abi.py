"""The C-ABI library loads and exports every symbol include/inpaint.h
declares; host-only argument checks (no device work) behave as documented."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "inpaint.h")
LIB = os.path.join(ROOT, "paper_1403_4238_amd", "libinpaint.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(inpaint_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} not built (run __graft_entry__.build())")
    return LIB


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["inpaint_create", "inpaint_find_exemplar", "inpaint_step", "inpaint_run",
                     "inpaint_workspace_bytes", "inpaint_batch_step", "inpaint_destroy",
                     "inpaint_import_state"]:
        assert required in names


def test_library_exports_every_declared_symbol(so):
    out = subprocess.run(["nm", "-D", "--defined-only", so], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(inpaint_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    # C linkage: no mangled inpaint symbols leak out
    assert not re.search(r"\sT\s_Z\w*inpaint_(create|run|step)\b", out)


def test_library_loads_and_host_only_calls(so):
    L = ctypes.CDLL(so)
    L.inpaint_status_string.restype = ctypes.c_char_p
    assert L.inpaint_status_string(0) == b"ok"
    assert L.inpaint_status_string(-2).startswith(b"no valid source")

    from paper_1403_4238_amd.binding import inpaint_params, inpaint_rect
    p = inpaint_params()
    p.patch_radius = 4
    p.alpha_den = 1
    b = ctypes.c_uint64()
    f = L.inpaint_workspace_bytes
    f.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(inpaint_params), ctypes.POINTER(ctypes.c_uint64)]
    assert f(1920, 1080, ctypes.byref(p), ctypes.byref(b)) == 0
    n = 1920 * 1080
    npad = ((8 + 1920 + 84 + 7) // 8 * 8) * (8 + 1080 + 72)
    # RGBX + gray + hole + original hole + validity + confidence + cached
    # priority terms (C, D), the padded search planes (RGBX + validity), plus
    # small tables
    base = 4 * n + 4 * n + 8 * n + 16 * n + 5 * npad
    assert base <= b.value < base + 2_000_000
    p.log_capacity = 1000
    b2 = ctypes.c_uint64()
    assert f(1920, 1080, ctypes.byref(p), ctypes.byref(b2)) == 0
    assert b2.value - b.value >= 64 * 1000 - 256
    # argument checks
    assert f(8, 8, ctypes.byref(p), ctypes.byref(b)) == -1         # smaller than the 9x9 patch
    p.patch_radius = 9
    assert f(100, 100, ctypes.byref(p), ctypes.byref(b)) == -1     # radius out of range
    p.patch_radius = 4
    p.tile_rows = 5
    assert f(100, 100, ctypes.byref(p), ctypes.byref(b)) == -1
    p.tile_rows = 0
    p.search_mode = 2
    p.rect = inpaint_rect(10, 0, 5, 10)
    assert f(100, 100, ctypes.byref(p), ctypes.byref(b)) == -1     # x0 > x1
    p.search_mode = 1
    p.alpha_den = 0
    assert f(100, 100, ctypes.byref(p), ctypes.byref(b)) == -1
    p.alpha_den = 1
    p.reserved[0] = 3
    assert f(100, 100, ctypes.byref(p), ctypes.byref(b)) == -1
    p.reserved[0] = 0
    # iterations per dispatch: a persistent dispatch counts them in 25 bits
    p.form = 3
    for ipc, ok in ((1, True), ((1 << 25) - 2, True), ((1 << 25) - 1, False), (0, False)):
        p.iters_per_check = ipc
        assert (f(100, 100, ctypes.byref(p), ctypes.byref(b)) == 0) == ok, ipc


def test_step_record_layout():
    from paper_1403_4238_amd.binding import STEP_DTYPE, inpaint_params
    import oracle
    assert STEP_DTYPE.itemsize == 64
    assert ctypes.sizeof(inpaint_params) == 4 * 16
    assert oracle.STEP_DTYPE.names == STEP_DTYPE.names


def test_create_rejects_empty_and_full_masks_before_device_work(so):
    # The caller's mask is counted on the host first: an empty or full mask
    # is an argument error, returned before any upload or kernel (the
    # workspace pointer below is host memory and is never used).
    import numpy as np
    from paper_1403_4238_amd.binding import inpaint_image, inpaint_params
    L = ctypes.CDLL(so)
    L.inpaint_create.argtypes = [ctypes.POINTER(inpaint_image), ctypes.c_void_p, ctypes.c_int32,
                                 ctypes.POINTER(inpaint_params), ctypes.c_void_p, ctypes.c_uint64,
                                 ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    L.inpaint_last_error.restype = ctypes.c_char_p
    L.inpaint_last_error.argtypes = [ctypes.c_void_p]
    W, H = 40, 30
    rgb = np.zeros((H, W, 3), np.uint8)
    img = inpaint_image()
    img.data = rgb.ctypes.data
    img.width, img.height, img.channels, img.stride_bytes = W, H, 3, 3 * W
    p = inpaint_params()
    p.patch_radius = 2
    p.alpha_den = 1
    need = ctypes.c_uint64()
    L.inpaint_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(inpaint_params),
                                          ctypes.POINTER(ctypes.c_uint64)]
    assert L.inpaint_workspace_bytes(W, H, ctypes.byref(p), ctypes.byref(need)) == 0
    host = np.zeros(int(need.value) + 256, np.uint8)
    ws = (host.ctypes.data + 255) // 256 * 256
    out = ctypes.c_void_p()
    for fill, why in ((0, b"mask is empty"), (1, b"mask covers the whole image")):
        mask = np.full((H, W), fill, np.uint8)
        st = L.inpaint_create(ctypes.byref(img), mask.ctypes.data, W, ctypes.byref(p), ws, need.value, None,
                              ctypes.byref(out))
        assert st == -1 and out.value is None
        assert L.inpaint_last_error(None) == why
