"""Python access to the CPU oracle (oracle.c).

THIS IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.  It
loads ``liboracle.so`` built from ``oracle.c`` in this directory and shares no
code with the HIP library.

Functions without an independent pin: none (every oracle function is pinned by
the CPU tests; see ``tests/test_oracle_pins.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OK, DONE, INVALID_ARGUMENT, NO_CANDIDATE, OUT_OF_MEMORY = 0, 1, -1, -2, -3
SEARCH_FULL, SEARCH_ALPHA, SEARCH_RECT = 0, 1, 2
SOURCE_ORIGINAL, SOURCE_CURRENT = 0, 1
SCORE_WHOLE, SCORE_INTERSECT = 0, 1

# One fill-iteration record (matches oracle_step_info in oracle.c).
STEP_DTYPE = np.dtype([
    ("target_index", "<i8"), ("source_index", "<i8"), ("ssd", "<u4"),
    ("known_k", "<i4"), ("n_filled", "<i4"), ("reserved", "<i4"),
    ("priority", "<f8"), ("confidence", "<f8"), ("data_term", "<f8"),
    ("remaining", "<i8"),
])


def build(force: bool = False) -> str:
    """Compile liboracle.so with contraction off and no fast-math."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.oracle_create.argtypes = [i32, i32, vp, i32, i32, vp, i32, i32, i32, i32, i32, vp,
                                    i32, i32, ctypes.POINTER(vp)]
        L.oracle_create.restype = i32
        L.oracle_destroy.argtypes = [vp]
        L.oracle_destroy.restype = None
        L.oracle_front.argtypes = [vp, vp, i64]
        L.oracle_front.restype = i64
        L.oracle_priority.argtypes = [vp, i32, i32, vp, vp, vp]
        L.oracle_priority.restype = i32
        L.oracle_select.argtypes = [vp, vp, vp, vp, vp]
        L.oracle_select.restype = i32
        L.oracle_find_exemplar.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp]
        L.oracle_find_exemplar.restype = i32
        L.oracle_step.argtypes = [vp, vp]
        L.oracle_step.restype = i32
        L.oracle_run.argtypes = [vp, i64, vp, vp, i64]
        L.oracle_run.restype = i32
        L.oracle_read.argtypes = [vp, vp, vp, vp, vp]
        L.oracle_read.restype = i32
        L.oracle_valid_map.argtypes = [vp, i32, vp]
        L.oracle_valid_map.restype = i32
        L.oracle_get_rect.argtypes = [vp, vp]
        L.oracle_get_rect.restype = i32
        L.oracle_remaining.argtypes = [vp]
        L.oracle_remaining.restype = i64
        L.oracle_import_state.argtypes = [vp, vp, i32, i32, vp, i32, vp, i64]
        L.oracle_import_state.restype = i32
        L.oracle_iterations.argtypes = [vp]
        L.oracle_iterations.restype = i64
        L.oracle_step_info_size.argtypes = []
        L.oracle_step_info_size.restype = i32
        assert L.oracle_step_info_size() == STEP_DTYPE.itemsize
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


class Oracle:
    """One removal job on the CPU oracle."""

    def __init__(self, rgb: np.ndarray, mask: np.ndarray, patch_radius: int,
                 search_mode: int = SEARCH_FULL, alpha=(0, 1), rect=None,
                 source_policy: int = SOURCE_ORIGINAL, scoring: int = SCORE_WHOLE):
        rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        H, W, ch = rgb.shape
        assert mask.shape == (H, W)
        self.W, self.H, self.r = W, H, patch_radius
        rect_a = np.asarray(rect if rect is not None else (0, 0, 0, 0), dtype=np.int32)
        h = ctypes.c_void_p()
        st = lib().oracle_create(W, H, _ptr(rgb), W * ch, ch, _ptr(mask), W, patch_radius,
                                 search_mode, int(alpha[0]), int(alpha[1]), _ptr(rect_a),
                                 source_policy, scoring, ctypes.byref(h))
        if st != OK:
            raise OracleError(st, "oracle_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    # ---- queries
    def front(self) -> np.ndarray:
        n = lib().oracle_front(self._h, None, 0)
        out = np.zeros(max(n, 1), dtype=np.int32)
        lib().oracle_front(self._h, _ptr(out), n)
        return out[:n]

    def priority(self, x: int, y: int):
        c, d, p = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        st = lib().oracle_priority(self._h, x, y, ctypes.byref(c), ctypes.byref(d), ctypes.byref(p))
        if st != OK:
            raise OracleError(st, "oracle_priority")
        return c.value, d.value, p.value

    def select(self):
        i = ctypes.c_int64()
        c, d, p = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        st = lib().oracle_select(self._h, ctypes.byref(i), ctypes.byref(c), ctypes.byref(d),
                                 ctypes.byref(p))
        if st != OK:
            return None
        return i.value, c.value, d.value, p.value

    def find_exemplar(self, x: int, y: int, r: int | None = None, rect=None):
        """Returns (source_index, ssd, known_k) or raises OracleError."""
        r = self.r if r is None else r
        rect_a = np.asarray(rect if rect is not None else self.rect(), dtype=np.int32)
        i, s, k = ctypes.c_int64(), ctypes.c_uint32(), ctypes.c_int32()
        st = lib().oracle_find_exemplar(self._h, x, y, r, _ptr(rect_a), ctypes.byref(i),
                                        ctypes.byref(s), ctypes.byref(k))
        if st != OK:
            raise OracleError(st, "oracle_find_exemplar")
        return i.value, s.value, k.value

    def step(self):
        rec = np.zeros(1, dtype=STEP_DTYPE)
        st = lib().oracle_step(self._h, _ptr(rec))
        if st == DONE:
            return None
        if st != OK:
            raise OracleError(st, "oracle_step")
        return rec[0]

    def run(self, max_iters: int = -1, log_cap: int | None = None):
        """Runs until the hole is empty (or max_iters); returns the log."""
        cap = int(log_cap if log_cap is not None else max(self.remaining(), 1))
        if max_iters >= 0:
            cap = min(cap, max(max_iters, 1))
        log = np.zeros(cap, dtype=STEP_DTYPE)
        done = ctypes.c_int64()
        st = lib().oracle_run(self._h, max_iters, ctypes.byref(done), _ptr(log), cap)
        if st not in (OK, DONE):
            raise OracleError(st, "oracle_run")
        return log[:min(done.value, cap)]

    def read(self):
        n = self.W * self.H
        rgb = np.zeros((self.H, self.W, 3), dtype=np.uint8)
        gray = np.zeros((self.H, self.W), dtype=np.uint8)
        hole = np.zeros((self.H, self.W), dtype=np.uint8)
        conf = np.zeros((self.H, self.W), dtype=np.float64)
        lib().oracle_read(self._h, _ptr(rgb), _ptr(gray), _ptr(hole), _ptr(conf))
        assert n == hole.size
        return rgb, gray, hole, conf

    def valid_map(self, r: int | None = None) -> np.ndarray:
        out = np.zeros((self.H, self.W), dtype=np.uint8)
        st = lib().oracle_valid_map(self._h, self.r if r is None else r, _ptr(out))
        if st != OK:
            raise OracleError(st, "oracle_valid_map")
        return out

    def rect(self):
        out = np.zeros(4, dtype=np.int32)
        lib().oracle_get_rect(self._h, _ptr(out))
        return tuple(int(v) for v in out)

    def remaining(self) -> int:
        return int(lib().oracle_remaining(self._h))

    def iterations(self) -> int:
        return int(lib().oracle_iterations(self._h))

    def export_state(self):
        """(rgb, hole, conf, iterations): what import_state takes back."""
        rgb, _, hole, conf = self.read()
        return rgb, hole, conf, self.iterations()

    def import_state(self, rgb: np.ndarray, hole: np.ndarray, conf: np.ndarray, iterations: int):
        """Continues from a checkpoint of the same removal (see oracle.c)."""
        rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
        hole = np.ascontiguousarray(hole, dtype=np.uint8)
        conf = np.ascontiguousarray(conf, dtype=np.float64)
        assert rgb.shape[:2] == hole.shape == conf.shape == (self.H, self.W)
        ch = rgb.shape[2]
        st = lib().oracle_import_state(self._h, _ptr(rgb), self.W * ch, ch, _ptr(hole), self.W, _ptr(conf),
                                       int(iterations))
        if st != OK:
            raise OracleError(st, "oracle_import_state")
