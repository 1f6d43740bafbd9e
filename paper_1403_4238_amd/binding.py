"""Thin Python binding of libinpaint.so (include/inpaint.h).

Argument marshalling only: every step of the removal runs in the library's
HIP kernels.  PyTorch provides the device workspace (a uint8 tensor) and the
stream.  torch is imported before the library is loaded so that both share
one HIP runtime.  There is no CPU fallback: if the library is missing, or no
GPU is visible, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library will share)

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libinpaint.so")

OK, DONE = 0, 1
INVALID_ARGUMENT, NO_CANDIDATE, OUT_OF_MEMORY, DEVICE = -1, -2, -3, -4
SEARCH_FULL, SEARCH_ALPHA, SEARCH_RECT = 0, 1, 2
PATH_AUTO, PATH_SIMT, PATH_MFMA, PATH_SIMT_DIRECT = 0, 1, 2, 3
SOURCE_ORIGINAL, SOURCE_CURRENT = 0, 1
SCORE_WHOLE, SCORE_INTERSECT = 0, 1
FORM_PLAIN, FORM_STREAM, FORM_GRAPH, FORM_PERSISTENT = 0, 1, 2, 3
FORMS = {"plain": FORM_PLAIN, "stream": FORM_STREAM, "graph": FORM_GRAPH, "persistent": FORM_PERSISTENT}
FORM_NAMES = {v: k for k, v in FORMS.items()}


class inpaint_image(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("stride_bytes", ctypes.c_int32), ("channels", ctypes.c_int32)]


class inpaint_rect(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_int32), ("y0", ctypes.c_int32), ("x1", ctypes.c_int32),
                ("y1", ctypes.c_int32)]


class inpaint_params(ctypes.Structure):
    _fields_ = [("patch_radius", ctypes.c_int32), ("search_mode", ctypes.c_int32),
                ("alpha_num", ctypes.c_int32), ("alpha_den", ctypes.c_int32),
                ("rect", inpaint_rect), ("path", ctypes.c_int32), ("form", ctypes.c_int32),
                ("iters_per_check", ctypes.c_int32), ("log_capacity", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32), ("source_policy", ctypes.c_int32),
                ("scoring", ctypes.c_int32), ("reserved", ctypes.c_int32 * 1)]


class inpaint_batch_params(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int32), ("graph_iters", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("form", ctypes.c_int32),
                ("tune_cache", ctypes.c_char_p)]


# inpaint_step_info as a numpy record (64 bytes).
STEP_DTYPE = np.dtype([
    ("target_index", "<i8"), ("source_index", "<i8"), ("ssd", "<u4"),
    ("known_k", "<i4"), ("n_filled", "<i4"), ("reserved", "<i4"),
    ("priority", "<f8"), ("confidence", "<f8"), ("data_term", "<f8"),
    ("remaining", "<i8"),
])

_lib = None


def lib() -> ctypes.CDLL:
    """Loads libinpaint.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "or `python -m paper_1403_4238_amd.csrc.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    P = ctypes.POINTER
    sig = {
        "inpaint_workspace_bytes": (i32, [i32, i32, P(inpaint_params), P(u64)]),
        "inpaint_create": (i32, [P(inpaint_image), vp, i32, P(inpaint_params), vp, u64, vp, P(vp)]),
        "inpaint_find_exemplar": (i32, [vp, i32, i32, i32, inpaint_rect, P(i64), P(ctypes.c_uint32)]),
        "inpaint_find_exemplar_static": (i32, [vp, i32, i32, i32, inpaint_rect, P(i64), P(ctypes.c_uint32)]),
        "inpaint_step": (i32, [vp, vp]),
        "inpaint_run": (i32, [vp, i64, P(i64), vp, i64]),
        "inpaint_read_log": (i32, [vp, i64, i64, vp]),
        "inpaint_read_image": (i32, [vp, vp, i32]),
        "inpaint_read_state": (i32, [vp, vp, vp]),
        "inpaint_remaining": (i32, [vp, P(i64)]),
        "inpaint_search_info": (i32, [vp, P(inpaint_rect), P(i64)]),
        "inpaint_progress": (i32, [vp, P(i64), P(i64)]),
        "inpaint_batch_status": (i32, [vp, i32, P(i32)]),
        "inpaint_profile_search": (i32, [vp, i32]),
        "inpaint_search_time": (i32, [vp, P(ctypes.c_double), P(i64)]),
        "inpaint_run_form": (i32, [vp, P(i32)]),
        "inpaint_import_state": (i32, [vp, vp, i32, i32, vp, i32, vp, i64]),
        "inpaint_destroy": (i32, [vp]),
        "inpaint_status_string": (ctypes.c_char_p, [i32]),
        "inpaint_last_error": (ctypes.c_char_p, [vp]),
        "inpaint_batch_create": (i32, [P(inpaint_batch_params), vp, P(vp)]),
        "inpaint_batch_attach": (i32, [vp, vp, P(i32)]),
        "inpaint_batch_detach": (i32, [vp, vp]),
        "inpaint_batch_step": (i32, [vp, i32, P(i64)]),
        "inpaint_batch_form": (i32, [vp, P(i32)]),
        "inpaint_batch_room": (i32, [vp, vp, i32, P(i32)]),
        "inpaint_batch_destroy": (i32, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class InpaintError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str = ""):
        msg = f"{what}: {inpaint_status_string(status)}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)
        self.status = status


def inpaint_status_string(status: int) -> str:
    return lib().inpaint_status_string(status).decode()


def inpaint_last_error(ctx) -> str:
    s = lib().inpaint_last_error(ctx)
    return s.decode() if s else ""


def make_params(patch_radius: int, search_mode: int = SEARCH_FULL, alpha=(0, 1), rect=(0, 0, 0, 0),
                path: int = PATH_AUTO, form: str = "plain", iters_per_check: int = 16,
                log_capacity: int = 0, tile_rows: int = 0, source_policy: int = SOURCE_ORIGINAL,
                scoring: int = SCORE_WHOLE) -> inpaint_params:
    p = inpaint_params()
    p.patch_radius = patch_radius
    p.search_mode = search_mode
    p.alpha_num, p.alpha_den = int(alpha[0]), int(alpha[1])
    p.rect = inpaint_rect(*rect)
    p.path = path
    p.form = FORMS[form]
    p.iters_per_check = iters_per_check
    p.log_capacity = log_capacity
    p.tile_rows = tile_rows
    p.source_policy = source_policy
    p.scoring = scoring
    return p


def inpaint_workspace_bytes(width: int, height: int, params: inpaint_params) -> int:
    out = ctypes.c_uint64()
    st = lib().inpaint_workspace_bytes(width, height, ctypes.byref(params), ctypes.byref(out))
    if st != OK:
        raise InpaintError(st, "inpaint_workspace_bytes")
    return out.value


def current_stream_handle() -> int:
    return torch.cuda.current_stream().cuda_stream


class Inpainter:
    """One removal job: a context plus the torch workspace it lives in."""

    def __init__(self, rgb: np.ndarray, mask: np.ndarray, patch_radius: int,
                 search_mode: int = SEARCH_FULL, alpha=(0, 1), rect=(0, 0, 0, 0),
                 path: int = PATH_AUTO, form: str = "plain", iters_per_check: int = 16,
                 log_capacity: int | None = None, tile_rows: int = 0, device: str = "cuda",
                 stream=None, source_policy: int = SOURCE_ORIGINAL, scoring: int = SCORE_WHOLE):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: libinpaint has no CPU path")
        rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        H, W, ch = rgb.shape
        if mask.shape != (H, W):
            raise ValueError("mask shape does not match the image")
        if log_capacity is None:
            log_capacity = int(np.count_nonzero(mask))
        self.params = make_params(patch_radius, search_mode, alpha, rect, path, form,
                                  iters_per_check, log_capacity, tile_rows, source_policy, scoring)
        self.width, self.height = W, H
        self.ws_bytes = inpaint_workspace_bytes(W, H, self.params)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        img = inpaint_image(rgb.ctypes.data, W, H, W * ch, ch)
        h = ctypes.c_void_p()
        st = lib().inpaint_create(ctypes.byref(img), mask.ctypes.data, W, ctypes.byref(self.params),
                                  self.workspace.data_ptr(), self.ws_bytes, self.stream.cuda_stream,
                                  ctypes.byref(h))
        if st != OK:
            raise InpaintError(st, "inpaint_create", inpaint_last_error(None))
        self.ctx = h

    # ---- lifetime
    def close(self):
        if getattr(self, "ctx", None):
            lib().inpaint_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, what: str) -> int:
        if st < 0:
            raise InpaintError(st, what, inpaint_last_error(self.ctx))
        return st

    # ---- calls
    def find_exemplar(self, x: int, y: int, patch_radius: int | None = None, rect=None):
        r = self.params.patch_radius if patch_radius is None else patch_radius
        rc = inpaint_rect(*(rect if rect is not None else (0, 0, self.width, self.height)))
        idx, ssd = ctypes.c_int64(), ctypes.c_uint32()
        self._check(lib().inpaint_find_exemplar(self.ctx, x, y, r, rc, ctypes.byref(idx),
                                                ctypes.byref(ssd)), "inpaint_find_exemplar")
        return idx.value, ssd.value

    def find_exemplar_static(self, x: int, y: int, patch_radius: int | None = None, rect=None):
        """find_exemplar through the allocation-free entry point."""
        r = self.params.patch_radius if patch_radius is None else patch_radius
        rc = inpaint_rect(*(rect if rect is not None else (0, 0, self.width, self.height)))
        idx, ssd = ctypes.c_int64(), ctypes.c_uint32()
        self._check(lib().inpaint_find_exemplar_static(self.ctx, x, y, r, rc, ctypes.byref(idx),
                                                       ctypes.byref(ssd)), "inpaint_find_exemplar_static")
        return idx.value, ssd.value

    def step(self):
        rec = np.zeros(1, dtype=STEP_DTYPE)
        st = self._check(lib().inpaint_step(self.ctx, rec.ctypes.data), "inpaint_step")
        return None if st == DONE else rec[0]

    def run(self, max_iters: int = -1, log_cap: int = 0):
        log = np.zeros(max(log_cap, 1), dtype=STEP_DTYPE)
        done = ctypes.c_int64()
        st = self._check(lib().inpaint_run(self.ctx, max_iters, ctypes.byref(done),
                                           log.ctypes.data if log_cap > 0 else None, log_cap),
                         "inpaint_run")
        n = min(done.value, log_cap)
        return st, done.value, log[:n]

    def read_log(self, first: int, count: int):
        out = np.zeros(max(count, 1), dtype=STEP_DTYPE)
        self._check(lib().inpaint_read_log(self.ctx, first, count, out.ctypes.data), "inpaint_read_log")
        return out[:count]

    def read_image(self) -> np.ndarray:
        out = np.zeros((self.height, self.width, 3), dtype=np.uint8)
        self._check(lib().inpaint_read_image(self.ctx, out.ctypes.data, self.width * 3), "inpaint_read_image")
        return out

    def read_state(self):
        mask = np.zeros((self.height, self.width), dtype=np.uint8)
        conf = np.zeros((self.height, self.width), dtype=np.float64)
        self._check(lib().inpaint_read_state(self.ctx, mask.ctypes.data, conf.ctypes.data), "inpaint_read_state")
        return mask, conf

    def remaining(self) -> int:
        out = ctypes.c_int64()
        self._check(lib().inpaint_remaining(self.ctx, ctypes.byref(out)), "inpaint_remaining")
        return out.value

    def progress(self):
        """(iterations committed, hole pixels left)."""
        it, rem = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().inpaint_progress(self.ctx, ctypes.byref(it), ctypes.byref(rem)), "inpaint_progress")
        return it.value, rem.value

    def export_state(self):
        """(rgb, hole, conf, iterations): a checkpoint that import_state takes back."""
        hole, conf = self.read_state()
        return self.read_image(), hole, conf, self.progress()[0]

    def import_state(self, rgb: np.ndarray, hole: np.ndarray, conf: np.ndarray, iterations: int):
        """Continues this removal from a checkpoint of it (inpaint_import_state)."""
        rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
        hole = np.ascontiguousarray(hole, dtype=np.uint8)
        conf = np.ascontiguousarray(conf, dtype=np.float64)
        if rgb.shape[:2] != (self.height, self.width) or hole.shape != rgb.shape[:2] or conf.shape != hole.shape:
            raise ValueError("checkpoint shape does not match the context")
        ch = rgb.shape[2]
        self._check(lib().inpaint_import_state(self.ctx, rgb.ctypes.data, self.width * ch, ch, hole.ctypes.data,
                                               self.width, conf.ctypes.data, int(iterations)),
                    "inpaint_import_state")

    def profile_search(self, enable: bool = True):
        self._check(lib().inpaint_profile_search(self.ctx, 1 if enable else 0), "inpaint_profile_search")

    def search_time(self):
        """(summed search-kernel milliseconds, searches timed)."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._check(lib().inpaint_search_time(self.ctx, ctypes.byref(ms), ctypes.byref(n)), "inpaint_search_time")
        return ms.value, n.value

    def run_form(self) -> str:
        """The execution form inpaint_run uses ("persistent" may become "stream")."""
        f = ctypes.c_int32()
        self._check(lib().inpaint_run_form(self.ctx, ctypes.byref(f)), "inpaint_run_form")
        return FORM_NAMES[f.value]

    def search_info(self):
        rc, n = inpaint_rect(), ctypes.c_int64()
        self._check(lib().inpaint_search_info(self.ctx, ctypes.byref(rc), ctypes.byref(n)), "inpaint_search_info")
        return (rc.x0, rc.y0, rc.x1, rc.y1), n.value


class Batch:
    """Many contexts advanced together by the persistent, graph-replayed form."""

    def __init__(self, capacity: int, graph_iters: int = 8, autotune: bool = True,
                 tune_cache: str | None = None, stream=None, form: str = "auto"):
        fid = {"auto": 0, "graph": FORMS["graph"], "persistent": FORMS["persistent"]}[form]
        self.params = inpaint_batch_params(capacity, graph_iters, 1 if autotune else 0, fid,
                                           tune_cache.encode() if tune_cache else None)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        st = lib().inpaint_batch_create(ctypes.byref(self.params), self.stream.cuda_stream, ctypes.byref(h))
        if st != OK:
            raise InpaintError(st, "inpaint_batch_create")
        self.h = h
        self.members = {}

    def attach(self, job: Inpainter) -> int:
        slot = ctypes.c_int32()
        st = lib().inpaint_batch_attach(self.h, job.ctx, ctypes.byref(slot))
        if st != OK:
            raise InpaintError(st, "inpaint_batch_attach", inpaint_last_error(job.ctx))
        self.members[slot.value] = job
        return slot.value

    def slot_of(self, job: Inpainter) -> int:
        for k, v in self.members.items():
            if v is job:
                return k
        raise KeyError("job is not attached")

    def status(self, job: Inpainter) -> int:
        """Slot state after the last step: 1 running, 2 finished, 3 error."""
        out = ctypes.c_int32()
        st = lib().inpaint_batch_status(self.h, self.slot_of(job), ctypes.byref(out))
        if st != OK:
            raise InpaintError(st, "inpaint_batch_status")
        return out.value

    def detach(self, job: Inpainter):
        st = lib().inpaint_batch_detach(self.h, job.ctx)
        if st != OK:
            raise InpaintError(st, "inpaint_batch_detach")
        for k, v in list(self.members.items()):
            if v is job:
                del self.members[k]

    def last_form(self) -> str:
        """Form the last step ran in: "persistent" or "graph"."""
        out = ctypes.c_int32()
        st = lib().inpaint_batch_form(self.h, ctypes.byref(out))
        if st != OK:
            raise InpaintError(st, "inpaint_batch_form")
        return {v: k for k, v in FORMS.items()}[out.value]

    def room(self, job: Inpainter, tiles_per_group: int = 1) -> bool:
        """Whether the running images and ``job`` (not attached) fit the
        persistent form with at most ``tiles_per_group`` search tiles per
        search work-group (1: every tile resident)."""
        out = ctypes.c_int32()
        st = lib().inpaint_batch_room(self.h, job.ctx, int(tiles_per_group), ctypes.byref(out))
        if st != OK:
            raise InpaintError(st, "inpaint_batch_room")
        return bool(out.value)

    def step(self, G: int | None = None) -> int:
        active = ctypes.c_int64()
        st = lib().inpaint_batch_step(self.h, int(G or self.params.graph_iters), ctypes.byref(active))
        if st != OK:
            raise InpaintError(st, "inpaint_batch_step")
        return active.value

    def close(self):
        if getattr(self, "h", None):
            lib().inpaint_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
