"""ctypes binding of the fbcorr C ABI (``include/fbcorr.h``, ``include/fbnn.h``).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libfbcorr.so``.  torch is imported first so that the library's
``libamdhip64``/``libhiprtc`` dependencies resolve to the copies torch has
already loaded (one HIP runtime per process; torch's stream handles are then
valid in the library).  There is no fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (load order: torch's HIP runtime first)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfbcorr.so")

FBCORR_OK = 0
STATUS_NAMES = {
    0: "FBCORR_OK", 1: "FBCORR_ERR_INVALID_ARGUMENT", 2: "FBCORR_ERR_SHAPE",
    3: "FBCORR_ERR_UNSUPPORTED", 4: "FBCORR_ERR_COMPILE", 5: "FBCORR_ERR_LAUNCH",
    6: "FBCORR_ERR_WORKSPACE", 7: "FBCORR_ERR_NO_DEVICE", 8: "FBCORR_ERR_INTERNAL",
}
PRECISIONS = {"fp32": 0, "bf16": 1, "fp16": 2}
ALGOS = {"auto": 0, "direct": 1, "igemm": 2}
ROLES = {"forward": 0, "backward_x": 1, "backward_w": 2}

# Every entry point declared in include/fbcorr.h.
EXPORTS = (
    "fbcorr_plan", "fbcorr_plan_destroy", "fbcorr_workspace_size", "fbcorr_forward", "fbcorr_forward_noalloc",
    "fbcorr_backward", "fbcorr_tune", "fbcorr_plan_batched", "fbcorr_forward_batched",
    "fbcorr_plan_get_config", "fbcorr_plan_set_config", "fbcorr_plan_set_epilogue", "fbcorr_plan_enable_timing",
    "fbcorr_plan_read_timing", "fbcorr_codegen", "fbcorr_compile_check", "fbcorr_compile_check_batched",
    "fbcorr_cache_stats", "fbcorr_cache_clear",
    "fbcorr_last_error", "fbcorr_status_string", "fbcorr_version",
)
# Every entry point declared in include/fbnn.h.
NN_EXPORTS = (
    "fbnn_plan", "fbnn_plan_destroy", "fbnn_workspace_size", "fbnn_search", "fbnn_tune",
    "fbnn_plan_get_config", "fbnn_plan_set_config", "fbnn_plan_enable_timing", "fbnn_plan_read_timing",
    "fbnn_compile_check",
)


class NNDesc(ctypes.Structure):
    _fields_ = [("n_targets", ctypes.c_int64), ("n_neighbors", ctypes.c_int64), ("dim", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class Desc(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("D", ctypes.c_int32), ("N", ctypes.c_int32), ("fh", ctypes.c_int32),
                ("fw", ctypes.c_int32), ("precision", ctypes.c_int32), ("algo", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class TuneOpts(ctypes.Structure):
    _fields_ = [("warmup", ctypes.c_int32), ("reps", ctypes.c_int32),
                ("max_candidates", ctypes.c_int32), ("role", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class TuneReport(ctypes.Structure):
    _fields_ = [("n_tried", ctypes.c_int32), ("n_compiled", ctypes.c_int32),
                ("n_rejected_resources", ctypes.c_int32), ("n_rejected_parity", ctypes.c_int32),
                ("n_failed", ctypes.c_int32), ("best_ms", ctypes.c_double),
                ("default_ms", ctypes.c_double), ("best_cfg", ctypes.c_char * 256),
                ("default_cfg", ctypes.c_char * 256)]

    def as_dict(self):
        return {k: (getattr(self, k).decode() if isinstance(getattr(self, k), bytes) else getattr(self, k))
                for k, _ in self._fields_}


class FbcorrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(message)
        self.status = status
        self.status_name = STATUS_NAMES.get(status, str(status))


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libfbcorr.so (built in-tree by ``paper_0911_3456_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("fbcorr native library not built: %s (run __graft_entry__.build())" % path)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    st = ctypes.c_int
    sz = ctypes.c_size_t
    lib.fbcorr_plan.argtypes = [ctypes.POINTER(Desc), ctypes.c_int, ctypes.POINTER(P)]
    lib.fbcorr_plan_destroy.argtypes = [P]
    lib.fbcorr_workspace_size.argtypes = [P, ctypes.c_int, ctypes.POINTER(sz)]
    lib.fbcorr_forward.argtypes = [P, P, P, P, P, sz, P]
    lib.fbcorr_backward.argtypes = [P, P, P, P, P, P, P, sz, P]
    lib.fbcorr_tune.argtypes = [P, P, P, P, P, sz, P, ctypes.POINTER(TuneOpts), ctypes.POINTER(TuneReport)]
    lib.fbcorr_plan_batched.argtypes = [ctypes.c_int32, ctypes.POINTER(Desc), ctypes.c_int, ctypes.POINTER(P)]
    lib.fbcorr_forward_batched.argtypes = [P, P, P, P, P, sz, P, ctypes.c_int]
    lib.fbcorr_plan_get_config.argtypes = [P, ctypes.c_int, ctypes.c_char_p, sz]
    lib.fbcorr_plan_set_config.argtypes = [P, ctypes.c_int, ctypes.c_char_p]
    lib.fbcorr_plan_set_epilogue.argtypes = [P, ctypes.c_char_p]
    lib.fbcorr_plan_enable_timing.argtypes = [P, ctypes.c_int]
    lib.fbcorr_plan_read_timing.argtypes = [P, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    lib.fbcorr_codegen.argtypes = [ctypes.POINTER(Desc), ctypes.c_int, ctypes.c_char_p, ctypes.c_char_p,
                                   ctypes.POINTER(sz), ctypes.c_char_p, ctypes.POINTER(sz)]
    lib.fbcorr_compile_check.argtypes = [ctypes.POINTER(Desc), ctypes.c_int, ctypes.c_char_p,
                                         ctypes.c_char_p, ctypes.POINTER(sz)]
    lib.fbcorr_compile_check_batched.argtypes = [ctypes.c_int32, ctypes.POINTER(Desc), ctypes.c_char_p,
                                                 ctypes.POINTER(sz)]
    lib.fbcorr_cache_stats.argtypes = [ctypes.POINTER(ctypes.c_int64)] * 4
    lib.fbcorr_cache_clear.argtypes = []
    lib.fbcorr_last_error.restype = ctypes.c_char_p
    lib.fbcorr_last_error.argtypes = []
    lib.fbcorr_status_string.restype = ctypes.c_char_p
    lib.fbcorr_status_string.argtypes = [ctypes.c_int]
    lib.fbcorr_version.restype = ctypes.c_int
    lib.fbnn_plan.argtypes = [ctypes.POINTER(NNDesc), ctypes.c_int, ctypes.POINTER(P)]
    lib.fbnn_plan_destroy.argtypes = [P]
    lib.fbnn_workspace_size.argtypes = [P, ctypes.c_int, ctypes.POINTER(sz)]
    lib.fbnn_search.argtypes = [P, P, P, P, P, P, sz, P]
    lib.fbnn_tune.argtypes = [P, P, P, P, sz, P, ctypes.POINTER(TuneOpts), ctypes.POINTER(TuneReport)]
    lib.fbnn_plan_get_config.argtypes = [P, ctypes.c_char_p, sz]
    lib.fbnn_plan_set_config.argtypes = [P, ctypes.c_char_p]
    lib.fbnn_plan_enable_timing.argtypes = [P, ctypes.c_int]
    lib.fbnn_plan_read_timing.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                          ctypes.c_int]
    lib.fbnn_compile_check.argtypes = [ctypes.POINTER(NNDesc), ctypes.c_char_p, ctypes.c_char_p,
                                       ctypes.POINTER(sz)]
    for name in NN_EXPORTS:
        getattr(lib, name).restype = st
    for name in EXPORTS:
        if name not in ("fbcorr_last_error", "fbcorr_status_string", "fbcorr_version"):
            getattr(lib, name).restype = st
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != FBCORR_OK:
        msg = (_lib.fbcorr_last_error() or b"").decode(errors="replace")
        raise FbcorrError(status, msg or STATUS_NAMES.get(status, str(status)))


FLAG_OVERLAP_BACKWARD = 1


def make_desc(batch, H, W, D, N, fh, fw, precision="fp32", algo="auto", flags=0) -> Desc:
    return Desc(batch, H, W, D, N, fh, fw, PRECISIONS[precision], ALGOS[algo], flags)


def codegen(desc: Desc, role: str = "forward", cfg: str | None = None):
    """Generated HIP source and -D options of a role (host only)."""
    lib = load()
    sl, ol = ctypes.c_size_t(0), ctypes.c_size_t(0)
    c = cfg.encode() if cfg else None
    check(lib.fbcorr_codegen(ctypes.byref(desc), ROLES[role], c, None, ctypes.byref(sl), None, ctypes.byref(ol)))
    sb, ob = ctypes.create_string_buffer(sl.value), ctypes.create_string_buffer(ol.value)
    check(lib.fbcorr_codegen(ctypes.byref(desc), ROLES[role], c, sb, ctypes.byref(sl), ob, ctypes.byref(ol)))
    return sb.value.decode(), ob.value.decode()


def compile_check(desc: Desc, role: str = "forward", cfg: str | None = None, arch: str = "gfx950") -> int:
    """Compile a role's kernels with hiprtc for ``arch`` without a device."""
    lib = load()
    n = ctypes.c_size_t(0)
    check(lib.fbcorr_compile_check(ctypes.byref(desc), ROLES[role], cfg.encode() if cfg else None,
                                   arch.encode(), ctypes.byref(n)))
    return n.value


def compile_check_batched(descs, arch: str = "gfx950") -> int:
    """Generate and compile the persistent batched kernel for a list of
    descriptors without a device."""
    lib = load()
    arr = (Desc * len(descs))(*descs)
    n = ctypes.c_size_t(0)
    check(lib.fbcorr_compile_check_batched(len(descs), arr, arch.encode(), ctypes.byref(n)))
    return n.value


def nn_compile_check(n_targets: int, n_neighbors: int, dim: int, cfg: str | None = None,
                     arch: str = "gfx950") -> int:
    """Compile the nearest-neighbour kernels with hiprtc without a device."""
    lib = load()
    n = ctypes.c_size_t(0)
    d = NNDesc(n_targets, n_neighbors, dim, 0)
    check(lib.fbnn_compile_check(ctypes.byref(d), cfg.encode() if cfg else None, arch.encode(), ctypes.byref(n)))
    return n.value


def cache_stats():
    lib = load()
    a, b, c, d = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    check(lib.fbcorr_cache_stats(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
    return {"hits": a.value, "misses": b.value, "entries": c.value, "disk_hits": d.value}


def cache_clear() -> None:
    check(load().fbcorr_cache_clear())
