"""CPU oracles for the filter-bank correlation and the exact nearest-neighbour
search (test infrastructure).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the benchmark's CPU-baseline leg may import this package.  The GPU library
(``paper_0911_3456_amd``) never imports it and shares no code with it.

What it computes (Sec. 6.2, "Computational Visual Neuroscience", and the
table "Performance of RTCG auto-tuning on 3D filter-bank convolutions"): a
bank of N filters fh x fw x D, each spanning the input's full depth D, is
correlated with an H x W x D input over the two spatial axes; valid extent,
stride one, no flip (readings recorded in the design notes).  The arithmetic
is the plain definition written out in ``fbcorr_oracle.c`` and run in double
precision on the exact float32 input values.

The second oracle, ``nearest_oracle.c`` (Sec. 6.4, the natural-image entropy
application), is exhaustive exact nearest-neighbour search over 8-bit patches
in 64-bit integers, lowest index on ties.

Besides the loops this module holds the oracle-side helpers the tests
need: the normalised error metric, round-to-nearest-even casts to bfloat16
and float16 (for an oracle on rounded operands), per-filter power-of-two
scales, and windowed central finite differences of L = sum(g * y).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "fbcorr_oracle.c"), os.path.join(_HERE, "nearest_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, *_SRCS])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            i64 = ctypes.c_int64
            lib.fbo_forward.argtypes = [dp, dp, dp] + [i64] * 7
            lib.fbo_backward_x.argtypes = [dp, dp, dp] + [i64] * 7
            lib.fbo_backward_w.argtypes = [dp, dp, dp] + [i64] * 7
            lib.nno_search.argtypes = [ctypes.c_void_p, ctypes.c_void_p, i64, i64, i64,
                                       ctypes.c_void_p, ctypes.c_void_p]
            lib.fbo_set_threads.argtypes = [ctypes.c_int]
            lib.fbo_max_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as4(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x)
    if x.ndim == 3:
        x = x[None]
    if x.ndim != 4:
        raise ValueError("input must be [H,W,D] or [B,H,W,D]")
    return np.ascontiguousarray(x, dtype=np.float64)


def set_threads(n: int) -> None:
    _load().fbo_set_threads(int(n))


def max_threads() -> int:
    return int(_load().fbo_max_threads())


def forward(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """y[b,i,j,n] = sum_{u,v,d} x[b,i+u,j+v,d] * w[n,u,v,d]  (float64)."""
    squeeze = np.asarray(x).ndim == 3
    x = _as4(x)
    w = np.ascontiguousarray(w, dtype=np.float64)
    B, H, W, D = x.shape
    N, fh, fw, Dw = w.shape
    if Dw != D:
        raise ValueError("filter depth %d != input depth %d" % (Dw, D))
    if fh > H or fw > W:
        raise ValueError("filter larger than input")
    y = np.empty((B, H - fh + 1, W - fw + 1, N), dtype=np.float64)
    _load().fbo_forward(_p(x), _p(w), _p(y), B, H, W, D, N, fh, fw)
    return y[0] if squeeze else y


def backward(x: np.ndarray, w: np.ndarray, g: np.ndarray, want_dx=True, want_dw=True):
    """Adjoint of the forward map for L = sum(g * y), scatter form (float64)."""
    squeeze = np.asarray(x).ndim == 3
    x = _as4(x)
    g = _as4(g)
    w = np.ascontiguousarray(w, dtype=np.float64)
    B, H, W, D = x.shape
    N, fh, fw, _ = w.shape
    if g.shape != (B, H - fh + 1, W - fw + 1, N):
        raise ValueError("gradient shape mismatch")
    lib = _load()
    dx = dw = None
    if want_dx:
        dx = np.empty_like(x)
        lib.fbo_backward_x(_p(w), _p(g), _p(dx), B, H, W, D, N, fh, fw)
        if squeeze:
            dx = dx[0]
    if want_dw:
        dw = np.empty_like(w)
        lib.fbo_backward_w(_p(x), _p(g), _p(dw), B, H, W, D, N, fh, fw)
    return dx, dw


def nearest(targets: np.ndarray, neighbors: np.ndarray):
    """Exact nearest neighbour of every target row among the neighbour rows
    (Sec. 6.4): returns (idx, dist) as int64 arrays, dist the squared
    Euclidean distance, idx the lowest index at that distance."""
    t = np.ascontiguousarray(targets, dtype=np.uint8)
    n = np.ascontiguousarray(neighbors, dtype=np.uint8)
    if t.ndim != 2 or n.ndim != 2 or t.shape[1] != n.shape[1]:
        raise ValueError("targets [T, D] and neighbors [M, D] with the same D")
    if n.shape[0] == 0:
        raise ValueError("empty neighbour set")
    idx = np.empty(t.shape[0], np.int64)
    dist = np.empty(t.shape[0], np.int64)
    _load().nno_search(t.ctypes.data, n.ctypes.data, t.shape[0], n.shape[0], t.shape[1],
                       idx.ctypes.data, dist.ctypes.data)
    return idx, dist


# --------------------------------------------------------------------------
# Error metric.  Any summation order is a correct result, so the error of an
# output is measured against the size of the terms that were summed:
#   e = |y_hat - y_ref| / A,  A = sum over the same index set of |a|*|b|.
# 0/0 counts as 0 and a non-zero error over A = 0 as infinity.
# --------------------------------------------------------------------------

def forward_scale(x, w):
    return forward(np.abs(np.asarray(x, np.float64)), np.abs(np.asarray(w, np.float64)))


def backward_scales(x, w, g):
    return backward(np.abs(np.asarray(x, np.float64)), np.abs(np.asarray(w, np.float64)),
                    np.abs(np.asarray(g, np.float64)))


def normalised_error(y_hat, y_ref, scale):
    """Return (max, mean, argmax index) of |y_hat - y_ref| / scale."""
    y_hat = np.asarray(y_hat, np.float64)
    y_ref = np.asarray(y_ref, np.float64)
    scale = np.asarray(scale, np.float64)
    if y_hat.shape != y_ref.shape or y_ref.shape != scale.shape:
        raise ValueError("shape mismatch %s %s %s" % (y_hat.shape, y_ref.shape, scale.shape))
    if y_ref.size == 0:
        return 0.0, 0.0, None
    diff = np.abs(y_hat - y_ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(scale > 0, diff / np.where(scale > 0, scale, 1.0),
                     np.where(diff > 0, np.inf, 0.0))
    idx = np.unravel_index(int(np.argmax(e)), e.shape)
    return float(e.max()), float(e.mean()), tuple(int(i) for i in idx)


# --------------------------------------------------------------------------
# Reduced-precision operand rounding (oracle side).  Round to nearest, ties
# to even, from float32; used to build an oracle on the rounded operands so
# that accumulation error can be told apart from operand rounding.
# --------------------------------------------------------------------------

def round_to_bf16(a) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    rounded = (bits + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return rounded.astype(np.uint32).view(np.float32).reshape(a.shape)


def round_to_fp16(a) -> np.ndarray:
    """float32 -> nearest IEEE half (ties to even), returned as float32."""
    return np.asarray(a, dtype=np.float32).astype(np.float16).astype(np.float32)


def filter_pow2_scales(w) -> np.ndarray:
    """s_n = 2**-floor(log2(max|w[n]|)), so that max|w[n]| * s_n is in [1, 2).

    A filter of zeros gets s_n = 1.
    """
    w = np.asarray(w, np.float64)
    m = np.abs(w.reshape(w.shape[0], -1)).max(axis=1)
    e = np.zeros_like(m)
    nz = m > 0
    e[nz] = np.floor(np.log2(m[nz]))
    return np.exp2(-e)


# --------------------------------------------------------------------------
# Windowed central finite differences of L(x, w) = sum(g * forward(x, w)).
# Perturbing x[b,p,q,d] changes only y[b] over an fh x fw window of output
# positions; perturbing w[n,...] changes only output channel n.  L is
# evaluated on exactly those outputs, so each difference stays cheap.
# --------------------------------------------------------------------------

def fd_grad_x(x, w, g, coords, h=1e-6):
    x = _as4(x)
    g = _as4(g)
    w = np.asarray(w, np.float64)
    _, H, W, _ = x.shape
    N, fh, fw, _ = w.shape
    Ho, Wo = H - fh + 1, W - fw + 1
    out = np.empty(len(coords))
    for t, (b, p, q, d) in enumerate(coords):
        i0, i1 = max(0, p - fh + 1), min(Ho - 1, p)
        j0, j1 = max(0, q - fw + 1), min(Wo - 1, q)
        if i0 > i1 or j0 > j1:
            out[t] = 0.0
            continue
        sub = x[b, i0:i1 + fh, j0:j1 + fw, :].copy()
        gw = g[b, i0:i1 + 1, j0:j1 + 1, :]
        orig = sub[p - i0, q - j0, d]
        sub[p - i0, q - j0, d] = orig + h
        lp = float(np.sum(gw * forward(sub, w)))
        sub[p - i0, q - j0, d] = orig - h
        lm = float(np.sum(gw * forward(sub, w)))
        out[t] = (lp - lm) / (2 * h)
    return out


def fd_grad_w(x, w, g, coords, h=1e-6):
    x = _as4(x)
    g = _as4(g)
    w = np.array(w, np.float64)
    out = np.empty(len(coords))
    for t, (n, u, v, d) in enumerate(coords):
        wn = w[n:n + 1].copy()
        gn = g[..., n:n + 1]
        orig = wn[0, u, v, d]
        wn[0, u, v, d] = orig + h
        lp = float(np.sum(gn * forward(x, wn)))
        wn[0, u, v, d] = orig - h
        lm = float(np.sum(gn * forward(x, wn)))
        out[t] = (lp - lm) / (2 * h)
    return out
