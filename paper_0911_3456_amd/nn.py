"""Exact brute-force nearest-neighbour search over 8-bit patches
(``include/fbnn.h``; Sec. 6.4, the natural-image entropy application).

Argument marshalling only: the search runs in the HIP kernels of
``libfbcorr.so``.
"""
from __future__ import annotations

import ctypes

import torch

from . import _native as nat
from .plan import _ptr, _stream_handle


def _check_u8(t: torch.Tensor, shape, name: str) -> None:
    if not t.is_cuda or t.dtype != torch.uint8 or not t.is_contiguous():
        raise ValueError("%s must be a contiguous uint8 GPU tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    if t.data_ptr() % 16:
        raise ValueError("%s must be 16-byte aligned" % name)


class NNPlan:
    """A compiled nearest-neighbour search for T targets, M neighbours and
    D bytes per patch."""

    def __init__(self, n_targets: int, n_neighbors: int, dim: int = 64, device=None):
        self.lib = nat.load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        self.shape = (n_targets, n_neighbors, dim)
        self.desc = nat.NNDesc(n_targets, n_neighbors, dim, 0)
        h = ctypes.c_void_p()
        nat.check(self.lib.fbnn_plan(ctypes.byref(self.desc), self.device.index, ctypes.byref(h)))
        self.handle = h
        self._ws = {}

    @property
    def ops(self) -> int:
        """Integer operations of the exhaustive comparison: one multiply and
        one add per pixel pair."""
        T, M, D = self.shape
        return 2 * T * M * D

    def workspace_size(self, pass_: int = 0) -> int:
        n = ctypes.c_size_t()
        nat.check(self.lib.fbnn_workspace_size(self.handle, pass_, ctypes.byref(n)))
        return n.value

    def workspace(self, pass_: int = 0) -> torch.Tensor:
        n = self.workspace_size(pass_)
        t = self._ws.get(pass_)
        if t is None or t.numel() < n:
            t = torch.empty(n + 256, dtype=torch.uint8, device=self.device)
            off = (-t.data_ptr()) % 256
            t = t[off:off + n]
            self._ws[pass_] = t
        return t

    def search(self, targets: torch.Tensor, neighbors: torch.Tensor, idx=None, dist=None):
        """Return (idx, dist) int32 tensors: nearest neighbour row and squared
        distance of every target (lowest index on ties)."""
        T, M, D = self.shape
        _check_u8(targets, (T, D), "targets")
        _check_u8(neighbors, (M, D), "neighbors")
        if idx is None:
            idx = torch.empty(max(T, 1), dtype=torch.int32, device=self.device)[:T]
        if dist is None:
            dist = torch.empty(max(T, 1), dtype=torch.int32, device=self.device)[:T]
        ws = self.workspace(0)
        nat.check(self.lib.fbnn_search(self.handle, _ptr(targets), _ptr(neighbors), _ptr(idx), _ptr(dist),
                                       _ptr(ws), ws.numel(), ctypes.c_void_p(_stream_handle(self.device))))
        return idx, dist

    def tune(self, targets, neighbors, warmup=2, reps=10, max_candidates=0, record=False):
        T, M, D = self.shape
        _check_u8(targets, (T, D), "targets")
        _check_u8(neighbors, (M, D), "neighbors")
        ws = self.workspace(1)
        opts = nat.TuneOpts(warmup, reps, max_candidates, 0, 2 if record else 0)
        rep = nat.TuneReport()
        nat.check(self.lib.fbnn_tune(self.handle, _ptr(targets), _ptr(neighbors), _ptr(ws), ws.numel(),
                                     ctypes.c_void_p(_stream_handle(self.device)), ctypes.byref(opts),
                                     ctypes.byref(rep)))
        return rep.as_dict()

    def get_config(self) -> str:
        buf = ctypes.create_string_buffer(512)
        nat.check(self.lib.fbnn_plan_get_config(self.handle, buf, 512))
        return buf.value.decode()

    def set_config(self, cfg: str) -> None:
        nat.check(self.lib.fbnn_plan_set_config(self.handle, cfg.encode()))

    def enable_timing(self, on=True) -> None:
        nat.check(self.lib.fbnn_plan_enable_timing(self.handle, 1 if on else 0))

    def read_timing(self, reset=True):
        """{'prepare'|'scan'|'final': (total ms, searches)}"""
        ms = (ctypes.c_double * 3)()
        calls = (ctypes.c_int64 * 3)()
        nat.check(self.lib.fbnn_plan_read_timing(self.handle, ms, calls, 1 if reset else 0))
        return {k: (ms[i], calls[i]) for i, k in enumerate(("prepare", "scan", "final"))}

    def close(self) -> None:
        if getattr(self, "handle", None):
            self.lib.fbnn_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nearest(targets: torch.Tensor, neighbors: torch.Tensor):
    """One-shot exact nearest-neighbour search (plans are not cached)."""
    plan = NNPlan(targets.shape[0], neighbors.shape[0], targets.shape[1], device=targets.device)
    try:
        return plan.search(targets, neighbors)
    finally:
        torch.cuda.current_stream(plan.device).synchronize()
        plan.close()
