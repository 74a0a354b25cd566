"""Plans over torch tensors, and the autograd wrapper.

torch provides device memory (inputs, outputs, workspaces) and streams;
every arithmetic step runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import _native as nat


def _stream_handle(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check_tensor(t: torch.Tensor, shape, name: str) -> None:
    if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError("%s must be a contiguous float32 GPU tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    if t.data_ptr() % 16:
        raise ValueError("%s must be 16-byte aligned" % name)


class Plan:
    """A compiled plan for one problem shape (see include/fbcorr.h)."""

    def __init__(self, batch, H, W, D, N, fh, fw, precision="fp32", algo="auto", device=None,
                 overlap_backward=False):
        self.lib = nat.load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        self.desc = nat.make_desc(batch, H, W, D, N, fh, fw, precision, algo,
                                  nat.FLAG_OVERLAP_BACKWARD if overlap_backward else 0)
        self.shape = (batch, H, W, D, N, fh, fw)
        self.precision = precision
        h = ctypes.c_void_p()
        nat.check(self.lib.fbcorr_plan(ctypes.byref(self.desc), self.device.index, ctypes.byref(h)))
        self.handle = h
        self._ws = {}

    # -- shapes
    @property
    def x_shape(self):
        b, H, W, D, _, _, _ = self.shape
        return (b, H, W, D)

    @property
    def w_shape(self):
        _, _, _, D, N, fh, fw = self.shape
        return (N, fh, fw, D)

    @property
    def y_shape(self):
        b, H, W, _, N, fh, fw = self.shape
        return (b, H - fh + 1, W - fw + 1, N)

    @property
    def flops(self) -> int:
        b, Ho, Wo, N = self.y_shape
        _, _, _, D, _, fh, fw = self.shape
        return 2 * b * Ho * Wo * N * fh * fw * D

    # -- workspace
    def workspace_size(self, pass_: int) -> int:
        n = ctypes.c_size_t()
        nat.check(self.lib.fbcorr_workspace_size(self.handle, pass_, ctypes.byref(n)))
        return n.value

    def workspace(self, pass_: int) -> torch.Tensor | None:
        n = self.workspace_size(pass_)
        if n == 0:
            return None
        t = self._ws.get(pass_)
        if t is None or t.numel() < n:
            t = torch.empty(n + 256, dtype=torch.uint8, device=self.device)
            off = (-t.data_ptr()) % 256
            t = t[off:off + n]
            self._ws[pass_] = t
        return t

    # -- compute
    def forward(self, x: torch.Tensor, w: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
        _check_tensor(x, self.x_shape, "x")
        _check_tensor(w, self.w_shape, "w")
        if y is None:
            y = torch.empty(self.y_shape, dtype=torch.float32, device=self.device)
        _check_tensor(y, self.y_shape, "y")
        ws = self.workspace(0)
        nat.check(self.lib.fbcorr_forward(self.handle, _ptr(x), _ptr(w), _ptr(y), _ptr(ws),
                                          ws.numel() if ws is not None else 0,
                                          ctypes.c_void_p(_stream_handle(self.device))))
        return y

    def forward_noalloc(self, x: torch.Tensor, w: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
        """fbcorr_forward_noalloc: the forward pass with the library's static
        device scratch instead of a workspace (y must be given: nothing is
        allocated)."""
        _check_tensor(x, self.x_shape, "x")
        _check_tensor(w, self.w_shape, "w")
        _check_tensor(y, self.y_shape, "y")
        nat.check(self.lib.fbcorr_forward_noalloc(self.handle, _ptr(x), _ptr(w), _ptr(y),
                                                  ctypes.c_void_p(_stream_handle(self.device))))
        return y

    def backward(self, x, w, dy, need_dx=True, need_dw=True, dx=None, dw=None):
        _check_tensor(dy, self.y_shape, "dy")
        if need_dx:
            _check_tensor(w, self.w_shape, "w")
            dx = torch.empty(self.x_shape, dtype=torch.float32, device=self.device) if dx is None else dx
            _check_tensor(dx, self.x_shape, "dx")
        else:
            dx = None
        if need_dw:
            _check_tensor(x, self.x_shape, "x")
            dw = torch.empty(self.w_shape, dtype=torch.float32, device=self.device) if dw is None else dw
            _check_tensor(dw, self.w_shape, "dw")
        else:
            dw = None
        ws = self.workspace(1)
        nat.check(self.lib.fbcorr_backward(self.handle, _ptr(x), _ptr(w), _ptr(dy), _ptr(dx), _ptr(dw),
                                           _ptr(ws), ws.numel() if ws is not None else 0,
                                           ctypes.c_void_p(_stream_handle(self.device))))
        return dx, dw

    def tune(self, x, w, y, role="forward", warmup=2, reps=10, max_candidates=0, with_direct=False,
             direct_only=False, record=False):
        ws = self.workspace(2)
        flags = (1 if with_direct else 0) | (2 if record else 0) | (4 if direct_only else 0)
        opts = nat.TuneOpts(warmup, reps, max_candidates, nat.ROLES[role], flags)
        rep = nat.TuneReport()
        nat.check(self.lib.fbcorr_tune(self.handle, _ptr(x), _ptr(w), _ptr(y), _ptr(ws),
                                       ws.numel() if ws is not None else 0,
                                       ctypes.c_void_p(_stream_handle(self.device)),
                                       ctypes.byref(opts), ctypes.byref(rep)))
        self._ws.pop(0, None)
        self._ws.pop(1, None)
        return rep.as_dict()

    # -- configuration and timing
    def get_config(self, role="forward") -> str:
        buf = ctypes.create_string_buffer(1024)
        nat.check(self.lib.fbcorr_plan_get_config(self.handle, nat.ROLES[role], buf, 1024))
        return buf.value.decode()

    def set_config(self, role: str, cfg: str) -> None:
        nat.check(self.lib.fbcorr_plan_set_config(self.handle, nat.ROLES[role], cfg.encode()))

    def set_epilogue(self, expr: str | None) -> None:
        """Fuse an elementwise C expression of v (value) and c (filter) into
        the forward kernel's store; None removes it."""
        nat.check(self.lib.fbcorr_plan_set_epilogue(self.handle, expr.encode() if expr else None))

    def enable_timing(self, on=True) -> None:
        nat.check(self.lib.fbcorr_plan_enable_timing(self.handle, 1 if on else 0))

    def read_timing(self, reset=True):
        ms = (ctypes.c_double * 3)()
        calls = (ctypes.c_int64 * 3)()
        nat.check(self.lib.fbcorr_plan_read_timing(self.handle, ms, calls, 1 if reset else 0))
        return {r: (ms[i], calls[i]) for r, i in nat.ROLES.items()}

    def close(self) -> None:
        if getattr(self, "handle", None):
            self.lib.fbcorr_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_plans: dict = {}


def get_plan(batch, H, W, D, N, fh, fw, precision="fp32", algo="auto", device=None) -> Plan:
    dev = torch.cuda.current_device() if device is None else torch.device(device).index or 0
    key = (batch, H, W, D, N, fh, fw, precision, algo, dev)
    p = _plans.get(key)
    if p is None:
        p = Plan(batch, H, W, D, N, fh, fw, precision, algo, device=dev)
        _plans[key] = p
    return p


class FbCorrFunction(torch.autograd.Function):
    """y = fbcorr(x, w) with hand-written adjoint kernels for dx and dw."""

    @staticmethod
    def forward(ctx, x, w, plan):
        ctx.plan = plan
        ctx.save_for_backward(x, w)
        return plan.forward(x, w)

    @staticmethod
    def backward(ctx, gy):
        x, w = ctx.saved_tensors
        need_dx, need_dw = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        dx, dw = ctx.plan.backward(x, w, gy.contiguous(), need_dx=need_dx, need_dw=need_dw)
        return dx, dw, None


def fbcorr(x: torch.Tensor, w: torch.Tensor, precision: str = "fp32", algo: str = "auto") -> torch.Tensor:
    """Filter-bank correlation of x [B,H,W,D] (or [H,W,D]) with w [N,fh,fw,D]."""
    squeeze = x.dim() == 3
    if squeeze:
        x = x.unsqueeze(0)
    B, H, W, D = x.shape
    N, fh, fw, Dw = w.shape
    if Dw != D:
        raise ValueError("filter depth %d != input depth %d" % (Dw, D))
    plan = get_plan(B, H, W, D, N, fh, fw, precision, algo, device=x.device)
    y = FbCorrFunction.apply(x.contiguous(), w.contiguous(), plan)
    return y[0] if squeeze else y


class BatchedPlan:
    """Many independent problems (each its own image and filter bank) in one
    persistent launch, optionally replayed from a captured HIP graph."""

    def __init__(self, shapes, device=None):
        """shapes: sequence of (H, W, D, N, fh, fw)."""
        self.lib = nat.load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        descs = [nat.make_desc(1, *s) for s in self.shapes]
        arr = (nat.Desc * len(descs))(*descs)
        h = ctypes.c_void_p()
        nat.check(self.lib.fbcorr_plan_batched(len(descs), arr, self.device.index, ctypes.byref(h)))
        self.handle = h
        self.ws = self._workspace(0)
        # device arrays of pointers; their addresses stay fixed for graph replay
        k = len(self.shapes)
        self.px = torch.zeros(k, dtype=torch.int64, device=self.device)
        self.pw = torch.zeros(k, dtype=torch.int64, device=self.device)
        self.py = torch.zeros(k, dtype=torch.int64, device=self.device)

    def _workspace(self, pass_: int):
        n = ctypes.c_size_t()
        nat.check(self.lib.fbcorr_workspace_size(self.handle, pass_, ctypes.byref(n)))
        ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        return ws[off:off + n.value]

    def tune(self, max_candidates=40, warmup=1, reps=5, record=False):
        """Tune every (fh, fw, D, N) variant on its largest image (four-wave
        candidates) and regenerate the persistent kernel."""
        ws = self._workspace(2)
        opts = nat.TuneOpts(warmup, reps, max_candidates, 0, 2 if record else 0)
        rep = nat.TuneReport()
        nat.check(self.lib.fbcorr_tune(self.handle, None, None, None, _ptr(ws), ws.numel(),
                                       ctypes.c_void_p(_stream_handle(self.device)),
                                       ctypes.byref(opts), ctypes.byref(rep)))
        del ws
        self.ws = self._workspace(0)     # the work table may have changed size
        return rep.as_dict()

    @property
    def flops(self) -> int:
        return sum(2 * (H - fh + 1) * (W - fw + 1) * N * fh * fw * D for H, W, D, N, fh, fw in self.shapes)

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(1 << 16)
        nat.check(self.lib.fbcorr_plan_get_config(self.handle, 0, buf, 1 << 16))
        return buf.value.decode()

    def output_buffers(self):
        return [torch.empty((H - fh + 1, W - fw + 1, N), dtype=torch.float32, device=self.device)
                for H, W, D, N, fh, fw in self.shapes]

    def set_pointers(self, xs, ws, ys) -> None:
        for i, (H, W, D, N, fh, fw) in enumerate(self.shapes):
            _check_tensor(xs[i], (H, W, D), "xs[%d]" % i)
            _check_tensor(ws[i], (N, fh, fw, D), "ws[%d]" % i)
            _check_tensor(ys[i], (H - fh + 1, W - fw + 1, N), "ys[%d]" % i)
        ptrs = torch.tensor([[t.data_ptr() for t in xs], [t.data_ptr() for t in ws],
                             [t.data_ptr() for t in ys]], dtype=torch.int64)
        self.px.copy_(ptrs[0])
        self.pw.copy_(ptrs[1])
        self.py.copy_(ptrs[2])

    def forward(self, xs, ws, ys=None, use_graph=False):
        ys = self.output_buffers() if ys is None else ys
        self.set_pointers(xs, ws, ys)
        self.launch(use_graph)
        return ys

    def launch(self, use_graph=False) -> None:
        """Run with the pointers last set (a graph replays them as they are)."""
        nat.check(self.lib.fbcorr_forward_batched(
            self.handle, _ptr(self.px), _ptr(self.pw), _ptr(self.py), _ptr(self.ws), self.ws.numel(),
            ctypes.c_void_p(_stream_handle(self.device)), 1 if use_graph else 0))

    def enable_timing(self, on=True) -> None:
        nat.check(self.lib.fbcorr_plan_enable_timing(self.handle, 1 if on else 0))

    def read_timing(self, reset=True):
        ms = (ctypes.c_double * 3)()
        calls = (ctypes.c_int64 * 3)()
        nat.check(self.lib.fbcorr_plan_read_timing(self.handle, ms, calls, 1 if reset else 0))
        return ms[0], calls[0]

    def close(self) -> None:
        if getattr(self, "handle", None):
            self.lib.fbcorr_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
