"""The allocation-free forward entry point (fbcorr_forward_noalloc) through
the C ABI: its output equals fbcorr_forward's (with a caller workspace) bit
for bit, on two calls in a row, the second with a smaller input; a plan
whose forward scratch exceeds the static array is refused with
FBCORR_ERR_WORKSPACE and nothing is launched.
"""
import ctypes

import numpy as np
import pytest

import workloads as wl
from _gpu_util import host, need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _noalloc(plan, xt, wt, y):
    import torch
    from paper_0911_3456_amd import _native as nat
    lib = nat.load()
    fn = lib.fbcorr_forward_noalloc
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p] * 5
    st = fn(plan.handle, ctypes.c_void_p(xt.data_ptr()), ctypes.c_void_p(wt.data_ptr()),
            ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return nat.STATUS_NAMES.get(st, str(st))


CASES = [
    # (shape, precision, forward configuration or None for the shipped one)
    (wl.Shape(1, 512, 512, 16, 128, 13, 13), "bf16", None),
    (wl.Shape(2, 64, 70, 16, 64, 5, 5), "fp16", "algo=rgemm"),
]


def test_noalloc_matches_forward_two_calls():
    need_gpu()
    import torch
    from paper_0911_3456_amd import Plan
    for k, (s, prec, cfg) in enumerate(CASES):
        x, w, _ = wl.draw_single(s, seed=40 + k)
        xt, wt = to_dev(x, w)
        plan = Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, precision=prec)
        if cfg:
            plan.set_config("forward", cfg)
        assert plan.workspace_size(0) > 0          # the role does use scratch
        ref = host(plan.forward(xt, wt))
        y = torch.full(plan.y_shape, float("nan"), device="cuda")
        assert _noalloc(plan, xt, wt, y) == "FBCORR_OK"
        got = host(y)
        print("call %d: %s %s, %d outputs, scratch %d B" % (k, prec, plan.get_config("forward"), got.size,
                                                             plan.workspace_size(0)))
        np.testing.assert_array_equal(got, ref)
        plan.close()


def test_noalloc_refuses_oversized_scratch():
    need_gpu()
    import torch
    from paper_0911_3456_amd import Plan
    s = wl.Shape(1, 40, 40, 64, 1024, 13, 13)       # 1024 x 10816 bf16 weights: 22 MB packed
    plan = Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, precision="bf16")
    assert plan.workspace_size(0) > 16 << 20
    xt = torch.zeros((s.batch, s.H, s.W, s.D), device="cuda")
    wt = torch.zeros((s.N, s.fh, s.fw, s.D), device="cuda")
    y = torch.full(plan.y_shape, 7.0, device="cuda")
    assert _noalloc(plan, xt, wt, y) == "FBCORR_ERR_WORKSPACE"
    assert float(host(y).min()) == 7.0 == float(host(y).max())    # nothing ran
    plan.close()
