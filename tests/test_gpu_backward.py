"""GPU parity of the gradient kernels (dX, dW) and the autograd wrapper.

The oracle's gradient is the scatter-form adjoint in FP64; the bar is the
same normalised error as the forward (A = sum|dy||w| for dX, sum|dy||x| for
dW), and bit-for-bit equality on integer data with exact partial sums.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from _gpu_util import host, need_gpu, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _plan(s, **kw):
    from paper_0911_3456_amd import Plan
    return Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, **kw)


def _grads(plan, x, w, g, need_dx=True, need_dw=True):
    xt, wt, gt = to_dev(x, w, g)
    dx, dw = plan.backward(xt, wt, gt, need_dx=need_dx, need_dw=need_dw)
    return (host(dx) if dx is not None else None), (host(dw) if dw is not None else None)


SHAPES = [
    (1, 64, 64, 4, 16, 5, 5),
    (2, 37, 45, 3, 7, 3, 4),
    (1, 40, 70, 8, 64, 9, 9),
    (3, 20, 21, 1, 1, 1, 1),
    (1, 9, 11, 5, 33, 9, 11),
    (2, 30, 34, 16, 64, 7, 7),
    (1, 24, 100, 2, 5, 8, 8),
    (1, 26, 29, 32, 128, 3, 3),
]


@pytest.mark.parametrize("shape", SHAPES)
def test_random_fp32(shape):
    need_gpu()
    s = wl.Shape(*shape)
    x, w, rng = wl.draw_single(s, seed=300 + sum(shape))
    g = wl.draw_grad(s, rng)
    dx, dw = _grads(_plan(s), x, w, g)
    rx, rw = oracle.backward(x, w, g)
    sx, sw = oracle.backward_scales(x, w, g)
    ex = oracle.normalised_error(dx, rx, sx)
    ew = oracle.normalised_error(dw, rw, sw)
    assert ex[0] <= TOL, ("dx", ex)
    assert ew[0] <= TOL, ("dw", ew)


@pytest.mark.parametrize("shape", SHAPES)
def test_integer_exact(shape):
    need_gpu()
    s = wl.Shape(*shape)
    x, w, rng = wl.draw_integer(s, seed=400 + sum(shape), xmax=3, wmax=3)
    g = rng.integers(-3, 4, size=(s.batch, s.Ho, s.Wo, s.N)).astype(np.float32)
    dx, dw = _grads(_plan(s), x, w, g)
    rx, rw = oracle.backward(x, w, g)
    np.testing.assert_array_equal(dx, rx.astype(np.float32))
    np.testing.assert_array_equal(dw, rw.astype(np.float32))


def test_one_gradient_at_a_time():
    need_gpu()
    s = wl.Shape(2, 33, 35, 8, 32, 5, 5)
    x, w, rng = wl.draw_integer(s, seed=5, xmax=3, wmax=3)
    g = rng.integers(-3, 4, size=(s.batch, s.Ho, s.Wo, s.N)).astype(np.float32)
    plan = _plan(s)
    rx, rw = oracle.backward(x, w, g)
    dx, dw = _grads(plan, x, w, g, need_dw=False)
    assert dw is None
    np.testing.assert_array_equal(dx, rx.astype(np.float32))
    dx, dw = _grads(plan, x, w, g, need_dx=False)
    assert dx is None
    np.testing.assert_array_equal(dw, rw.astype(np.float32))


BX_CFGS = ["mf=16 kc=4 s=2 mr=4 mt=2 nt=1 wm=2 wn=1 ks=4", "mf=16 kc=8 s=1 mr=2 mt=1 nt=1 wm=2 wn=1 ks=2",
           "kc=4 s=4 mr=4 mt=1 nt=1 wm=1 wn=1 ks=4", "kc=4 s=4 mr=2 mt=2 nt=1 wm=1 wn=1 ks=2 ustage=3",
           "kc=8 s=2 mr=4 mt=1 nt=1 wm=2 wn=1 ks=3", "kc=8 s=4 mt=1 nt=1 wm=4 wn=1", "kc=8 s=2 mr=1 ks=1 mt=2 nt=1 wm=2 wn=1 ustage=3",
           "kc=4 s=8 mt=1 nt=1 wm=2 wn=1 xcd=0", "kc=8 s=1 mt=1 nt=1 wm=4 wn=1",
           # the flip fused into the staging
           "mf=16 kc=16 s=2 mr=1 mt=1 nt=1 wm=8 wn=1 ks=2 ustage=3 flip=1",
           "kc=4 s=4 mr=4 mt=1 nt=1 wm=1 wn=1 ks=4 flip=1", "kc=8 s=2 mr=4 mt=1 nt=1 wm=2 wn=1 ks=3 flip=1",
           # filter rows of a stage unrolled (stages of 3, and of 2 with a ragged last stage)
           "mf=16 kc=16 s=2 mr=1 mt=1 nt=1 wm=8 wn=1 ks=2 ustage=3 flip=1 uunr=1",
           "kc=4 s=4 mr=2 mt=2 nt=1 wm=1 wn=1 ks=2 ustage=2 uunr=1"]
BW_CFGS = ["rh=2 rw=32 nw=4 tpb=21 np=64 pf=1", "rh=4 rw=16 nw=8 tpb=42 np=7 pf=0",
           "rh=1 rw=64 nw=2 tpb=8 np=1 gpad=0 xpad=0 pf=1", "rh=2 rw=32 nw=8 tpb=14 np=300 pf=1",
           "rh=2 rw=32 nw=8 tpb=21 np=64 pf=2", "rh=1 rw=64 nw=2 tpb=8 np=1 gpad=0 xpad=0 pf=2",
           "rh=4 rw=16 nw=14 tpb=42 np=7 pf=2",
           # balanced split of the left-over tiles: five left over, none left
           # over, a wave range of odd length, a short last workgroup row
           # with only left-over tiles, one full round plus one left over
           "rh=2 rw=32 nw=8 tpb=21 np=64 pf=1 bal=1", "rh=4 rw=16 nw=14 tpb=42 np=7 pf=2 bal=1",
           "rh=1 rw=62 nw=16 tpb=42 np=9 pf=1 bal=1", "rh=2 rw=30 nw=8 tpb=20 np=13 pf=0 bal=1",
           "rh=1 rw=8 nw=4 tpb=5 np=40 pf=1 bal=1",
           # step loop unrolled completely, or by a factor that leaves a rest
           "rh=2 rw=30 nw=8 tpb=21 np=13 pf=1 unr=0", "rh=1 rw=62 nw=8 tpb=21 np=9 pf=2 bal=1 unr=0",
           "rh=2 rw=16 nw=4 tpb=14 np=20 pf=0 unr=3",
           # padded rows of the staged tiles (the default keeps them contiguous)
           "rh=2 rw=32 nw=8 tpb=21 np=64 pf=2 gpad=4 xpad=4", "rh=2 rw=61 nw=8 tpb=25 np=16 pf=2 bal=1 gpad=8 xpad=12",
           # waves with an empty last slot skip its products
           "rh=2 rw=30 nw=8 tpb=21 np=13 pf=1 unr=0 skipe=1", "rh=1 rw=32 nw=4 tpb=14 np=20 pf=2 skipe=1"]


@pytest.mark.parametrize("cfg", BX_CFGS)
def test_dx_configs_integer_exact(cfg):
    need_gpu()
    s = wl.Shape(2, 41, 67, 8, 64, 9, 9)
    x, w, rng = wl.draw_integer(s, seed=9, xmax=2, wmax=2)
    g = rng.integers(-2, 3, size=(s.batch, s.Ho, s.Wo, s.N)).astype(np.float32)
    plan = _plan(s)
    plan.set_config("backward_x", "algo=igemm " + cfg)
    dx, _ = _grads(plan, x, w, g, need_dw=False)
    rx, _ = oracle.backward(x, w, g, want_dw=False)
    np.testing.assert_array_equal(dx, rx.astype(np.float32))


@pytest.mark.parametrize("cfg", BW_CFGS)
def test_dw_configs_integer_exact(cfg):
    need_gpu()
    s = wl.Shape(2, 41, 67, 8, 64, 9, 9)
    x, w, rng = wl.draw_integer(s, seed=10, xmax=2, wmax=2)
    g = rng.integers(-2, 3, size=(s.batch, s.Ho, s.Wo, s.N)).astype(np.float32)
    plan = _plan(s)
    plan.set_config("backward_w", "algo=dw " + cfg)
    _, dw = _grads(plan, x, w, g, need_dx=False)
    _, rw = oracle.backward(x, w, g, want_dx=False)
    np.testing.assert_array_equal(dw, rw.astype(np.float32))


def test_fp32_workload_full_size():
    """256x256x8 input, 64 filters 9x9x8: full gradients against the oracle."""
    need_gpu()
    wk = wl.WORKLOADS["fp32"]
    x, w, rng = wl.draw_single(wk.shape, wk.seed)
    g = wl.draw_grad(wk.shape, rng)
    dx, dw = _grads(_plan(wk.shape), x, w, g)
    rx, rw = oracle.backward(x, w, g)
    sx, sw = oracle.backward_scales(x, w, g)
    ex = oracle.normalised_error(dx, rx, sx)
    ew = oracle.normalised_error(dw, rw, sw)
    print("fp32 workload dx %.3e dw %.3e" % (ex[0], ew[0]))
    assert ex[0] <= TOL and ew[0] <= TOL


def test_deterministic_repeat():
    need_gpu()
    s = wl.Shape(4, 64, 64, 16, 64, 7, 7)
    x, w, rng = wl.draw_single(s, seed=11)
    g = wl.draw_grad(s, rng)
    plan = _plan(s)
    a = _grads(plan, x, w, g)
    b = _grads(plan, x, w, g)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_autograd_function_matches_oracle():
    need_gpu()
    import torch
    from paper_0911_3456_amd import fbcorr
    s = wl.Shape(2, 30, 28, 4, 12, 5, 3)
    x, w, rng = wl.draw_single(s, seed=12)
    g = wl.draw_grad(s, rng)
    xt, wt, gt = to_dev(x, w, g)
    xt.requires_grad_(True)
    wt.requires_grad_(True)
    y = fbcorr(xt, wt)
    (y * gt).sum().backward()
    torch.cuda.synchronize()
    rx, rw = oracle.backward(x, w, g)
    sx, sw = oracle.backward_scales(x, w, g)
    assert oracle.normalised_error(host(y), oracle.forward(x, w), oracle.forward_scale(x, w))[0] <= TOL
    assert oracle.normalised_error(host(xt.grad), rx, sx)[0] <= TOL
    assert oracle.normalised_error(host(wt.grad), rw, sw)[0] <= TOL
    # only one input requiring grad
    xt2 = xt.detach().clone()
    wt2 = wt.detach().clone().requires_grad_(True)
    (fbcorr(xt2, wt2) * gt).sum().backward()
    np.testing.assert_array_equal(host(wt2.grad), host(wt.grad))


def _abs_scale_x(x, w, g, c):
    """sum over the terms of dx[b,p,q,d] of |dy| |w| (error normaliser)."""
    b, p, q, d = c
    _, fh, fw, _ = w.shape
    Ho, Wo = g.shape[1], g.shape[2]
    tot = 0.0
    for u in range(fh):
        for v in range(fw):
            i, j = p - u, q - v
            if 0 <= i < Ho and 0 <= j < Wo:
                tot += float(np.abs(g[b, i, j, :]).astype(np.float64) @ np.abs(w[:, u, v, d]).astype(np.float64))
    return tot


def _abs_scale_w(x, g, c, s):
    """sum over the terms of dw[n,u,v,d] of |dy| |x| (error normaliser)."""
    n, u, v, d = c
    return float(np.sum(np.abs(g[..., n]).astype(np.float64) *
                        np.abs(x[:, u:u + s.Ho, v:v + s.Wo, d]).astype(np.float64)))


def test_differentiation_workload():
    """32 inputs 128x128x16, 64 filters 7x7x16, dy ~ N(0,1): GPU gradients
    against windowed FP64 central finite differences at 200 coordinates
    (100 in x, 100 in w).  Every element against the oracle's gradient is
    compared in test_gpu_fullsize.py."""
    need_gpu()
    wk = wl.WORKLOADS["differentiation"]
    s = wk.shape
    x, w, rng = wl.draw_single(s, wk.seed)
    g = wl.draw_grad(s, rng)
    cx, cw = wl.fd_coordinates(s, rng, nx=100, nw=100)
    dx, dw = _grads(_plan(s), x, w, g)
    fdx = oracle.fd_grad_x(x, w, g, cx, h=1e-6)
    fdw = oracle.fd_grad_w(x, w, g, cw, h=1e-6)
    gx = np.array([dx[tuple(c)] for c in cx])
    gw = np.array([dw[tuple(c)] for c in cw])
    ax = np.array([_abs_scale_x(x, w, g, c) for c in cx])
    aw = np.array([_abs_scale_w(x, g, c, s) for c in cw])
    ex = np.max(np.abs(gx - fdx) / ax)
    ew = np.max(np.abs(gw - fdw) / aw)
    print("FD: dx %.3e dw %.3e" % (ex, ew))
    assert ex <= TOL and ew <= TOL


@pytest.mark.parametrize("overlap", [False, True])
def test_concurrent_backward_from_two_threads(overlap):
    """One plan used from two host threads on two streams with separate
    workspaces (the documented concurrency contract): both results exact,
    with the gradients in sequence or overlapped on the side stream.  The
    plan is fresh: both threads' first calls compile the gradient kernels
    concurrently (one compiles, the other waits and uses that build)."""
    need_gpu()
    import threading
    import torch
    from paper_0911_3456_amd import Plan
    s = wl.Shape(2, 60, 70, 8, 64, 7, 7)
    # workspace size from a second plan of the same problem, so that the
    # plan under test has no gradient kernels yet when the threads start
    sizer = Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, overlap_backward=overlap)
    need = sizer.workspace_size(1)
    sizer.close()
    plan = Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, overlap_backward=overlap)
    data, refs, outs = [], [], [None, None]
    for t in range(2):
        x, w, rng = wl.draw_integer(s, seed=50 + t, xmax=3, wmax=3)
        g = rng.integers(-3, 4, size=(s.batch, s.Ho, s.Wo, s.N)).astype(np.float32)
        data.append(to_dev(x, w, g))
        refs.append(oracle.backward(x, w, g))
    import ctypes
    from paper_0911_3456_amd import _native as nat

    def worker(t):
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            xt, wt, gt = data[t]
            ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
            wsp = ws.data_ptr() + (-ws.data_ptr()) % 256
            dx, dw = torch.empty_like(xt), torch.empty_like(wt)
            for _ in range(5):
                nat.check(plan.lib.fbcorr_backward(plan.handle, ctypes.c_void_p(xt.data_ptr()),
                                                   ctypes.c_void_p(wt.data_ptr()), ctypes.c_void_p(gt.data_ptr()),
                                                   ctypes.c_void_p(dx.data_ptr()), ctypes.c_void_p(dw.data_ptr()),
                                                   ctypes.c_void_p(wsp), need,
                                                   ctypes.c_void_p(stream.cuda_stream)))
            stream.synchronize()
            outs[t] = (dx.cpu().numpy(), dw.cpu().numpy())

    torch.cuda.synchronize()
    th = [threading.Thread(target=worker, args=(t,)) for t in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for t in range(2):
        np.testing.assert_array_equal(outs[t][0], refs[t][0].astype(np.float32))
        np.testing.assert_array_equal(outs[t][1], refs[t][1].astype(np.float32))


def test_overlapped_backward_matches_sequential():
    """The side-stream overlap changes only the schedule: dx and dw are bit
    for bit those of the sequential path."""
    need_gpu()
    from paper_0911_3456_amd import Plan
    wk = wl.WORKLOADS["fp32"]
    s = wk.shape
    x, w, rng = wl.draw_single(s, wk.seed)
    g = wl.draw_grad(s, rng)
    xt, wt, gt = to_dev(x, w, g)
    res = []
    for overlap in (False, True):
        plan = Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, overlap_backward=overlap)
        dx, dw = plan.backward(xt, wt, gt)
        res.append((host(dx), host(dw)))
    np.testing.assert_array_equal(res[0][0], res[1][0])
    np.testing.assert_array_equal(res[0][1], res[1][1])


@pytest.mark.parametrize("shape", [(1, 30, 33, 3, 7, 5, 4), (2, 21, 26, 5, 16, 3, 3), (1, 40, 40, 12, 33, 7, 7)])
def test_fused_flip_ragged_channels(shape):
    """The fused flip with channel counts that are not multiples of four
    (one channel per staged item) and ragged tiles: exact on integers."""
    need_gpu()
    from paper_0911_3456_amd import Plan
    s = wl.Shape(*shape)
    x, w, rng = wl.draw_integer(s, seed=61, xmax=2, wmax=2)
    g = rng.integers(-2, 3, size=(s.batch, s.Ho, s.Wo, s.N)).astype(np.float32)
    plan = Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw)
    plan.set_config("backward_x", plan.get_config("backward_x") + " flip=1")
    assert "flip=1" in plan.get_config("backward_x")
    xt, wt, gt = to_dev(x, w, g)
    dx, _ = plan.backward(xt, wt, gt, need_dw=False)
    rdx, _ = oracle.backward(x, w, g, want_dw=False)
    np.testing.assert_array_equal(host(dx), rdx.astype(np.float32))
