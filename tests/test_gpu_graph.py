"""Forward + backward captured into a HIP graph (through torch.cuda.graph)
and replayed: every replay equals the eager result bit for bit.

The library only enqueues kernel launches on the caller's stream (no
memsets, no host synchronisation, no allocation), so a caller can capture a
whole step.  Replays are interleaved with the program's own eager work and
synchronisations, and each one is checked.
"""
import numpy as np
import pytest

import workloads as wl
from _gpu_util import host, need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("overlap", [False, True])
def test_captured_step_matches_eager(overlap):
    need_gpu()
    import torch
    from paper_0911_3456_amd import Plan
    s = wl.Shape(2, 70, 90, 8, 64, 9, 9)
    x, w, rng = wl.draw_single(s, seed=41)
    g = wl.draw_grad(s, rng)
    xt, wt, gt = to_dev(x, w, g)
    plan = Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, overlap_backward=overlap)
    y = torch.empty(plan.y_shape, device="cuda")
    dx, dw = torch.empty_like(xt), torch.empty_like(wt)

    plan.forward(xt, wt, y)
    plan.backward(xt, wt, gt, dx=dx, dw=dw)
    ref = (host(y), host(dx), host(dw))

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):                 # warm-up on the capture stream
        plan.forward(xt, wt, y)
        plan.backward(xt, wt, gt, dx=dx, dw=dw)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.forward(xt, wt, y)
        plan.backward(xt, wt, gt, dx=dx, dw=dw)
    torch.cuda.synchronize()

    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(4):
        y.zero_()
        dx.zero_()
        dw.zero_()
        junk.mul_(1.0001).add_(0.5)               # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = (host(y), host(dx), host(dw))
        for a, b, name in zip(got, ref, ("y", "dx", "dw")):
            np.testing.assert_array_equal(a, b, err_msg="replay %d, %s" % (rep, name))
    # eager calls still work after the capture, and still agree
    plan.forward(xt, wt, y)
    plan.backward(xt, wt, gt, dx=dx, dw=dw)
    np.testing.assert_array_equal(host(dw), ref[2])


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_captured_lowp_forward_matches_eager(prec):
    """The 16-bit forward (filter pack into the workspace, then the
    correlation) captured and replayed; the filters change between replays
    so each replay must re-pack them."""
    need_gpu()
    import torch
    from paper_0911_3456_amd import Plan
    s = wl.Shape(1, 60, 75, 16, 64, 7, 7)
    x, w, _ = wl.draw_single(s, seed=43)
    xt, wt = to_dev(x, w)
    plan = Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, precision=prec)
    y = torch.empty(plan.y_shape, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.forward(xt, wt, y)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.forward(xt, wt, y)
    torch.cuda.synchronize()
    for rep in range(4):
        wt.mul_(0.5 if rep % 2 else 3.0)          # new filters (new per-filter scales)
        ref = host(plan.forward(xt, wt))         # eager result for these filters
        y.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(y), ref, err_msg="replay %d" % rep)
