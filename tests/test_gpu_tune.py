"""The tuner: every installed variant keeps oracle parity."""
import numpy as np
import pytest

import oracle
import workloads as wl
from _gpu_util import forward_error, host, need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _plan(s, **kw):
    from paper_0911_3456_amd import Plan
    return Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, **kw)


@pytest.mark.parametrize("role", ["forward", "backward_x", "backward_w"])
def test_tune_role_keeps_parity(role):
    need_gpu()
    s = wl.Shape(1, 70, 90, 8, 64, 9, 9)
    x, w, rng = wl.draw_single(s, seed=31)
    g = wl.draw_grad(s, rng)
    plan = _plan(s)
    xt, wt, gt = to_dev(x, w, g)
    y = plan.forward(xt, wt)
    buf = gt.clone() if role != "forward" else y
    rep = plan.tune(xt, wt, buf, role=role, warmup=1, reps=3, max_candidates=12,
                    with_direct=(role == "forward"))
    print(role, rep)
    assert rep["n_compiled"] >= 1 and rep["best_ms"] > 0
    assert rep["n_rejected_parity"] == 0
    cfg = plan.get_config(role)
    assert cfg.split(" (")[0] == rep["best_cfg"]
    if role == "forward":
        e, _, _ = forward_error(host(plan.forward(xt, wt)), x, w)
        assert e <= 1e-5
    else:
        dx, dw = plan.backward(xt, wt, gt)
        rx, rw = oracle.backward(x, w, g)
        sx, sw = oracle.backward_scales(x, w, g)
        assert oracle.normalised_error(host(dx), rx, sx)[0] <= 1e-5
        assert oracle.normalised_error(host(dw), rw, sw)[0] <= 1e-5


def test_timing_counters():
    need_gpu()
    s = wl.Shape(1, 64, 64, 4, 16, 5, 5)
    x, w, rng = wl.draw_single(s, seed=1)
    g = wl.draw_grad(s, rng)
    plan = _plan(s)
    xt, wt, gt = to_dev(x, w, g)
    plan.enable_timing(True)
    for _ in range(3):
        plan.forward(xt, wt)
        plan.backward(xt, wt, gt)
    t = plan.read_timing()
    assert t["forward"][1] == 3 and t["backward_x"][1] == 3 and t["backward_w"][1] == 3
    assert all(v[0] > 0 for v in t.values())
    assert plan.read_timing()["forward"][1] == 0


def test_error_paths_on_device():
    need_gpu()
    import torch
    from paper_0911_3456_amd import FbcorrError
    from paper_0911_3456_amd import _native as nat
    import ctypes
    s = wl.Shape(1, 32, 32, 4, 8, 3, 3)
    plan = _plan(s)
    x = torch.zeros(s.batch, s.H, s.W, s.D, device="cuda")
    w = torch.zeros(s.N, s.fh, s.fw, s.D, device="cuda")
    y = torch.zeros(s.batch, s.Ho, s.Wo, s.N, device="cuda")
    lib = nat.load()
    # misaligned pointer
    st = lib.fbcorr_forward(plan.handle, ctypes.c_void_p(x.data_ptr() + 4), ctypes.c_void_p(w.data_ptr()),
                            ctypes.c_void_p(y.data_ptr()), None, 0, None)
    assert nat.STATUS_NAMES[st] == "FBCORR_ERR_INVALID_ARGUMENT"
    # workspace too small for the backward pass
    need = plan.workspace_size(1)
    assert need > 0
    st = lib.fbcorr_backward(plan.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                             ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                             ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(x.data_ptr()), need - 1, None)
    assert nat.STATUS_NAMES[st] == "FBCORR_ERR_WORKSPACE"
    # the plan is still usable afterwards
    plan.forward(x, w, y)
    torch.cuda.synchronize()
    with pytest.raises(FbcorrError):
        plan.set_config("forward", "algo=igemm s=3")
    with pytest.raises(FbcorrError) as e:
        plan.set_config("forward", "algo=igemm inject_error=1")
    assert e.value.status_name == "FBCORR_ERR_COMPILE"
    plan.forward(x, w, y)
    torch.cuda.synchronize()
    with pytest.raises(ValueError):
        plan.forward(x[:, :-1].contiguous(), w)
