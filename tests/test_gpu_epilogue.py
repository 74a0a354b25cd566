"""Fused elementwise epilogue of the forward pass (through the C ABI).

The vision model family of Sec. 6.2 follows each filtering stage with a
static elementwise nonlinearity (Fig. 5b); the library generates it into the
forward kernel's store, like the paper's elementwise kernels (Sec. 5.2).
The oracle side applies the same function to the oracle's forward result.
Clamping is 1-Lipschitz and the channel scale is exact up to one rounding,
so the forward bars carry over unchanged.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from _gpu_util import host, need_gpu, to_dev

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
LOWP_TOL = 1e-2

CLAMP = "fminf(fmaxf(v, 0.f), 1.f)"
CHANNEL = "v * (1.0f + 0.25f * (float)c)"


def _plan(s, **kw):
    from paper_0911_3456_amd import Plan
    return Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, **kw)


def _clamp(y):
    return np.clip(y, 0.0, 1.0)


def _channel(y):
    return y * (1.0 + 0.25 * np.arange(y.shape[-1]))


CASES = [
    ("fp32", None, CLAMP, _clamp, False),
    ("fp32", "algo=direct", CLAMP, _clamp, False),
    ("fp32", "algo=igemm mf=16 kc=8 s=2 mr=1 mt=1 nt=1 wm=4 wn=1 ks=1", CLAMP, _clamp, False),
    ("fp32", None, CHANNEL, _channel, True),
    ("fp32", "algo=direct", CHANNEL, _channel, True),
    ("bf16", None, CLAMP, _clamp, False),
    ("fp16", None, CHANNEL, _channel, True),
]


@pytest.mark.parametrize("prec,cfg,expr,fn,scaled", CASES)
def test_epilogue_matches_oracle(prec, cfg, expr, fn, scaled):
    need_gpu()
    s = wl.Shape(2, 45, 70, 8, 40, 7, 7)          # ragged tiles in every dimension
    x, w, _ = wl.draw_single(s, seed=901)
    plan = _plan(s, precision=prec)
    if cfg:
        plan.set_config("forward", cfg)
    plan.set_epilogue(expr)
    y = host(plan.forward(*to_dev(x, w)))
    ref = oracle.forward(x, w)
    scale = oracle.forward_scale(x, w)
    if scaled:                                      # the channel factor scales the bound too
        scale = _channel(scale)
    e, m, idx = oracle.normalised_error(y, fn(ref), scale)
    print(prec, cfg, expr, plan.get_config(), "max %.3e mean %.3e at %s" % (e, m, idx))
    assert e <= (FP32_TOL if prec == "fp32" else LOWP_TOL)
    if expr == CLAMP:
        assert y.min() >= 0.0 and y.max() <= 1.0


def test_epilogue_integer_exact_and_removable():
    need_gpu()
    s = wl.Shape(1, 40, 52, 8, 33, 5, 5)
    x, w, _ = wl.draw_integer(s, seed=902)
    plan = _plan(s)
    xt, wt = to_dev(x, w)
    plain = host(plan.forward(xt, wt))
    plan.set_epilogue("fmaxf(v, 0.f) + (float)c")
    fused = host(plan.forward(xt, wt))
    ref = oracle.forward(x, w)
    np.testing.assert_array_equal(fused, np.maximum(ref, 0.0) + np.arange(s.N))
    plan.set_epilogue(None)
    np.testing.assert_array_equal(host(plan.forward(xt, wt)), plain)
    np.testing.assert_array_equal(plain, ref)


def test_epilogue_survives_config_change_and_tuning():
    need_gpu()
    s = wl.Shape(1, 40, 52, 8, 33, 5, 5)
    x, w, _ = wl.draw_integer(s, seed=903)
    plan = _plan(s)
    plan.set_epilogue("fmaxf(v, 0.f)")
    xt, wt = to_dev(x, w)
    want = np.maximum(oracle.forward(x, w), 0.0)
    plan.set_config("forward", "algo=direct")
    np.testing.assert_array_equal(host(plan.forward(xt, wt)), want)
    yt = plan.forward(xt, wt)
    plan.tune(xt, wt, yt, role="forward", max_candidates=6, record=False)
    np.testing.assert_array_equal(host(plan.forward(xt, wt)), want)


def test_epilogue_errors():
    need_gpu()
    from paper_0911_3456_amd._native import FbcorrError
    s = wl.Shape(1, 30, 30, 4, 16, 3, 3)
    x, w, _ = wl.draw_integer(s, seed=904)
    plan = _plan(s)
    xt, wt = to_dev(x, w)
    plan.set_epilogue("fmaxf(v, 0.f)")
    for bad in ("v\n+1", "#v", "v \\"):
        with pytest.raises(FbcorrError) as ei:
            plan.set_epilogue(bad)
        assert ei.value.status == 1                  # FBCORR_ERR_INVALID_ARGUMENT
    with pytest.raises(FbcorrError) as ei:
        plan.set_epilogue("v +* undefined_name")      # does not compile
    assert ei.value.status == 4                      # FBCORR_ERR_COMPILE
    # the previous kernel (with its epilogue) is still installed
    np.testing.assert_array_equal(host(plan.forward(xt, wt)), np.maximum(oracle.forward(x, w), 0.0))
    dy = np.ones((1, s.Ho, s.Wo, s.N), np.float32)
    with pytest.raises(FbcorrError) as ei:
        plan.backward(xt, wt, to_dev(dy)[0])
    assert ei.value.status == 3                      # FBCORR_ERR_UNSUPPORTED
