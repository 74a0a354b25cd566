"""GPU parity of the register-streamed implicit-GEMM kernel (algo=rgemm:
filter fragments loaded from L2 straight into registers, input tile in LDS)
against the FP64 oracle, through the C ABI, as the forward correlation and
as the input gradient (flipped bank packed from the forward filters).

* integer-valued inputs (every partial sum exact in fp32; 16-bit operands
  exact after the power-of-two filter scale): bit-for-bit equality, fp32,
  bf16 and fp16, over ragged shapes and explicit tile configurations
  (chunk widths, tile rows, per-wave tiles, ring depths, padding, register
  budgets, filter banks that fill part of a column block);
* random inputs: fp32 within 1e-5 normalised; bf16 / fp16 within their
  closed-form bounds against the oracle on the fp32 operands and within
  1e-5 against the oracle on the rounded operands.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from _gpu_util import forward_error, host, need_gpu, to_dev

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
BOUND = {"bf16": 2 * 2.0 ** -9 + 1e-5, "fp16": 2 * 2.0 ** -11 + 1e-5}


def _plan(s, precision="fp32", cfg=""):
    from paper_0911_3456_amd import Plan
    p = Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, precision=precision)
    p.set_config("forward", ("algo=rgemm " + cfg).strip())
    assert p.get_config("forward").startswith("algo=rgemm"), p.get_config("forward")
    return p


def _run(plan, x, w):
    xt, wt = to_dev(x, w)
    return host(plan.forward(xt, wt))


SHAPES = [
    # batch, H, W, D, N, fh, fw  -- ragged tails, odd depths, small banks
    (1, 64, 64, 4, 16, 5, 5),
    (2, 37, 45, 3, 7, 3, 4),
    (1, 40, 70, 8, 64, 9, 9),
    (1, 33, 33, 16, 40, 13, 13),
    (3, 20, 21, 1, 1, 1, 1),
    (1, 9, 11, 5, 33, 9, 11),      # filter as large as the input: 1x1 output
    (1, 50, 66, 32, 128, 3, 3),
    (2, 24, 100, 2, 5, 8, 8),      # even filter size
    (1, 30, 41, 24, 96, 7, 7),     # 24 channels: a partial chunk of 16
]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_integer_exact(shape, prec):
    need_gpu()
    s = wl.Shape(*shape)
    x, w, _ = wl.draw_integer(s, seed=300 + sum(shape))
    plan = _plan(s, prec)
    y = _run(plan, x, w)
    np.testing.assert_array_equal(y, oracle.forward(x, w).astype(np.float32))


RGEMM_CFGS = [
    "kc=4 mr=1 mt=1 nt=1 wm=1 wn=1 pf=1",
    "mf=16 kc=4 mr=1 mt=4 nt=1 wm=2 wn=2 pf=3",
    "mf=16 kc=8 mr=2 mt=2 nt=2 wm=2 wn=1 pf=2",
    "mf=16 kc=16 mr=4 mt=8 nt=1 wm=1 wn=4 pf=4 xpadc=1",
    "kc=8 mr=2 mt=4 nt=2 wm=2 wn=1 pf=3",
    "kc=8 mr=4 mt=2 nt=1 wm=4 wn=2 pf=2 xpadc=1",
    "kc=16 mr=1 mt=2 nt=2 wm=2 wn=1 pf=4 wpe=1",
    "kc=4 mr=8 mt=1 nt=1 wm=2 wn=2 pf=6",
    "kc=8 mr=2 mt=8 nt=1 wm=1 wn=2 pf=2 xcd=0",
    "kc=16 mr=2 mt=4 nt=2 wm=2 wn=2 pf=3",          # 128 columns for a 64-filter bank: half empty
    # column shifts: 16 filters x 2 shifts, 8 filters x 4 shifts per block
    "mf=32 s=2 kc=8 mr=2 mt=4 nt=1 wm=2 wn=1 pf=3",
    "mf=16 s=4 kc=4 mr=1 mt=4 nt=1 wm=2 wn=2 pf=2",
    "mf=16 s=2 kc=8 mr=2 mt=2 nt=2 wm=2 wn=1 pf=4 xpadc=1",
    # interior tiles stored through LDS as 16-byte vectors (edge tiles as before)
    "kc=8 mr=2 mt=4 nt=2 wm=2 wn=1 pf=3 ste=1",
    "mf=16 kc=8 mr=1 mt=4 nt=2 wm=2 wn=2 pf=2 ste=1 nts=1",
    "kc=16 mr=4 mt=2 nt=1 wm=2 wn=2 pf=3 ste=1",
]


@pytest.mark.parametrize("cfg", RGEMM_CFGS)
def test_fp32_configs_integer_exact(cfg):
    need_gpu()
    s = wl.Shape(2, 45, 77, 8, 64, 9, 9)
    x, w, _ = wl.draw_integer(s, seed=9)
    plan = _plan(s, "fp32", cfg)
    y = _run(plan, x, w)
    np.testing.assert_array_equal(y, oracle.forward(x, w).astype(np.float32))


LOWP_CFGS = [
    "kc=8 mr=2 mt=4 nt=2 wm=2 wn=2 pf=3",
    "mf=16 kc=8 mr=1 mt=4 nt=2 wm=2 wn=2 pf=3",
    "mf=16 kc=16 mr=2 mt=8 nt=1 wm=2 wn=4 pf=2",
    "mf=16 kc=32 mr=4 mt=2 nt=2 wm=4 wn=1 pf=4 xpadc=1",
    "kc=16 mr=1 mt=2 nt=1 wm=4 wn=1 pf=2",
    "kc=16 mr=4 mt=4 nt=1 wm=2 wn=4 pf=4 xpadc=1",
    "kc=32 mr=2 mt=2 nt=2 wm=2 wn=2 pf=6 wpe=1",
    "kc=8 mr=2 mt=8 nt=1 wm=1 wn=2 pf=3",
    "mf=32 s=2 kc=16 mr=2 mt=4 nt=2 wm=2 wn=1 pf=3",
    "mf=16 s=4 kc=8 mr=1 mt=4 nt=1 wm=2 wn=2 pf=2",
    "kc=16 mr=2 mt=4 nt=2 wm=2 wn=2 pf=3 ste=1",
    "kc=16 mr=4 mt=4 nt=2 wm=2 wn=2 pf=4 ste=1 nts=1",
    "kc=16 mr=1 mt=8 nt=1 wm=1 wn=4 pf=4 ste=1 nts=1",
    # one wave per SIMD with 16 accumulator tiles (accumulators in AGPRs)
    "kc=16 mr=2 mt=4 nt=4 wm=2 wn=1 pf=3 wpe=1 ste=1",
    "kc=8 mr=2 mt=8 nt=2 wm=1 wn=2 pf=3 wpe=1",
]


@pytest.mark.parametrize("cfg", LOWP_CFGS)
@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_lowp_configs_integer_exact(cfg, prec):
    need_gpu()
    s = wl.Shape(1, 50, 61, 32, 128, 7, 7)
    x, w, _ = wl.draw_integer(s, seed=11)
    plan = _plan(s, prec, cfg)
    y = _run(plan, x, w)
    np.testing.assert_array_equal(y, oracle.forward(x, w).astype(np.float32))


@pytest.mark.parametrize("shape", SHAPES[:5])
def test_random_fp32(shape):
    need_gpu()
    s = wl.Shape(*shape)
    x, w, _ = wl.draw_single(s, seed=400 + sum(shape))
    e, _, idx = forward_error(_run(_plan(s, "fp32"), x, w), x, w)
    assert e <= FP32_TOL, (e, idx)


def _rounded_operands(x, w, prec):
    sc = oracle.filter_pow2_scales(w)
    rnd = oracle.round_to_bf16 if prec == "bf16" else oracle.round_to_fp16
    xr = rnd(x).astype(np.float64)
    wr = rnd((w.astype(np.float64) * sc[:, None, None, None]).astype(np.float32)).astype(np.float64)
    return xr, wr / sc[:, None, None, None]


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_random_lowp_bounds(prec):
    need_gpu()
    s = wl.Shape(1, 60, 57, 16, 128, 13, 13)
    x, w, _ = wl.draw_single(s, seed=23)
    y = _run(_plan(s, prec), x, w)
    e, m, idx = forward_error(y, x, w)
    print("rgemm %s vs fp64 oracle: max %.3e mean %.3e at %s" % (prec, e, m, idx))
    assert e <= BOUND[prec]
    xr, wr = _rounded_operands(x, w, prec)
    e2, _, idx2 = oracle.normalised_error(y, oracle.forward(xr, wr), oracle.forward_scale(xr, wr))
    assert e2 <= FP32_TOL, (e2, idx2)


def test_filters_change_between_calls():
    """The packed bank is rebuilt on every call: a second call with other
    filters gives the second result, not a cached one."""
    need_gpu()
    s = wl.Shape(1, 40, 40, 16, 64, 5, 5)
    x, w1, _ = wl.draw_integer(s, seed=31)
    _, w2, _ = wl.draw_integer(s, seed=32)
    plan = _plan(s, "bf16")
    xt, w1t, w2t = to_dev(x, w1, w2)
    y1 = host(plan.forward(xt, w1t))
    y2 = host(plan.forward(xt, w2t))
    np.testing.assert_array_equal(y1, oracle.forward(x, w1).astype(np.float32))
    np.testing.assert_array_equal(y2, oracle.forward(x, w2).astype(np.float32))


# ------------------------------------------------------------ input gradient

DX_SHAPES = [
    (1, 64, 64, 4, 16, 5, 5),
    (2, 37, 45, 3, 7, 3, 4),
    (1, 40, 70, 8, 64, 9, 9),
    (3, 20, 21, 1, 1, 1, 1),
    (1, 9, 11, 5, 33, 9, 11),
    (2, 30, 34, 16, 64, 7, 7),
    (1, 24, 100, 2, 5, 8, 8),
    (1, 26, 29, 32, 128, 3, 3),
]

DX_CFGS = [
    "",                                               # the role's rgemm default
    "mf=16 kc=16 mr=1 mt=8 nt=1 wm=4 wn=1 pf=3",
    "mf=16 kc=8 mr=2 mt=4 nt=1 wm=2 wn=2 pf=2 xpadc=1",
    "mf=32 kc=16 mr=2 mt=4 nt=1 wm=2 wn=1 pf=3",
    "mf=16 kc=4 mr=4 mt=2 nt=1 wm=1 wn=1 pf=6 wpe=1",
    # column shifts for the 16-channel input gradient
    "mf=32 s=2 kc=16 mr=2 mt=4 nt=1 wm=2 wn=1 pf=3",
    "mf=16 s=2 kc=16 mr=1 mt=8 nt=1 wm=4 wn=1 pf=3",
    "mf=16 s=4 kc=8 mr=2 mt=2 nt=2 wm=2 wn=1 pf=4 xpadc=1",
    "mf=16 kc=16 mr=1 mt=8 nt=1 wm=4 wn=1 pf=3 ste=1",
]


def _dx(s, x, w, g, cfg):
    from paper_0911_3456_amd import Plan
    plan = Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw)
    plan.set_config("backward_x", ("algo=rgemm " + cfg).strip())
    assert plan.get_config("backward_x").startswith("algo=rgemm")
    xt, wt, gt = to_dev(x, w, g)
    dx, _ = plan.backward(xt, wt, gt, need_dw=False)
    return host(dx)


@pytest.mark.parametrize("shape", DX_SHAPES)
def test_dx_integer_exact(shape):
    need_gpu()
    s = wl.Shape(*shape)
    x, w, rng = wl.draw_integer(s, seed=500 + sum(shape), xmax=3, wmax=3)
    g = rng.integers(-3, 4, size=(s.batch, s.Ho, s.Wo, s.N)).astype(np.float32)
    rx, _ = oracle.backward(x, w, g, want_dw=False)
    np.testing.assert_array_equal(_dx(s, x, w, g, ""), rx.astype(np.float32))


@pytest.mark.parametrize("cfg", DX_CFGS)
def test_dx_configs_integer_exact(cfg):
    need_gpu()
    s = wl.Shape(2, 41, 67, 16, 64, 7, 7)
    x, w, rng = wl.draw_integer(s, seed=13, xmax=2, wmax=2)
    g = rng.integers(-2, 3, size=(s.batch, s.Ho, s.Wo, s.N)).astype(np.float32)
    rx, _ = oracle.backward(x, w, g, want_dw=False)
    np.testing.assert_array_equal(_dx(s, x, w, g, cfg), rx.astype(np.float32))


def test_dx_random_fp32():
    need_gpu()
    s = wl.Shape(2, 50, 47, 16, 64, 7, 7)
    x, w, rng = wl.draw_single(s, seed=29)
    g = wl.draw_grad(s, rng)
    rx, _ = oracle.backward(x, w, g, want_dw=False)
    sx, _ = oracle.backward_scales(x, w, g)
    e = oracle.normalised_error(_dx(s, x, w, g, ""), rx, sx)
    assert e[0] <= FP32_TOL, e


SHIFT_SHAPES = [
    # (shape, precision, configuration): banks narrower than a block
    ((1, 60, 61, 16, 7, 5, 5), "fp32", "mf=16 s=2 kc=16 mr=2 mt=2 nt=1 wm=2 wn=2 pf=3"),
    ((2, 37, 45, 3, 7, 3, 4), "fp32", "mf=32 s=4 kc=4 mr=2 mt=2 nt=1 wm=2 wn=1 pf=2"),
    ((1, 64, 64, 4, 16, 5, 5), "bf16", "mf=32 s=2 kc=8 mr=2 mt=4 nt=1 wm=2 wn=1 pf=3"),
    ((1, 50, 47, 8, 8, 9, 9), "fp16", "mf=16 s=2 kc=8 mr=1 mt=4 nt=1 wm=4 wn=1 pf=3"),
]


@pytest.mark.parametrize("shape,prec,cfg", SHIFT_SHAPES)
def test_column_shift_integer_exact(shape, prec, cfg):
    need_gpu()
    s = wl.Shape(*shape)
    x, w, _ = wl.draw_integer(s, seed=700 + sum(shape))
    y = _run(_plan(s, prec, cfg), x, w)
    np.testing.assert_array_equal(y, oracle.forward(x, w).astype(np.float32))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_stores_through_lds_with_epilogue(prec):
    """A fused epilogue (clamp to [0, 2]) on the LDS-transposed stores of
    interior tiles and the direct stores of edge tiles: exact on integers."""
    need_gpu()
    s = wl.Shape(1, 53, 70, 16, 64, 5, 5)
    x, w, _ = wl.draw_integer(s, seed=81, xmax=2, wmax=2)
    plan = _plan(s, prec, "kc=16 mr=2 mt=2 nt=2 wm=2 wn=1 pf=3 ste=1")
    plan.set_epilogue("fminf(fmaxf(v, 0.f), 2.f)")
    y = _run(plan, x, w)
    np.testing.assert_array_equal(y, np.clip(oracle.forward(x, w), 0, 2).astype(np.float32))
