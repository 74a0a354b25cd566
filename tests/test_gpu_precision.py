"""BF16/FP16 matrix-core forward against the FP64 oracle.

Operands are rounded to nearest-even after a per-filter power-of-two scale
(exact), products accumulate in fp32.  Bars: normalised error <= 1e-2
against the oracle on the original fp32 operands (worst-case closed form for
bf16: 2 * 2^-9 + fp32 accumulation ~ 3.9e-3), and ~fp32-accumulation level
against an oracle run on the rounded operands.  On small integers the 16-bit
path is exact.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from _gpu_util import forward_error, host, need_gpu, sample_sites, sampled_forward_error, to_dev

pytestmark = pytest.mark.gpu

LOWP_TOL = 1e-2
BF16_BOUND = 2 * 2.0 ** -9 + 1e-5
FP16_BOUND = 2 * 2.0 ** -11 + 1e-5


def _plan(s, **kw):
    from paper_0911_3456_amd import Plan
    return Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, **kw)


def _rounded_operands(x, w, prec):
    sc = oracle.filter_pow2_scales(w)
    rnd = oracle.round_to_bf16 if prec == "bf16" else oracle.round_to_fp16
    xr = rnd(x).astype(np.float64)
    wr = rnd((w.astype(np.float64) * sc[:, None, None, None]).astype(np.float32)).astype(np.float64)
    wr = wr / sc[:, None, None, None]
    return xr, wr


SHAPES = [(1, 64, 64, 16, 128, 13, 13), (2, 40, 51, 8, 64, 9, 9), (1, 33, 70, 16, 32, 5, 5),
          (1, 30, 30, 32, 48, 3, 3), (1, 20, 20, 4, 16, 5, 5)]


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("shape", SHAPES)
def test_lowp_error_bounds(shape, prec):
    need_gpu()
    s = wl.Shape(*shape)
    x, w, _ = wl.draw_single(s, seed=500 + sum(shape))
    y = host(_plan(s, precision=prec).forward(*to_dev(x, w)))
    e, m, _ = forward_error(y, x, w)
    bound = BF16_BOUND if prec == "bf16" else FP16_BOUND
    print(prec, shape, "max %.3e mean %.3e (bound %.3e)" % (e, m, bound))
    assert e <= LOWP_TOL and e <= bound
    # against the oracle on the rounded operands: only accumulation error left
    xr, wr = _rounded_operands(x, w, prec)
    e2, _, _ = oracle.normalised_error(y, oracle.forward(xr, wr), oracle.forward_scale(xr, wr))
    assert e2 <= 1e-5


LOWP_CFGS = [None, "algo=igemm mf=16 kc=16 s=1 mr=4 mt=2 nt=2 wm=2 wn=1 ks=1",
             "algo=igemm mf=32 kc=8 s=1 mr=2 mt=2 nt=2 wm=2 wn=1 ks=2",
             # 512-pixel workgroup (eight waves of 2x2 tiles)
             "algo=igemm mf=32 kc=8 s=1 mr=2 mt=2 nt=2 wm=8 wn=1 ks=1 xpad=8 wpad=8",
             # whole 16-channel chunks, 32-channel blocks
             "algo=igemm mf=32 kc=16 s=1 mr=2 mt=2 nt=1 wm=8 wn=1 ks=1 xpad=24 wpad=8",
             # the same with the swizzled tile, and a 16x16-tile variant of it
             "algo=igemm mf=32 kc=16 s=1 mr=2 mt=2 nt=1 wm=8 wn=1 ks=1 xpad=24 wpad=8 swz=1",
             "algo=igemm mf=16 kc=16 s=1 mr=4 mt=2 nt=2 wm=2 wn=1 ks=1 swz=1"]


@pytest.mark.parametrize("cfg", LOWP_CFGS)
@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_lowp_integer_exact(prec, cfg):
    need_gpu()
    s = wl.Shape(2, 45, 60, 16, 64, 7, 7)
    x, w, _ = wl.draw_integer(s, seed=77)
    w[3] = 0.0        # an all-zero filter (scale 1)
    w[5] *= 0.125     # power-of-two scaled filter
    plan = _plan(s, precision=prec)
    if cfg:
        plan.set_config("forward", cfg)
    y = host(plan.forward(*to_dev(x, w)))
    np.testing.assert_array_equal(y, oracle.forward(x, w).astype(np.float32))


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_swizzled_tile_ragged_channels(prec):
    """18 input channels: the second 16-channel chunk is mostly zero padding
    and the tile is staged element by element (the swizzle must be applied
    on that path too)."""
    need_gpu()
    s = wl.Shape(2, 33, 41, 18, 32, 5, 5)
    x, w, _ = wl.draw_integer(s, seed=78)
    plan = _plan(s, precision=prec)
    plan.set_config("forward", "algo=igemm mf=32 kc=16 s=1 mr=2 mt=2 nt=1 wm=8 wn=1 ks=1 xpad=24 wpad=8 swz=1")
    y = host(plan.forward(*to_dev(x, w)))
    np.testing.assert_array_equal(y, oracle.forward(x, w).astype(np.float32))


def test_precision_workload_sampled():
    """512x512x16 input, 128 filters 13x13x16: fp32 (matrix-core and direct)
    and bf16/fp16 outputs at sampled sites (and the four corners) against
    the oracle."""
    need_gpu()
    wk = wl.WORKLOADS["precision"]
    s = wk.shape
    x, w, rng = wl.draw_single(s, wk.seed)
    sites = sample_sites(np.random.default_rng(99), s, 400)
    xt, wt = to_dev(x, w)
    for prec, algo, tol in [("fp32", "igemm", 1e-5), ("fp32", "direct", 1e-5),
                            ("bf16", "igemm", BF16_BOUND), ("fp16", "igemm", FP16_BOUND)]:
        y = host(_plan(s, precision=prec, algo=algo).forward(xt, wt))
        e, m, _ = sampled_forward_error(y, x, w, sites)
        print("precision workload", prec, algo, "max %.3e mean %.3e" % (e, m))
        assert e <= tol


# fp16 inputs beyond its range: the per-tensor power-of-two input scale keeps
# them finite (reading c-10); both matrix-core algorithms.
FP16_RANGE_CFGS = ["algo=igemm", "algo=rgemm"]


@pytest.mark.parametrize("cfg", FP16_RANGE_CFGS)
def test_fp16_input_beyond_range_integer_exact(cfg):
    """Integer inputs times 2^16 (up to 2^19, far past fp16's 65504): scaled
    by 2^-5 while staged they stay integers below 2^15, so the result is
    exact and equal to the oracle's."""
    need_gpu()
    s = wl.Shape(1, 37, 41, 16, 64, 5, 5)
    x, w, _ = wl.draw_integer(s, seed=61)
    x = (x * 65536.0).astype(np.float32)
    plan = _plan(s, precision="fp16")
    plan.set_config("forward", cfg)
    y = host(plan.forward(*to_dev(x, w)))
    assert np.isfinite(y).all()
    np.testing.assert_array_equal(y, oracle.forward(x, w).astype(np.float32))


@pytest.mark.parametrize("cfg", FP16_RANGE_CFGS)
def test_fp16_input_beyond_range_error_bound(cfg):
    """Random inputs scaled to +-3e5: finite, within the fp16 bound of the
    oracle; unscaled inputs give the same result divided by the scale."""
    need_gpu()
    s = wl.Shape(1, 40, 43, 16, 64, 7, 7)
    x, w, _ = wl.draw_single(s, seed=62)
    big = (x * 3.0e5).astype(np.float32)
    plan = _plan(s, precision="fp16")
    plan.set_config("forward", cfg)
    y = host(plan.forward(*to_dev(big, w)))
    assert np.isfinite(y).all()
    e, m, idx = forward_error(y, big, w)
    print("fp16 %s, |x| up to 3e5: max %.3e mean %.3e at %s" % (cfg, e, m, idx))
    assert e <= FP16_BOUND
