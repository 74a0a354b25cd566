"""GPU parity of the forward kernels against the FP64 oracle (through the C ABI).

Bar: max normalised error <= 1e-5 for fp32 (|y - y*| / sum|x||w| over the
summed terms), and bit-for-bit equality on integer-valued inputs whose
partial sums stay below 2**24 (exact in any summation order).
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from _gpu_util import forward_error, host, need_gpu, to_dev

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5


def _plan(s, **kw):
    from paper_0911_3456_amd import Plan
    return Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, **kw)


def _run(plan, x, w):
    xt, wt = to_dev(x, w)
    return host(plan.forward(xt, wt))


def test_tiny_workload_default():
    need_gpu()
    wk = wl.WORKLOADS["tiny"]
    x, w, _ = wl.draw_single(wk.shape, wk.seed)
    plan = _plan(wk.shape)
    e, m, idx = forward_error(_run(plan, x, w), x, w)
    print("tiny igemm", plan.get_config(), "max %.3e mean %.3e at %s" % (e, m, idx))
    assert e <= FP32_TOL


def test_tiny_workload_direct():
    need_gpu()
    wk = wl.WORKLOADS["tiny"]
    x, w, _ = wl.draw_single(wk.shape, wk.seed)
    plan = _plan(wk.shape, algo="direct")
    e, m, idx = forward_error(_run(plan, x, w), x, w)
    print("tiny direct", plan.get_config(), "max %.3e" % e)
    assert e <= FP32_TOL


SHAPES = [
    # batch, H, W, D, N, fh, fw  -- ragged tails, odd depths, tiny banks
    (1, 64, 64, 4, 16, 5, 5),
    (2, 37, 45, 3, 7, 3, 4),
    (1, 40, 70, 8, 64, 9, 9),
    (1, 33, 33, 16, 40, 13, 13),
    (3, 20, 21, 1, 1, 1, 1),
    (1, 9, 11, 5, 33, 9, 11),      # filter as large as the input: 1x1 output
    (1, 50, 66, 32, 128, 3, 3),
    (2, 24, 100, 2, 5, 8, 8),      # even filter size
]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("algo", ["igemm", "direct"])
def test_integer_exact(shape, algo):
    need_gpu()
    s = wl.Shape(*shape)
    if algo == "direct" and s.N % 4 and s.N > 4:
        pass
    x, w, _ = wl.draw_integer(s, seed=100 + sum(shape))
    plan = _plan(s, algo=algo)
    y = _run(plan, x, w)
    np.testing.assert_array_equal(y, oracle.forward(x, w).astype(np.float32))


@pytest.mark.parametrize("shape", SHAPES)
def test_random_fp32(shape):
    need_gpu()
    s = wl.Shape(*shape)
    x, w, _ = wl.draw_single(s, seed=200 + sum(shape))
    for algo in ("igemm", "direct"):
        plan = _plan(s, algo=algo)
        e, _, idx = forward_error(_run(plan, x, w), x, w)
        assert e <= FP32_TOL, (algo, e, idx)


IGEMM_CFGS = [
    "mf=16 kc=8 s=1 mr=4 mt=2 nt=2 wm=2 wn=1 ks=1",
    "mf=16 kc=4 s=2 mr=2 mt=1 nt=1 wm=2 wn=2 ks=2 ustage=3",
    "mf=16 kc=8 s=1 mr=16 mt=1 nt=4 wm=1 wn=1 ks=3",
    "kc=8 s=1 mr=4 mt=1 nt=2 wm=2 wn=1 ks=2",
    "kc=4 s=2 mr=2 mt=2 nt=1 wm=1 wn=2 ks=2 ustage=1",
    "kc=8 s=1 mr=8 mt=1 nt=1 wm=1 wn=2 ks=3 ustage=1 xpad=0",
    "kc=2 s=1 mr=32 mt=1 nt=2 wm=2 wn=1 ks=1",
    "kc=4 s=1 mt=1 nt=2 wm=4 wn=1",
    "kc=8 s=1 mt=2 nt=2 wm=2 wn=1 ustage=3",
    "kc=8 s=1 mt=1 nt=1 wm=2 wn=2 xpad=0 wpad=0",
    "kc=8 s=2 mt=2 nt=1 wm=2 wn=2",
    "kc=2 s=4 mt=1 nt=1 wm=4 wn=1 xcd=0",
    # filter rows of a stage unrolled; 9 rows in stages of 3, and of 4 (the
    # last stage ragged)
    "kc=8 s=1 mt=2 nt=2 wm=2 wn=1 ustage=3 uunr=1",
    "mf=16 kc=4 s=2 mr=2 mt=1 nt=1 wm=2 wn=2 ks=2 ustage=4 uunr=1",
]


@pytest.mark.parametrize("cfg", IGEMM_CFGS)
def test_igemm_configs_integer_exact(cfg):
    need_gpu()
    s = wl.Shape(2, 45, 77, 8, 64, 9, 9)
    x, w, _ = wl.draw_integer(s, seed=7)
    plan = _plan(s, algo="igemm")
    plan.set_config("forward", "algo=igemm " + cfg)
    y = _run(plan, x, w)
    np.testing.assert_array_equal(y, oracle.forward(x, w).astype(np.float32))


DIRECT_CFGS = [
    "th=4 tw=32 p=4 q=16 nb=64 layout=0",
    "th=8 tw=16 p=2 q=8 nb=32 layout=1 ds=2",
    "th=16 tw=16 p=4 q=16 nb=16 layout=1 ud=2",
    "th=8 tw=32 p=8 q=8 nb=64 layout=0 ds=4 xpad=0",
    "th=16 tw=16 p=4 q=8 nb=32 layout=1 fsrc=1",            # scalar weights, 4 filter groups
    "th=8 tw=32 p=4 q=16 nb=16 layout=0 fsrc=1 ud=2",       # scalar weights, one group
    "th=16 tw=32 p=8 q=4 nb=12 layout=1 fsrc=1",            # N not a multiple of nb: zero-padded copy
    # staging loads issued in batches (input tile and filter slices)
    "th=8 tw=16 p=2 q=8 nb=64 layout=1 ds=2 sb=1",
    "th=16 tw=32 p=8 q=8 nb=64 layout=1 sb=1",
    "th=8 tw=32 p=4 q=16 nb=16 layout=0 fsrc=1 ud=2 sb=1",
]


@pytest.mark.parametrize("cfg", DIRECT_CFGS)
def test_direct_configs_integer_exact(cfg):
    need_gpu()
    s = wl.Shape(2, 45, 77, 8, 64, 9, 9)
    x, w, _ = wl.draw_integer(s, seed=8)
    plan = _plan(s, algo="direct")
    plan.set_config("forward", "algo=direct " + cfg)
    y = _run(plan, x, w)
    np.testing.assert_array_equal(y, oracle.forward(x, w).astype(np.float32))


def test_fp32_workload_full_size():
    """256x256x8 input, 64 filters 9x9x8: every output against the oracle."""
    need_gpu()
    wk = wl.WORKLOADS["fp32"]
    x, w, _ = wl.draw_single(wk.shape, wk.seed)
    y_ref = oracle.forward(x, w)
    for algo in ("igemm", "direct"):
        plan = _plan(wk.shape, algo=algo)
        e, m, idx = forward_error(_run(plan, x, w), x, w, y_ref=y_ref)
        print("fp32 workload", algo, "max %.3e mean %.3e" % (e, m))
        assert e <= FP32_TOL


def test_deterministic_repeat():
    need_gpu()
    wk = wl.WORKLOADS["fp32"]
    x, w, _ = wl.draw_single(wk.shape, wk.seed)
    plan = _plan(wk.shape)
    xt, wt = to_dev(x, w)
    a = host(plan.forward(xt, wt))
    b = host(plan.forward(xt, wt))
    np.testing.assert_array_equal(a, b)


# the four shapes of the paper's auto-tuning table (input, filter bank)
PAPER_SHAPES = [wl.Shape(1, 256, 256, 8, 64, 9, 9), wl.Shape(1, 512, 512, 4, 32, 13, 13),
                wl.Shape(1, 1024, 1024, 8, 16, 5, 5), wl.Shape(1, 2048, 2048, 4, 4, 8, 8)]


@pytest.mark.parametrize("algo", ["auto", "direct"])
@pytest.mark.parametrize("s", PAPER_SHAPES, ids=lambda s: "%dx%dx%d_%dx%dx%d" % (s.H, s.W, s.D, s.N, s.fh, s.fw))
def test_paper_shapes_shipped_configs_integer_exact(s, algo):
    """The tuning database's configurations for the paper's four shapes
    (matrix-core and direct), bit for bit on integer inputs."""
    need_gpu()
    x, w, _ = wl.draw_integer(s, seed=17, xmax=2, wmax=2)
    plan = _plan(s, algo=algo)
    y = _run(plan, x, w)
    np.testing.assert_array_equal(y, oracle.forward(x, w).astype(np.float32))
