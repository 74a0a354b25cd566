"""Full-size parity: every output of the benchmarked workloads against the
FP64 oracle, in the launch configuration the benchmark times (the library's
shipped configuration for each shape, replayed from a captured HIP graph).

* differentiation workload (32 inputs 128x128x16, 64 filters 7x7x16):
  forward, dX and dW, every element, normalised error <= 1e-5;
* precision workload (512x512x16, 128 filters 13x13x16): fp32 matrix-core
  and direct kernels (<= 1e-5), bf16 and fp16 (closed-form bounds against
  the oracle on the fp32 operands, <= 1e-5 against the oracle on the
  rounded operands), every output;
* batching workload (256 uneven images, own bank each): one image of every
  variant key (the cheapest image of that key, 78 images) at every output,
  plus 10^4 random sites over the other images;
* nearest neighbour at the largest size of the paper's table (4096 targets,
  1,048,576 neighbours): idx and dist of every target, bit-exact.

Each test prints its error summary; the oracle runs on the host's cores.
"""
import os

import numpy as np
import pytest

import oracle
import workloads as wl
from _gpu_util import host, need_gpu, sample_sites, sampled_forward_error, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-5
BF16_BOUND = 2 * 2.0 ** -9 + 1e-5
FP16_BOUND = 2 * 2.0 ** -11 + 1e-5


def _replayed(fn):
    """Run fn's launches once eagerly on a side stream (warm-up), capture
    them into a HIP graph, replay twice; return after the last replay."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fn()
    for _ in range(2):
        graph.replay()
    torch.cuda.synchronize()
    return graph


# ------------------------------------------------------------ differentiation

@pytest.fixture(scope="module")
def diff_results():
    need_gpu()
    import torch
    from paper_0911_3456_amd import Plan
    wk = wl.WORKLOADS["differentiation"]
    s = wk.shape
    x, w, rng = wl.draw_single(s, wk.seed)
    g = wl.draw_grad(s, rng)
    xt, wt, gt = to_dev(x, w, g)
    plan = Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw)
    y = torch.empty(plan.y_shape, device="cuda")
    dx, dw = torch.empty_like(xt), torch.empty_like(wt)

    def step():
        plan.forward(xt, wt, y)
        plan.backward(xt, wt, gt, dx=dx, dw=dw)

    graph = _replayed(step)
    out = {"x": x, "w": w, "g": g, "y": host(y), "dx": host(dx), "dw": host(dw),
           "cfg": {r: plan.get_config(r) for r in ("forward", "backward_x", "backward_w")}}
    del graph
    plan.close()
    return out


def test_differentiation_forward_every_output(diff_results):
    r = diff_results
    y_ref = oracle.forward(r["x"], r["w"])
    e, m, idx = oracle.normalised_error(r["y"], y_ref, oracle.forward_scale(r["x"], r["w"]))
    print("differentiation forward [%s]: max %.3e mean %.3e at %s" % (r["cfg"]["forward"], e, m, idx))
    assert e <= TOL


def test_differentiation_dx_every_element(diff_results):
    r = diff_results
    rx, _ = oracle.backward(r["x"], r["w"], r["g"], want_dw=False)
    sx, _ = oracle.backward(np.abs(r["x"]), np.abs(r["w"]), np.abs(r["g"]), want_dw=False)
    e, m, idx = oracle.normalised_error(r["dx"], rx, sx)
    print("differentiation dX [%s]: max %.3e mean %.3e at %s" % (r["cfg"]["backward_x"], e, m, idx))
    assert e <= TOL


def test_differentiation_dw_every_element(diff_results):
    r = diff_results
    _, rw = oracle.backward(r["x"], r["w"], r["g"], want_dx=False)
    _, sw = oracle.backward(np.abs(r["x"]), np.abs(r["w"]), np.abs(r["g"]), want_dx=False)
    e, m, idx = oracle.normalised_error(r["dw"], rw, sw)
    print("differentiation dW [%s]: max %.3e mean %.3e at %s" % (r["cfg"]["backward_w"], e, m, idx))
    assert e <= TOL


# ------------------------------------------------------------------ precision

@pytest.fixture(scope="module")
def precision_data():
    need_gpu()
    wk = wl.WORKLOADS["precision"]
    s = wk.shape
    x, w, _ = wl.draw_single(s, wk.seed)
    return {"s": s, "x": x, "w": w, "y_ref": oracle.forward(x, w), "a": oracle.forward_scale(x, w)}


def _precision_gpu(d, prec, algo):
    import torch
    from paper_0911_3456_amd import Plan
    s = d["s"]
    xt, wt = to_dev(d["x"], d["w"])
    plan = Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, precision=prec, algo=algo)
    y = torch.empty(plan.y_shape, device="cuda")
    graph = _replayed(lambda: plan.forward(xt, wt, y))
    out = host(y)
    cfg = plan.get_config("forward")
    del graph
    plan.close()
    return out, cfg


def _rounded_operands(x, w, prec):
    sc = oracle.filter_pow2_scales(w)
    rnd = oracle.round_to_bf16 if prec == "bf16" else oracle.round_to_fp16
    xr = rnd(x).astype(np.float64)
    wr = rnd((w.astype(np.float64) * sc[:, None, None, None]).astype(np.float32)).astype(np.float64)
    return xr, wr / sc[:, None, None, None]


@pytest.mark.parametrize("algo", ["igemm", "direct"])
def test_precision_fp32_every_output(precision_data, algo):
    d = precision_data
    y, cfg = _precision_gpu(d, "fp32", algo)
    e, m, idx = oracle.normalised_error(y, d["y_ref"], d["a"])
    print("precision fp32 %s [%s]: max %.3e mean %.3e at %s" % (algo, cfg, e, m, idx))
    assert e <= TOL


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_precision_lowp_every_output(precision_data, prec):
    d = precision_data
    y, cfg = _precision_gpu(d, prec, "igemm")
    e, m, idx = oracle.normalised_error(y, d["y_ref"], d["a"])
    bound = BF16_BOUND if prec == "bf16" else FP16_BOUND
    print("precision %s [%s] vs fp64 oracle on fp32 operands: max %.3e mean %.3e at %s (bound %.3e)"
          % (prec, cfg, e, m, idx, bound))
    assert e <= 1e-2 and e <= bound
    xr, wr = _rounded_operands(d["x"], d["w"], prec)
    e2, m2, idx2 = oracle.normalised_error(y, oracle.forward(xr, wr), oracle.forward_scale(xr, wr))
    print("precision %s vs fp64 oracle on rounded operands: max %.3e mean %.3e at %s" % (prec, e2, m2, idx2))
    assert e2 <= TOL


# ------------------------------------------------------------------- batching

def _full_subset(shapes, count=None):
    """One image per variant key (the cheapest image of that key); with
    `count`, only the keys whose cheapest image costs least."""
    best = {}
    for i, s in enumerate(shapes):
        key = (s.fh, s.fw, s.D, s.N)
        if key not in best or s.macs < shapes[best[key]].macs:
            best[key] = i
    chosen = sorted(best.values(), key=lambda i: shapes[i].macs)
    return sorted(chosen if count is None else chosen[:count])


def test_batching_workload_full_subset_and_sites():
    """The 256-image persistent launch replayed from a HIP graph: one image
    of every variant key (78 keys) compared at every output, and 10^4 random
    output sites (all filters each) over the other 178 images."""
    need_gpu()
    import torch
    from paper_0911_3456_amd import BatchedPlan
    shapes, xs, fs = wl.draw_batched()
    plan = BatchedPlan([(s.H, s.W, s.D, s.N, s.fh, s.fw) for s in shapes])
    xd = [torch.from_numpy(a).cuda() for a in xs]
    fd = [torch.from_numpy(a).cuda() for a in fs]
    ys = plan.output_buffers()
    plan.set_pointers(xd, fd, ys)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        for _ in range(2):
            plan.launch(use_graph=True)
    side.synchronize()
    full = _full_subset(shapes)
    keys = {(shapes[i].fh, shapes[i].D, shapes[i].N) for i in full}
    assert len(keys) == len(full) == len({(s.fh, s.D, s.N) for s in shapes})
    worst = 0.0
    for i in full:
        e, m, idx = oracle.normalised_error(host(ys[i]), oracle.forward(xs[i], fs[i]),
                                            oracle.forward_scale(xs[i], fs[i]))
        worst = max(worst, e)
        assert e <= TOL, (i, shapes[i], e, idx)
    print("batching: %d images in full (%d keys), worst %.3e" % (len(full), len(keys), worst))
    rest = [i for i in range(len(shapes)) if i not in set(full)]
    rng = np.random.default_rng(2024)
    owner = rng.choice(rest, size=10000)
    worst = 0.0
    nsites = 0
    for i in rest:
        k = int((owner == i).sum())
        if k == 0:
            continue
        s = shapes[i]
        sites = np.stack([np.zeros(k, np.int64), rng.integers(0, s.Ho, k), rng.integers(0, s.Wo, k)], axis=1)
        ii = torch.from_numpy(sites[:, 1]).cuda()
        jj = torch.from_numpy(sites[:, 2]).cuda()
        got = host(ys[i][ii, jj])
        yfull = np.zeros((1, s.Ho, s.Wo, s.N), np.float32)
        yfull[0, sites[:, 1], sites[:, 2]] = got
        e, _, _ = sampled_forward_error(yfull, xs[i][None], fs[i], sites)
        worst = max(worst, e)
        nsites += k
    print("batching: %d random sites over %d other images, worst %.3e" % (nsites, len(rest), worst))
    assert nsites == 10000 and worst <= TOL


# ----------------------------------------------------------- nearest neighbour

def test_nearest_neighbour_paper_size_every_target():
    """4096 targets against 1,048,576 neighbours in the benchmark's
    configuration: every target's idx and dist equal the oracle's."""
    need_gpu()
    import torch
    from paper_0911_3456_amd import NNPlan
    T, M = wl.NN_TARGETS, wl.NN_NEIGHBOURS[-1]
    t, n = wl.draw_nn(T, M, seed=7)
    plan = NNPlan(T, M, t.shape[1])
    idx, dist = plan.search(torch.from_numpy(t).cuda(), torch.from_numpy(n).cuda())
    torch.cuda.synchronize()
    idx = idx.cpu().numpy().astype(np.int64)
    dist = dist.cpu().numpy().astype(np.int64)
    ri, rd = oracle.nearest(t, n)
    bad = np.flatnonzero((idx != ri) | (dist != rd))
    print("nearest neighbour [%s]: %d of %d targets differ" % (plan.get_config(), bad.size, T))
    assert bad.size == 0
    plan.close()


# ---------------------------------------------- batched variants, clamped knobs

# Keys of a batched plan with tuned entries that ask for three filter rows
# per stage and the unrolled stage loop (two with fewer filter rows than
# that); the generated constants are checked on the host by
# tests/test_abi.py before any GPU run.
CLAMP_SHAPES = [wl.Shape(1, 50, 47, 16, 32, 1, 1), wl.Shape(1, 61, 40, 8, 64, 2, 2),
                wl.Shape(1, 40, 44, 8, 32, 3, 3)]
CLAMP_DB_LINES = [
    "gfx950 batched fp32 1 0 0 16 32 1 1 : algo=igemm kc=16 ks=1 mf=32 mr=2 mt=2 nt=1 s=1 ustage=3 uunr=1 "
    "wm=4 wn=1 wpad=4 xcd=1 xpad=4",
    "gfx950 batched fp32 1 0 0 8 64 2 2 : algo=igemm kc=8 ks=1 mf=32 mr=2 mt=1 nt=2 s=1 ustage=3 uunr=1 "
    "wm=4 wn=1 wpad=4 xcd=1 xpad=4",
    "gfx950 batched fp32 1 0 0 8 32 3 3 : algo=igemm kc=8 ks=1 mf=32 mr=2 mt=2 nt=1 s=1 ustage=3 uunr=1 "
    "wm=4 wn=1 wpad=4 xcd=1 xpad=4",
]

def test_batched_variant_constants_match_standalone(tmp_path):
    """A batched key tuned with more filter rows per stage than its filter
    has (ustage=3 with fh=1 and fh=2) and the unrolled stage loop: the
    persistent kernel takes the clamped value and the unrolling switch from
    the standalone build, so its LDS fits and every output is exact."""
    need_gpu()
    from paper_0911_3456_amd import BatchedPlan
    from paper_0911_3456_amd import _native as nat
    shapes, lines = CLAMP_SHAPES, CLAMP_DB_LINES
    db = tmp_path / "tuning_db.txt"
    db.write_text("\n".join(lines) + "\n")
    old = os.environ.get("FBCORR_TUNING_DB")
    os.environ["FBCORR_TUNING_DB"] = str(db)
    nat.cache_clear()
    try:
        rng = np.random.default_rng(77)
        xs = [rng.integers(-4, 5, size=(s.H, s.W, s.D)).astype(np.float32) for s in shapes]
        fs = [rng.integers(-4, 5, size=(s.N, s.fh, s.fw, s.D)).astype(np.float32) for s in shapes]
        plan = BatchedPlan([(s.H, s.W, s.D, s.N, s.fh, s.fw) for s in shapes])
        desc = plan.describe()
        print(desc)
        assert desc.count("ustage=3") == 3 and desc.count("uunr=1") == 3
        import torch
        ys = plan.forward([torch.from_numpy(a).cuda() for a in xs], [torch.from_numpy(a).cuda() for a in fs])
        for i in range(len(shapes)):
            np.testing.assert_array_equal(host(ys[i]), oracle.forward(xs[i], fs[i]).astype(np.float32))
        plan.close()
    finally:
        if old is None:
            del os.environ["FBCORR_TUNING_DB"]
        else:
            os.environ["FBCORR_TUNING_DB"] = old
        nat.cache_clear()
