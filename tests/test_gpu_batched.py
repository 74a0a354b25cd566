"""The persistent batched launch: many uneven images, each with its own
filter bank, in one kernel, eager and replayed from a HIP graph."""
import numpy as np
import pytest

import oracle
import workloads as wl
from _gpu_util import host, need_gpu, sample_sites, sampled_forward_error

pytestmark = pytest.mark.gpu


def _draw(shapes, seed):
    rng = np.random.default_rng(seed)
    xs, fs = [], []
    for s in shapes:
        x, f, rng = wl.draw_single(s, seed, normalised=False, rng=rng)
        xs.append(x[0])
        fs.append(f)
    return xs, fs


def _dev(arrs):
    import torch
    return [torch.from_numpy(a).cuda() for a in arrs]


SMALL = [wl.Shape(1, 40, 37, 4, 16, 3, 3), wl.Shape(1, 64, 64, 8, 64, 9, 9),
         wl.Shape(1, 33, 50, 16, 32, 5, 5), wl.Shape(1, 40, 41, 4, 16, 3, 3),
         wl.Shape(1, 96, 96, 32, 128, 11, 11), wl.Shape(1, 20, 70, 8, 64, 9, 9),
         wl.Shape(1, 25, 25, 16, 32, 7, 7), wl.Shape(1, 11, 11, 4, 16, 11, 11)]


def test_batched_matches_oracle_and_single_plans():
    need_gpu()
    from paper_0911_3456_amd import BatchedPlan, Plan
    xs, fs = _draw(SMALL, seed=41)
    plan = BatchedPlan([(s.H, s.W, s.D, s.N, s.fh, s.fw) for s in SMALL])
    desc = plan.describe()
    print(desc)
    ys = plan.forward(_dev(xs), _dev(fs))
    out = [host(y) for y in ys]
    for i, s in enumerate(SMALL):
        e, _, idx = oracle.normalised_error(out[i], oracle.forward(xs[i], fs[i]),
                                            oracle.forward_scale(xs[i], fs[i]))
        assert e <= 1e-5, (i, e, idx)
    # the same variant through a single-image plan gives the same bits
    variants = {}
    for part in desc.split(" | ")[1:]:
        head, cfg = part.split(" algo=")
        toks = dict(t.split("=") for t in head.split()[1:])
        variants[(int(toks["fh"]), int(toks["D"]), int(toks["N"]))] = "algo=" + cfg
    for i, s in enumerate(SMALL[:4]):
        p1 = Plan(1, s.H, s.W, s.D, s.N, s.fh, s.fw)
        p1.set_config("forward", variants[(s.fh, s.D, s.N)])
        import torch
        y1 = host(p1.forward(torch.from_numpy(xs[i][None]).cuda(), torch.from_numpy(fs[i]).cuda()))[0]
        np.testing.assert_array_equal(out[i], y1)


def test_batched_integer_exact_and_graph_replay():
    need_gpu()
    import torch
    from paper_0911_3456_amd import BatchedPlan
    rng = np.random.default_rng(5)
    xs = [rng.integers(-4, 5, size=(s.H, s.W, s.D)).astype(np.float32) for s in SMALL]
    fs = [rng.integers(-4, 5, size=(s.N, s.fh, s.fw, s.D)).astype(np.float32) for s in SMALL]
    plan = BatchedPlan([(s.H, s.W, s.D, s.N, s.fh, s.fw) for s in SMALL])
    xd, fd = _dev(xs), _dev(fs)
    eager = [host(y) for y in plan.forward(xd, fd)]
    for i in range(len(SMALL)):
        np.testing.assert_array_equal(eager[i], oracle.forward(xs[i], fs[i]).astype(np.float32))
    ys = plan.output_buffers()
    plan.set_pointers(xd, fd, ys)
    from paper_0911_3456_amd import FbcorrError
    with pytest.raises(FbcorrError):
        plan.launch(use_graph=True)          # the null stream cannot be captured
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        for rep in range(3):
            for y in ys:
                y.fill_(float("nan"))
            plan.launch(use_graph=True)
            side.synchronize()
            for i in range(len(SMALL)):
                np.testing.assert_array_equal(host(ys[i]), eager[i])
            # eager work between replays
            plan.launch(use_graph=False)
            side.synchronize()
        # new contents behind the same pointer arrays are picked up at replay
        ys2 = plan.output_buffers()
        plan.set_pointers(xd, fd, ys2)
        side.synchronize()
        plan.launch(use_graph=True)
        side.synchronize()
    for i in range(len(SMALL)):
        np.testing.assert_array_equal(host(ys2[i]), eager[i])


def test_batching_workload_sampled():
    """256 images, sides 96..512, D in {4,8,16,32}, N in {16..128},
    f in {3..11}, own bank each: sampled sites of every image against the
    oracle, through a captured graph."""
    need_gpu()
    import torch
    from paper_0911_3456_amd import BatchedPlan
    shapes, xs, fs = wl.draw_batched()
    plan = BatchedPlan([(s.H, s.W, s.D, s.N, s.fh, s.fw) for s in shapes])
    xd, fd = _dev(xs), _dev(fs)
    ys = plan.output_buffers()
    plan.set_pointers(xd, fd, ys)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        plan.launch(use_graph=True)
    side.synchronize()
    rng = np.random.default_rng(123)
    worst = 0.0
    for i, s in enumerate(shapes):
        sites = sample_sites(rng, s, 6)
        ii = torch.from_numpy(sites[:, 1]).cuda()
        jj = torch.from_numpy(sites[:, 2]).cuda()
        got = host(ys[i][ii, jj])                     # [sites, N], gathered on the GPU
        full = np.zeros((1, s.Ho, s.Wo, s.N), np.float32)
        full[0, sites[:, 1], sites[:, 2]] = got
        e, _, _ = sampled_forward_error(full, xs[i][None], fs[i], sites)
        worst = max(worst, e)
    print("batching workload: worst sampled normalised error %.3e" % worst)
    assert worst <= 1e-5


def test_batched_per_key_tuning_keeps_parity():
    """Tuning picks a four-wave variant per key; results stay exact."""
    need_gpu()
    from paper_0911_3456_amd import BatchedPlan
    shapes = SMALL[:4]
    rng = np.random.default_rng(8)
    xs = [rng.integers(-4, 5, size=(s.H, s.W, s.D)).astype(np.float32) for s in shapes]
    fs = [rng.integers(-4, 5, size=(s.N, s.fh, s.fw, s.D)).astype(np.float32) for s in shapes]
    plan = BatchedPlan([(s.H, s.W, s.D, s.N, s.fh, s.fw) for s in shapes])
    before = plan.describe()
    rep = plan.tune(max_candidates=6, warmup=1, reps=2)
    print(rep, plan.describe())
    assert rep["n_compiled"] >= 1 and rep["n_rejected_parity"] == 0
    ys = plan.forward(_dev(xs), _dev(fs))
    for i in range(len(shapes)):
        np.testing.assert_array_equal(host(ys[i]), oracle.forward(xs[i], fs[i]).astype(np.float32))
    assert "variants=3" in before
