"""Benchmark: filter-bank correlation forward + backward on one MI355X.

A step is one pass of the hot path over one batch: the forward correlation,
the input gradient dX and the filter gradient dW, in fp32, on the
differentiation workload -- a batch of 32 inputs 128x128x16 and one bank of
64 filters 7x7x16 (normalised), upstream gradient N(0,1) -- the
configuration the fwd+bwd metric is quoted on.  Inputs are seeded synthetic
data resident in GPU memory before timing starts.  value = 3 * 2 *
multiply-adds of one forward pass / seconds per step, the step's launches
captured once into a HIP graph and replayed (--no-graph: eager launches;
the eager time is reported beside it).

Also printed in the same JSON line:
  roofline      the dominant role (forward, dX or dW -- every kernel the role
                launches, so dW includes the fixed-order sum of its partials):
                algorithmic flops per execution over its average duration
                from HIP events on the launch stream (eager pass, after the
                warm-ups), against the MI355X fp32 matrix peak; traffic from
                the committed rocprofv3 counter summary when it was taken on
                exactly these kernels.
  cpu_baseline  the FP64 oracle timed on this host: all cores on the whole
                step, and one thread on one image of the batch.
  fp32_table_shape  the same step on the 256x256x8 input with 64 filters
                9x9x8 (the first shape of the paper's table "Performance of
                RTCG auto-tuning on 3D filter-bank convolutions").
  direct_fp32   the plain fp32 direct kernel (vector ALU, auto-tuned) on that
                shape's forward pass, against the 157.3 TFLOP/s fp32 vector
                peak.
  precision     the 512x512x16 / 128x13x13x16 forward: fp32 direct
                (fp32_direct), fp32, bf16 and fp16 on the matrix cores
                (fp32_mfma, bf16_mfma, fp16_mfma) times, the bf16/fp16
                speedups over the fp32 direct kernel, and each one's
                normalised error against FP64 oracle values stored at 132
                sites x 128 filters (tests/golden/precision_sites.npz, written
                by a script that runs only the oracle).
  batched       256 uneven images with their own banks in one persistent
                launch, replayed from a HIP graph, with its roofline.
  nearest_neighbour  exact brute-force nearest-neighbour search of 4096
                8x8-pixel target patches against 4096 ... 1,048,576
                neighbours (the sizes of the paper's search-time table,
                Sec. 6.4), with the paper's GTX 295 times for context; the
                int8 matrix-core scan kernel against the int8 peak.
  plan_cache    plan + compile time of the step's plan with an empty code
                cache (hiprtc for every kernel) and from the on-disk cache.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks (256 CUs, 2.4 GHz).
FP32_MATRIX_PEAK_TFLOPS = 157.3     # dense fp32 matrix cores
FP32_VECTOR_PEAK_TFLOPS = 157.3     # fp32 vector ALU: 256 CUs x 256 flop/clk x 2.4 GHz
BF16_MATRIX_PEAK_TFLOPS = 2500.0    # dense bf16 / fp16 matrix cores
INT8_MATRIX_PEAK_TOPS = 5000.0
# Search times of the paper's nearest-neighbour table (Sec. 6.4), seconds:
# one GPU of a GTX 295, and one core of a 2.4 GHz Core2 (C, gcc -O).
PAPER_NN_GTX295_S = {4096: 0.089, 16384: 0.299, 65536: 1.146, 262144: 4.508, 1048576: 17.989}
PAPER_NN_CPU_S = {4096: 3.76, 16384: 15.03, 65536: 60.16, 262144: 242.13, 1048576: 969.00}
ROLES = ("forward", "backward_x", "backward_w")
METRIC = "filterbank-correlation GFLOP/s fwd+bwd, % roofline; BF16-MFMA vs FP32 at stated err"
STEP_WORKLOAD = "differentiation"
TABLE_WORKLOAD = "fp32"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tune", action="store_true", help="run the tuner for every role of the step first")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-table", action="store_true", help="skip the 256x256x8 table-shape step and direct leg")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-nn", action="store_true")
    ap.add_argument("--no-plan-cache", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="time the step as eager launches instead of replaying a captured HIP graph")
    ap.add_argument("--workload", choices=[STEP_WORKLOAD, TABLE_WORKLOAD], default=STEP_WORKLOAD,
                    help="profiling aid: the workload of the timed step")
    ap.add_argument("--paper-table", action="store_true",
                    help="default vs auto-tuned forward on the paper's four table shapes, then exit")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run the kernels for a rocprofv3 counter pass and exit")
    ap.add_argument("--only", choices=["step", "forward", "backward_x", "backward_w"], default="step",
                    help="profiling aid: time one role only")
    ap.add_argument("--plan-probe", action="store_true", help=argparse.SUPPRESS)
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _code_only(src: str) -> str:
    """Kernel source without its comments, so that a comment edit does not
    orphan the counter summaries taken on unchanged code."""
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return re.sub(r"//[^\n]*", "", src)


def kernel_fingerprint(plan, role: str) -> str:
    """Hash of the generated source (comments aside) and options of a role's
    main kernel."""
    import paper_0911_3456_amd as fb
    cfg = plan.get_config(role).split(" (")[0]
    src, opts = fb.codegen(plan.desc, role, cfg)
    return hashlib.sha256((_code_only(src) + "\0" + opts).encode()).hexdigest()[:16]


def nn_fingerprint(plan) -> str:
    """Hash of the nearest-neighbour kernel template (comments aside),
    configuration and shape."""
    src = open(os.path.join(ROOT, "paper_0911_3456_amd", "csrc", "kernels", "nn.hip")).read()
    return hashlib.sha256((_code_only(src) + "\0" + plan.get_config() + "\0" + repr(plan.shape)).encode()).hexdigest()[:16]


def batched_fingerprint(plan) -> str:
    """Hash of the batched plan's configuration (every variant) and the
    igemm template its kernel is generated from (comments aside)."""
    src = open(os.path.join(ROOT, "paper_0911_3456_amd", "csrc", "kernels", "igemm.hip")).read()
    return hashlib.sha256((_code_only(src) + "\0" + plan.describe()).encode()).hexdigest()[:16]


TRAFFIC_FILES = {
    STEP_WORKLOAD: "traffic_fp32_32x128x128x16_64x7x7x16.txt",
    TABLE_WORKLOAD: "traffic_fp32_256x256x8_64x9x9x8.txt",
    "nn": "traffic_nn_4096x1048576x64.txt",
    "batched": "traffic_batched_256.txt",
    "precision_bf16": "traffic_bf16_512x512x16_128x13x13x16.txt",
    "precision_fp16": "traffic_fp16_512x512x16_128x13x13x16.txt",
}


def load_traffic(role: str, fingerprint: str, name: str):
    """HBM bytes per execution (fetch + write) from the committed rocprofv3
    counter summary, if it was taken on exactly this kernel (same generated
    source and options); None otherwise."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    for line in open(path):
        f = line.split("#")[0].split()
        if len(f) == 4 and f[0] == role and f[1] == fingerprint:
            return int(f[2]) + int(f[3])
    return None


COPY_BYTES = 256 << 20


def traffic_probe():
    """For counter runs (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE): the step
    workloads' kernels three times each, the 16-bit forwards of the precision
    workload, the batched launch and the nearest-neighbour search, plus a
    device copy of COPY_BYTES after each execution whose counter readings
    calibrate the counters (it moves COPY_BYTES in and COPY_BYTES out)."""
    import torch
    import workloads as wl
    from paper_0911_3456_amd import BatchedPlan, NNPlan, Plan
    dev = torch.device("cuda", 0)
    a = torch.ones(COPY_BYTES // 4, device=dev)
    b = torch.empty_like(a)
    for name in (STEP_WORKLOAD, TABLE_WORKLOAD):
        wk = wl.WORKLOADS[name]
        s = wk.shape
        x, w, rng = wl.draw_single(s, wk.seed)
        g = wl.draw_grad(s, rng)
        xt, wt, gt = (torch.from_numpy(v).to(dev) for v in (x, w, g))
        plan = Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, device=dev)
        y = torch.empty(plan.y_shape, device=dev)
        dx, dw = torch.empty_like(xt), torch.empty_like(wt)
        for _ in range(3):
            plan.forward(xt, wt, y)
            plan.backward(xt, wt, gt, dx=dx, dw=dw)
            b.copy_(a)
        torch.cuda.synchronize()
        for r in ROLES:
            print(name, r, kernel_fingerprint(plan, r), plan.get_config(r), flush=True)
        plan.close()
    wk = wl.WORKLOADS["precision"]
    s = wk.shape
    x, w, _ = wl.draw_single(s, wk.seed)
    xt, wt = torch.from_numpy(x).to(dev), torch.from_numpy(w).to(dev)
    for prec in ("bf16", "fp16"):
        plan = Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, precision=prec, device=dev)
        y = torch.empty(plan.y_shape, device=dev)
        for _ in range(3):
            plan.forward(xt, wt, y)
            b.copy_(a)
        torch.cuda.synchronize()
        print("precision_" + prec, "forward", kernel_fingerprint(plan, "forward"), plan.get_config("forward"),
              flush=True)
        plan.close()
    del xt, wt
    shapes, xs, fs = wl.draw_batched()
    bplan = BatchedPlan([(s.H, s.W, s.D, s.N, s.fh, s.fw) for s in shapes], device=dev)
    xd = [torch.from_numpy(v).to(dev) for v in xs]
    fd = [torch.from_numpy(v).to(dev) for v in fs]
    bplan.set_pointers(xd, fd, bplan.output_buffers())
    for _ in range(3):
        bplan.launch(use_graph=False)
    torch.cuda.synchronize()
    print("batched", batched_fingerprint(bplan), flush=True)
    bplan.close()
    T, M, D = wl.NN_TARGETS, wl.NN_NEIGHBOURS[-1], wl.NN_PATCH * wl.NN_PATCH
    t, n = wl.draw_nn(T, M, seed=7)
    tt, nt = torch.from_numpy(t).to(dev), torch.from_numpy(n).to(dev)
    nplan = NNPlan(T, M, D, device=dev)
    for _ in range(3):
        nplan.search(tt, nt)
    torch.cuda.synchronize()
    print("nn_scan", nn_fingerprint(nplan), nplan.get_config(), flush=True)


def time_steps(fn, steps: int, warmup: int):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def timed_roles(plan, fn, steps: int, warmup: int):
    """Wall time per call of fn over `steps` calls after `warmup` untimed
    ones, and the plan's per-role event times (ms per execution) over
    exactly the timed calls."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    plan.read_timing(reset=True)
    plan.enable_timing(True)
    sec = time_steps(fn, steps, 0)
    plan.enable_timing(False)
    t = plan.read_timing(reset=True)
    return sec, {r: t[r][0] / t[r][1] for r in t if t[r][1] > 0}


def captured(fn, dev):
    """fn's launches captured once into a HIP graph (after a warm-up call on
    a side stream, as graph capture requires)."""
    import torch
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fn()
    return graph


def step_leg(name: str, steps: int, warmup: int, use_graph: bool = True, only: str = "step",
             tune: bool = False):
    """forward + dX + dW of a workload: graph-replayed time per step, eager
    time, per-role event times and the roofline of the dominant role."""
    import torch
    import workloads as wl
    from paper_0911_3456_amd import Plan
    wk = wl.WORKLOADS[name]
    s = wk.shape
    x, w, rng = wl.draw_single(s, wk.seed)
    g = wl.draw_grad(s, rng)
    dev = torch.device("cuda", 0)
    xt, wt, gt = (torch.from_numpy(a).to(dev) for a in (x, w, g))
    t0 = time.perf_counter()
    plan = Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, device=dev)
    y = torch.empty(plan.y_shape, device=dev)
    dx, dw = torch.empty_like(xt), torch.empty_like(wt)
    plan.backward(xt, wt, gt, dx=dx, dw=dw)        # compiles the gradient roles
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    tune_reports = {}
    if tune:
        for role in ROLES:
            buf = y if role == "forward" else gt.clone()
            rep = plan.tune(xt, wt, buf, role=role, warmup=2, reps=10, with_direct=(role == "forward"))
            tune_reports[role] = {"default_ms": round(rep["default_ms"], 4), "best_ms": round(rep["best_ms"], 4),
                                  "boost": round(rep["default_ms"] / rep["best_ms"] - 1, 4),
                                  "tried": rep["n_tried"], "compiled": rep["n_compiled"], "best": rep["best_cfg"]}
            log("tuned", role, rep["best_cfg"], "%.4f ms (default %.4f ms)" % (rep["best_ms"], rep["default_ms"]))

    def step():
        plan.forward(xt, wt, y)
        plan.backward(xt, wt, gt, dx=dx, dw=dw)

    fns = {"step": step, "forward": lambda: plan.forward(xt, wt, y),
           "backward_x": lambda: plan.backward(xt, wt, gt, need_dw=False, dx=dx),
           "backward_w": lambda: plan.backward(xt, wt, gt, need_dx=False, dw=dw)}
    fn = fns[only]
    sec_eager, role_ms = timed_roles(plan, fn, steps, warmup)
    sec, graph_used = sec_eager, False
    if use_graph:
        graph = captured(fn, dev)
        sec = time_steps(graph.replay, steps, warmup)
        graph_used = True
        del graph
    flops = (3 if only == "step" else 1) * s.flops
    dom = max(role_ms, key=role_ms.get)
    achieved = s.flops / (role_ms[dom] * 1e-3) / 1e12
    fp = kernel_fingerprint(plan, dom)
    out = {
        "shape": s, "plan_s": plan_s, "ms": sec * 1e3, "eager_ms": sec_eager * 1e3, "graph": graph_used,
        "gflops": flops / sec / 1e9,
        "kernels": {r: plan.get_config(r) for r in ROLES},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP32_MATRIX_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP32_MATRIX_PEAK_TFLOPS, 4),
                     "traffic": load_traffic(dom, fp, TRAFFIC_FILES[name]), "kernel": dom,
                     "kernel_ms": round(role_ms[dom], 5),
                     "per_role_ms": {r: round(v, 5) for r, v in role_ms.items()},
                     "per_role_tflops": {r: round(s.flops / (v * 1e-3) / 1e12, 3) for r, v in role_ms.items()},
                     "per_role_frac": {r: round(s.flops / (v * 1e-3) / 1e12 / FP32_MATRIX_PEAK_TFLOPS, 4)
                                       for r, v in role_ms.items()},
                     "fingerprint": fp},
    }
    if tune_reports:
        out["tune"] = tune_reports
    plan.close()
    return out, (x, w, g)


def cpu_baseline(shape, x, w, g):
    """The FP64 oracle (as it stands) on this host: the whole step (forward
    + dX + dW of the batch) on all cores, and one image of the batch on one
    thread."""
    import oracle
    threads = oracle.max_threads()
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass

    def run(xs, gs):
        t0 = time.perf_counter()
        oracle.forward(xs, w)
        oracle.backward(xs, w, gs)
        return time.perf_counter() - t0

    t_all = run(x, g)
    per_image = 3 * shape.flops / shape.batch
    oracle.set_threads(1)
    try:
        t_one = run(x[:1], g[:1])
    finally:
        oracle.set_threads(threads)
    return {"value": round(3 * shape.flops / t_all / 1e9, 4), "unit": "GFLOP/s", "cores": threads,
            "kind": "oracle",
            "sample": "the whole step: forward + dX + dW of all %d images (FP64 C loops, OpenMP over "
                      "independent outputs), one run, %.1f s" % (shape.batch, t_all),
            "single_thread": {"value": round(per_image / t_one / 1e9, 4), "unit": "GFLOP/s", "cores": 1,
                              "sample": "forward + dX + dW of one image of the batch, one run, %.1f s" % t_one},
            "cpu_model": model}


def direct_leg(steps: int, warmup: int):
    """The plain fp32 direct kernel (vector ALU, auto-tuned configuration
    from the database) on the table shape's forward pass."""
    import torch
    import workloads as wl
    from paper_0911_3456_amd import Plan
    wk = wl.WORKLOADS[TABLE_WORKLOAD]
    s = wk.shape
    x, w, _ = wl.draw_single(s, wk.seed)
    dev = torch.device("cuda", 0)
    xt, wt = torch.from_numpy(x).to(dev), torch.from_numpy(w).to(dev)
    plan = Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, algo="direct", device=dev)
    y = torch.empty(plan.y_shape, device=dev)
    t, role_ms = timed_roles(plan, lambda: plan.forward(xt, wt, y), max(5, steps // 2), warmup)
    k_ms = role_ms["forward"]
    tf = s.flops / k_ms / 1e9
    cfg = plan.get_config("forward")
    plan.close()
    return {"workload": "forward of the 256x256x8 / 64x9x9x8 shape on the vector-ALU direct kernel",
            "ms": round(t * 1e3, 4), "kernel_ms": round(k_ms, 4), "tflops": round(tf, 2),
            "roofline": {"bound": "alu", "achieved": round(tf, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(tf / FP32_VECTOR_PEAK_TFLOPS, 4)},
            "config": cfg}


def precision_leg(steps: int, warmup: int, use_graph: bool = True):
    import numpy as np
    import torch
    import workloads as wl
    from paper_0911_3456_amd import Plan
    wk = wl.WORKLOADS["precision"]
    s = wk.shape
    x, w, _ = wl.draw_single(s, wk.seed)
    dev = torch.device("cuda", 0)
    xt, wt = torch.from_numpy(x).to(dev), torch.from_numpy(w).to(dev)
    # FP64 oracle values at 132 sites x all filters (written by
    # tests/golden/make_precision_sites.py, which runs only the oracle)
    ref = np.load(os.path.join(ROOT, "tests", "golden", "precision_sites.npz"))
    si = torch.from_numpy(ref["sites"][:, 0].astype(np.int64)).to(dev)
    sj = torch.from_numpy(ref["sites"][:, 1].astype(np.int64)).to(dev)
    out = {}
    for prec, algo in (("fp32", "direct"), ("fp32", "igemm"), ("bf16", "igemm"), ("fp16", "igemm")):
        plan = Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, precision=prec, algo=algo, device=dev)
        y = torch.empty(plan.y_shape, device=dev)
        reps = max(3, steps // 5)
        t_eager, role_ms = timed_roles(plan, lambda: plan.forward(xt, wt, y), reps, warmup)
        k_ms = role_ms["forward"]
        # per call: the whole forward (filter pack for bf16/fp16 and the
        # correlation) replayed from a HIP graph, as in the step
        t, replayed = t_eager, False
        if use_graph:
            graph = captured(lambda: plan.forward(xt, wt, y), dev)
            t = time_steps(graph.replay, reps, warmup)
            replayed = True
            del graph               # before the plan's kernels are unloaded
        got = y[0][si, sj].double().cpu().numpy()
        err = np.abs(got - ref["y"]) / ref["a"]
        arg = np.unravel_index(int(np.argmax(err)), err.shape)
        row = {"ms": round(t * 1e3, 4), "eager_ms": round(t_eager * 1e3, 4), "graph": replayed,
               "kernel_ms": round(k_ms, 4), "tflops": round(s.flops / k_ms / 1e9, 2),
               "config": plan.get_config("forward"),
               "err_vs_fp64_oracle": {"max": float(err.max()), "mean": float(err.mean()),
                                      "argmax": {"i": int(ref["sites"][arg[0], 0]),
                                                 "j": int(ref["sites"][arg[0], 1]), "n": int(arg[1])},
                                      "outputs_compared": int(err.size)}}
        if algo == "igemm" and prec != "fp32":
            fp = kernel_fingerprint(plan, "forward")
            row["roofline"] = {"bound": "mfma", "achieved": row["tflops"], "peak": BF16_MATRIX_PEAK_TFLOPS,
                               "unit": "TFLOP/s", "frac": round(row["tflops"] / BF16_MATRIX_PEAK_TFLOPS, 4),
                               "traffic": load_traffic("forward", fp, TRAFFIC_FILES["precision_" + prec]),
                               "fingerprint": fp}
        elif algo == "igemm":
            row["roofline"] = {"bound": "mfma", "achieved": row["tflops"], "peak": FP32_MATRIX_PEAK_TFLOPS,
                               "unit": "TFLOP/s", "frac": round(row["tflops"] / FP32_MATRIX_PEAK_TFLOPS, 4)}
        else:
            row["roofline"] = {"bound": "alu", "achieved": row["tflops"], "peak": FP32_VECTOR_PEAK_TFLOPS,
                               "unit": "TFLOP/s", "frac": round(row["tflops"] / FP32_VECTOR_PEAK_TFLOPS, 4)}
        # "mfma": the plan's matrix-core kernel (the database's choice of the
        # LDS-staged or the register-streamed implicit GEMM, named in "config")
        out["%s_%s" % (prec, "mfma" if algo == "igemm" else algo)] = row
        torch.cuda.synchronize()
        plan.close()
    base = out["fp32_direct"]["ms"]
    for k in ("fp32_mfma", "bf16_mfma", "fp16_mfma"):
        out[k]["speedup_vs_fp32_direct"] = round(base / out[k]["ms"], 3)
    out["err_tolerance"] = {"fp32": 1e-5, "bf16": 1e-2, "fp16": 1e-2}
    out["err_metric"] = ("|y - y_fp64| / sum |x||w| over each output's terms, at 132 sites x 128 filters "
                         "(every output is compared in the GPU tests)")
    out["workload"] = "512x512x16 input, 128 filters 13x13x16 (forward only)"
    return out


def batched_leg(steps: int, warmup: int):
    """256 uneven images (own bank each) in one persistent launch replayed
    from a HIP graph: throughput over the whole batch; roofline from the
    persistent kernel's own duration (eager launches, events around it)."""
    import torch
    import workloads as wl
    from paper_0911_3456_amd import BatchedPlan
    shapes, xs, fs = wl.draw_batched()
    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    plan = BatchedPlan([(s.H, s.W, s.D, s.N, s.fh, s.fw) for s in shapes], device=dev)
    plan_s = time.perf_counter() - t0
    xd = [torch.from_numpy(a).to(dev) for a in xs]
    fd = [torch.from_numpy(a).to(dev) for a in fs]
    ys = plan.output_buffers()
    plan.set_pointers(xd, fd, ys)
    side = torch.cuda.Stream(device=dev)
    reps = max(3, steps // 10)
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        for _ in range(max(1, warmup // 2)):
            plan.launch(use_graph=False)
            plan.launch(use_graph=True)
        side.synchronize()
        # the persistent kernel alone (eager launches, events around it)
        plan.read_timing(reset=True)
        plan.enable_timing(True)
        for _ in range(reps):
            plan.launch(use_graph=False)
        side.synchronize()
        plan.enable_timing(False)
        k_ms, k_calls = plan.read_timing(reset=True)
        k_ms /= max(k_calls, 1)
        # the whole launch replayed from the graph (counter reset + kernel)
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.launch(use_graph=True)
        side.synchronize()
        sec = (time.perf_counter() - t0) / reps
    desc = plan.describe()
    nvar = int(desc.split("variants=")[1].split()[0])
    achieved = plan.flops / (k_ms * 1e-3) / 1e12
    fp = batched_fingerprint(plan)
    out = {"workload": "256 images, sides 96..512, D 4..32, N 16..128, f 3..11, own bank each (forward)",
           "gflop": round(plan.flops / 1e9, 2), "ms": round(sec * 1e3, 3),
           "kernel_ms": round(k_ms, 3),
           "tflops": round(plan.flops / sec / 1e12, 2), "variants": nvar,
           "plan_s": round(plan_s, 2),
           "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP32_MATRIX_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / FP32_MATRIX_PEAK_TFLOPS, 4),
                        "traffic": load_traffic("batched", fp, TRAFFIC_FILES["batched"]),
                        "kernel": "fbcorr_batched", "fingerprint": fp}}
    plan.close()
    return out


def plan_probe():
    """(Child process of plan_cache_leg.)  Create the step's plan and compile
    all three roles; print the seconds it took and the cache counters."""
    import torch
    import workloads as wl
    from paper_0911_3456_amd import Plan, cache_stats
    s = wl.WORKLOADS[STEP_WORKLOAD].shape
    dev = torch.device("cuda", 0)
    torch.cuda.init()
    t0 = time.perf_counter()
    plan = Plan(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, device=dev)
    for r in ROLES:
        plan.get_config(r)                    # compiles and loads the role
    dt = time.perf_counter() - t0
    print(json.dumps({"plan_s": dt, "cache": cache_stats()}), flush=True)
    plan.close()


def plan_cache_leg():
    """Plan + compile time of the step's plan (three roles, four kernels)
    in a fresh process: once with an empty on-disk code cache (every kernel
    compiled by hiprtc) and once from the populated cache."""
    import tempfile
    res = {}
    with tempfile.TemporaryDirectory() as tmp:
        env = dict(os.environ, FBCORR_CACHE_DIR=tmp)
        for label in ("cold", "warm"):
            p = subprocess.run([sys.executable, os.path.abspath(__file__), "--plan-probe"], env=env,
                               capture_output=True, text=True, timeout=600)
            if p.returncode != 0:
                return {"error": p.stderr[-400:]}
            r = json.loads(p.stdout.strip().splitlines()[-1])
            res[label + "_s"] = round(r["plan_s"], 3)
            res[label + "_cache"] = r["cache"]
    res["what"] = ("fbcorr_plan + first use of dX and dW for the step's workload in a fresh process; "
                   "cold: empty code cache, every kernel compiled by hiprtc; warm: loaded from the "
                   "on-disk cache")
    return res


def fmt_step(leg, with_shape=True):
    s = leg["shape"]
    out = {"ms_per_step": round(leg["ms"], 5), "eager_ms_per_step": round(leg["eager_ms"], 5),
           "graph": leg["graph"], "gflops": round(leg["gflops"], 3), "kernels": leg["kernels"],
           "roofline": leg["roofline"]}
    if with_shape:
        out["workload"] = ("input %dx%dx%d, %d filters %dx%dx%d, step = forward + dX + dW"
                           % (s.H, s.W, s.D, s.N, s.fh, s.fw, s.D))
    return out


PAPER_SHAPES = [  # (H, W, D, N, fh, fw): the four shapes of the paper's fbconv3 table
    (256, 256, 8, 64, 9, 9), (512, 512, 4, 32, 13, 13), (1024, 1024, 8, 16, 5, 5), (2048, 2048, 4, 4, 8, 8)]


def nn_leg(steps: int, warmup: int):
    """Exact nearest-neighbour search at every neighbour-set size of the
    paper's table; the largest carries the scan kernel's roofline."""
    import torch
    import workloads as wl
    from paper_0911_3456_amd import NNPlan
    dev = torch.device("cuda", 0)
    T, D = wl.NN_TARGETS, wl.NN_PATCH * wl.NN_PATCH
    t, n = wl.draw_nn(T, wl.NN_NEIGHBOURS[-1], seed=7)
    tt, nt = torch.from_numpy(t).to(dev), torch.from_numpy(n).to(dev)
    rows = []
    for m in wl.NN_NEIGHBOURS:
        plan = NNPlan(T, m, D, device=dev)
        nm = nt[:m]
        idx, dist = plan.search(tt, nm)
        reps = max(3, steps // 5) if m < wl.NN_NEIGHBOURS[-1] else max(3, steps // 2)
        for _ in range(warmup):
            plan.search(tt, nm, idx, dist)
        torch.cuda.synchronize()
        plan.read_timing(reset=True)
        plan.enable_timing(True)
        sec = time_steps(lambda: plan.search(tt, nm, idx, dist), reps, 0)
        plan.enable_timing(False)
        tm = plan.read_timing(reset=True)
        k = {name: v[0] / max(v[1], 1) for name, v in tm.items()}
        ops = 2 * T * m * D
        row = {"neighbours": m, "ms": round(sec * 1e3, 4), "gops": round(ops / sec / 1e9, 1),
               "kernel_ms": {name: round(v, 4) for name, v in k.items()},
               "scan_tops": round(ops / (k["scan"] * 1e-3) / 1e12, 2),
               "paper_gtx295_s": PAPER_NN_GTX295_S[m], "speedup_vs_paper_gtx295": round(
                   PAPER_NN_GTX295_S[m] / sec, 1), "config": plan.get_config()}
        rows.append(row)
        log("nn", m, row["ms"], "ms", row["scan_tops"], "TOP/s scan")
        big_fp = nn_fingerprint(plan)
        plan.close()
    big = rows[-1]
    achieved = big["scan_tops"]
    return {"workload": "4096 target patches 8x8 (uint8) against 4096 ... 1,048,576 neighbours, exact",
            "ops_per_search": "2 * T * M * D (one multiply and one add per pixel pair)",
            "rows": rows,
            "roofline": {"bound": "mfma", "kernel": "fbnn_scan", "achieved": achieved,
                         "peak": INT8_MATRIX_PEAK_TOPS, "unit": "TOP/s",
                         "frac": round(achieved / INT8_MATRIX_PEAK_TOPS, 4),
                         "traffic": load_traffic("nn_scan", big_fp, TRAFFIC_FILES["nn"]), "fingerprint": big_fp}}


def paper_table(reps: int):
    """The paper's experiment on this GPU: per table shape, the hand-written
    default direct kernel vs the auto-tuned direct kernel ("boost"), and the
    auto-tuned matrix-core kernel, forward GFLOP/s."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_0911_3456_amd import Plan
    dev = torch.device("cuda", 0)
    rows, kept = [], []
    for H, W, D, N, fh, fw in PAPER_SHAPES:
        s = wl.Shape(1, H, W, D, N, fh, fw)
        x, w, _ = wl.draw_single(s, seed=6)
        xt, wt = torch.from_numpy(x).to(dev), torch.from_numpy(w).to(dev)
        row = {"input": "%dx%dx%d" % (H, W, D), "filter_bank": "%dx%dx%dx%d" % (N, fh, fw, D)}
        pd = Plan(1, H, W, D, N, fh, fw, algo="direct", device=dev)
        y = torch.empty(pd.y_shape, device=dev)
        rep = pd.tune(xt, wt, y, warmup=2, reps=reps, direct_only=True)
        row["direct_default_gflops"] = round(s.flops / rep["default_ms"] / 1e6, 1)
        row["direct_tuned_gflops"] = round(s.flops / rep["best_ms"] / 1e6, 1)
        row["boost"] = round(rep["default_ms"] / rep["best_ms"] - 1, 4)
        row["direct_tuned_cfg"] = rep["best_cfg"]
        pi = Plan(1, H, W, D, N, fh, fw, device=dev)
        rep2 = pi.tune(xt, wt, y, warmup=2, reps=reps, max_candidates=300)
        row["igemm_default_gflops"] = round(s.flops / rep2["default_ms"] / 1e6, 1)
        row["igemm_tuned_gflops"] = round(s.flops / rep2["best_ms"] / 1e6, 1)
        row["igemm_tuned_cfg"] = rep2["best_cfg"]
        row["candidates"] = {"direct": rep["n_compiled"], "igemm": rep2["n_compiled"]}
        print(json.dumps(row), flush=True)
        rows.append(row)
        kept.append((s, pd, xt, wt, y, rep["best_cfg"]))
        pi.close()
    # Per-input optimum: each shape run with every other shape's tuned direct
    # configuration (the paper reports that the best variant differs per input
    # and per GPU).  penalty = time(foreign) / time(own) - 1; null where the
    # foreign configuration does not fit this shape.
    def fwd_ms(pd, xt, wt, y):
        for _ in range(2):
            pd.forward(xt, wt, y)
        pd.enable_timing(True)
        pd.read_timing(reset=True)
        for _ in range(reps):
            pd.forward(xt, wt, y)
        ms, calls = pd.read_timing(reset=True)["forward"]
        pd.enable_timing(False)
        return ms / max(calls, 1)
    own = [fwd_ms(pd, xt, wt, y) for _, pd, xt, wt, y, _ in kept]
    for a, (s, pd, xt, wt, y, cfg) in enumerate(kept):
        pen = {}
        for b, other in enumerate(kept):
            if a == b:
                continue
            try:
                pd.set_config("forward", other[5])
                pen[rows[b]["input"] + "/" + rows[b]["filter_bank"]] = round(fwd_ms(pd, xt, wt, y) / own[a] - 1, 4)
            except Exception:
                pen[rows[b]["input"] + "/" + rows[b]["filter_bank"]] = None
        pd.set_config("forward", cfg)
        rows[a]["foreign_optimum_penalty"] = pen
        print(json.dumps({"input": rows[a]["input"], "filter_bank": rows[a]["filter_bank"],
                          "foreign_optimum_penalty": pen}), flush=True)
    for k in kept:
        k[1].close()
    return rows


def main():
    args = parse()
    if args.plan_probe:
        plan_probe()
        return
    if args.traffic_probe:
        traffic_probe()
        return
    if args.paper_table:
        paper_table(10)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(sharding is described in DESIGN.md); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    name = args.workload
    log("step: %s workload ..." % name)
    leg, (x, w, g) = step_leg(name, args.steps, args.warmup, use_graph=not args.no_graph, only=args.only,
                              tune=args.tune)
    s = leg["shape"]
    log("step %.4f ms (eager %.4f ms), roles %s" % (leg["ms"], leg["eager_ms"], leg["roofline"]["per_role_ms"]))
    if name == STEP_WORKLOAD:
        workload = ("differentiation: batch of %d inputs %dx%dx%d, one bank of %d filters %dx%dx%d "
                    "(normalised), upstream gradient N(0,1); step = forward + dX + dW in fp32"
                    % (s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, s.D))
    else:
        workload = ("fp32: input %dx%dx%d, %d filters %dx%dx%d, step = forward + dX + dW"
                    % (s.H, s.W, s.D, s.N, s.fh, s.fw, s.D))
    result = {
        "metric": METRIC,
        "value": round(leg["gflops"], 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(leg["ms"], 5),
        "eager_ms_per_step": round(leg["eager_ms"], 5),
        "graph": leg["graph"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded uniform[-1,1] inputs, normalised filters, N(0,1) upstream gradient)",
        "config": {"workload": workload, "batch": s.batch, "H": s.H, "W": s.W, "D": s.D, "N": s.N,
                   "fh": s.fh, "fw": s.fw, "role": args.only, "kernels": leg["kernels"]},
        "roofline": leg["roofline"],
    }
    if "tune" in leg:
        result["tune"] = leg["tune"]
    full = args.only == "step" and name == STEP_WORKLOAD
    if full and not args.no_table:
        log("table-shape step (256x256x8, 64 filters 9x9x8) ...")
        tleg, _ = step_leg(TABLE_WORKLOAD, args.steps, args.warmup, use_graph=not args.no_graph)
        result["fp32_table_shape"] = fmt_step(tleg)
        log("direct fp32 kernel ...")
        result["direct_fp32"] = direct_leg(args.steps, args.warmup)
    if full and not args.no_precision:
        log("precision leg ...")
        result["precision"] = precision_leg(args.steps, args.warmup, use_graph=not args.no_graph)
    if full and not args.no_batched:
        log("batched leg ...")
        result["batched"] = batched_leg(args.steps, args.warmup)
    if full and not args.no_nn:
        log("nearest-neighbour leg ...")
        result["nearest_neighbour"] = nn_leg(args.steps, args.warmup)
    if full and not args.no_plan_cache:
        log("plan cache (cold / warm) ...")
        result["plan_cache"] = plan_cache_leg()
    if full and not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle) ...")
        result["cpu_baseline"] = cpu_baseline(s, x, w, g)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
