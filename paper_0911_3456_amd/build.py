"""Build the fbcorr native library in-tree.

Steps: embed the HIP kernel templates (``csrc/kernels/*.hip``) as strings in a
generated header, compile the host library (C++17, hipcc) into
``libfbcorr.so`` next to this file, and compile every kernel template for
gfx950 with hipcc (device only) as a syntax/resource check.  At run time the
library generates each kernel's specialised variant and compiles it with
hiprtc.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
KDIR = os.path.join(CSRC, "kernels")
HDIR = os.path.join(CSRC, "host")
INC = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libfbcorr.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
ARCH = "gfx950"
NO_PACKED_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

# Representative specialisations used only for the offline compile check.
CHECK_DEFINES = {
    "igemm.hip": ["-DFB_BATCH=1 -DFB_FH=9 -DFB_FW=9 -DFB_CIN=8 -DFB_COUT=64 -DFB_HI=256 -DFB_WI=256 -DFB_HO=248 -DFB_WO=248 "
                  "-DFB_PADH=0 -DFB_PADW=0 -DFB_MF=32 -DFB_KC=8 -DFB_S=1 -DFB_MR=1 -DFB_KS=1 -DFB_MT=1 -DFB_NT=2 -DFB_WM=4 -DFB_WN=1 -DFB_DT=0 -DFB_XPAD=4 "
                  "-DFB_WPAD=4 -DFB_USTAGE=1 -DFB_XCDMAP=1 -DFB_EPILOGUE(v,c)=fmaxf(v,0.f)",
                  "-DFB_BATCH=1 -DFB_FH=13 -DFB_FW=13 -DFB_CIN=16 -DFB_COUT=128 -DFB_HI=512 -DFB_WI=512 -DFB_HO=500 -DFB_WO=500 "
                  "-DFB_PADH=0 -DFB_PADW=0 -DFB_MF=32 -DFB_KC=16 -DFB_S=1 -DFB_MR=2 -DFB_KS=1 -DFB_MT=2 -DFB_NT=1 -DFB_WM=8 -DFB_WN=1 -DFB_DT=2 -DFB_XPAD=24 "
                  "-DFB_WPAD=8 -DFB_USTAGE=1 -DFB_XCDMAP=1 -DFB_XMOFF=128"],
    "direct.hip": ["-DFB_BATCH=1 -DFB_FH=9 -DFB_FW=9 -DFB_D=8 -DFB_N=64 -DFB_H=256 -DFB_W=256 -DFB_HO=248 -DFB_WO=248 "
                   "-DFB_TH=8 -DFB_TW=32 -DFB_P=4 -DFB_Q=16 -DFB_NB=64 -DFB_DS=1 -DFB_LAYOUT=1 -DFB_XPAD=1 -DFB_WPAD=4 "
                   "-DFB_UD=1 -DFB_XCDMAP=1 -DFB_EPILOGUE(v,c)=fmaxf(v,0.f)",
                   "-DFB_BATCH=1 -DFB_FH=9 -DFB_FW=9 -DFB_D=8 -DFB_N=64 -DFB_H=256 -DFB_W=256 -DFB_HO=248 -DFB_WO=248 "
                   "-DFB_TH=16 -DFB_TW=32 -DFB_P=8 -DFB_Q=16 -DFB_NB=32 -DFB_DS=1 -DFB_LAYOUT=1 -DFB_XPAD=1 -DFB_WPAD=4 "
                   "-DFB_UD=1 -DFB_XCDMAP=1 -DFB_FSRC=1 -DFB_NPAD=64"],
    "dw.hip": ["-DFB_BATCH=1 -DFB_FH=9 -DFB_FW=9 -DFB_D=8 -DFB_N=64 -DFB_H=256 -DFB_W=256 -DFB_HO=248 -DFB_WO=248 "
               "-DFB_RH=2 -DFB_RW=32 -DFB_NW=8 -DFB_TPB=21 -DFB_NP=128 -DFB_GPAD=4 -DFB_XPAD=4 -DFB_PF=1",
               "-DFB_BATCH=1 -DFB_FH=9 -DFB_FW=9 -DFB_D=8 -DFB_N=64 -DFB_H=256 -DFB_W=256 -DFB_HO=248 -DFB_WO=248 "
               "-DFB_RH=2 -DFB_RW=64 -DFB_NW=8 -DFB_TPB=21 -DFB_NP=128 -DFB_GPAD=4 -DFB_XPAD=4 -DFB_PF=2"],
    "nn.hip": ["-DFB_NN_NORMS -DFB_NN_OFFSETS -DFB_NN_SCATTER -DFB_T=4096 -DFB_M=1048576 -DFB_D=64 -DFB_SPLIT=1",
               "-DFB_NN_NORMS -DFB_T=4096 -DFB_M=4096 -DFB_D=64 -DFB_SPLIT=0",
               "-DFB_NN_SCAN -DFB_T=4096 -DFB_M=1048576 -DFB_D=64 -DFB_SPLIT=1 -DFB_NT=8 -DFB_WV=4 -DFB_CH=128 "
               "-DFB_BT=4 -DFB_TG=2 -DFB_XCDMAP=1",
               "-DFB_NN_SCAN -DFB_T=4096 -DFB_M=4096 -DFB_D=64 -DFB_SPLIT=0 -DFB_NT=8 -DFB_WV=4 -DFB_CH=2 "
               "-DFB_BT=2 -DFB_TG=1 -DFB_XCDMAP=1",
               "-DFB_NN_FINAL -DFB_T=4096 -DFB_M=1048576 -DFB_D=64 -DFB_SPLIT=1 -DFB_FW=4 -DFB_TG=2 -DFB_NCHK=513",
               "-DFB_NN_FINAL -DFB_T=4096 -DFB_M=4096 -DFB_D=64 -DFB_SPLIT=0 -DFB_FW=4 -DFB_TG=1 -DFB_NCHK=128"],
    "rgemm.hip": ["-DFB_BATCH=1 -DFB_FH=13 -DFB_FW=13 -DFB_CIN=16 -DFB_COUT=128 -DFB_HI=512 -DFB_WI=512 -DFB_HO=500 "
                  "-DFB_WO=500 -DFB_PADH=0 -DFB_PADW=0 -DFB_DT=1 -DFB_KC=16 -DFB_MR=2 -DFB_MT=4 -DFB_NT=2 -DFB_WM=2 "
                  "-DFB_WN=2 -DFB_PF=3 -DFB_XPADC=0 -DFB_WPE=2 -DFB_XCDMAP=1 -DFB_KNAME=fbcorr_fwd_rgemm "
                  "-DFB_EPILOGUE(v,c)=fmaxf(v,0.f)",
                  "-DFB_BATCH=32 -DFB_FH=7 -DFB_FW=7 -DFB_CIN=16 -DFB_COUT=64 -DFB_HI=128 -DFB_WI=128 -DFB_HO=122 "
                  "-DFB_WO=122 -DFB_PADH=0 -DFB_PADW=0 -DFB_DT=0 -DFB_KC=16 -DFB_MR=2 -DFB_MT=4 -DFB_NT=2 -DFB_WM=2 "
                  "-DFB_WN=1 -DFB_PF=3 -DFB_XPADC=0 -DFB_WPE=2 -DFB_XCDMAP=1 -DFB_KNAME=fbcorr_fwd_rgemm",
                  "-DFB_BATCH=1 -DFB_FH=5 -DFB_FW=5 -DFB_CIN=3 -DFB_COUT=7 -DFB_HI=20 -DFB_WI=19 -DFB_HO=16 "
                  "-DFB_WO=15 -DFB_PADH=0 -DFB_PADW=0 -DFB_DT=2 -DFB_KC=8 -DFB_MR=1 -DFB_MT=1 -DFB_NT=1 -DFB_WM=1 "
                  "-DFB_WN=1 -DFB_PF=2 -DFB_XPADC=1 -DFB_WPE=1 -DFB_XCDMAP=0 -DFB_KNAME=fbcorr_fwd_rgemm",
                  "-DFB_BATCH=1 -DFB_FH=13 -DFB_FW=13 -DFB_CIN=16 -DFB_COUT=128 -DFB_HI=512 -DFB_WI=512 -DFB_HO=500 "
                  "-DFB_WO=500 -DFB_PADH=0 -DFB_PADW=0 -DFB_DT=2 -DFB_KC=16 -DFB_MR=2 -DFB_MT=4 -DFB_NT=2 -DFB_WM=2 "
                  "-DFB_WN=2 -DFB_PF=3 -DFB_XPADC=0 -DFB_WPE=2 -DFB_XCDMAP=1 -DFB_KNAME=fbcorr_fwd_rgemm -DFB_XMOFF=128",
                  "-DFB_PACK_FRAG -DFB_FH=13 -DFB_FW=13 -DFB_CIN=16 -DFB_COUT=128 -DFB_DT=1 -DFB_KC=16 -DFB_PF=3",
                  "-DFB_PACK_FRAG -DFB_FH=7 -DFB_FW=7 -DFB_CIN=64 -DFB_COUT=16 -DFB_DT=0 -DFB_KC=16 -DFB_PF=3 -DFB_FLIP"],
    "util.hip": "-DFB_SUM_PARTIALS -DFB_L=41472 -DFB_NP=256 -DFB_RS=16 -DFB_LANES=16 -DFB_FLIP_FILTERS -DFB_N=64 -DFB_FH=9 -DFB_FW=9 -DFB_D=8 "
                "-DFB_PACK_LOWP -DFB_LOWP=1 -DFB_FILL_INT -DFB_TRANSPOSE_FILTERS -DFB_NPAD=64 -DFB_ABSMAX",
}


def _run(cmd, **kw):
    print("+", " ".join(cmd), flush=True)
    subprocess.check_call(cmd, **kw)


def embed_kernels() -> str:
    out = os.path.join(HDIR, "kernels_embed.h")
    files = sorted(glob.glob(os.path.join(KDIR, "*.hip")))
    parts = ["// Generated by build.py from csrc/kernels/*.hip; do not edit.",
             "#pragma once", "#include <cstddef>", "namespace fbc {",
             "struct EmbeddedKernel { const char* name; const char* text; };",
             "static const EmbeddedKernel kEmbedded[] = {"]
    for f in files:
        name = os.path.splitext(os.path.basename(f))[0]
        text = open(f).read()
        if ")FBCK\"" in text:
            raise RuntimeError("delimiter clash in " + f)
        parts.append('    {"%s", R"FBCK(%s)FBCK"},' % (name, text))
    parts += ["};", "static const size_t kEmbeddedCount = sizeof(kEmbedded) / sizeof(kEmbedded[0]);",
              "}  // namespace fbc", ""]
    new = "\n".join(parts)
    if not os.path.exists(out) or open(out).read() != new:
        with open(out, "w") as fh:
            fh.write(new)
    return out


def build_host() -> str:
    embed_kernels()
    srcs = sorted(glob.glob(os.path.join(HDIR, "*.cpp")))
    tmp = LIB + ".tmp%d" % os.getpid()
    # The one HIP source of the host library (the allocation-free entry
    # point's device scratch array): hipcc, device code for gfx950.
    objdir = os.path.join(CSRC, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for f in sorted(glob.glob(os.path.join(HDIR, "*.hip"))):
        o = os.path.join(objdir, os.path.basename(f) + ".o")
        _run([HIPCC, "--offload-arch=" + ARCH, "-O2", "-fPIC", "-std=c++17", "-fvisibility=hidden",
              *NO_PACKED_FP32, "-I" + INC, "-I" + HDIR, "-c", f, "-o", o])
        objs.append(o)
    # Everything else is host code: plain g++ against the HIP runtime and
    # hiprtc.
    _run(["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-Wall", "-Wno-unused-result", "-fvisibility=hidden",
          "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"),
          "-I" + INC, "-I" + HDIR, *srcs, *objs, "-o", tmp,
          "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-lhiprtc", "-pthread",
          "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    os.replace(tmp, LIB)
    return LIB


def check_kernels(outdir: str | None = None) -> None:
    outdir = outdir or os.path.join(CSRC, "_build")
    os.makedirs(outdir, exist_ok=True)
    for f in sorted(glob.glob(os.path.join(KDIR, "*.hip"))):
        base = os.path.basename(f)
        variants = CHECK_DEFINES.get(base, "")
        for k, defs in enumerate([variants] if isinstance(variants, str) else variants):
            _run([HIPCC, "--offload-arch=" + ARCH, "-O3", "--cuda-device-only", "--no-gpu-bundle-output",
                  "-c", f, "-o", os.path.join(outdir, "%s.%d.co" % (base, k)), *NO_PACKED_FP32, *defs.split()])


def warm_cache() -> None:
    """Compile (through the library, as a plan would) the kernels of the
    benchmark and smoke workloads into a fresh on-disk code-object cache, so
    a fresh process finds them there instead of running hiprtc."""
    cache = os.path.join(HERE, "_rtc_cache")
    if os.path.isdir(cache):
        shutil.rmtree(cache)          # drop entries of earlier kernel versions
    sys.path.insert(0, ROOT)
    import workloads as wl
    from paper_0911_3456_amd import _native as nat
    nat.load()
    jobs = []
    for name in ("tiny", "fp32", "differentiation"):
        s = wl.WORKLOADS[name].shape
        d = nat.make_desc(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw)
        jobs += [(d, "forward", None), (d, "forward", "algo=direct"), (d, "backward_x", None),
                 (d, "backward_w", None)]
    s = wl.WORKLOADS["precision"].shape
    for prec in ("fp32", "bf16", "fp16"):
        jobs.append((nat.make_desc(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, precision=prec), "forward", None))
    jobs.append((nat.make_desc(s.batch, s.H, s.W, s.D, s.N, s.fh, s.fw, algo="direct"), "forward", None))
    for d, role, cfg in jobs:
        nat.compile_check(d, role, cfg)
    for m in wl.NN_NEIGHBOURS:
        nat.nn_compile_check(wl.NN_TARGETS, m, wl.NN_PATCH * wl.NN_PATCH)
    shapes, _ = wl.draw_batched_list()
    nat.compile_check_batched([nat.make_desc(1, s.H, s.W, s.D, s.N, s.fh, s.fw) for s in shapes])
    print("code-object cache:", nat.cache_stats(), flush=True)


def build(check: bool = True, warm: bool = True) -> str:
    lib = build_host()
    if check:
        check_kernels()
    if warm:
        warm_cache()
    return lib


if __name__ == "__main__":
    build(check="--no-check" not in sys.argv, warm="--no-warm" not in sys.argv)
