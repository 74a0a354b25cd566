"""Host-side tests of the C-ABI library (no GPU needed).

The library loads, exports every entry point include/fbcorr.h declares,
generates deterministic specialised sources, compiles every role for gfx950
with hiprtc without a device, and turns bad input into status codes.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_0911_3456_amd import _native
    return _native, _native.load()


def _header_symbols():
    text = open(os.path.join(ROOT, "include", "fbcorr.h")).read()
    return sorted(set(re.findall(r"FBCORR_API\s+[\w\s\*]+?\b(fbcorr_\w+)\s*\(", text)))


def test_header_symbols_exported():
    nat, lib = _lib()
    syms = _header_symbols()
    assert len(syms) >= 18
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(nat.EXPORTS) == syms


def test_status_strings_and_version():
    nat, lib = _lib()
    for code, name in nat.STATUS_NAMES.items():
        assert lib.fbcorr_status_string(code).decode() == name
    assert lib.fbcorr_version() >= 100


def test_codegen_is_deterministic_and_specialised():
    from paper_0911_3456_amd import codegen, make_desc
    d = make_desc(1, 256, 256, 8, 64, 9, 9)
    s1, o1 = codegen(d)
    s2, o2 = codegen(d)
    assert s1 == s2 and o1 == o2
    assert "-DFB_FH=9" in o1 and "-DFB_CIN=8" in o1 and "-DFB_COUT=64" in o1
    _, o3 = codegen(make_desc(1, 256, 256, 8, 64, 7, 7))
    assert o3 != o1 and "-DFB_FH=7" in o3
    _, od = codegen(d, "forward", "algo=direct th=4")
    assert "-DFB_TH=4" in od
    _, ob = codegen(d, "backward_x")
    assert "-DFB_PADH=8" in ob and "-DFB_CIN=64" in ob and "-DFB_COUT=8" in ob


@pytest.mark.parametrize("shape,prec", [
    ((1, 64, 64, 4, 16, 5, 5), "fp32"),
    ((1, 256, 256, 8, 64, 9, 9), "fp32"),
    ((1, 512, 512, 16, 128, 13, 13), "bf16"),
    ((1, 512, 512, 16, 128, 13, 13), "fp16"),
    ((32, 128, 128, 16, 64, 7, 7), "fp32"),
    ((2, 37, 45, 3, 7, 3, 4), "fp32"),
])
def test_compile_every_role_for_gfx950(shape, prec):
    from paper_0911_3456_amd import compile_check, make_desc
    d = make_desc(*shape, precision=prec)
    assert compile_check(d, "forward") > 0
    if prec == "fp32":
        assert compile_check(d, "forward", "algo=direct") > 0
        assert compile_check(d, "backward_x") > 0
        assert compile_check(d, "backward_w") > 0


def test_compile_cache_hits():
    from paper_0911_3456_amd import cache_stats, compile_check, make_desc
    d = make_desc(1, 30, 31, 4, 8, 3, 3)
    compile_check(d)
    before = cache_stats()
    compile_check(d)
    after = cache_stats()
    assert after["hits"] > before["hits"]
    assert after["entries"] == before["entries"]


def test_invalid_descriptors_map_to_status():
    from paper_0911_3456_amd import FbcorrError, codegen, make_desc
    with pytest.raises(FbcorrError) as e:
        codegen(make_desc(1, 8, 8, 4, 4, 9, 3))
    assert e.value.status_name == "FBCORR_ERR_SHAPE"
    with pytest.raises(FbcorrError) as e:
        codegen(make_desc(1, 0, 8, 4, 4, 3, 3))
    assert e.value.status_name == "FBCORR_ERR_INVALID_ARGUMENT"
    with pytest.raises(FbcorrError) as e:
        codegen(make_desc(1, 8, 8, 4, 4, 3, 3, precision="bf16", algo="direct"))
    assert e.value.status_name == "FBCORR_ERR_UNSUPPORTED"
    with pytest.raises(FbcorrError) as e:
        codegen(make_desc(1, 8, 8, 4, 4, 3, 3, flags=2))
    assert e.value.status_name == "FBCORR_ERR_INVALID_ARGUMENT"
    assert codegen(make_desc(1, 8, 8, 4, 4, 3, 3, flags=1))[0]     # FBCORR_FLAG_OVERLAP_BACKWARD


def test_bad_configs_rejected_before_compiling():
    from paper_0911_3456_amd import FbcorrError, codegen, make_desc
    d = make_desc(1, 256, 256, 8, 64, 9, 9)
    for cfg in ["algo=igemm s=3", "algo=igemm wm=32", "algo=direct p=3", "algo=igemm kc=8 xpad=1",
                "algo=igemm mt=4 nt=4", "bogus", "algo=nope", "algo=igemm mtt=2"]:
        with pytest.raises(FbcorrError):
            codegen(d, "forward", cfg)
    with pytest.raises(FbcorrError) as e:
        codegen(make_desc(1, 256, 256, 64, 128, 13, 13), "forward", "algo=igemm kc=64 ustage=13 nt=4")
    assert e.value.status_name == "FBCORR_ERR_UNSUPPORTED"    # LDS over the device limit


def test_kernel_knobs_accepted_and_checked():
    """The filter-gradient knobs (unr, bal, skipe) and the implicit-GEMM
    knobs (uunr, swz) reach the generated options; out-of-range values and
    a swizzle without 16-bit operands are refused before compiling."""
    from paper_0911_3456_amd import FbcorrError, codegen, make_desc
    d = make_desc(1, 256, 256, 8, 64, 9, 9)
    _, o = codegen(d, "backward_w", "algo=dw rh=2 rw=62 nw=8 tpb=21 np=124 unr=0 skipe=1")
    assert "-DFB_UNR=0" in o and "-DFB_SKIPE=1" in o and "-DFB_BAL" not in o
    _, o = codegen(d, "backward_w", "algo=dw rh=2 rw=32 nw=8 tpb=25 np=64 bal=1")
    assert "-DFB_BAL=1" in o
    _, o = codegen(d, "forward", "algo=igemm kc=8 ustage=3 uunr=1")
    assert "-DFB_UUNR=1" in o
    lp = make_desc(1, 128, 128, 16, 64, 7, 7, precision="bf16")
    _, o = codegen(lp, "forward", "algo=igemm kc=16 mr=2 mt=2 nt=1 wm=8 xpad=24 swz=1")
    assert "-DFB_SWZ=1" in o
    for role, cfg in [("backward_w", "algo=dw unr=-1"), ("backward_w", "algo=dw bal=2"),
                      ("backward_w", "algo=dw nw=2 tpb=42 bal=1"),       # more than 8 slots per wave
                      ("forward", "algo=igemm kc=8 swz=1")]:           # fp32 operands
        with pytest.raises(FbcorrError):
            codegen(d, role, cfg)
    with pytest.raises(FbcorrError):
        codegen(lp, "forward", "algo=igemm kc=8 swz=1")                # 8-channel chunks


def test_rgemm_knobs_accepted_and_checked():
    """The register-streamed kernel's knobs reach the generated options of
    the main kernel and of its filter pack (the pack flips the bank for the
    input gradient); impossible values are refused before compiling."""
    from paper_0911_3456_amd import FbcorrError, codegen, make_desc
    lp = make_desc(1, 512, 512, 16, 128, 13, 13, precision="bf16")
    _, o = codegen(lp, "forward", "algo=rgemm mf=32 kc=16 mr=2 mt=4 nt=2 wm=2 wn=2 pf=3 wpe=2")
    for k in ("-DFB_KNAME=fbcorr_fwd_rgemm", "-DFB_DT=1", "-DFB_MF=32", "-DFB_KC=16", "-DFB_PF=3", "-DFB_WPE=2"):
        assert k in o, k
    d = make_desc(2, 45, 77, 16, 64, 7, 7)
    _, o = codegen(d, "backward_x", "algo=rgemm mf=16 kc=16 mr=1 mt=8 nt=1 wm=4 wn=1")
    assert "-DFB_KNAME=fbcorr_dx_rgemm" in o and "-DFB_PADH=6" in o and "-DFB_CIN=64" in o and "-DFB_COUT=16" in o
    for role, cfg in [("forward", "algo=rgemm kc=12"),            # not the cell width times a power of two
                      ("forward", "algo=rgemm mf=8"),
                      ("forward", "algo=rgemm mr=3"),
                      ("forward", "algo=rgemm pf=9"),
                      ("forward", "algo=rgemm mt=8 nt=4 wpe=2"),  # accumulators over the register budget
                      ("forward", "algo=rgemm flip=1"),           # flip is the input gradient's
                      ("forward", "algo=rgemm s=3"),
                      ("forward", "algo=rgemm mf=16 nt=1 wn=1 s=32"),
                      ("forward", "algo=rgemm mf=32 s=2 mt=4 nt=1 wm=2 wn=1 ste=1"),   # ste needs s=1
                      ("backward_w", "algo=rgemm")]:
        with pytest.raises(FbcorrError):
            codegen(lp if role == "forward" else d, role, cfg)
    # stores through LDS and streaming stores reach the options; ste needs a
    # multiple of 4 output channels (16-byte rows)
    _, o = codegen(lp, "forward", "algo=rgemm mf=32 kc=16 mr=2 mt=4 nt=2 wm=2 wn=2 pf=3 ste=1 nts=1")
    assert "-DFB_STE=1" in o and "-DFB_NTS=1" in o
    with pytest.raises(FbcorrError):
        codegen(make_desc(1, 40, 40, 8, 30, 5, 5), "forward", "algo=rgemm mf=32 mt=2 nt=1 wm=2 wn=1 ste=1")


def test_fp16_forward_has_input_scale():
    """fp16 forward roles (both matrix-core algorithms) read the partial
    maxima of |x| for the per-tensor input scale; bf16 and fp32 do not."""
    from paper_0911_3456_amd import codegen, make_desc
    for algo in ("igemm", "rgemm"):
        _, o = codegen(make_desc(1, 40, 43, 16, 64, 7, 7, precision="fp16"), "forward", "algo=" + algo)
        assert "-DFB_XMOFF=" in o
        _, o = codegen(make_desc(1, 40, 43, 16, 64, 7, 7, precision="bf16"), "forward", "algo=" + algo)
        assert "-DFB_XMOFF" not in o
    _, o = codegen(make_desc(1, 40, 43, 16, 64, 7, 7), "forward", "algo=igemm")
    assert "-DFB_XMOFF" not in o


def test_compile_error_is_reported():
    """An injected code-generation failure comes back as FBCORR_ERR_COMPILE
    with the compiler log, and the library stays usable."""
    nat, lib = _lib()
    d = nat.make_desc(1, 16, 16, 4, 4, 3, 3)
    n = ctypes.c_size_t(0)
    for role in (0, 1, 2):
        st = lib.fbcorr_compile_check(ctypes.byref(d), role, b"inject_error=1", b"gfx950", ctypes.byref(n))
        assert nat.STATUS_NAMES[st] == "FBCORR_ERR_COMPILE"
        assert b"injected code-generation failure" in lib.fbcorr_last_error()
    assert lib.fbcorr_compile_check(ctypes.byref(d), 0, None, b"gfx950", ctypes.byref(n)) == 0
    st = lib.fbcorr_compile_check(ctypes.byref(d), 0, None, b"gfx_not_a_gpu", ctypes.byref(n))
    assert nat.STATUS_NAMES[st] == "FBCORR_ERR_UNSUPPORTED"


def test_null_arguments():
    nat, lib = _lib()
    assert nat.STATUS_NAMES[lib.fbcorr_plan(None, 0, None)] == "FBCORR_ERR_INVALID_ARGUMENT"
    assert lib.fbcorr_plan_destroy(None) == 0
    n = ctypes.c_size_t(0)
    assert nat.STATUS_NAMES[lib.fbcorr_workspace_size(None, 0, ctypes.byref(n))] == "FBCORR_ERR_INVALID_ARGUMENT"
    assert nat.STATUS_NAMES[lib.fbcorr_forward(None, None, None, None, None, 0, None)] == \
        "FBCORR_ERR_INVALID_ARGUMENT"


def test_plan_without_device_reports_no_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    nat, lib = _lib()
    d = nat.make_desc(1, 16, 16, 4, 4, 3, 3)
    h = ctypes.c_void_p()
    st = lib.fbcorr_plan(ctypes.byref(d), 0, ctypes.byref(h))
    assert nat.STATUS_NAMES[st] == "FBCORR_ERR_NO_DEVICE"
    assert not h.value


def test_gpu_test_configurations_are_valid():
    """Every explicit configuration the GPU tests install fits the device
    limits (checked here, on the host, before any GPU run)."""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import paper_0911_3456_amd as fb
    import test_gpu_backward as tb
    import test_gpu_forward as tf
    d = fb.make_desc(2, 45, 77, 8, 64, 9, 9)
    for c in tf.IGEMM_CFGS:
        fb.codegen(d, "forward", "algo=igemm " + c)
    for c in tf.DIRECT_CFGS:
        fb.codegen(d, "forward", "algo=direct " + c)
    d = fb.make_desc(2, 41, 67, 8, 64, 9, 9)
    for c in tb.BX_CFGS:
        fb.codegen(d, "backward_x", "algo=igemm " + c)
    for c in tb.BW_CFGS:
        fb.codegen(d, "backward_w", "algo=dw " + c)
    import test_gpu_precision as tp
    d = fb.make_desc(2, 45, 60, 16, 64, 7, 7, precision="bf16")
    for c in tp.LOWP_CFGS:
        if c:
            fb.codegen(d, "forward", c)
    import test_gpu_rgemm as tr
    d = fb.make_desc(2, 45, 77, 8, 64, 9, 9)
    for c in tr.RGEMM_CFGS:
        fb.codegen(d, "forward", "algo=rgemm " + c)
    for prec in ("bf16", "fp16"):
        d = fb.make_desc(1, 50, 61, 32, 128, 7, 7, precision=prec)
        for c in tr.LOWP_CFGS:
            fb.codegen(d, "forward", "algo=rgemm " + c)
    for sh in tr.SHAPES:
        for prec in ("fp32", "bf16", "fp16"):
            fb.codegen(fb.make_desc(*sh, precision=prec), "forward", "algo=rgemm")
    d = fb.make_desc(2, 41, 67, 16, 64, 7, 7)
    for c in tr.DX_CFGS:
        fb.codegen(d, "backward_x", ("algo=rgemm " + c).strip())
    for sh, prec, c in tr.SHIFT_SHAPES:
        fb.codegen(fb.make_desc(*sh, precision=prec), "forward", "algo=rgemm " + c)
    for sh in tr.DX_SHAPES:
        fb.codegen(fb.make_desc(*sh), "backward_x", "algo=rgemm")


def test_disk_cache_reuse_and_corruption(tmp_path, monkeypatch):
    """Compiled code persists on disk keyed by source, options, architecture
    and compiler version; a damaged entry is recompiled and rewritten."""
    from paper_0911_3456_amd import cache_clear, cache_stats, compile_check, make_desc
    monkeypatch.setenv("FBCORR_CACHE_DIR", str(tmp_path))
    d = make_desc(1, 23, 29, 4, 8, 3, 5)
    cache_clear()
    s0 = cache_stats()
    compile_check(d)
    s1 = cache_stats()
    files = sorted(tmp_path.glob("*.co"))
    assert len(files) >= 1 and s1["misses"] > s0["misses"]
    cache_clear()
    compile_check(d)
    s2 = cache_stats()
    assert s2["disk_hits"] > s1["disk_hits"] and s2["misses"] == s1["misses"]
    # damage every entry: it must be recompiled, not loaded
    for f in files:
        raw = bytearray(f.read_bytes())
        raw[-1] ^= 0xFF
        f.write_bytes(bytes(raw))
    cache_clear()
    compile_check(d)
    s3 = cache_stats()
    assert s3["misses"] > s2["misses"]
    cache_clear()
    compile_check(d)
    assert cache_stats()["disk_hits"] > s3["disk_hits"]     # rewritten and valid again
    monkeypatch.setenv("FBCORR_CACHE", "0")
    cache_clear()
    s5 = cache_stats()
    compile_check(d)
    assert cache_stats()["disk_hits"] == s5["disk_hits"]


def test_cache_entry_shared_by_kernels_of_one_code_object(tmp_path, monkeypatch):
    """The cache key names the template, not the kernel: the persistent
    batched kernel and its counter-reset kernel (one generated source) share
    one on-disk entry, so a plan never recompiles the module for the second
    kernel."""
    import workloads as wl
    from paper_0911_3456_amd import _native as nat
    monkeypatch.setenv("FBCORR_CACHE_DIR", str(tmp_path))
    nat.cache_clear()
    shapes, _ = wl.draw_batched_list(count=6, seed=31)
    nat.compile_check_batched([nat.make_desc(1, s.H, s.W, s.D, s.N, s.fh, s.fw) for s in shapes])
    names = [f.name for f in tmp_path.glob("*.co")]
    assert len(names) == 1 and names[0].startswith("batched-"), names
    nat.cache_clear()


def test_kept_sources(tmp_path, monkeypatch):
    """FBCORR_KEEP_SOURCE keeps every generated source that is compiled, with
    its options; the batched source keeps each variant's body a function of
    its own and asks for two waves per SIMD."""
    import workloads as wl
    from paper_0911_3456_amd import _native as nat
    keep = tmp_path / "keep"
    keep.mkdir()
    monkeypatch.setenv("FBCORR_CACHE_DIR", str(tmp_path / "cache"))
    monkeypatch.setenv("FBCORR_KEEP_SOURCE", str(keep))
    nat.cache_clear()
    nat.compile_check(nat.make_desc(1, 30, 40, 4, 16, 3, 3), "forward")
    kept = sorted(keep.glob("igemm-*.hip"))
    assert len(kept) == 1
    text = kept[0].read_text()
    assert text.startswith("// options:") and "-DFB_FH=3" in text.splitlines()[0]
    assert "igemm_body" in text
    shapes, _ = wl.draw_batched_list(count=4, seed=32)
    nat.compile_check_batched([nat.make_desc(1, s.H, s.W, s.D, s.N, s.fh, s.fw) for s in shapes])
    (bsrc,) = keep.glob("batched-*.hip")
    btext = bsrc.read_text()
    assert "#define FB_BATCHED 1" in btext and "__attribute__((noinline))" in btext
    assert "amdgpu_waves_per_eu(2)" in btext
    monkeypatch.delenv("FBCORR_KEEP_SOURCE")
    nat.cache_clear()


def test_tuning_database_supplies_defaults(tmp_path, monkeypatch):
    from paper_0911_3456_amd import cache_clear, codegen, make_desc
    db = tmp_path / "db.txt"
    db.write_text("# test\ngfx950 forward fp32 1 40 50 8 64 5 5 : algo=igemm kc=4 mr=2 nt=1 wm=2 wn=2\n")
    monkeypatch.setenv("FBCORR_TUNING_DB", str(db))
    cache_clear()
    _, opts = codegen(make_desc(1, 40, 50, 8, 64, 5, 5))
    assert "-DFB_KC=4" in opts and "-DFB_MR=2" in opts and "-DFB_WN=2" in opts
    _, opts2 = codegen(make_desc(1, 40, 51, 8, 64, 5, 5))      # other shape: heuristic
    assert "-DFB_WN=2" not in opts2
    db.write_text("gfx950 forward fp32 1 40 50 8 64 5 5 : algo=igemm s=3\n")   # invalid entry
    cache_clear()
    _, opts3 = codegen(make_desc(1, 40, 50, 8, 64, 5, 5))
    assert "-DFB_S=1" in opts3
    monkeypatch.delenv("FBCORR_TUNING_DB")
    cache_clear()


def test_batched_kernel_generation_compiles():
    from paper_0911_3456_amd import compile_check_batched, make_desc
    import workloads as wl
    shapes, _ = wl.draw_batched_list(count=6, seed=9)
    descs = [make_desc(1, s.H, s.W, s.D, s.N, s.fh, s.fw) for s in shapes]
    assert compile_check_batched(descs) > 0


def test_batched_variants_take_the_standalone_constants(tmp_path, monkeypatch):
    """A batched variant is compiled with exactly the constants of its
    standalone kernel: a tuned ustage larger than the filter height is
    clamped (as the standalone kernel's LDS budget assumes) and the unrolled
    stage loop is kept.  Uses the tuning entries of the GPU test."""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import test_gpu_fullsize as tfs
    from paper_0911_3456_amd import _native as nat
    db = tmp_path / "db.txt"
    db.write_text("\n".join(tfs.CLAMP_DB_LINES) + "\n")
    keep = tmp_path / "keep"
    keep.mkdir()
    monkeypatch.setenv("FBCORR_TUNING_DB", str(db))
    monkeypatch.setenv("FBCORR_CACHE_DIR", str(tmp_path / "cache"))
    monkeypatch.setenv("FBCORR_KEEP_SOURCE", str(keep))
    nat.cache_clear()
    shapes = tfs.CLAMP_SHAPES
    nat.compile_check_batched([nat.make_desc(1, s.H, s.W, s.D, s.N, s.fh, s.fw) for s in shapes])
    (bsrc,) = keep.glob("batched-*.hip")
    text = bsrc.read_text()
    parts = text.split("// ---- variant ")[1:]
    assert len(parts) == 3
    for part, s in zip(parts, shapes):
        head = part.splitlines()[0]
        assert "fh=%d" % s.fh in head and "ustage=3" in head and "uunr=1" in head
        assert "#define FB_USTAGE %d\n" % min(3, s.fh) in part
        assert "#define FB_UUNR 1\n" in part
        assert "#define FB_HI" not in part and "#define FB_KNAME" not in part
    monkeypatch.delenv("FBCORR_KEEP_SOURCE")
    monkeypatch.delenv("FBCORR_TUNING_DB")
    nat.cache_clear()
