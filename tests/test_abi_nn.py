"""Host-side tests of the nearest-neighbour entry points (no GPU needed):
exports, run-time kernel generation for gfx950, and status codes."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_0911_3456_amd import _native
    return _native, _native.load()


def test_header_symbols_exported():
    nat, lib = _lib()
    text = open(os.path.join(ROOT, "include", "fbnn.h")).read()
    syms = sorted(set(re.findall(r"FBCORR_API\s+[\w\s\*]+?\b(fbnn_\w+)\s*\(", text)))
    assert len(syms) == 10
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(nat.NN_EXPORTS) == syms


@pytest.mark.parametrize("T,M,D", [(4096, 1048576, 64), (4096, 4096, 64), (1, 1, 16), (37, 1000, 48),
                                   (5, 77, 512), (0, 50, 64)])
def test_compile_for_gfx950(T, M, D):
    from paper_0911_3456_amd import nn_compile_check
    for split in (0, 1):
        assert nn_compile_check(T, M, D, "split=%d" % split) > 1000


def test_bad_configs_and_descriptors():
    from paper_0911_3456_amd import FbcorrError, nn_compile_check
    for cfg in ["nt=0", "nt=9", "wv=0", "wv=17", "ch=0", "pf=1", "xcd=3", "fw=0", "bogus", "algo=igemm",
                "nt=4 mt=2", "bt=3", "bt=2 tg=4", "tg=3", "split=2"]:
        with pytest.raises(FbcorrError):
            nn_compile_check(64, 1000, 64, cfg)
    with pytest.raises(FbcorrError) as e:
        nn_compile_check(64, 1000, 512, "nt=4")      # target fragments over the register budget
    assert e.value.status_name == "FBCORR_ERR_UNSUPPORTED"
    with pytest.raises(FbcorrError) as e:
        nn_compile_check(64, 1000, 512, "nt=1 bt=16")  # LDS batch over the device limit
    assert e.value.status_name == "FBCORR_ERR_UNSUPPORTED"
    for T, M, D in [(1, 1, 15), (1, 1, 0), (1, 1, 528), (1, 0, 64), (-1, 5, 64)]:
        with pytest.raises(FbcorrError) as e:
            nn_compile_check(T, M, D)
        assert e.value.status_name == "FBCORR_ERR_INVALID_ARGUMENT"
    with pytest.raises(FbcorrError) as e:
        nn_compile_check(1, 2 ** 31 - 8, 64)
    assert e.value.status_name == "FBCORR_ERR_UNSUPPORTED"


def test_compile_error_is_reported():
    nat, lib = _lib()
    d = nat.NNDesc(64, 1000, 64, 0)
    n = ctypes.c_size_t(0)
    st = lib.fbnn_compile_check(ctypes.byref(d), b"inject_error=1", b"gfx950", ctypes.byref(n))
    assert nat.STATUS_NAMES[st] == "FBCORR_ERR_COMPILE"
    assert b"injected code-generation failure" in lib.fbcorr_last_error()
    assert lib.fbnn_compile_check(ctypes.byref(d), None, b"gfx950", ctypes.byref(n)) == 0
    st = lib.fbnn_compile_check(ctypes.byref(d), None, b"gfx_not_a_gpu", ctypes.byref(n))
    assert nat.STATUS_NAMES[st] == "FBCORR_ERR_UNSUPPORTED"
    d.flags = 1
    assert nat.STATUS_NAMES[lib.fbnn_compile_check(ctypes.byref(d), None, None, None)] == \
        "FBCORR_ERR_INVALID_ARGUMENT"


def test_null_arguments_and_no_device():
    import torch
    nat, lib = _lib()
    assert nat.STATUS_NAMES[lib.fbnn_plan(None, 0, None)] == "FBCORR_ERR_INVALID_ARGUMENT"
    assert lib.fbnn_plan_destroy(None) == 0
    n = ctypes.c_size_t(0)
    assert nat.STATUS_NAMES[lib.fbnn_workspace_size(None, 0, ctypes.byref(n))] == "FBCORR_ERR_INVALID_ARGUMENT"
    assert nat.STATUS_NAMES[lib.fbnn_search(None, None, None, None, None, None, 0, None)] == \
        "FBCORR_ERR_INVALID_ARGUMENT"
    assert nat.STATUS_NAMES[lib.fbnn_tune(None, None, None, None, 0, None, None, None)] == \
        "FBCORR_ERR_INVALID_ARGUMENT"
    if torch.cuda.is_available():
        return
    d = nat.NNDesc(64, 1000, 64, 0)
    h = ctypes.c_void_p()
    assert nat.STATUS_NAMES[lib.fbnn_plan(ctypes.byref(d), 0, ctypes.byref(h))] == "FBCORR_ERR_NO_DEVICE"
    assert not h.value


def test_gpu_test_configurations_are_valid():
    from test_gpu_nn import NN_CFGS
    from paper_0911_3456_amd import nn_compile_check
    for cfg in NN_CFGS:
        assert nn_compile_check(300, 5000, 64, cfg) > 0
        assert nn_compile_check(37, 777, 48, cfg) > 0
