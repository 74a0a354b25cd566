"""fbcorr — run-time-specialised multi-channel 2-D filter-bank correlation
for AMD MI355X (gfx950).

The hot path of the GPU run-time code generation method applied to the
"3D filter-bank convolution" of Sec. 6.2 (Computational Visual
Neuroscience): kernels are generated and compiled at plan time with hiprtc,
specialised on the problem and tile constants, cached, and auto-tuned.
The computation lives in ``libfbcorr.so`` (C ABI in ``include/fbcorr.h``);
this package only marshals torch tensors and streams into it.

The same library holds a second run-time generated workload, the exact
brute-force nearest-neighbour search of Sec. 6.4 (``include/fbnn.h``,
``NNPlan``).
"""
from . import _native
from ._native import (FbcorrError, codegen, compile_check, compile_check_batched, cache_stats, cache_clear, make_desc,
                      load, nn_compile_check)
from .nn import NNPlan, nearest
from .plan import BatchedPlan, FbCorrFunction, Plan, fbcorr, get_plan

__all__ = ["BatchedPlan", "FbcorrError", "FbCorrFunction", "Plan", "fbcorr", "get_plan", "codegen",
           "compile_check", "compile_check_batched", "cache_stats", "cache_clear", "make_desc", "load",
           "NNPlan", "nearest", "nn_compile_check"]
