"""Helpers shared by the GPU tests (marshalling and comparisons only)."""
import numpy as np
import pytest
import torch

import oracle


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev():
    return torch.device("cuda", 0)


def to_dev(*arrs):
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).to(dev()) for a in arrs)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def forward_error(y_gpu, x, w, y_ref=None):
    y_ref = oracle.forward(x, w) if y_ref is None else y_ref
    return oracle.normalised_error(y_gpu, y_ref, oracle.forward_scale(x, w))
