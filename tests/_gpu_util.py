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


def sample_sites(rng, shape, count):
    """Random output sites (b, i, j) of a valid correlation."""
    b = rng.integers(0, shape.batch, count)
    i = rng.integers(0, shape.Ho, count)
    j = rng.integers(0, shape.Wo, count)
    # always include the four corners of the first image (ragged tile tails)
    b = np.concatenate([[0, 0, 0, 0], b])
    i = np.concatenate([[0, 0, shape.Ho - 1, shape.Ho - 1], i])
    j = np.concatenate([[0, shape.Wo - 1, 0, shape.Wo - 1], j])
    return np.stack([b, i, j], axis=1)


def sampled_forward_error(y_gpu, x, w, sites):
    """Oracle on one input patch per site; normalised error over all filters."""
    fh, fw = w.shape[1], w.shape[2]
    got, ref, scl = [], [], []
    for b, i, j in sites:
        patch = x[b, i:i + fh, j:j + fw, :]
        ref.append(oracle.forward(patch, w)[0, 0])
        scl.append(oracle.forward_scale(patch, w)[0, 0])
        got.append(y_gpu[b, i, j])
    return oracle.normalised_error(np.array(got), np.array(ref), np.array(scl))
