"""Write the FP64 oracle's outputs at sampled sites of the precision workload.

The benchmark reports the normalised error of every precision's forward
(fp32 direct, fp32 / bf16 / fp16 matrix cores) against the FP64 oracle; it
may not run the oracle itself, so it reads the oracle's values from the file
this script writes.  Only ``oracle/`` computes them (and ``workloads`` draws
the input, seed 3: 512x512x16 input, 128 normalised filters 13x13x16).

Sites: the four corners of the output plus 128 random (i, j) from
``default_rng(2023)``; at each site all 128 filters.  Stored: sites [K, 2]
(int32), y [K, 128] = the oracle's outputs, a [K, 128] = the error
normaliser sum |x| |w| over each output's terms (both float64).

Run from the repository root:  python tests/golden/make_precision_sites.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as wl  # noqa: E402

OUT = os.path.join(HERE, "precision_sites.npz")
N_RANDOM = 128


def sites(shape):
    rng = np.random.default_rng(2023)
    corners = [(0, 0), (0, shape.Wo - 1), (shape.Ho - 1, 0), (shape.Ho - 1, shape.Wo - 1)]
    rand = np.stack([rng.integers(0, shape.Ho, N_RANDOM), rng.integers(0, shape.Wo, N_RANDOM)], axis=1)
    return np.concatenate([np.array(corners), rand]).astype(np.int32)


def compute(x, w, st):
    fh, fw = w.shape[1], w.shape[2]
    y, a = [], []
    for i, j in st:
        patch = x[0, i:i + fh, j:j + fw, :]
        y.append(oracle.forward(patch, w)[0, 0])
        a.append(oracle.forward_scale(patch, w)[0, 0])
    return np.array(y), np.array(a)


def main():
    wk = wl.WORKLOADS["precision"]
    x, w, _ = wl.draw_single(wk.shape, wk.seed)
    st = sites(wk.shape)
    y, a = compute(x, w, st)
    np.savez(OUT, sites=st, y=y, a=a)
    print("wrote %s: %d sites x %d filters" % (OUT, len(st), y.shape[1]))


if __name__ == "__main__":
    main()
