"""Seeded synthetic inputs for the filter-bank correlation workloads.

This module only draws numbers.  It holds none of the correlation's
arithmetic, so both the CPU oracle (under ``oracle/``) and the GPU library
can be fed from it without sharing any of the method's code.

Workloads follow the shapes of the 3-D filter-bank convolution experiment of
the "Computational Visual Neuroscience" application (Sec. 6.2 and the table
"Performance of RTCG auto-tuning on 3D filter-bank convolutions"): an input
image H x W x D and a bank of N filters fh x fw x D that span the full depth.
The paper names no dataset for this experiment, so uniform values stand in
for images and filters.

Conventions (fixed here, used by tests and the benchmark):

* ``numpy.random.default_rng(seed)``; draw order is X, then F, then the
  upstream gradient G, then finite-difference coordinates.
* X and F are ``uniform(-1, 1)`` in float64, then cast to float32.
* "Normalised" filters: per filter, over all fh*fw*D taps, in float64,
  subtract the mean and divide by the L2 norm, then cast to float32
  (round-to-nearest-even).
* G is ``standard_normal`` in float32.
* Layouts are C-contiguous: X[b][H][W][D], F[N][fh][fw][D],
  Y/G[b][Ho][Wo][N].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Shape", "WORKLOADS", "normalise_filters", "draw_single", "draw_grad",
    "draw_integer", "draw_batched_list", "draw_batched", "fd_coordinates",
]


@dataclass(frozen=True)
class Shape:
    batch: int
    H: int
    W: int
    D: int
    N: int
    fh: int
    fw: int

    @property
    def Ho(self) -> int:
        return self.H - self.fh + 1

    @property
    def Wo(self) -> int:
        return self.W - self.fw + 1

    @property
    def macs(self) -> int:
        """Multiply-adds of one valid forward pass."""
        return self.batch * self.Ho * self.Wo * self.N * self.fh * self.fw * self.D

    @property
    def flops(self) -> int:
        """Two flops per multiply-add over the valid output."""
        return 2 * self.macs


@dataclass(frozen=True)
class Workload:
    name: str
    seed: int
    shape: Shape | None
    normalised: bool
    note: str = field(default="")


# The five workloads.  Seeds are the 1-based workload index.
WORKLOADS = {
    "tiny": Workload("tiny", 1, Shape(1, 64, 64, 4, 16, 5, 5), True,
                     "64x64x4 input, 16 filters 5x5x4"),
    "fp32": Workload("fp32", 2, Shape(1, 256, 256, 8, 64, 9, 9), True,
                     "256x256x8 input, 64 filters 9x9x8 (the table's first shape)"),
    "precision": Workload("precision", 3, Shape(1, 512, 512, 16, 128, 13, 13), True,
                          "512x512x16 input, 128 filters 13x13x16"),
    "batching": Workload("batching", 4, None, False,
                         "256 square images, S in {96..512 step 32}, D in {4,8,16,32}, "
                         "N in {16,32,64,128}, f in {3,5,7,9,11}; own bank per image"),
    "differentiation": Workload("differentiation", 5, Shape(32, 128, 128, 16, 64, 7, 7), True,
                                "32 inputs 128x128x16, 64 filters 7x7x16, G ~ N(0,1)"),
}


def normalise_filters(f64: np.ndarray) -> np.ndarray:
    """Per filter: zero mean and unit L2 norm over all taps, in float64."""
    n = f64.shape[0]
    flat = f64.reshape(n, -1)
    flat = flat - flat.mean(axis=1, keepdims=True)
    norms = np.sqrt((flat * flat).sum(axis=1, keepdims=True))
    norms[norms == 0] = 1.0
    return (flat / norms).reshape(f64.shape)


def draw_single(shape: Shape, seed: int, normalised: bool = True,
                rng: np.random.Generator | None = None):
    """Draw X[b][H][W][D] and F[N][fh][fw][D] as float32 arrays."""
    rng = np.random.default_rng(seed) if rng is None else rng
    x = rng.uniform(-1.0, 1.0, size=(shape.batch, shape.H, shape.W, shape.D))
    f = rng.uniform(-1.0, 1.0, size=(shape.N, shape.fh, shape.fw, shape.D))
    if normalised:
        f = normalise_filters(f)
    return x.astype(np.float32), f.astype(np.float32), rng


def draw_grad(shape: Shape, rng: np.random.Generator) -> np.ndarray:
    """Upstream gradient G[b][Ho][Wo][N], standard normal, float32."""
    return rng.standard_normal(size=(shape.batch, shape.Ho, shape.Wo, shape.N),
                               dtype=np.float32)


def draw_integer(shape: Shape, seed: int, xmax: int = 8, wmax: int = 8):
    """Integer-valued float32 inputs, |x| <= xmax and |w| <= wmax.

    While every partial sum stays below 2**24 in magnitude, float32
    accumulation is exact in any order, so results must match bit for bit.
    """
    rng = np.random.default_rng(seed)
    x = rng.integers(-xmax, xmax + 1, size=(shape.batch, shape.H, shape.W, shape.D))
    f = rng.integers(-wmax, wmax + 1, size=(shape.N, shape.fh, shape.fw, shape.D))
    return x.astype(np.float32), f.astype(np.float32), rng


BATCH_SIDES = tuple(range(96, 513, 32))
BATCH_DEPTHS = (4, 8, 16, 32)
BATCH_BANKS = (16, 32, 64, 128)
BATCH_FSIZES = (3, 5, 7, 9, 11)


def draw_batched_list(count: int = 256, seed: int = 4,
                      sides=BATCH_SIDES, depths=BATCH_DEPTHS,
                      banks=BATCH_BANKS, fsizes=BATCH_FSIZES):
    """Per image, draw (S, D, N, f) in that order; return the list of Shapes.

    Only the shape list is drawn here (cheap); ``draw_batched`` draws the data
    with the same generator state.
    """
    rng = np.random.default_rng(seed)
    shapes = []
    for _ in range(count):
        s = int(rng.choice(sides))
        d = int(rng.choice(depths))
        n = int(rng.choice(banks))
        f = int(rng.choice(fsizes))
        shapes.append(Shape(1, s, s, d, n, f, f))
    return shapes, rng


def draw_batched(count: int = 256, seed: int = 4, **kw):
    """Shapes, then per image X_b and F_b (plain uniform, not normalised)."""
    shapes, rng = draw_batched_list(count, seed, **kw)
    xs, fs = [], []
    for s in shapes:
        x, f, rng = draw_single(s, seed, normalised=False, rng=rng)
        xs.append(x[0])
        fs.append(f)
    return shapes, xs, fs


def fd_coordinates(shape: Shape, rng: np.random.Generator, nx: int = 100, nw: int = 100):
    """Coordinates for finite-difference checks: nx in X, nw in F."""
    cx = np.stack([rng.integers(0, shape.batch, nx), rng.integers(0, shape.H, nx),
                   rng.integers(0, shape.W, nx), rng.integers(0, shape.D, nx)], axis=1)
    cw = np.stack([rng.integers(0, shape.N, nw), rng.integers(0, shape.fh, nw),
                   rng.integers(0, shape.fw, nw), rng.integers(0, shape.D, nw)], axis=1)
    return cx, cw


# --------------------------------------------------------------------------
# Nearest-neighbour search over image patches (Sec. 6.4 and its table of
# search times: 4096 target patches of 8 x 8 pixels, neighbour sets of 4096
# to 1,048,576 patches).  The natural-image database that application used
# is not available here, so synthetic images with the best-known statistic of
# natural scenes stand in: an amplitude spectrum falling as 1/f (power 1/f^2)
# with random phases, scaled to mean 128 and standard deviation 48, clipped
# to [0, 255] and rounded to 8-bit pixels.  Patches are cut at distinct
# random positions (without replacement inside an image); targets come from
# images of their own, disjoint from the neighbours' images.
# --------------------------------------------------------------------------

NN_TARGETS = 4096
NN_NEIGHBOURS = (4096, 16384, 65536, 262144, 1048576)
NN_PATCH = 8
NN_IMAGE_SIDE = 512
NN_PER_IMAGE = 16384


def draw_images(count: int, rng: np.random.Generator, side: int = NN_IMAGE_SIDE) -> np.ndarray:
    """count images side x side of 8-bit pixels with a 1/f amplitude spectrum."""
    fy = np.fft.fftfreq(side)[:, None]
    fx = np.fft.rfftfreq(side)[None, :]
    f = np.sqrt(fx * fx + fy * fy)
    f[0, 0] = 1.0
    out = np.empty((count, side, side), np.uint8)
    for k in range(count):
        spec = np.fft.rfft2(rng.standard_normal((side, side))) / f
        spec[0, 0] = 0.0
        img = np.fft.irfft2(spec, s=(side, side))
        img = 128.0 + 48.0 * (img - img.mean()) / img.std()
        out[k] = np.clip(np.rint(img), 0, 255).astype(np.uint8)
    return out


def draw_patches(count: int, seed: int, patch: int = NN_PATCH, per_image: int = NN_PER_IMAGE,
                 side: int = NN_IMAGE_SIDE) -> np.ndarray:
    """count patches [count, patch*patch] (uint8, row-major pixels) cut from
    ceil(count / per_image) synthetic images at distinct positions."""
    rng = np.random.default_rng(seed)
    out = np.empty((count, patch * patch), np.uint8)
    npos = side - patch + 1
    done = 0
    while done < count:
        img = draw_images(1, rng, side)[0]
        take = min(per_image, count - done)
        pos = rng.choice(npos * npos, size=take, replace=False)
        ii, jj = pos // npos, pos % npos
        win = np.lib.stride_tricks.sliding_window_view(img, (patch, patch))
        out[done:done + take] = win[ii, jj].reshape(take, patch * patch)
        done += take
    return out


def draw_nn(n_targets: int, n_neighbours: int, seed: int = 7, patch: int = NN_PATCH):
    """Targets and neighbours for one search (separate image draws)."""
    targets = draw_patches(n_targets, seed * 1000 + 1, patch)
    neighbours = draw_patches(n_neighbours, seed * 1000 + 2, patch)
    return targets, neighbours
