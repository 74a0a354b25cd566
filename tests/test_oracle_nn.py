"""Pins of the nearest-neighbour oracle (CPU only).

What the oracle computes (Sec. 6.4): for every target patch, the exact
nearest neighbour by squared Euclidean distance, lowest index on ties.  The
pins below do not re-run the oracle's own loop: a hand-worked example,
pure-Python enumeration, a k-d tree (a different exact algorithm), a sorted
search in one dimension, and invariants of the problem.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "nn_hand_example.json")


def test_hand_example():
    g = json.load(open(GOLDEN))
    idx, dist = oracle.nearest(np.array(g["targets"], np.uint8), np.array(g["neighbors"], np.uint8))
    assert idx.tolist() == g["expected_idx"]
    assert dist.tolist() == g["expected_dist"]


def _python_nearest(t, n):
    out_i, out_d = [], []
    for a in t.tolist():
        best, bi = None, None
        for m, b in enumerate(n.tolist()):
            s = sum((p - q) * (p - q) for p, q in zip(a, b))
            if best is None or s < best:
                best, bi = s, m
        out_i.append(bi)
        out_d.append(best)
    return out_i, out_d


@pytest.mark.parametrize("T,M,D,vmax", [(7, 13, 4, 256), (5, 40, 16, 4), (9, 33, 64, 256), (3, 1, 8, 256),
                                        (6, 50, 2, 3)])
def test_enumeration(T, M, D, vmax):
    rng = np.random.default_rng(T * 100 + M + D)
    t = rng.integers(0, vmax, (T, D), dtype=np.uint8)
    n = rng.integers(0, vmax, (M, D), dtype=np.uint8)
    idx, dist = oracle.nearest(t, n)
    ei, ed = _python_nearest(t, n)
    assert idx.tolist() == ei and dist.tolist() == ed


def test_kd_tree_distances():
    from scipy.spatial import cKDTree
    t, n = wl.draw_nn(300, 5000, seed=3)
    idx, dist = oracle.nearest(t, n)
    dd, ii = cKDTree(n.astype(np.float64)).query(t.astype(np.float64), k=1)
    np.testing.assert_array_equal(dist, np.rint(dd * dd).astype(np.int64))
    # the returned index attains the distance
    got = ((t.astype(np.int64) - n[idx].astype(np.int64)) ** 2).sum(1)
    np.testing.assert_array_equal(got, dist)
    # where the tree's answer is the only one at that distance, indices agree
    tree_d = ((t.astype(np.int64) - n[ii].astype(np.int64)) ** 2).sum(1)
    np.testing.assert_array_equal(tree_d, dist)


def test_one_dimension_sorted_search():
    rng = np.random.default_rng(11)
    n = rng.integers(0, 256, (400, 1), dtype=np.uint8)
    t = np.arange(256, dtype=np.uint8)[:, None]
    idx, dist = oracle.nearest(t, n)
    vals = np.unique(n[:, 0]).astype(np.int64)
    first = {int(v): int(np.flatnonzero(n[:, 0] == v)[0]) for v in vals}
    for v in range(256):
        k = np.searchsorted(vals, v)
        cands = [vals[j] for j in (k - 1, k) if 0 <= j < len(vals)]
        dmin = min((v - c) ** 2 for c in cands)
        best = min(first[int(c)] for c in cands if (v - c) ** 2 == dmin)
        assert (idx[v], dist[v]) == (best, dmin)


def test_self_match_and_duplicates():
    t, n = wl.draw_nn(64, 2000, seed=5)
    n = n.copy()
    n[1500] = n[100]            # duplicate: the lower index must win
    q = n[[100, 7, 1999, 0]]
    idx, dist = oracle.nearest(q, n)
    assert dist.tolist() == [0, 0, 0, 0]
    assert idx.tolist() == [100, 7, 1999, 0]


def test_permutation_and_translation():
    t, n = wl.draw_nn(200, 3000, seed=6)
    idx, dist = oracle.nearest(t, n)
    perm = np.random.default_rng(1).permutation(len(n))
    pidx, pdist = oracle.nearest(t, n[perm])
    np.testing.assert_array_equal(pdist, dist)
    # the permuted answer is the same row whenever the nearest row is unique
    d_all = ((t[:, None, :].astype(np.int64) - n[None].astype(np.int64)) ** 2).sum(-1)
    unique = (d_all == dist[:, None]).sum(1) == 1
    np.testing.assert_array_equal(perm[pidx][unique], idx[unique])
    # shifting every pixel of both sets by the same amount changes nothing
    lo = min(int(t.min()), int(n.min()))
    sidx, sdist = oracle.nearest((t.astype(np.int64) - lo).astype(np.uint8),
                                 (n.astype(np.int64) - lo).astype(np.uint8))
    np.testing.assert_array_equal(sdist, dist)
    np.testing.assert_array_equal(sidx, idx)


def test_planted_neighbour():
    rng = np.random.default_rng(21)
    n = rng.integers(0, 64, (1000, 64), dtype=np.uint8)
    t = rng.integers(192, 256, (10, 64), dtype=np.uint8)
    plant = rng.integers(0, 1000, 10)
    for k in range(10):
        n[plant[k]] = t[k]
        n[plant[k], k] = t[k, k] - 3       # distance 9 exactly
    idx, dist = oracle.nearest(t, n)
    assert idx.tolist() == plant.tolist()
    assert dist.tolist() == [9] * 10


def test_growing_neighbour_sets():
    # the application doubles the neighbour set; distances never grow, and an
    # unchanged distance keeps the earlier (lower-index) answer
    t, n = wl.draw_nn(128, 8192, seed=8)
    prev = None
    for m in (1024, 2048, 4096, 8192):
        idx, dist = oracle.nearest(t, n[:m])
        if prev is not None:
            assert (dist <= prev[1]).all()
            same = dist == prev[1]
            np.testing.assert_array_equal(idx[same], prev[0][same])
            assert (idx[~same] >= m // 2).all()
        prev = (idx, dist)


def test_empty_inputs():
    idx, dist = oracle.nearest(np.zeros((0, 64), np.uint8), np.zeros((5, 64), np.uint8))
    assert idx.shape == (0,)
    with pytest.raises(ValueError):
        oracle.nearest(np.zeros((3, 64), np.uint8), np.zeros((0, 64), np.uint8))


def test_patch_generator():
    a = wl.draw_patches(5000, seed=9)
    b = wl.draw_patches(5000, seed=9)
    np.testing.assert_array_equal(a, b)
    assert a.dtype == np.uint8 and a.shape == (5000, 64)
    assert abs(a.mean() - 128) < 4 and 40 < a.std() < 50
    # amplitude spectrum of the synthetic images falls roughly as 1/f
    img = wl.draw_images(1, np.random.default_rng(0), 256)[0].astype(np.float64)
    amp = np.abs(np.fft.fft2(img - img.mean()))
    f = np.hypot(*np.meshgrid(np.fft.fftfreq(256), np.fft.fftfreq(256)))
    lo = amp[(f > 0.02) & (f < 0.04)].mean()
    hi = amp[(f > 0.16) & (f < 0.32)].mean()
    ratio = lo / hi
    assert 4 < ratio < 16          # 1/f over an 8x frequency span: ~8
