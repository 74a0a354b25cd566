"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test fixes part of the oracle by something independent of its loops:
a hand-worked example, exhaustive integer enumeration, library routines on
special cases (scipy's 2-D correlation, numpy products, FFT), closed forms,
invariants (delta filters, linearity, shift equivariance, the adjoint
identity) and finite differences.  A dropped term, a wrong sign or index, or
a transposed operand in the oracle fails at least one of them.
"""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.signal

import oracle
import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand(rng, *shape):
    return rng.uniform(-1, 1, size=shape)


# ---------------------------------------------------------------- worked example

def test_hand_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "hand_example.json")))
    x = np.array(g["x_hwd"], np.float64)
    w = np.array(g["w_nuvd"], np.float64)
    y = oracle.forward(x, w)
    np.testing.assert_array_equal(y, np.array(g["y_ijn"], np.float64))


# ------------------------------------------------------------ brute enumeration

def _brute_forward(x, w):
    """Exact Python-integer enumeration of every (i, j, n, u, v, d) term."""
    B, H, W, D = x.shape
    N, fh, fw, _ = w.shape
    Ho, Wo = H - fh + 1, W - fw + 1
    y = [[[[0] * N for _ in range(Wo)] for _ in range(Ho)] for _ in range(B)]
    for b, i, j, n, u, v, d in itertools.product(range(B), range(Ho), range(Wo), range(N),
                                                  range(fh), range(fw), range(D)):
        y[b][i][j][n] += int(x[b, i + u, j + v, d]) * int(w[n, u, v, d])
    return np.array(y, dtype=np.float64).reshape(B, Ho, Wo, N)


def test_brute_force_all_tiny_shapes():
    rng = np.random.default_rng(123)
    count = 0
    for H, W in itertools.product(range(1, 6), range(1, 6)):
        for fh, fw in itertools.product(range(1, H + 1), range(1, W + 1)):
            for D, N, B in itertools.product((1, 2, 3), (1, 3), (1, 2)):
                x = rng.integers(-3, 4, size=(B, H, W, D)).astype(np.float64)
                w = rng.integers(-3, 4, size=(N, fh, fw, D)).astype(np.float64)
                np.testing.assert_array_equal(oracle.forward(x, w), _brute_forward(x, w))
                count += 1
    assert count == 225 * 12


def test_backward_equals_exact_forward_differences():
    """L = sum(g*y) is linear in x and in w, so on integer data the change of
    L under a unit step of one coordinate IS the gradient, exactly."""
    rng = np.random.default_rng(7)
    for (B, H, W, D, N, fh, fw) in [(1, 4, 5, 2, 3, 2, 3), (2, 5, 4, 3, 2, 3, 1),
                                    (1, 3, 3, 1, 1, 3, 3), (2, 4, 4, 2, 2, 1, 2)]:
        x = rng.integers(-3, 4, size=(B, H, W, D)).astype(np.float64)
        w = rng.integers(-3, 4, size=(N, fh, fw, D)).astype(np.float64)
        g = rng.integers(-3, 4, size=(B, H - fh + 1, W - fw + 1, N)).astype(np.float64)
        L0 = float(np.sum(g * oracle.forward(x, w)))
        dx, dw = oracle.backward(x, w, g)
        for idx in itertools.product(*map(range, x.shape)):
            xp = x.copy()
            xp[idx] += 1
            assert float(np.sum(g * oracle.forward(xp, w))) - L0 == dx[idx]
        for idx in itertools.product(*map(range, w.shape)):
            wp = w.copy()
            wp[idx] += 1
            assert float(np.sum(g * oracle.forward(x, wp))) - L0 == dw[idx]


# ------------------------------------------------------------ library special cases

def test_single_channel_is_scipy_correlate2d():
    rng = np.random.default_rng(1)
    x = _rand(rng, 17, 23)
    f = _rand(rng, 4, 6)
    y = oracle.forward(x[:, :, None], f[None, :, :, None])[:, :, 0]
    ref = scipy.signal.correlate2d(x, f, mode="valid")
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-13)


def test_multichannel_is_sum_of_correlate2d():
    rng = np.random.default_rng(2)
    x = _rand(rng, 2, 12, 15, 3)
    w = _rand(rng, 4, 3, 5, 3)
    y = oracle.forward(x, w)
    for b in range(2):
        for n in range(4):
            ref = sum(scipy.signal.correlate2d(x[b, :, :, d], w[n, :, :, d], mode="valid")
                      for d in range(3))
            np.testing.assert_allclose(y[b, :, :, n], ref, rtol=0, atol=1e-13)


def test_one_by_one_filters_are_a_matrix_product():
    rng = np.random.default_rng(3)
    x = _rand(rng, 9, 7, 5)
    w = _rand(rng, 6, 1, 1, 5)
    y = oracle.forward(x, w)
    ref = (x.reshape(-1, 5) @ w.reshape(6, 5).T).reshape(9, 7, 6)
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-14)


def test_full_size_filter_is_a_dot_product():
    rng = np.random.default_rng(4)
    x = _rand(rng, 6, 5, 3)
    w = _rand(rng, 2, 6, 5, 3)
    y = oracle.forward(x, w)
    assert y.shape == (1, 1, 2)
    for n in range(2):
        assert abs(y[0, 0, n] - np.dot(x.ravel(), w[n].ravel())) < 1e-14


def test_fft_convolution_with_flipped_filter():
    rng = np.random.default_rng(5)
    x = _rand(rng, 40, 33, 2)
    w = _rand(rng, 3, 7, 4, 2)
    y = oracle.forward(x, w)
    for n in range(3):
        ref = sum(scipy.signal.fftconvolve(x[:, :, d], w[n, ::-1, ::-1, d], mode="valid")
                  for d in range(2))
        np.testing.assert_allclose(y[:, :, n], ref, rtol=0, atol=1e-12)


def test_backward_special_cases_scipy():
    rng = np.random.default_rng(6)
    B, H, W, D, N, fh, fw = 2, 11, 9, 3, 4, 4, 3
    x = _rand(rng, B, H, W, D)
    w = _rand(rng, N, fh, fw, D)
    g = _rand(rng, B, H - fh + 1, W - fw + 1, N)
    dx, dw = oracle.backward(x, w, g)
    for b in range(B):
        for d in range(D):
            ref = sum(scipy.signal.convolve2d(g[b, :, :, n], w[n, :, :, d], mode="full")
                      for n in range(N))
            np.testing.assert_allclose(dx[b, :, :, d], ref, rtol=0, atol=1e-12)
    for n in range(N):
        for d in range(D):
            ref = sum(scipy.signal.correlate2d(x[b, :, :, d], g[b, :, :, n], mode="valid")
                      for b in range(B))
            np.testing.assert_allclose(dw[n, :, :, d], ref, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- invariants

def test_delta_filter_selects_shifted_input():
    rng = np.random.default_rng(8)
    x = _rand(rng, 2, 13, 10, 4)
    fh, fw = 5, 3
    taps = [(0, 0, 0), (4, 2, 3), (2, 1, 1), (1, 2, 2)]
    w = np.zeros((len(taps), fh, fw, 4))
    for n, (u, v, d) in enumerate(taps):
        w[n, u, v, d] = 1.0
    y = oracle.forward(x, w)
    Ho, Wo = 13 - fh + 1, 10 - fw + 1
    for n, (u, v, d) in enumerate(taps):
        np.testing.assert_array_equal(y[..., n], x[:, u:u + Ho, v:v + Wo, d])


def test_linearity_in_input_and_filters():
    rng = np.random.default_rng(9)
    x1, x2 = _rand(rng, 1, 20, 18, 3), _rand(rng, 1, 20, 18, 3)
    w1, w2 = _rand(rng, 5, 4, 4, 3), _rand(rng, 5, 4, 4, 3)
    a, b = 0.75, -1.5
    scale = oracle.forward_scale(np.abs(a * x1) + np.abs(b * x2), np.abs(w1) + np.abs(w2))
    lhs = oracle.forward(a * x1 + b * x2, w1)
    rhs = a * oracle.forward(x1, w1) + b * oracle.forward(x2, w1)
    assert np.max(np.abs(lhs - rhs) / scale) < 1e-13
    lhs = oracle.forward(x1, a * w1 + b * w2)
    rhs = a * oracle.forward(x1, w1) + b * oracle.forward(x1, w2)
    assert np.max(np.abs(lhs - rhs) / scale) < 1e-13


def test_constant_input_gives_filter_sum():
    s = wl.Shape(1, 16, 16, 4, 6, 5, 5)
    _, w, _ = wl.draw_single(s, seed=11)
    w = w.astype(np.float64)
    c = 0.625
    y = oracle.forward(np.full((16, 16, 4), c), w)
    closed = c * w.reshape(6, -1).sum(axis=1)
    atol = 1e-15 * c * np.abs(w).reshape(6, -1).sum(axis=1)
    assert np.all(np.abs(y - closed) <= atol + 1e-300)
    assert np.all(np.abs(closed) < 1e-6)   # normalised filters have zero mean


def test_self_match_gives_squared_norm():
    s = wl.Shape(1, 20, 20, 3, 4, 6, 5)
    x, w, _ = wl.draw_single(s, seed=12)
    x = x[0].astype(np.float64)
    w = w.astype(np.float64)
    i0, j0 = 7, 9
    for n in range(4):
        xx = x.copy()
        xx[i0:i0 + 6, j0:j0 + 5, :] = w[n]
        y = oracle.forward(xx, w)
        assert abs(y[i0, j0, n] - np.sum(w[n] * w[n])) < 1e-14
        assert abs(y[i0, j0, n] - 1.0) < 1e-6    # unit norm up to the float32 cast


def test_shift_equivariance():
    rng = np.random.default_rng(13)
    x = _rand(rng, 30, 28, 2)
    w = _rand(rng, 3, 5, 4, 2)
    a, b = 3, 5
    y = oracle.forward(x, w)
    ys = oracle.forward(x[a:, b:], w)
    np.testing.assert_array_equal(ys, y[a:, b:])


def test_adjoint_identity():
    rng = np.random.default_rng(14)
    B, H, W, D, N, fh, fw = 3, 15, 12, 4, 5, 3, 4
    x = _rand(rng, B, H, W, D)
    w = _rand(rng, N, fh, fw, D)
    g = _rand(rng, B, H - fh + 1, W - fw + 1, N)
    y = oracle.forward(x, w)
    dx, dw = oracle.backward(x, w, g)
    lhs = float(np.sum(g * y))
    mag = float(np.sum(np.abs(g) * oracle.forward_scale(x, w)))
    assert abs(lhs - float(np.sum(dx * x))) < 1e-13 * mag
    assert abs(lhs - float(np.sum(dw * w))) < 1e-13 * mag


def test_delta_gradient_cases():
    rng = np.random.default_rng(15)
    B, H, W, D, N, fh, fw = 1, 9, 8, 3, 4, 3, 2
    x = _rand(rng, B, H, W, D)
    w = _rand(rng, N, fh, fw, D)
    Ho, Wo = H - fh + 1, W - fw + 1
    i0, j0, n0 = 4, 5, 2
    g = np.zeros((B, Ho, Wo, N))
    g[0, i0, j0, n0] = 1.0
    dx, dw = oracle.backward(x, w, g)
    expect_dw = np.zeros_like(w)
    expect_dw[n0] = x[0, i0:i0 + fh, j0:j0 + fw, :]
    np.testing.assert_array_equal(dw, expect_dw)
    expect_dx = np.zeros_like(x)
    expect_dx[0, i0:i0 + fh, j0:j0 + fw, :] = w[n0]
    np.testing.assert_array_equal(dx, expect_dx)
    # a delta filter makes dx the gradient shifted into place
    wd = np.zeros((1, fh, fw, D))
    wd[0, 2, 1, 0] = 1.0
    gg = _rand(rng, B, Ho, Wo, 1)
    dx, _ = oracle.backward(x, wd, gg, want_dw=False)
    expect = np.zeros_like(x)
    expect[0, 2:2 + Ho, 1:1 + Wo, 0] = gg[0, :, :, 0]
    np.testing.assert_array_equal(dx, expect)


def test_finite_differences_match_backward():
    s = wl.Shape(2, 14, 12, 3, 4, 5, 3)
    x, w, rng = wl.draw_single(s, seed=16)
    g = wl.draw_grad(s, rng)
    cx, cw = wl.fd_coordinates(s, rng, nx=30, nw=30)
    dx, dw = oracle.backward(x, w, g)
    fdx = oracle.fd_grad_x(x, w, g, cx)
    fdw = oracle.fd_grad_w(x, w, g, cw)
    ex = np.array([dx[tuple(c)] for c in cx])
    ew = np.array([dw[tuple(c)] for c in cw])
    sx, sw = oracle.backward_scales(x, w, g)
    assert np.max(np.abs(fdx - ex) / np.array([sx[tuple(c)] for c in cx])) < 1e-7
    assert np.max(np.abs(fdw - ew) / np.array([sw[tuple(c)] for c in cw])) < 1e-7


# ---------------------------------------------------------------- helpers

def test_normalised_error_conventions():
    e, m, idx = oracle.normalised_error([1.0, 2.0, 0.0], [1.0, 2.5, 0.0], [1.0, 5.0, 0.0])
    assert e == pytest.approx(0.1) and idx == (1,)
    e, _, _ = oracle.normalised_error([1e-30], [0.0], [0.0])
    assert e == np.inf
    e, _, _ = oracle.normalised_error([0.0], [0.0], [0.0])
    assert e == 0.0


def test_bf16_rounding_ties_to_even():
    one = 1.0
    cases = {
        one: one,
        one + 2.0 ** -8: one,                          # halfway, even stays
        one + 3 * 2.0 ** -8: one + 2.0 ** -6,          # halfway, rounds up to even
        one + 2.0 ** -8 + 2.0 ** -20: one + 2.0 ** -7,  # above halfway
        -(one + 3 * 2.0 ** -8): -(one + 2.0 ** -6),
    }
    src = np.array(list(cases), np.float32)
    np.testing.assert_array_equal(oracle.round_to_bf16(src), np.array(list(cases.values()), np.float32))


def test_bf16_and_fp16_rounding_match_torch_cpu():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(17)
    a = (rng.standard_normal(100000) * np.exp2(rng.integers(-20, 20, 100000))).astype(np.float32)
    tb = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    th = torch.from_numpy(a).to(torch.float16).to(torch.float32).numpy()
    np.testing.assert_array_equal(oracle.round_to_bf16(a), tb)
    np.testing.assert_array_equal(oracle.round_to_fp16(a), th)


def test_filter_pow2_scales():
    rng = np.random.default_rng(18)
    w = _rand(rng, 7, 3, 3, 2) * np.exp2(rng.integers(-10, 10, 7))[:, None, None, None]
    w[3] = 0.0
    s = oracle.filter_pow2_scales(w)
    m = np.abs(w.reshape(7, -1)).max(axis=1)
    for n in range(7):
        assert np.log2(s[n]) == np.round(np.log2(s[n]))
        if n == 3:
            assert s[n] == 1.0
        else:
            assert 1.0 <= m[n] * s[n] < 2.0


def test_workload_generators():
    wk = wl.WORKLOADS["fp32"]
    x, w, _ = wl.draw_single(wk.shape, wk.seed)
    assert x.shape == (1, 256, 256, 8) and x.dtype == np.float32
    assert w.shape == (64, 9, 9, 8)
    flat = w.reshape(64, -1).astype(np.float64)
    assert np.all(np.abs(flat.mean(axis=1)) < 1e-8)
    assert np.all(np.abs(np.sqrt((flat ** 2).sum(axis=1)) - 1) < 1e-6)
    x2, w2, _ = wl.draw_single(wk.shape, wk.seed)
    np.testing.assert_array_equal(x, x2)
    shapes, _ = wl.draw_batched_list()
    assert len(shapes) == 256
    assert all(s.H in wl.BATCH_SIDES and s.D in wl.BATCH_DEPTHS and s.N in wl.BATCH_BANKS
               and s.fh in wl.BATCH_FSIZES for s in shapes)
    assert wl.WORKLOADS["fp32"].shape.flops == 2 * 248 * 248 * 64 * 9 * 9 * 8


def test_stored_precision_sites_are_the_oracles():
    """tests/golden/precision_sites.npz (read by the benchmark to state the
    16-bit error against FP64) holds exactly what the oracle computes at its
    sites: recomputed here for a few sites, bit for bit."""
    import importlib.util
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_precision_sites",
                                                  os.path.join(here, "make_precision_sites.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    data = np.load(os.path.join(here, "precision_sites.npz"))
    wk = wl.WORKLOADS["precision"]
    st = mk.sites(wk.shape)
    np.testing.assert_array_equal(data["sites"], st)
    x, w, _ = wl.draw_single(wk.shape, wk.seed)
    pick = [0, 3, 4, len(st) - 1]
    y, a = mk.compute(x, w, st[pick])
    np.testing.assert_array_equal(data["y"][pick], y)
    np.testing.assert_array_equal(data["a"][pick], a)
