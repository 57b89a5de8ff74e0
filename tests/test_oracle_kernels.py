"""Pins of the oracle's kernel entries and product (Sec. 2.1, Sec. 4.1)."""
import math

import numpy as np
import pytest

from oracle import kernels as K

KINDS = [K.GAUSSIAN, K.LAPLACE]


def brute(X, Y, kind, sigma):
    out = [[0.0] * len(Y) for _ in range(len(X))]
    for i, x in enumerate(X):
        for j, y in enumerate(Y):
            if kind == K.GAUSSIAN:
                s = sum((float(a) - float(b)) ** 2 for a, b in zip(x, y))
                out[i][j] = math.exp(-s / (2 * sigma * sigma))
            else:
                s = sum(abs(float(a) - float(b)) for a, b in zip(x, y))
                out[i][j] = math.exp(-s / sigma)
    return np.array(out)


@pytest.mark.parametrize("kind", KINDS)
def test_block_matches_brute_force(kind):
    g = np.random.default_rng(0)
    X = g.standard_normal((9, 5))
    Y = g.standard_normal((7, 5))
    np.testing.assert_allclose(K.block(X, Y, kind, 1.7), brute(X, Y, kind, 1.7), rtol=1e-14, atol=0)
    v = g.standard_normal(7)
    np.testing.assert_allclose(K.matvec(X, Y, v, kind, 1.7), brute(X, Y, kind, 1.7) @ v, rtol=1e-13)


@pytest.mark.parametrize("kind", KINDS)
def test_separable_product_form(kind):
    # Both kernels factor over coordinates: K(x,y) = prod_l k(x_l, y_l).
    g = np.random.default_rng(1)
    X = g.standard_normal((30, 4))
    Y = g.standard_normal((20, 4))
    s = 2.3
    P = np.ones((30, 20))
    for l in range(4):
        dl = X[:, l][:, None] - Y[:, l][None, :]
        P *= np.exp(-dl ** 2 / (2 * s * s)) if kind == K.GAUSSIAN else np.exp(-np.abs(dl) / s)
    np.testing.assert_allclose(K.block(X, Y, kind, s), P, rtol=1e-13)


@pytest.mark.parametrize("kind", KINDS)
def test_identical_points_all_ones(kind):
    X = np.tile(np.array([[0.3, -1.2, 2.0]]), (11, 1))
    v = np.arange(11.0)
    np.testing.assert_array_equal(K.matvec(X, X, v, kind, 1.0), np.full(11, v.sum()))


@pytest.mark.parametrize("kind", KINDS)
def test_two_far_clusters_rank_two_block(kind):
    # The rank-2 block matrix of the uniform-sampling failure example (Sec. 3.1).
    n1, n2 = 12, 3
    X = np.vstack([np.zeros((n1, 2)), np.full((n2, 2), 1e3)])
    A = K.block(X, X, kind, 1.0)
    E = np.zeros((n1 + n2, n1 + n2))
    E[:n1, :n1] = 1
    E[n1:, n1:] = 1
    np.testing.assert_array_equal(A, E)
    assert np.linalg.matrix_rank(A) == 2


def test_laplace_1d_grid_is_kms_matrix():
    # 1-D equispaced grid, spacing h: A_ij = rho^|i-j|, rho = exp(-h/sigma),
    # whose inverse is tridiagonal in closed form.
    n, h, s = 40, 0.25, 0.8
    X = (np.arange(n) * h)[:, None]
    A = K.block(X, X, K.LAPLACE, s)
    rho = math.exp(-h / s)
    Ainv = np.zeros((n, n))
    for i in range(n):
        Ainv[i, i] = 1 + rho * rho if 0 < i < n - 1 else 1.0
        if i + 1 < n:
            Ainv[i, i + 1] = Ainv[i + 1, i] = -rho
    Ainv /= 1 - rho * rho
    np.testing.assert_allclose(A @ Ainv, np.eye(n), atol=1e-12)
    y = np.sin(np.arange(n))
    np.testing.assert_allclose(A @ (Ainv @ y), y, atol=1e-12)


@pytest.mark.parametrize("kind", KINDS)
def test_symmetry_of_product(kind):
    g = np.random.default_rng(2)
    X = g.standard_normal((50, 6))
    u, v = g.standard_normal(50), g.standard_normal(50)
    a = u @ K.matvec(X, X, v, kind, 2.0)
    b = v @ K.matvec(X, X, u, kind, 2.0)
    assert abs(a - b) <= 1e-12 * (abs(a) + 1)


@pytest.mark.parametrize("kind", KINDS)
def test_bandwidth_limits(kind):
    # sigma -> 0 gives the identity, sigma -> infinity the all-ones matrix (Sec. 2.1.2).
    g = np.random.default_rng(3)
    X = g.standard_normal((15, 3))
    np.testing.assert_array_equal(K.block(X, X, kind, 1e-3), np.eye(15))
    np.testing.assert_allclose(K.block(X, X, kind, 1e9), np.ones((15, 15)), atol=1e-8)


def test_shifted_product_and_diag():
    g = np.random.default_rng(4)
    X = g.standard_normal((20, 3))
    v = g.standard_normal((20, 2))
    w = K.matvec(X, X, v, K.GAUSSIAN, 1.0, shift=0.5)
    np.testing.assert_allclose(w, brute(X, X, K.GAUSSIAN, 1.0) @ v + 0.5 * v, rtol=1e-13)
    np.testing.assert_array_equal(K.diag(X, K.LAPLACE, 1.0), np.ones(20))


def test_fast_expansion_mode_matches_direct_differences():
    """The oracle's BLAS-expansion timing mode against its exact mode: each
    exponent of the expansion carries at most about (d + 4) eps s
    (||x - c||^2 + ||y - c||^2) (rounding of the two norms, the d-term dot
    product and the sum; c = column mean), so entries agree to that relative
    amount; Laplace blocks are the direct form itself."""
    g = np.random.default_rng(77)
    eps = 2.0 ** -52
    for d, sigma, shift in ((3, 0.7, 0.0), (16, 4.0, 2.0), (32, 1.5, 0.5)):
        Xr = g.standard_normal((300, d)) + shift
        Xc = g.standard_normal((500, d)) + shift
        Ke = K.block(Xr, Xc, K.GAUSSIAN, sigma)
        Kf = K.block_fast(Xr, Xc, K.GAUSSIAN, sigma)
        c = Xc.mean(axis=0)
        nr = np.sum((Xr - c) ** 2, axis=1)[:, None]
        nc = np.sum((Xc - c) ** 2, axis=1)[None, :]
        bound = 2 * (d + 4) * eps * (nr + nc) / (2 * sigma ** 2) * np.maximum(Ke, Kf) + 1e-300
        assert np.all(np.abs(Kf - Ke) <= bound), np.max(np.abs(Kf - Ke) / bound)
        V = g.standard_normal((500, 2))
        np.testing.assert_allclose(K.matvec(Xr, Xc, V, K.GAUSSIAN, sigma, fast=True),
                                   K.matvec(Xr, Xc, V, K.GAUSSIAN, sigma),
                                   rtol=1e-12, atol=1e-13 * np.abs(Ke).sum(axis=1).max())
    Xr = g.standard_normal((50, 5))
    np.testing.assert_array_equal(K.block_fast(Xr, Xr, K.LAPLACE, 2.0),
                                  K.block(Xr, Xr, K.LAPLACE, 2.0))


def test_fast_mode_dropped_factor_is_caught():
    """A plausible mistake in the fast mode (sigma^2 instead of 2 sigma^2)
    trips the cross-check above."""
    import pytest
    orig = K.block_fast
    try:
        K.block_fast = lambda Xr, Xc, kind, sigma: orig(Xr, Xc, kind, sigma / np.sqrt(2.0))
        with pytest.raises(AssertionError):
            test_fast_expansion_mode_matches_direct_differences()
    finally:
        K.block_fast = orig
