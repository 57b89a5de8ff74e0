"""Pins of the oracle's prediction functions (Sec. 2, Sec. 2.2) and SMAPE
(Sec. 4.1) against what the KRR equations and the definitions fix."""
import math

import numpy as np

from oracle import direct
from oracle import kernels as OK
from oracle import predict as OP


def test_single_expansion_point_closed_form():
    # one training point: f(x) = beta K(x1, x), written out with math.exp
    x1 = np.array([[0.3, -1.2, 2.0]])
    xt = np.array([[1.0, 0.5, -0.5], [0.3, -1.2, 2.0]])
    b = np.array([2.5])
    s = 1.7
    g = OP.predict_full(x1, b, xt, OK.GAUSSIAN, s)
    l = OP.predict_full(x1, b, xt, OK.LAPLACE, s)
    d2 = (1.0 - 0.3) ** 2 + (0.5 + 1.2) ** 2 + (-0.5 - 2.0) ** 2
    d1 = abs(1.0 - 0.3) + abs(0.5 + 1.2) + abs(-0.5 - 2.0)
    assert math.isclose(g[0], 2.5 * math.exp(-d2 / (2 * s * s)), rel_tol=1e-14)
    assert math.isclose(l[0], 2.5 * math.exp(-d1 / s), rel_tol=1e-14)
    assert g[1] == 2.5 and l[1] == 2.5  # K(x, x) = 1


def test_full_data_fit_satisfies_the_normal_equations():
    # (A + mu I) beta = y  =>  f(X) = A beta = y - mu beta (Sec. 2, eq. exact_eqn)
    g = np.random.default_rng(1)
    X = g.standard_normal((300, 4))
    y = np.sin(X.sum(axis=1))
    for kind, sigma, mu in ((OK.GAUSSIAN, 2.0, 1e-2), (OK.LAPLACE, 4.0, 0.3)):
        beta = direct.full_krr(X, y, kind, sigma, mu)
        f = OP.predict_full(X, beta, X, kind, sigma)
        np.testing.assert_allclose(f, y - mu * beta, rtol=0, atol=1e-9 * np.abs(y).max())


def test_restricted_fit_satisfies_the_normal_equations():
    # restricted KRR (Sec. 2.2): (A(S,:)A(:,S) + mu A(S,S)) beta = A(S,:) y, so
    # A(S,:) (f(X) - y) = -mu A(S,S) beta with f(X) = A(:,S) beta
    g = np.random.default_rng(2)
    X = g.standard_normal((400, 3))
    y = np.cos(2 * X[:, 0]) + X[:, 1]
    S = np.sort(g.choice(400, 25, replace=False))
    kind, sigma, mu = OK.GAUSSIAN, 1.5, 0.5
    ANS = OK.block(X, X[S], kind, sigma)
    ASS = OK.block(X[S], X[S], kind, sigma)
    beta = direct.restricted_krr(ANS.T @ ANS + mu * ASS, ANS.T @ y)
    f = OP.predict_restricted(X, S, beta, X, kind, sigma)
    lhs = ANS.T @ (f - y)
    np.testing.assert_allclose(lhs, -mu * ASS @ beta, rtol=0, atol=1e-8 * np.abs(ANS.T @ y).max())
    # and a test point predicted from the centres only
    xt = g.standard_normal((5, 3))
    f_t = OP.predict_restricted(X, S, beta, xt, kind, sigma)
    brute = [sum(beta[j] * OK.entry(X[S[j]], xt[i], kind, sigma) for j in range(len(S)))
             for i in range(5)]
    np.testing.assert_allclose(f_t, brute, rtol=1e-13)


def test_smape_definition_values():
    assert OP.smape([1.0, 3.0], [3.0, 1.0]) == 1.0      # |2| / 2 each
    assert OP.smape([2.0, -5.0], [2.0, -5.0]) == 0.0
    assert OP.smape([-1.0, 4.0], [1.0, -4.0]) == 2.0    # the maximum
    assert OP.smape([0.0, 1.0], [0.0, 3.0]) == 0.5      # 0/0 pair counts 0
    assert math.isclose(OP.smape([1.1], [1.0]), 0.1 / 1.05, rel_tol=1e-15)
