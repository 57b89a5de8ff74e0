"""Pins of the oracle's blocked RPCholesky (Alg. 3) and Nystrom
preconditioner (Alg. 1; Sec. 5.1 bounds)."""
import math
import os

import numpy as np
import pytest
from scipy.stats import chisquare

from oracle import kernels as K
from oracle import rpcholesky as RP
from oracle import pcg as PCG
from oracle.rng import sm, key, u53, TAG_PIVOT
from synth import c1

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")


def golden(name):
    for l in open(GOLD):
        if l.strip() and not l.startswith("#"):
            k, v = l.split()
            if k == name:
                return float(v)
    raise KeyError(name)


def test_block_size_rule_matches_paper():
    assert RP.default_block(1000) == golden("block_size_at_r1000")
    assert RP.default_block(100) == 10 and RP.default_block(2000) == 100 and RP.default_block(5) == 1


def test_sampler_distribution_is_proportional_to_d():
    d = np.array([0.5, 0.0, 2.0, 1.0, 0.25])
    O = RP.prefix_tables(d)
    g = np.random.default_rng(5)
    n = 40000
    counts = np.zeros(5)
    for u in g.random(n):
        counts[RP.sample_index(d, O, float(u))] += 1
    assert counts[1] == 0
    nz = d > 0
    p = d[nz] / d.sum()
    assert chisquare(counts[nz], p * n).pvalue > 1e-3


def test_sampler_edges():
    d = np.zeros(3000)
    d[[5, 1500, 2999]] = [1.0, 2.0, 3.0]
    O = RP.prefix_tables(d)
    assert RP.sample_index(d, O, 0.0) == 5
    assert RP.sample_index(d, O, 1.0 - 2.0 ** -53) == 2999
    assert RP.sample_index(d, O, 1.0 / 6.0) == 1500  # t == c_5 exactly -> next index
    # prefix tables: chunk totals summed left to right
    assert O[-1] == 6.0 and O[1] == 1.0 and O[2] == 3.0


def test_first_block_is_uniform_closed_form():
    # diag(A) = 1 for both kernels, so c_i = i + 1 exactly and draw = floor(u N).
    N = 3000
    d = np.ones(N)
    draws = RP.draw_block(d, seed=77, b=0, count=50)
    kb = sm(key(77, TAG_PIVOT), 0)
    assert draws == [int(math.floor(u53(sm(kb, t)) * N)) for t in range(50)]


def test_chol_drop_matches_library_without_drops_and_drops_duplicates():
    g = np.random.default_rng(6)
    Z = g.standard_normal((8, 8))
    G = Z @ Z.T + 0.1 * np.eye(8)
    R, acc = RP.chol_drop(G, 1e-12)
    assert acc == list(range(8))
    np.testing.assert_allclose(R, np.linalg.cholesky(G).T, rtol=1e-12, atol=1e-14)
    v = g.standard_normal((4, 1))
    Gd = np.hstack([v, v, g.standard_normal((4, 1))])
    Gd = Gd.T @ Gd  # rank 2; position 1 duplicates position 0
    R2, acc2 = RP.chol_drop(Gd, 1e-10 * np.trace(Gd))
    assert acc2 == [0, 2]
    np.testing.assert_allclose(R2.T @ R2, Gd[np.ix_([0, 2], [0, 2])], rtol=1e-12)


@pytest.mark.parametrize("kind", [K.GAUSSIAN, K.LAPLACE])
def test_nystrom_identity_psd_residual_and_monotone_trace(kind):
    p = c1(n=400)
    rec = []
    F, piv = RP.rpcholesky(p.X, kind, p.sigma, r=60, B=7, seed=11, record=rec)
    A = K.block(p.X, p.X, kind, p.sigma)
    assert F.shape[1] == len(piv) == 60
    assert len(set(piv)) == 60
    # F F^T = A(:,S) A(S,S)^{-1} A(S,:) (column Nystrom form, Sec. 3.1)
    S = np.array(piv)
    Nys = A[:, S] @ np.linalg.solve(A[np.ix_(S, S)], A[S, :])
    np.testing.assert_allclose(F @ F.T, Nys, atol=1e-9)
    # A - F F^T is psd (the Nystrom approximation is bounded by A, Sec. 5.1)
    lam = np.linalg.eigvalsh(A - F @ F.T)
    assert lam.min() >= -1e-12 * 400
    # residual trace is non-increasing block to block
    T = [b["T"] for b in rec]
    assert all(T[i + 1] <= T[i] + 1e-12 for i in range(len(T) - 1))
    assert abs(np.trace(A - F @ F.T) - np.sum(np.maximum(np.diag(A - F @ F.T), 0))) < 1e-9


def test_exact_recovery_and_early_stop():
    # q distinct points, each repeated: rank(A) = q; RPCholesky recovers A
    # exactly once the rank is reached (Sec. 5.1) and stops early.
    g = np.random.default_rng(7)
    q = 6
    base = g.standard_normal((q, 3)) * 3
    X = base[g.integers(0, q, size=200)]
    X[:q] = base
    A = K.block(X, X, K.GAUSSIAN, 1.0)
    F, piv = RP.rpcholesky(X, K.GAUSSIAN, 1.0, r=40, B=5, seed=3)
    assert F.shape[1] == q
    np.testing.assert_allclose(F @ F.T, A, atol=1e-10)


def woodbury(F, mu, z):
    r = F.shape[1]
    core = mu * np.eye(r) + F.T @ F
    return (z - F @ np.linalg.solve(core, F.T @ z)) / mu


def test_preconditioner_forms_agree_and_bounds_hold():
    p = c1(n=300)
    mu = 0.05
    F, _ = RP.rpcholesky(p.X, p.kind, p.sigma, r=30, seed=5)
    P = RP.NystromPreconditioner(F, mu)
    g = np.random.default_rng(8)
    Z = g.standard_normal((300, 3))
    dense = np.linalg.solve(F @ F.T + mu * np.eye(300), Z)
    np.testing.assert_allclose(P.apply(Z), dense, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(woodbury(F, mu, Z), dense, rtol=1e-9, atol=1e-9)
    # eq. condition: 1 <= lambda(P^{-1/2}(A+mu I)P^{-1/2}) <= 1 + tr(A - Ahat)/mu
    A = K.block(p.X, p.X, p.kind, p.sigma)
    Pm = F @ F.T + mu * np.eye(300)
    w, V = np.linalg.eigh(Pm)
    Pmh = V @ np.diag(w ** -0.5) @ V.T
    lam = np.linalg.eigvalsh(Pmh @ (A + mu * np.eye(300)) @ Pmh)
    assert lam.min() >= 1 - 1e-9
    assert lam.max() <= 1 + np.trace(A - F @ F.T) / mu + 1e-9


def test_full_rank_preconditioner_converges_in_one_iteration():
    g = np.random.default_rng(9)
    base = g.standard_normal((5, 2))
    X = base[g.integers(0, 5, size=60)]
    X[:5] = base
    F, _ = RP.rpcholesky(X, K.LAPLACE, 1.0, r=20, seed=1)
    mu = 1e-2
    A = K.block(X, X, K.LAPLACE, 1.0)
    P = RP.NystromPreconditioner(F, mu)
    y = g.standard_normal(60)
    x, info = PCG.pcg(lambda V: A @ V + mu * V, P.apply, y, 1e-10, 10)
    assert info["iters"][0] == 1
    np.testing.assert_allclose((A + mu * np.eye(60)) @ x, y, atol=1e-9)
