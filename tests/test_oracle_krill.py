"""Pins of the oracle's KRILL (Alg. 2), sparse sign embedding and centre
sampling (Sec. 2.2), against direct solves, closed forms and invariants."""
import math
import os

import numpy as np
import scipy.sparse as sp
from scipy.stats import chisquare

from oracle import kernels as K
from oracle import krill as KR
from oracle import pcg as PCG
from oracle import direct
from synth import c4

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")


def golden(name):
    for l in open(GOLD):
        if l.strip() and not l.startswith("#"):
            k, v = l.split()
            if k == name:
                return float(v)
    raise KeyError(name)


def test_default_zeta_natural_log():
    assert KR.default_zeta(1000) == 7 and KR.default_zeta(10_000) == 10 and KR.default_zeta(1) == 1


def test_sketch_structure():
    N, d, z = 3000, 64, 6
    Phi = KR.sketch_matrix(N, d, z, seed=12).tocsc()
    nnz = np.diff(Phi.indptr)
    assert np.all(nnz == z)
    np.testing.assert_allclose(np.abs(Phi.data), 1 / math.sqrt(z), rtol=0, atol=0)
    np.testing.assert_allclose(sp.linalg.norm(Phi, axis=0), np.ones(N), rtol=1e-15)
    frac_pos = np.mean(Phi.data > 0)
    assert abs(frac_pos - 0.5) < 0.02
    rows = Phi.indices
    counts = np.bincount(rows, minlength=d)
    assert chisquare(counts).pvalue > 1e-4  # rows uniform


def test_centers_uniform_without_replacement():
    N, k = 20, 5
    hits = np.zeros(N)
    for s in range(3000):
        c = KR.sample_centers(N, k, s)
        assert len(set(c.tolist())) == k and list(c) == sorted(c)
        hits[c] += 1
    assert chisquare(hits).pvalue > 1e-4
    assert abs(hits.sum() / (3000 * N) - k / N) < 1e-12


def small_problem(n=1500, k=120):
    p = c4(n=n, k=k)
    S = KR.sample_centers(n, k, p.algo_seed)
    return p, S


def test_krill_matches_direct_solve_and_psd_gap():
    p, S = small_problem()
    kr = KR.Krill(p.X, p.kind, p.sigma, p.mu, S, seed=p.algo_seed)
    G = kr.P - kr.H
    assert np.linalg.eigvalsh(G).min() >= -1e-10 * np.abs(G).max()
    b = kr.rhs(p.Y)
    M = kr.restricted_matrix()
    xd = direct.restricted_krr(M, b)
    x, info = PCG.pcg(kr.product, kr.precondition, b, 1e-12, 200)
    assert info["converged"] and info["relres_true"][0] < 1e-10
    # ||x - xd||_M <= (||b - M x|| + ||b - M xd||) / sqrt(lambda_min(M)),
    # and the fitted values satisfy ||A(:,S)(x - xd)|| <= ||x - xd||_M.
    e = (x - xd)[:, 0]
    lmin = np.linalg.eigvalsh(M).min()
    bound = (np.linalg.norm(b - M @ x) + np.linalg.norm(b - M @ xd)) / np.sqrt(lmin)
    assert np.sqrt(e @ M @ e) <= 1.01 * bound + 1e-14
    assert np.linalg.norm(kr.AnS @ e) <= 1.01 * bound + 1e-14
    assert info["iters"][0] < 60


def test_identity_sketch_gives_exact_preconditioner():
    p, S = small_problem(n=400, k=40)
    kr = KR.Krill(p.X, p.kind, p.sigma, p.mu, S, phi=sp.identity(400, format="csr"))
    np.testing.assert_allclose(kr.P, kr.restricted_matrix(), rtol=1e-12, atol=1e-12)
    b = kr.rhs(p.Y)
    x, info = PCG.pcg(kr.product, kr.precondition, b, 1e-8, 10)
    assert info["iters"][0] == 1


def test_all_points_as_centres_reduce_to_full_data_krr():
    # S = [N], A nonsingular: (A^2 + mu A) b = A y  ->  b = (A + mu I)^{-1} y (Sec. 2.2).
    g = np.random.default_rng(3)
    n = 150
    X = 3.0 * g.standard_normal((n, 3))   # well separated: A close to I
    y = g.standard_normal(n)
    mu = 0.3
    kr = KR.Krill(X, K.GAUSSIAN, 1.0, mu, np.arange(n), seed=4)
    b = kr.rhs(y)
    x, info = PCG.pcg(kr.product, kr.precondition, b, 1e-13, 300)
    xf = direct.full_krr(X, y, K.GAUSSIAN, 1.0, mu)
    A = K.block(X, X, K.GAUSSIAN, 1.0)
    assert np.linalg.eigvalsh(A).min() > 1e-3
    np.testing.assert_allclose(x, xf, rtol=1e-9, atol=1e-10 * np.abs(xf).max())


def test_sparse_sign_embedding_kappa_near_gaussian_model():
    # Sec. 2.2.3: with d = 2k the preconditioned spectrum follows a 2k x k
    # Gaussian matrix, kappa ~ (1+1/sqrt2)^2/(1-1/sqrt2)^2 ~ 34.0.  For an
    # orthonormal Q the embedded Gram (Phi Q)^T (Phi Q) shows the same spread.
    target = golden("krill_gaussian_kappa")
    assert abs((1 + 2 ** -0.5) ** 2 / (1 - 2 ** -0.5) ** 2 - target) < 0.05
    g = np.random.default_rng(5)
    N, k = 6000, 200
    Q, _ = np.linalg.qr(g.standard_normal((N, k)))
    kappas = []
    for s in range(3):
        Phi = KR.sketch_matrix(N, 2 * k, KR.default_zeta(k), seed=s)
        ev = np.linalg.eigvalsh((Phi @ Q).T @ (Phi @ Q))
        kappas.append(ev.max() / ev.min())
    km = float(np.median(kappas))
    assert 0.5 * target < km < 2.0 * target, kappas
