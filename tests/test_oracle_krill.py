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


def singular_centre_problem(n=2000, k=100, mu=1e-9):
    """The restricted workload with two pairs of centres made identical, so
    A(S,S) is singular with null vectors e_0 - e_1 and e_2 - e_3, and a ridge
    small enough that the shift of Alg. 2 is what keeps H nonsingular."""
    p = c4(n=n, k=k)
    X = p.X.copy()
    S = KR.sample_centers(n, k, p.algo_seed)
    X[S[1]] = X[S[0]]
    X[S[3]] = X[S[2]]
    return KR.Krill(X, p.kind, p.sigma, mu, S, seed=p.algo_seed), n, k


def test_krill_shift_on_singular_centres():
    """Alg. 2, steps 1-2: H = mu A_SS + N eps_mach tr(A_SS) I, with eps_mach
    about 2e-16 in double precision.  Both kernels have a unit diagonal, so
    tr(A_SS) = k.  Two identical centres give A_SS an exact null vector u:
    then H u is exactly the shift times u, and the shift is lambda_min(H)
    because mu A_SS is positive semidefinite."""
    kr, n, k = singular_centre_problem()
    eps_paper = golden("eps_mach_approx")
    assert abs(KR.EPS / eps_paper - 1.0) < 0.15
    for i, j in ((0, 1), (2, 3)):
        u = np.zeros(k)
        u[i], u[j] = 1.0, -1.0
        Hu = kr.H @ u
        lam = Hu[i]
        np.testing.assert_array_equal(Hu, lam * u)
        # the shift the paper prints, with its own approximate eps
        assert abs(lam / (n * eps_paper * k) - 1.0) < 0.15, lam
        # the same with eps = 2**-52 (the reading), to rounding
        assert abs(lam - n * 2.0 ** -52 * k) <= 4 * np.spacing(lam)
    ev = np.linalg.eigvalsh(kr.H)
    assert abs(ev[0] / lam - 1.0) < 1e-9 and abs(ev[1] / lam - 1.0) < 1e-9
    assert ev[2] > lam                                  # the other directions carry mu A_SS
    # H minus its shift is mu A_SS: symmetric, zero on the null vectors
    Hm = kr.H - lam * np.eye(k)
    np.testing.assert_array_equal(Hm, Hm.T)
    assert np.all(np.abs(np.diag(Hm) - kr.mu) <= 4 * np.spacing(kr.mu))


def test_krill_kappa_on_a_restricted_system_as_mu_vanishes():
    """Sec. 2.2.3: with a sketch of d = 2k rows and mu -> 0 the preconditioned
    restricted matrix behaves like the Gram matrix of a 2k x k Gaussian
    matrix, condition number (1 + 1/sqrt 2)^2 / (1 - 1/sqrt 2)^2 ~ 34.0,
    while the unpreconditioned system is badly conditioned (the paper's
    example sets mu/N = 1e-12).  Checked on the restricted workload's
    distribution (sigma = 4) through the generalised eigenvalues of (M, P)."""
    import scipy.linalg as sl
    target = golden("krill_gaussian_kappa")
    n, k = 6000, 200
    p = c4(n=n, k=k)
    S = KR.sample_centers(n, k, p.algo_seed)
    kappas = []
    for s in range(3):
        kr = KR.Krill(p.X, p.kind, p.sigma, 1e-12 * n, S, seed=s)
        M = kr.restricted_matrix()
        ev = sl.eigh(M, kr.P, eigvals_only=True)
        kappas.append(ev.max() / ev.min())
    assert np.linalg.cond(M) > 1e10
    km = float(np.median(kappas))
    assert 0.5 * target < km < 2.0 * target, kappas
