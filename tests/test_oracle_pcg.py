"""Pins of the oracle's PCG (Sec. 3, eq. psd_system and eq. rate) and of
the full-data solve of Alg. 1 against a dense Cholesky solve (eq. exact_eqn)."""
import numpy as np

from oracle import kernels as K
from oracle import rpcholesky as RP
from oracle import pcg as PCG
from oracle import direct
from synth import c1


def test_rpcholesky_pcg_matches_dense_cholesky_solve():
    p = c1(n=600)
    F, _ = RP.rpcholesky(p.X, p.kind, p.sigma, r=60, seed=p.algo_seed)
    P = RP.NystromPreconditioner(F, p.mu)
    prod = lambda V: K.matvec(p.X, p.X, V, p.kind, p.sigma, shift=p.mu)
    x, info = PCG.pcg(prod, P.apply, p.Y, 1e-12, 500)
    xd = direct.full_krr(p.X, p.Y, p.kind, p.sigma, p.mu)
    assert info["converged"]
    assert info["relres_true"][0] < 1e-10
    A = K.block(p.X, p.X, p.kind, p.sigma)
    # fitted values are well conditioned; coefficients carry kappa * eps
    np.testing.assert_allclose(A @ x, A @ xd, rtol=0, atol=1e-8 * np.abs(A @ xd).max())


def test_cg_exact_in_n_steps():
    g = np.random.default_rng(1)
    Q, _ = np.linalg.qr(g.standard_normal((20, 20)))
    M = Q @ np.diag(np.linspace(1, 30, 20)) @ Q.T
    b = g.standard_normal(20)
    x, info = PCG.pcg(lambda V: M @ V, lambda V: V, b, 1e-13, 20)
    np.testing.assert_allclose(M @ x, b, atol=1e-10)
    assert info["iters"][0] <= 20


def test_cg_three_distinct_eigenvalues_three_steps():
    g = np.random.default_rng(2)
    Q, _ = np.linalg.qr(g.standard_normal((30, 30)))
    ev = np.repeat([1.0, 4.0, 9.0], 10)
    M = Q @ np.diag(ev) @ Q.T
    b = g.standard_normal(30)
    x, info = PCG.pcg(lambda V: M @ V, lambda V: V, b, 1e-11, 50)
    assert info["iters"][0] == 3


def test_error_bound_of_eq_rate():
    g = np.random.default_rng(3)
    n = 120
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    M = Q @ np.diag(np.geomspace(1, 1e4, n)) @ Q.T
    Pm = np.diag(np.diag(M)) + 0.0
    Pinv = lambda V: V / np.diag(Pm)[:, None] if V.ndim == 2 else V / np.diag(Pm)
    b = g.standard_normal(n)
    xs = np.linalg.solve(M, b)
    ph = np.diag(np.diag(Pm) ** -0.5)
    lam = np.linalg.eigvalsh(ph @ M @ ph)
    kap = lam.max() / lam.min()
    rate = (np.sqrt(kap) - 1) / (np.sqrt(kap) + 1)
    nrm = lambda e: np.sqrt(e @ M @ e)
    for t in range(1, 25):
        x, _ = PCG.pcg(lambda V: M @ V, Pinv, b, 1e-300, t)
        assert nrm(x - xs) / nrm(xs) <= 2 * rate ** t * (1 + 1e-9)


def test_columns_are_independent_recurrences():
    g = np.random.default_rng(4)
    Z = g.standard_normal((50, 50))
    M = Z @ Z.T + 5 * np.eye(50)
    B = g.standard_normal((50, 3))
    B[:, 1] *= 1e-3
    X, info = PCG.pcg(lambda V: M @ V, lambda V: V, B, 1e-9, 200)
    for c in range(3):
        xc, ic = PCG.pcg(lambda V: M @ V, lambda V: V, B[:, c], 1e-9, 200)
        # same recurrence; only BLAS summation order differs (gemm vs gemv)
        np.testing.assert_allclose(X[:, c], xc, rtol=1e-9, atol=1e-12)
        assert ic["iters"][0] == info["iters"][c]
