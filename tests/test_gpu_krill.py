"""Parity of the KRILL build and restricted solve (Alg. 2) against the FP64
oracle.

Tolerances:
* centres, sketch rows and signs: bit-exact (integer work).
* H (FP64 kernel entries): 1e-13 relative to max |H|.
* B = Phi A(:,S): FP64 tiles 1e-12 * (|Phi| |A(:,S)|); FP32 tiles
  2e-5 * (|Phi| |A(:,S)|) (same entry bound as the product tiles).
* P = L L^T (FP64 tiles): 1e-10 relative to max |P|.
* restricted operator M v: FP64 1e-12, FP32 tiles 4e-5, relative to
  (|A_SN| |A_NS| |v| + |H| |v|).
* solutions: fitted values A(:,S) beta within 1e-6 (FP64) / 1e-4 (FP32) of
  the oracle's, relative 2-norm.
"""
import math

import numpy as np
import pytest
import torch

from oracle import kernels as OK
from oracle import krill as OKR
from oracle import pcg as OPCG
from oracle.rng import sm, key, below, TAG_SKETCH_ROW
import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def B():
    from paper_2304_12465_amd import binding
    return binding


def T(a, dtype=np.float64):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to(DEV)


def small(n=2000, k=100):
    return synth.c4(n=n, k=k)


def build(p, prec, centers=None, m_max=1, zeta=None):
    c = None if centers is None else T(centers, np.int64)
    return B().krill_build(p.kind, p.sigma, prec, T(p.X), p.mu, p.centers, centers=c,
                           sketch_rows=p.sketch_rows, zeta=zeta or p.zeta, seed=p.algo_seed,
                           m_max=m_max)


def test_centres_and_sketch_bit_exact():
    p = small()
    P = build(p, 0)
    S_o = OKR.sample_centers(p.X.shape[0], p.centers, p.algo_seed)
    assert P.pivots() == [int(v) for v in S_o]
    N, z = p.X.shape[0], p.zeta
    rows = B().krill_export(P, 0, (N, z), torch.int32).cpu().numpy()
    signs = B().krill_export(P, 1, (N, z), torch.int32).cpu().numpy()
    r_o, s_o = OKR.sketch_columns(N, p.sketch_rows, z, p.algo_seed)
    np.testing.assert_array_equal(rows, r_o)
    np.testing.assert_array_equal(signs, s_o.astype(np.int32))


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 2e-5), (2, 2e-5)])
def test_sketch_H_and_factor(prec, tol):
    # prec 2 (KRR_MIXED): the sketch on FP32 tiles, H and the factor in FP64
    p = small()
    P = build(p, prec)
    k = p.centers
    kr = OKR.Krill(p.X, p.kind, p.sigma, p.mu, np.array(P.pivots()), sketch_rows=p.sketch_rows,
                   zeta=p.zeta, seed=p.algo_seed)
    Bg = B().krill_export(P, 2, (p.sketch_rows, k), torch.float64).cpu().numpy()
    bound = tol * (np.abs(kr.Phi) @ np.abs(kr.AnS)) + 1e-300
    assert np.all(np.abs(Bg - kr.B) <= bound), np.max(np.abs(Bg - kr.B) / bound)
    Hg = B().krill_export(P, 3, (k, k), torch.float64).cpu().numpy()
    np.testing.assert_allclose(Hg, kr.H, rtol=0, atol=1e-13 * np.abs(kr.H).max())
    if prec == 0:
        L = B().krill_export(P, 4, (k, k), torch.float64).cpu().numpy()
        assert np.all(np.triu(L, 1) == 0)
        np.testing.assert_allclose(L @ L.T, kr.P, rtol=0, atol=1e-10 * np.abs(kr.P).max())
    if prec == 2:
        # P = B^T B + H from the FP32-tile B: with |dB| <= E = tol |Phi||A(:,S)|,
        # |dP| <= 2 |B|^T E + E^T E entrywise, plus the factorisation's rounding
        L = B().krill_export(P, 4, (k, k), torch.float64).cpu().numpy()
        assert np.all(np.triu(L, 1) == 0)
        E = tol * (np.abs(kr.Phi) @ np.abs(kr.AnS))
        dP = 2.0 * np.abs(kr.B).T @ E + E.T @ E + 1e-10 * np.abs(kr.P).max()
        assert np.all(np.abs(L @ L.T - kr.P) <= dP), np.max(np.abs(L @ L.T - kr.P) / dP)


@pytest.mark.parametrize("d", [3, 7, 16, 19, 23, 30])
def test_fp32_sketch_over_padded_dimensions(d):
    # FP32 sketch tiles at padded dimensions 4, 8, 16, 20, 24 and 32: the
    # multiples of 8 contract three bf16 slices per coordinate on the bf16
    # matrix cores, 4 and 20 run the FP32 ones; both within the FP32 tiles'
    # entry bound 2e-5 |Phi||A(:,S)| of the oracle's B
    p = synth.c4(n=3000, k=300, d=d)
    P = build(p, 1)
    kr = OKR.Krill(p.X, p.kind, p.sigma, p.mu, np.array(P.pivots()), sketch_rows=p.sketch_rows,
                   zeta=p.zeta, seed=p.algo_seed)
    Bg = B().krill_export(P, 2, (p.sketch_rows, p.centers), torch.float64).cpu().numpy()
    bound = 2e-5 * (np.abs(kr.Phi) @ np.abs(kr.AnS)) + 1e-300
    assert np.all(np.abs(Bg - kr.B) <= bound), np.max(np.abs(Bg - kr.B) / bound)


@pytest.mark.parametrize("n,k", [(6000, 1024), (6000, 1100), (8000, 2100)])
def test_factor_and_apply_past_one_outer_block(n, k):
    # k = 1,024, 1,100 and 2,100 centres: the Cholesky factor and the inverse
    # of L are built in two levels of blocks (outer steps of 512, the last one
    # whole or ragged, on two streams), so the outer panel solves and
    # trailing updates all run;
    # at k = 2,100 B^T B runs on 128 x 128 tiles.  sigma = 0.3 keeps kappa(P)
    # near 1e4-1e5, so the apply bound below is tight.
    p = small(n=n, k=k)
    p.sigma = 0.3
    P = build(p, 0, m_max=2)
    k = p.centers
    kr = OKR.Krill(p.X, p.kind, p.sigma, p.mu, np.array(P.pivots()), sketch_rows=p.sketch_rows,
                   zeta=p.zeta, seed=p.algo_seed)
    L = B().krill_export(P, 4, (k, k), torch.float64).cpu().numpy()
    assert np.all(np.triu(L, 1) == 0)
    np.testing.assert_allclose(L @ L.T, kr.P, rtol=0, atol=1e-10 * np.abs(kr.P).max())
    # P^{-1} z through the explicit inverse of L: forward error of an
    # SPD solve, 100 k eps kappa(P)
    Z = np.random.default_rng(11).standard_normal((k, 2))
    got = P.apply(T(Z)).cpu().numpy()
    ref = np.linalg.solve(kr.P, Z)
    kap = np.linalg.cond(kr.P)
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel <= 100 * k * 2.0 ** -52 * kap, (rel, kap)


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 4e-5), (2, 1e-12)])
def test_restricted_operator(prec, tol):
    p = small()
    P = build(p, prec, m_max=2)
    S = np.array(P.pivots())
    kr = OKR.Krill(p.X, p.kind, p.sigma, p.mu, S, sketch_rows=p.sketch_rows, zeta=p.zeta,
                   seed=p.algo_seed)
    V = np.random.default_rng(3).standard_normal((p.centers, 2))
    got = P.operator(T(V)).cpu().numpy()
    ref = kr.product(V)
    scale = np.abs(kr.AnS).T @ (np.abs(kr.AnS) @ np.abs(V)) + np.abs(kr.H) @ np.abs(V)
    assert np.all(np.abs(got - ref) <= tol * scale), np.max(np.abs(got - ref) / scale)


def test_restricted_solve_matches_oracle_fp64():
    p = small(n=3000, k=150)
    P = build(p, 0)
    S = np.array(P.pivots())
    kr = OKR.Krill(p.X, p.kind, p.sigma, p.mu, S, sketch_rows=p.sketch_rows, zeta=p.zeta,
                   seed=p.algo_seed)
    beta, info = P.solve(T(p.Y), p.tol, max_iter=200)
    b = kr.rhs(p.Y)
    xo, io = OPCG.pcg(kr.product, kr.precondition, b, p.tol, 200)
    assert info["converged"] and io["converged"]
    assert info["iters"] <= 60
    fit = kr.AnS @ beta.cpu().numpy()
    fit_o = kr.AnS @ xo
    rel = np.linalg.norm(fit - fit_o) / np.linalg.norm(fit_o)
    assert rel <= 1e-6, rel
    assert abs(info["iters"] - int(io["iters"][0])) <= 1


def test_restricted_solve_mixed_sketch():
    # KRR_MIXED: the FP64 build's restricted products, right-hand side and
    # checks, with the sketch on FP32 tiles.  The system is the FP64 one; only
    # the preconditioner differs (by the sketch's FP32 error).  So the oracle's
    # FP64 true residual of the returned beta meets 10 tol, the library's
    # true residual is the oracle's to within the FP64 tile error, the M-norm
    # distance to the oracle's solution is within (||b - M beta|| +
    # ||b - M x_o||) / sqrt(lambda_min(M)), and the iteration count stays
    # within 2 of the FP64 build's.
    p = small(n=3000, k=150)
    P = build(p, 2)
    P64 = build(p, 0)
    S = np.array(P.pivots())
    assert P64.pivots() == P.pivots()
    kr = OKR.Krill(p.X, p.kind, p.sigma, p.mu, S, sketch_rows=p.sketch_rows, zeta=p.zeta,
                   seed=p.algo_seed)
    beta, info = P.solve(T(p.Y), p.tol, max_iter=200)
    _, info64 = P64.solve(T(p.Y), p.tol, max_iter=200)
    assert info["converged"] and abs(info["iters"] - info64["iters"]) <= 2, (info, info64)
    beta = beta.cpu().numpy()
    b = kr.rhs(p.Y)
    M = kr.restricted_matrix()
    bn = np.linalg.norm(b)
    r_true = np.linalg.norm(b - M @ beta) / bn
    assert r_true <= 10 * p.tol, r_true
    Mabs = np.abs(kr.AnS).T @ np.abs(kr.AnS) + np.abs(kr.H)
    err = (3e-12 * np.linalg.norm(Mabs @ np.abs(beta))
           + 1e-12 * np.linalg.norm(np.abs(kr.AnS).T @ np.abs(p.Y))) / bn
    assert abs(info["relres_true"] - r_true) <= err + 1e-6 * r_true, (info, r_true, err)
    xo, io = OPCG.pcg(kr.product, kr.precondition, b, p.tol, 200)
    e = (beta - xo)[:, 0]
    bound = (r_true * bn + np.linalg.norm(b - M @ xo)) / np.sqrt(np.linalg.eigvalsh(M).min())
    assert np.sqrt(e @ M @ e) <= 1.01 * bound


def test_restricted_solve_fp32_tiles_within_derived_bounds():
    # FP32 tiles perturb the restricted operator by at most
    # delta * (|A_SN||A_NS| + |H|)|v| with delta = 4e-5 (test_restricted_operator).
    # The FP64 true residual of the returned beta is therefore bounded by
    # tol ||b|| + delta ||(|A_SN||A_NS| + |H|)|beta|||, and its distance to the
    # oracle's solution in the M-norm by (||b - M beta|| + ||b - M x_o||) /
    # sqrt(lambda_min(M)).  (With mu/N = 1e-5 the restricted matrix is
    # ill-conditioned, so fitted values can differ by more than the operator
    # error; the bounds above are what the arithmetic guarantees.)
    p = small(n=3000, k=150)
    P = build(p, 1)
    S = np.array(P.pivots())
    kr = OKR.Krill(p.X, p.kind, p.sigma, p.mu, S, sketch_rows=p.sketch_rows, zeta=p.zeta,
                   seed=p.algo_seed)
    beta, info = P.solve(T(p.Y), p.tol, max_iter=200)
    assert info["converged"] and info["iters"] <= 60
    beta = beta.cpu().numpy()
    b = kr.rhs(p.Y)
    M = kr.restricted_matrix()
    xo, io = OPCG.pcg(kr.product, kr.precondition, b, p.tol, 200)
    # refinement contract: the FP64 true residual meets tol (the library's own
    # FP64 product, then the oracle's, which differs from it by rounding)
    assert info["relres_true"] <= p.tol, info
    r_true = np.linalg.norm(b - M @ beta)
    assert r_true <= 10 * p.tol * np.linalg.norm(b), r_true / np.linalg.norm(b)
    e = (beta - xo)[:, 0]
    bound = (r_true + np.linalg.norm(b - M @ xo)) / np.sqrt(np.linalg.eigvalsh(M).min())
    assert np.sqrt(e @ M @ e) <= 1.01 * bound
    rel = np.linalg.norm(kr.AnS @ e) / np.linalg.norm(kr.AnS @ xo)
    print(f"fp32-tile fitted-value difference vs oracle: {rel:.2e}")


@pytest.mark.parametrize("m", [1, 3])
def test_carried_true_residual_matches_oracle(m):
    # 40,000 points x 250 centres: above the size of the short-solve bursts,
    # so every iteration is a step.  With FP64 tiles the step predicted to
    # converge, and the last step allowed, carry x beside p; the exit check
    # (b - M x) - alpha (M p) then needs no product of its own.  relres_true
    # must be the oracle's ||b - M beta|| / ||b|| of the returned beta, to
    # within the FP64 tile error of M x, M p (test_restricted_operator: 1e-12
    # of (|A_SN||A_NS| + |H|)|v|) and of b = A(S,:) y.
    p = small(n=40_000, k=250)
    P = build(p, 0, m_max=m)
    S = np.array(P.pivots())
    kr = OKR.Krill(p.X, p.kind, p.sigma, p.mu, S, sketch_rows=p.sketch_rows, zeta=p.zeta,
                   seed=p.algo_seed)
    g = np.random.default_rng(21)
    Y = np.column_stack([p.Y[:, 0]] + [g.standard_normal(p.X.shape[0]) for _ in range(m - 1)])
    b = kr.rhs(Y)
    M = kr.restricted_matrix()
    Mabs = np.abs(kr.AnS).T @ np.abs(kr.AnS) + np.abs(kr.H)
    bnorm = np.linalg.norm(b, axis=0)
    berr = 1e-12 * np.linalg.norm(np.abs(kr.AnS).T @ np.abs(Y), axis=0)
    for max_iter, tol in ((3, 1e-12), (200, 1e-8)):
        beta, info = P.solve(T(Y), tol, max_iter=max_iter)
        beta = beta.cpu().numpy().reshape(-1, m)
        res = np.linalg.norm(b - M @ beta, axis=0) / bnorm
        err = (3e-12 * np.linalg.norm(Mabs @ np.abs(beta), axis=0) + berr) / bnorm
        print(f"m={m} max_iter={max_iter}: iters {info['iters']} products {info['products']} "
              f"relres_true {info['relres_true']:.3e} oracle {res.max():.3e} bound {err.max():.1e}")
        assert abs(info["relres_true"] - res.max()) <= err.max() + 1e-6 * res.max(), (info, res)
        if max_iter == 3:
            assert not info["converged"] and info["iters"] == 3 and info["products"] == 3, info
        else:
            assert info["converged"] and info["products"] <= info["iters"] + 1, info
    # the same solve with no carried columns (m_max above the carrying limit):
    # the same iterates, and one more product for the exit check
    P5 = build(p, 0, m_max=5)
    beta5, info5 = P5.solve(T(Y), 1e-8, max_iter=200)
    assert info5["iters"] == info["iters"] and info5["products"] == info5["iters"] + 1, info5
    np.testing.assert_allclose(beta, beta5.cpu().numpy().reshape(-1, m), rtol=0,
                               atol=1e-10 * np.abs(beta).max())


def test_given_centres_and_multi_rhs():
    p = small()
    S = np.sort(np.random.default_rng(4).choice(p.X.shape[0], p.centers, replace=False))
    P = build(p, 0, centers=S, m_max=3)
    assert P.pivots() == [int(v) for v in S]
    Y = np.column_stack([p.Y[:, 0], np.random.default_rng(5).standard_normal(p.X.shape[0])])
    beta, info = P.solve(T(Y), 1e-8, 200)
    assert info["converged"]
    beta = beta.cpu().numpy()
    for c in range(2):
        b1, _ = P.solve(T(Y[:, c].copy()), 1e-8, 200)
        np.testing.assert_allclose(beta[:, c], b1.cpu().numpy(), rtol=1e-12, atol=1e-14)


def test_all_points_as_centres():
    # S = [N] with A well conditioned: (A^2 + mu A) b = A y gives
    # b = (A + mu I)^{-1} y (Sec. 2.2); same instance as the oracle's pin.
    g = np.random.default_rng(3)
    n = 150
    X = 3.0 * g.standard_normal((n, 3))
    y = g.standard_normal((n, 1))
    assert np.linalg.eigvalsh(OK.block(X, X, 0, 1.0)).min() > 1e-3
    p = synth.Problem("all", X, y, 0, 1.0, 0.3, centers=n, sketch_rows=2 * n, zeta=4)
    P = build(p, 0, centers=np.arange(n))
    beta, info = P.solve(T(y), 1e-13, 300)
    assert info["converged"]
    from oracle import direct
    xf = direct.full_krr(X, y, 0, 1.0, 0.3)
    np.testing.assert_allclose(beta.cpu().numpy(), xf, rtol=1e-8, atol=1e-9 * np.abs(xf).max())


def test_invalid_arguments():
    b = B()
    p = small(n=500, k=50)
    with pytest.raises(b.KrrError):
        b.krill_build(p.kind, p.sigma, 0, T(p.X), p.mu, 600)            # k > N
    with pytest.raises(b.KrrError):
        b.krill_build(p.kind, p.sigma, 0, T(p.X), p.mu, 50, sketch_rows=4, zeta=8)
    with pytest.raises(b.KrrError):
        b.krill_build(p.kind, p.sigma, 0, T(p.X), -1.0, 50)


def test_full_size_restricted_solve():
    # 2,000,000 points, d = 16, k = 10,000 centres, sketch 20,000 x 8.
    p = synth.c4()
    P = build(p, 1)
    N = p.X.shape[0]
    S_o = OKR.sample_centers(N, p.centers, p.algo_seed)
    assert P.pivots() == [int(v) for v in S_o]
    g = np.random.default_rng(8)
    cols = np.sort(g.choice(N, 64, replace=False))
    rows = B().krill_export(P, 0, (N, p.zeta), torch.int32).cpu().numpy()
    for j in cols:
        r, _ = OKR.sketch_column(int(j), p.sketch_rows, p.zeta, p.algo_seed)
        assert list(rows[j]) == r
    beta, info = P.solve(T(p.Y), p.tol, max_iter=100)
    assert info["converged"], info
    assert info["iters"] <= 60, info
    assert info["relres_true"] <= p.tol, info


@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_restricted_products_sampled(prec):
    # The two restricted products at the 2,000,000 x 10,000 shape, through the
    # product entry point: K(X, X_S) v on 64 sampled points and K(X_S, X) u on
    # 48 sampled centres against the oracle, at the product tolerances.
    p = synth.c4()
    N = p.X.shape[0]
    S = OKR.sample_centers(N, p.centers, p.algo_seed)
    C = p.X[S]
    g = np.random.default_rng(11)
    v = g.standard_normal((p.centers, 1))
    u = g.standard_normal((N, 1))
    b = B()
    tol = 1e-13 if prec == 0 else 3e-5
    Wt = b.kernel_matvec(p.kind, p.sigma, prec, T(p.X), T(C), T(v)).cpu().numpy()
    rows = np.sort(g.choice(N, 64, replace=False))
    Kb = OK.block(p.X[rows], C, p.kind, p.sigma)
    err = np.abs(Wt[rows] - Kb @ v)
    assert np.all(err <= tol * (np.abs(Kb) @ np.abs(v)) + 1e-300), err.max()
    Wc = b.kernel_matvec(p.kind, p.sigma, prec, T(C), T(p.X), T(u)).cpu().numpy()
    cs = np.sort(g.choice(p.centers, 48, replace=False))
    ref = np.zeros((48, 1))
    scale = np.zeros((48, 1))
    for j0 in range(0, N, 250_000):
        Kb = OK.block(C[cs], p.X[j0:j0 + 250_000], p.kind, p.sigma)
        ref += Kb @ u[j0:j0 + 250_000]
        scale += np.abs(Kb) @ np.abs(u[j0:j0 + 250_000])
    err = np.abs(Wc[cs] - ref)
    assert np.all(err <= tol * scale), (err / scale).max()


@pytest.mark.parametrize("prec", [2, 0])
def test_full_size_restricted_solve_fp64_oracle_residual(prec):
    # The headline configuration (KRR_MIXED: FP64 restricted products with the
    # sketch on FP32 tiles) and the all-FP64 build; both solve the same FP64
    # system, only their preconditioners differ.  The restricted residual
    # b - M beta, M = A(S,:)A(:,S) + H, is re-checked on 32 sampled centres:
    # the oracle forms their rows of A(S,:) against all 2,000,000 points (for
    # b = A(S,:)y and for A(S,:) t), t = A(:,S) beta comes from the FP64
    # product entry point (checked on sampled rows above), and their rows of
    # H = mu A_SS + N eps tr(A_SS) I from the oracle's kernel.
    p = synth.c4()
    N, k = p.X.shape[0], p.centers
    P = build(p, prec)
    beta, info = P.solve(T(p.Y), p.tol, max_iter=100)
    assert info["converged"] and info["relres_true"] <= 10 * p.tol, info
    beta_h = beta.cpu().numpy()
    S = np.array(P.pivots())
    C = p.X[S]
    t = B().kernel_matvec(p.kind, p.sigma, 0, T(p.X), T(C), beta).cpu().numpy()
    cs = np.sort(np.random.default_rng(12).choice(k, 32, replace=False))
    Yt = np.hstack([p.Y, t])
    acc = np.zeros((32, 2))
    for j0 in range(0, N, 250_000):
        acc += OK.block(C[cs], p.X[j0:j0 + 250_000], p.kind, p.sigma) @ Yt[j0:j0 + 250_000]
    Hrows = p.mu * OK.block(C[cs], C, p.kind, p.sigma)
    Hrows[np.arange(32), cs] += N * 2.0 ** -52 * k
    r = acc[:, 0] - acc[:, 1] - Hrows @ beta_h[:, 0]
    est = np.linalg.norm(r) / np.linalg.norm(acc[:, 0])
    assert est <= 20 * p.tol, est


def small_laplace(n=2000, k=100):
    # the restricted workload's points with the l1 Laplace kernel of Sec. 4.1
    p = synth.c4(n=n, k=k)
    p.kind, p.sigma = 1, 2.0
    return p


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 2e-5), (2, 2e-5)])
def test_laplace_sketch_H_factor_and_operator(prec, tol):
    # KRILL with the Laplace kernel: B = Phi A(:,S) (direct differences), H and
    # L against the oracle, then the restricted operator (FP32: the quantised
    # l1 tiles, exponent error <= dpad range / ((2^qbits - 1) sigma) plus FP32
    # rounding, well inside 4e-5 here)
    p = small_laplace()
    P = build(p, prec, m_max=2)
    k = p.centers
    S = np.array(P.pivots())
    assert list(S) == list(OKR.sample_centers(p.X.shape[0], k, p.algo_seed))
    kr = OKR.Krill(p.X, p.kind, p.sigma, p.mu, S, sketch_rows=p.sketch_rows, zeta=p.zeta,
                   seed=p.algo_seed)
    Bg = B().krill_export(P, 2, (p.sketch_rows, k), torch.float64).cpu().numpy()
    bound = tol * (np.abs(kr.Phi) @ np.abs(kr.AnS)) + 1e-300
    assert np.all(np.abs(Bg - kr.B) <= bound), np.max(np.abs(Bg - kr.B) / bound)
    Hg = B().krill_export(P, 3, (k, k), torch.float64).cpu().numpy()
    np.testing.assert_allclose(Hg, kr.H, rtol=0, atol=1e-13 * np.abs(kr.H).max())
    if prec == 0:
        L = B().krill_export(P, 4, (k, k), torch.float64).cpu().numpy()
        np.testing.assert_allclose(L @ L.T, kr.P, rtol=0, atol=1e-10 * np.abs(kr.P).max())
    V = np.random.default_rng(3).standard_normal((k, 2))
    got = P.operator(T(V)).cpu().numpy()
    ref = kr.product(V)
    scale = np.abs(kr.AnS).T @ (np.abs(kr.AnS) @ np.abs(V)) + np.abs(kr.H) @ np.abs(V)
    otol = 4e-5 if prec == 1 else 1e-12  # MIXED (2): FP64 restricted products
    assert np.all(np.abs(got - ref) <= otol * scale), np.max(np.abs(got - ref) / scale)


def test_laplace_restricted_solve_matches_oracle_fp64():
    p = small_laplace(n=3000, k=150)
    P = build(p, 0)
    S = np.array(P.pivots())
    kr = OKR.Krill(p.X, p.kind, p.sigma, p.mu, S, sketch_rows=p.sketch_rows, zeta=p.zeta,
                   seed=p.algo_seed)
    beta, info = P.solve(T(p.Y), p.tol, max_iter=200)
    b = kr.rhs(p.Y)
    xo, io = OPCG.pcg(kr.product, kr.precondition, b, p.tol, 200)
    assert info["converged"] and io["converged"]
    fit = kr.AnS @ beta.cpu().numpy()
    fit_o = kr.AnS @ xo
    assert np.linalg.norm(fit - fit_o) <= 1e-6 * np.linalg.norm(fit_o)
    assert abs(info["iters"] - int(io["iters"][0])) <= 1


@pytest.mark.parametrize("kind", [0, 1])
def test_shift_on_duplicated_centres(kind):
    # Alg. 2, steps 1-2, on the device: two pairs of identical centres give
    # A_SS exact null vectors u = e_i - e_j, so H u is exactly the shift
    # N eps tr(A_SS) times u (tr(A_SS) = k: unit diagonal), eps = 2^-52.
    p = synth.c4(n=2000, k=100)
    p.kind = kind
    p.mu = 1e-9
    S = OKR.sample_centers(2000, 100, p.algo_seed)
    X = p.X.copy()
    X[S[1]] = X[S[0]]
    X[S[3]] = X[S[2]]
    p.X = X
    P = build(p, 0, centers=S)
    Hg = B().krill_export(P, 3, (100, 100), torch.float64).cpu().numpy()
    lam = 2000 * 2.0 ** -52 * 100
    for i, j in ((0, 1), (2, 3)):
        u = np.zeros(100)
        u[i], u[j] = 1.0, -1.0
        Hu = Hg @ u
        assert np.all(np.abs(Hu - lam * u) <= 4 * np.spacing(lam)), Hu[:4]
    kr = OKR.Krill(X, p.kind, p.sigma, p.mu, S, seed=p.algo_seed)
    np.testing.assert_allclose(Hg, kr.H, rtol=0, atol=1e-13 * np.abs(kr.H).max())


def build_stored(p, prec, centers=None, m_max=1):
    c = None if centers is None else T(centers, np.int64)
    return B().krill_build(p.kind, p.sigma, prec, T(p.X), p.mu, p.centers, centers=c,
                           sketch_rows=p.sketch_rows, zeta=p.zeta, seed=p.algo_seed,
                           m_max=m_max, stored=True)


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_stored_block_and_operator(kind, prec):
    # prec 2 (KRR_MIXED): the FP64 block and operator with the sketch on FP32 tiles
    # Stored mode (Sec. 4.1 keeps A(:,S) in memory): the stored block against
    # the oracle's A(:,S), then the restricted operator over it for m = 1 (one
    # pass), 2 and 6 (two passes).  Gaussian blocks come from the product
    # tiles' expansion, whose guard holds the exponent's error to 400 eps (FP64)
    # or 200 eps_32 (FP32), plus a few ulps of exp and, in FP32, the exponent's
    # own rounding; Laplace blocks from direct differences (FP64: exp within an
    # ulp or two; FP32: |arg| (d + 2) 2^-24 plus FP32 rounding of the exp)
    p = small(n=3000, k=150)
    if kind == 1:
        p.kind, p.sigma = 1, 2.0
    P = build_stored(p, prec, m_max=6)
    S = np.array(P.pivots())
    kr = OKR.Krill(p.X, p.kind, p.sigma, p.mu, S, sketch_rows=p.sketch_rows, zeta=p.zeta,
                   seed=p.algo_seed)
    A = B().krill_export(P, 5, (p.X.shape[0], p.centers), torch.float64).cpu().numpy()
    arg = -np.log(np.maximum(kr.AnS, 1e-300))
    if kind == 0:
        if prec != 1:
            bound = 404 * 2.0 ** -53 * kr.AnS + 1e-300
        else:
            bound = (2 * (arg + 1) + 204) * 2.0 ** -24 * kr.AnS + 1e-38
        assert np.all(np.abs(A - kr.AnS) <= bound), np.max(np.abs(A - kr.AnS) / bound)
    elif prec != 1:
        np.testing.assert_allclose(A, kr.AnS, rtol=4e-16, atol=1e-300)
    else:
        d = p.X.shape[1]
        bound = ((arg + 1) * (d + 2) + 4) * 2.0 ** -24 * kr.AnS + 1e-38
        assert np.all(np.abs(A - kr.AnS) <= bound), np.max(np.abs(A - kr.AnS) / bound)
    # B, H as the recomputing build
    Bg = B().krill_export(P, 2, (p.sketch_rows, p.centers), torch.float64).cpu().numpy()
    tolB = 1e-12 if prec == 0 else 2e-5
    assert np.all(np.abs(Bg - kr.B) <= tolB * (np.abs(kr.Phi) @ np.abs(kr.AnS)) + 1e-300)
    otol = 4e-5 if prec == 1 else 1e-12
    for m in (1, 2, 6):
        V = np.random.default_rng(30 + m).standard_normal((p.centers, m))
        got = P.operator(T(V)).cpu().numpy()
        ref = kr.product(V)
        scale = np.abs(kr.AnS).T @ (np.abs(kr.AnS) @ np.abs(V)) + np.abs(kr.H) @ np.abs(V)
        assert np.all(np.abs(got - ref) <= otol * scale), (m, np.max(np.abs(got - ref) / scale))


@pytest.mark.parametrize("d", [7, 23, 30])
@pytest.mark.parametrize("prec", [0, 1])
def test_stored_gaussian_block_over_padded_dimensions(prec, d):
    # the Gaussian stored block from the expansion tiles' store variant at
    # padded dimensions 8, 24 and 32 (FP32: bf16 slices at 8 and 32, FP32
    # products at 24): entries within the expansion's bound, k = 150 centres
    # leave a ragged last chunk and the rows' padding columns zero (read back
    # through the operator, which streams whole padded rows)
    p = synth.c4(n=3000, k=150, d=d)
    P = build_stored(p, prec)
    S = np.array(P.pivots())
    kr = OKR.Krill(p.X, p.kind, p.sigma, p.mu, S, sketch_rows=p.sketch_rows, zeta=p.zeta,
                   seed=p.algo_seed)
    A = B().krill_export(P, 5, (p.X.shape[0], p.centers), torch.float64).cpu().numpy()
    arg = -np.log(np.maximum(kr.AnS, 1e-300))
    if prec == 0:
        bound = 404 * 2.0 ** -53 * kr.AnS + 1e-300
    else:
        bound = (2 * (arg + 1) + 204) * 2.0 ** -24 * kr.AnS + 1e-38
    assert np.all(np.abs(A - kr.AnS) <= bound), np.max(np.abs(A - kr.AnS) / bound)
    V = np.random.default_rng(40 + d).standard_normal((p.centers, 1))
    got = P.operator(T(V)).cpu().numpy()
    ref = kr.product(V)
    scale = np.abs(kr.AnS).T @ (np.abs(kr.AnS) @ np.abs(V)) + np.abs(kr.H) @ np.abs(V)
    otol = 4e-5 if prec == 1 else 1e-12
    assert np.all(np.abs(got - ref) <= otol * scale), np.max(np.abs(got - ref) / scale)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_stored_solve_matches_recomputed_and_oracle(prec):
    # the same KRILL preconditioner (same centres and sketch) with the block
    # stored and recomputed: FP64 iterations within one and fitted values
    # within 1e-6 of each other and of the oracle's PCG; FP32 storage meets tol
    # on the FP64 true residual (refinement with recomputed FP64 products)
    p = small(n=3000, k=150)
    Ps = build_stored(p, prec)
    Pr = build(p, prec)
    bs, is_ = Ps.solve(T(p.Y), p.tol, max_iter=200)
    br, ir = Pr.solve(T(p.Y), p.tol, max_iter=200)
    assert is_["converged"] and ir["converged"], (is_, ir)
    S = np.array(Ps.pivots())
    kr = OKR.Krill(p.X, p.kind, p.sigma, p.mu, S, sketch_rows=p.sketch_rows, zeta=p.zeta,
                   seed=p.algo_seed)
    if prec == 0:
        xo, io = OPCG.pcg(kr.product, kr.precondition, kr.rhs(p.Y), p.tol, 200)
        fit_o = kr.AnS @ xo
        for b_ in (bs, br):
            fit = kr.AnS @ b_.cpu().numpy()
            assert np.linalg.norm(fit - fit_o) <= 1e-6 * np.linalg.norm(fit_o)
        assert abs(is_["iters"] - ir["iters"]) <= 1
    elif prec == 2:
        # the same FP32-tile sketch on both sides, FP64 operators whose entries
        # agree to an ulp: the same iterates, the FP64 true residual within 10 tol
        assert abs(is_["iters"] - ir["iters"]) <= 1
        assert is_["relres_true"] <= 10 * p.tol and ir["relres_true"] <= 10 * p.tol
        fs, fr = kr.AnS @ bs.cpu().numpy(), kr.AnS @ br.cpu().numpy()
        assert np.linalg.norm(fs - fr) <= 1e-6 * np.linalg.norm(fr)
    else:
        assert is_["relres_true"] <= p.tol


def test_stored_two_pass_for_long_rows():
    # ld > 16,384 centres: the row does not fit the one-pass workgroup, so
    # one right-hand side takes the two passes (rows, then column sums);
    # against the recomputing FP64 operator of the same build
    n = k = 16_400
    p = synth.c4(n=n, k=k)
    p.sketch_rows = 2 * k
    Ps = build_stored(p, 0, centers=np.arange(n))
    Pr = build(p, 0, centers=np.arange(n))
    V = T(np.random.default_rng(9).standard_normal((k, 1)))
    gs = Ps.operator(V).cpu().numpy()
    gr = Pr.operator(V).cpu().numpy()
    assert np.max(np.abs(gs - gr)) <= 1e-12 * np.max(np.abs(gr)), np.max(np.abs(gs - gr))


def test_stored_export_needs_stored_build():
    p = small(n=500, k=50)
    P = build(p, 0)
    with pytest.raises(B().KrrError):
        B().krill_export(P, 5, (500, 50), torch.float64)
