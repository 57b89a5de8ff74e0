"""The uniform and greedy pivot rules (Sec. 3.1) on the GPU against the
oracle's block loop with the same rule.

* pivots: bit-exact.  Uniform draws use integer pool weights, whose prefix
  sums are exact on both sides; greedy compares residual diagonals that
  agree to ~1e-16 between the two sides, and the workloads here have no
  maxima that close (the rank-2 matrix's ties are exact on both sides).
* F: ||dF||_F / ||F||_F <= 100 r eps kappa(A(S,S)), as for RPCholesky.
* solves: PCG on the rule's preconditioner reaches tol, with the oracle's
  PCG on the oracle's factor of the same rule within one iteration (FP64).
"""
import numpy as np
import pytest
import torch

from oracle import kernels as OK
from oracle import rpcholesky as ORP
from oracle import pcg as OPCG
import synth

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -52
DEV = torch.device("cuda:0")
RULES = {"uniform": 1, "greedy": 2, "rpcholesky": 0}


def B():
    from paper_2304_12465_amd import binding
    return binding


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def build(X, kind, sigma, mu, r, rule, B_=0, seed=0, prec=0):
    return B().nystrom_build(kind, sigma, prec, T(X), mu, r, RULES[rule], B=B_, seed=seed)


@pytest.mark.parametrize("rule", ["uniform", "greedy"])
@pytest.mark.parametrize("kind", [0, 1])
def test_pivots_and_factor_match_oracle(rule, kind):
    p = synth.c2(n=3_000)
    sigma = p.sigma if kind == 1 else 6.0
    r, B_ = 150, 16
    P = build(p.X, kind, sigma, p.mu, r, rule, B_=B_, seed=21)
    F_o, piv_o = ORP.rpcholesky(p.X, kind, sigma, r, B=B_, seed=21, rule=rule)
    assert P.pivots() == piv_o
    F = P.factor().cpu().numpy().T
    S = np.array(piv_o)
    kap = np.linalg.cond(OK.block(p.X[S], p.X[S], kind, sigma))
    rel = np.linalg.norm(F - F_o) / np.linalg.norm(F_o)
    assert rel <= 100 * len(S) * EPS * kap, (rel, kap)


def test_rank2_block_matrix():
    # two far-apart clusters of identical points: the kernel matrix is the
    # rank-2 block matrix of the uniform-sampling failure example
    N, n2 = 1000, 10
    X = np.zeros((N, 2))
    X[N - n2:, 0] = 1000.0
    P = build(X, 0, 1.0, 1e-3, 2, "greedy")
    assert P.pivots() == [0, N - n2]
    P = build(X, 0, 1.0, 1e-3, 5, "greedy")  # stops once the residual is exhausted
    assert P.dims()[0] == 2
    for seed in range(4):
        P = build(X, 0, 1.0, 1e-3, 2, "rpcholesky", B_=1, seed=seed)
        assert sorted(q >= N - n2 for q in P.pivots()) == [False, True]
    misses = 0
    for seed in range(20):
        P = build(X, 0, 1.0, 1e-3, 10, "uniform", B_=1, seed=seed)
        _, piv_o = ORP.rpcholesky(X, 0, 1.0, 10, B=1, seed=seed, rule="uniform")
        assert P.pivots() == piv_o
        misses += all(q < N - n2 for q in piv_o)
    assert misses >= 10  # expected 0.904 * 20


@pytest.mark.parametrize("rule", ["uniform", "greedy"])
def test_solve_with_rule(rule):
    p = synth.c2(n=3_000)
    r = 200
    P = build(p.X, p.kind, p.sigma, p.mu, r, rule, seed=3)
    F_o, piv_o = ORP.rpcholesky(p.X, p.kind, p.sigma, r, seed=3, rule=rule)
    assert P.pivots() == piv_o
    beta, info = P.solve(T(p.Y), 1e-8, max_iter=600)
    assert info["converged"] and info["relres_true"] <= 1e-7
    Pc = ORP.NystromPreconditioner(F_o, p.mu)
    A = OK.block(p.X, p.X, p.kind, p.sigma)
    xo, io = OPCG.pcg(lambda V: A @ V + p.mu * V, Pc.apply, p.Y, 1e-8, 600)
    assert abs(info["iters"] - int(io["iters"][0])) <= 1
    fit, fit_o = A @ beta.cpu().numpy(), A @ xo
    assert np.linalg.norm(fit - fit_o) / np.linalg.norm(fit_o) <= 1e-6


def test_unknown_rule_rejected():
    b = B()
    X = T(np.zeros((10, 2)))
    ws = b.workspace(b.rpchol_ws(0, 0, 10, 2, 2, 0, 1), X.device)
    with pytest.raises(b.KrrError):
        b.nystrom_build(0, 1.0, 0, X, 1e-3, 2, 7, ws=ws)


@pytest.mark.parametrize("rule", ["uniform", "greedy"])
def test_full_rank_and_ragged_blocks(rule):
    # r = N: every index is drawn (uniform) or the residual is exhausted
    # (greedy); F F^T reproduces A, and the pivots equal the oracle's.  B = 7
    # leaves a ragged last block.
    # (a narrow bandwidth keeps A well conditioned, so no residual diagonal
    # sits near the drop threshold and greedy's maxima are well separated)
    g = np.random.default_rng(31)
    X = g.standard_normal((150, 3))
    P = build(X, 0, 0.3, 1e-2, 150, rule, B_=7, seed=4)
    F_o, piv_o = ORP.rpcholesky(X, 0, 0.3, 150, B=7, seed=4, rule=rule)
    assert P.pivots() == piv_o
    F = P.factor().cpu().numpy().T
    A = OK.block(X, X, 0, 0.3)
    assert np.max(np.abs(F @ F.T - A)) <= 1e-8
    if rule == "uniform":
        assert len(set(piv_o)) == len(piv_o)


def test_invalid_rank_rejected():
    b = B()
    X = T(np.random.default_rng(0).standard_normal((20, 2)))
    for r in (0, 21):
        with pytest.raises(b.KrrError):
            b.nystrom_build(0, 1.0, 0, X, 1e-3, r, RULES["greedy"],
                            ws=b.workspace(1 << 20, X.device))
