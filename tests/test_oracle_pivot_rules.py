"""Pins of the oracle's uniform and greedy pivot rules (Sec. 3.1's
alternatives to RPCholesky), run through the block loop of Alg. 3.

* The rank-2 block matrix of the uniform-sampling failure mode: greedy and
  RPCholesky recover it exactly with two pivots; uniform sampling of r
  indices misses the small block with the hypergeometric probability
  C(N - n2, r) / C(N, r).
* The matrix of the greedy failure mode, 1 1^T + blockdiag((1/2N) 1 1^T,
  (1/N) I): greedy takes every index of the identity block before any other
  (its residual diagonal stays the largest); RPCholesky and uniform sampling
  reach the large block at once.
* Greedy equals textbook Cholesky with diagonal pivoting written out here
  (pivot sequence and the Nystrom approximation).
* Uniform with B = 1 draws distinct indices, and with r = N reproduces A.
"""
from math import comb

import numpy as np
import pytest

from oracle import kernels as K
from oracle import rpcholesky as RP

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def run(A, r, rule, seed=0, B=None, record=None):
    return RP.nystrom_columns(np.diag(A).copy(), lambda S: A[:, S], r, B=B, seed=seed,
                              record=record, rule=rule)


def rank2_block(N, n2):
    A = np.zeros((N, N))
    A[:N - n2, :N - n2] = 1.0
    A[N - n2:, N - n2:] = 1.0
    return A


def greedy_trap(N, n2):
    A = np.ones((N, N))
    A[:N - n2, :N - n2] += 1.0 / (2 * N)
    A[N - n2:, N - n2:] += np.eye(n2) / N
    return A


def test_rank2_block_greedy_and_rpcholesky_recover_with_two_pivots():
    N, n2 = 1000, 10
    A = rank2_block(N, n2)
    F, piv = run(A, 2, "greedy")
    assert piv == [0, N - n2]  # first maximum, then the only nonzero block
    assert np.max(np.abs(F @ F.T - A)) <= 1e-15
    for seed in range(20):
        F, piv = run(A, 2, "rpcholesky", seed=seed, B=1)
        assert sorted(p >= N - n2 for p in piv) == [False, True]
        assert np.max(np.abs(F @ F.T - A)) <= 1e-15


def test_rank2_block_uniform_misses_the_small_block_hypergeometrically():
    N, n2, r, runs = 1000, 10, 10, 300
    A = rank2_block(N, n2)
    miss = 0
    for seed in range(runs):
        rec = []
        F, piv = run(A, r, "uniform", seed=seed, B=1, record=rec)
        drawn = [x for blk in rec for x in blk["drawn"]]
        assert len(set(drawn)) == len(drawn) <= r
        hit = any(x >= N - n2 for x in drawn)
        # the loop stops early only once the matrix is exhausted
        assert len(drawn) == r or hit
        assert hit == any(p >= N - n2 for p in piv)
        # the approximation is exact exactly when both blocks were drawn
        err = np.max(np.abs(F @ F.T - A))
        assert (err <= 1e-15) == hit
        miss += not hit
    p = comb(N - n2, r) / comb(N, r)  # 0.904
    assert abs(miss / runs - p) <= 4 * np.sqrt(p * (1 - p) / runs)


def test_greedy_trap_greedy_takes_the_identity_block_first():
    N, n2 = 1000, 100
    A = greedy_trap(N, n2)
    F, piv = run(A, n2, "greedy")
    assert sorted(piv) == list(range(N - n2, N))
    # the residual still carries the whole rank-one part of the large block
    d = np.diag(A - F @ F.T)[:N - n2]
    assert np.all(d > 1.0 / (2 * N))
    # one more greedy pivot finally reaches the large block
    _, piv2 = run(A, n2 + 1, "greedy")
    assert piv2[:n2] == piv and piv2[n2] < N - n2
    for seed in range(10):
        _, pr = run(A, 3, "rpcholesky", seed=seed, B=1)
        _, pu = run(A, 3, "uniform", seed=seed, B=1)
        assert min(pr) < N - n2 and min(pu) < N - n2


def textbook_diagonal_pivoting(A, r):
    """Partial Cholesky with diagonal pivoting, outer-product form."""
    R = A.copy()
    L = np.zeros((A.shape[0], r))
    piv = []
    for k in range(r):
        j = int(np.argmax(np.diag(R)))
        piv.append(j)
        L[:, k] = R[:, j] / np.sqrt(R[j, j])
        R = R - np.outer(L[:, k], L[:, k])
    return L, piv


@pytest.mark.parametrize("kind", [K.GAUSSIAN, K.LAPLACE])
def test_greedy_equals_diagonal_pivoting(kind):
    g = np.random.default_rng(4)
    X = g.standard_normal((300, 5))
    A = K.block(X, X, kind, 2.0)
    L, piv_ref = textbook_diagonal_pivoting(A, 40)
    F, piv = RP.rpcholesky(X, kind, 2.0, 40, rule="greedy")
    assert piv == piv_ref
    assert np.max(np.abs(F @ F.T - L @ L.T)) <= 1e-12


def test_uniform_without_replacement_reproduces_a_full_rank_matrix():
    g = np.random.default_rng(5)
    X = g.standard_normal((60, 4))
    A = K.block(X, X, K.GAUSSIAN, 1.0)
    rec = []
    F, piv = RP.rpcholesky(X, K.GAUSSIAN, 1.0, 60, B=1, seed=9, rule="uniform", record=rec)
    drawn = [x for blk in rec for x in blk["drawn"]]
    assert sorted(drawn) == list(range(60))
    assert np.max(np.abs(F @ F.T - A)) <= 1e-10


def test_uniform_blocks_budget_distinct_draws():
    g = np.random.default_rng(6)
    X = g.standard_normal((500, 3))
    rec = []
    F, piv = RP.rpcholesky(X, K.GAUSSIAN, 0.3, 120, B=25, seed=2, rule="uniform", record=rec)
    drawn = [sorted(set(blk["drawn"])) for blk in rec]
    flat = [x for blk in drawn for x in blk]
    assert len(flat) == 120 and len(set(flat)) == 120  # no index drawn twice across blocks
    assert set(piv) <= set(flat)


def test_unknown_rule_rejected():
    with pytest.raises(ValueError):
        RP.nystrom_columns(np.ones(3), lambda S: np.eye(3)[:, S], 2, rule="leverage")
