"""Blocked RPCholesky (Appendix A, Alg. 3) and the Nystrom preconditioner of
Alg. 1, oracle side, FP64.

Readings where the paper leaves a choice (each is restated in the design
notes, and the GPU library implements the same rules independently):

* Draws (Alg. 3, "sample i.i.d. indices ~ d / Sum(d)") are with replacement.
  Draw t of block b uses u = u53(sm(sm(key(seed,1), b), t)) and picks the
  smallest index i whose inclusive prefix sum c_i exceeds t = u * T.  Prefix
  sums are taken in a FIXED order so that both sides round identically:
  chunks of 1024 entries are summed left to right from 0 (chunk totals S_c),
  chunk offsets are a left-to-right running sum O_0 = 0, O_{c+1} = O_c + S_c,
  T = O_last, and c_i = O_c + p_i where p_i is the left-to-right running sum
  inside i's chunk.  If no c_i exceeds t (t rounded up to T), the last index
  with d_i > 0 is taken.
* Unique (Alg. 3) returns the distinct draws in ascending index order.
* The small Cholesky of G(S', S') proceeds pivot by pivot in that order; a
  pivot whose Schur complement diagonal is <= eps * tr(A) (eps = 2**-52) is
  dropped: it creates no column of F.  Only accepted pivots join S.
* After each block the residual diagonal of every drawn index is set to 0
  (its exact value) and d is clamped at 0 (rounding can leave -1e-16).
* The loop stops early when T <= eps * tr(A) (the matrix is exhausted;
  exact recovery, Sec. 5.1).

Two other pivot rules that Sec. 3.1 sets against RPCholesky (its failure
modes of uniform sampling and of greedy selection) run through the same
block loop, differing only in how a block's pivots are chosen:

* uniform: the block's draws are i.i.d. uniform over the indices never
  drawn before -- the same fixed-order prefix rule and random stream as
  above, applied to the weights w_i = 1 (never drawn) / 0 (drawn) instead
  of d; every drawn index (accepted or dropped) leaves the pool.  The rank
  r budgets the distinct indices drawn (r columns sampled uniformly, as the
  Nystrom approximation A(:,S) A(S,S)^+ A(S,:) takes them; dependent ones
  are dropped), not the accepted pivots.  With B = 1 this is uniform
  sampling of r indices without replacement.
* greedy: one pivot per block (B is ignored), the index of the largest
  residual diagonal entry (smallest index among equal maxima); the loop
  also stops when that entry is <= eps * tr(A), since no further pivot
  could be accepted.
"""
import numpy as np
from scipy.linalg import solve_triangular

from . import kernels
from .rng import sm, key, u53, TAG_PIVOT

EPS = 2.0 ** -52
CHUNK = 1024


def default_block(r):
    """Block size B = min(100, ceil(r/10)) (Alg. 1, first step)."""
    return min(100, -(-r // 10))


def prefix_tables(d):
    """Chunk offsets O (len nchunks+1) in the fixed summation order above."""
    d = np.asarray(d, dtype=np.float64)
    n = d.shape[0]
    nch = -(-n // CHUNK)
    S = np.empty(nch)
    for c in range(nch):
        S[c] = np.cumsum(d[c * CHUNK:(c + 1) * CHUNK])[-1]
    O = np.zeros(nch + 1)
    O[1:] = np.cumsum(S)
    return O


def sample_index(d, O, u):
    """One draw ~ d / sum(d) with the fixed-order prefix rule."""
    T = O[-1]
    t = u * T
    nch = O.shape[0] - 1
    c = int(np.searchsorted(O[1:], t, side="right"))
    if c >= nch:
        nz = np.nonzero(np.asarray(d) > 0)[0]
        return int(nz[-1])
    p = np.cumsum(d[c * CHUNK:(c + 1) * CHUNK])
    vals = O[c] + p
    i = int(np.searchsorted(vals, t, side="right"))
    return c * CHUNK + i


def draw_block(d, seed, b, count):
    O = prefix_tables(d)
    kb = sm(key(seed, TAG_PIVOT), b)
    return [sample_index(d, O, u53(sm(kb, t))) for t in range(count)]


def chol_drop(Gss, thresh):
    """Upper Cholesky of Gss = R^T R pivot by pivot, dropping weak pivots.

    Returns (R restricted to accepted pivots, list of accepted positions).
    """
    n = Gss.shape[0]
    R = np.zeros((n, n))
    acc = []
    for q in range(n):
        s = Gss[q, q] - sum(R[p, q] ** 2 for p in acc)
        if s <= thresh:
            continue
        rqq = np.sqrt(s)
        R[q, q] = rqq
        for q2 in range(q + 1, n):
            R[q, q2] = (Gss[q, q2] - sum(R[p, q] * R[p, q2] for p in acc)) / rqq
        acc.append(q)
    return R[np.ix_(acc, acc)], acc


RULES = ("rpcholesky", "uniform", "greedy")


def select_block(rule, d, pool, seed, b, count):
    """The draws of block b under ``rule``: ``count`` i.i.d. draws ~ d
    (RPCholesky) or ~ pool (uniform over the indices never drawn), or the
    single index of the largest residual diagonal entry (greedy)."""
    if rule == "greedy":
        return [int(np.argmax(d))]  # first index of the maximum
    if rule == "uniform":
        return draw_block(pool, seed, b, count)
    return draw_block(d, seed, b, count)


def rpcholesky(X, kind, sigma, r, B=None, seed=0, record=None, rule="rpcholesky"):
    """Blocked RPCholesky, Alg. 3: returns (F, pivots) with F F^T ~ A.

    ``record`` (optional list) receives per block: dict(T=..., drawn=...,
    accepted=...), used by invariant tests.  ``rule`` selects the pivot rule
    (RULES; see the module notes).
    """
    X = np.asarray(X, dtype=np.float64)
    return nystrom_columns(kernels.diag(X, kind, sigma),
                           lambda S: kernels.block(X, X[S], kind, sigma),
                           r, B=B, seed=seed, record=record, rule=rule)


def nystrom_columns(diag, columns, r, B=None, seed=0, record=None, rule="rpcholesky"):
    """The block loop of Alg. 3 on a PSD matrix A given by its diagonal
    (length N) and ``columns(S)`` -> A(:, S) (N x len(S)); returns (F, pivots).
    """
    if rule not in RULES:
        raise ValueError(f"unknown pivot rule {rule!r}")
    d = np.array(diag, dtype=np.float64)
    N = d.shape[0]
    if B is None or B <= 0:
        B = default_block(r)
    if rule == "greedy":
        B = 1
    F = np.zeros((N, r))
    trA = float(np.sum(d))
    thresh = EPS * trA
    pool = np.ones(N)  # uniform rule: 1 for indices never drawn
    pivots = []
    i = 0
    ndrawn = 0  # uniform rule: distinct indices drawn so far
    b = 0
    while (ndrawn if rule == "uniform" else i) < r and b <= N:
        O = prefix_tables(d)
        stop = O[-1] <= thresh
        if rule == "greedy":
            stop = stop or np.max(d) <= thresh
        elif rule == "uniform":
            stop = stop or not pool.any()
        if stop:
            if record is not None:
                record.append(dict(T=float(O[-1]), drawn=[], accepted=[]))
            break
        count = min(B, r - (ndrawn if rule == "uniform" else i))
        draws = select_block(rule, d, pool, seed, b, count)
        Sp = sorted(set(draws))
        pool[Sp] = 0.0
        ndrawn += len(Sp)
        G = columns(Sp) - F[:, :i] @ F[Sp, :i].T
        R, acc = chol_drop(G[Sp, :], thresh)
        if acc:
            Gacc = G[:, acc]
            # F_new R = G_acc  ->  R^T F_new^T = G_acc^T
            Fnew = solve_triangular(R, Gacc.T, trans="T", lower=False).T
            F[:, i:i + len(acc)] = Fnew
            d = d - np.sum(Fnew * Fnew, axis=1)
        d[Sp] = 0.0
        d = np.maximum(d, 0.0)
        accepted = [Sp[q] for q in acc]
        pivots.extend(accepted)
        if record is not None:
            record.append(dict(T=float(O[-1]), drawn=list(draws), accepted=accepted))
        i += len(acc)
        b += 1
    return F[:, :i], pivots


class NystromPreconditioner:
    """P^{-1} for P = F F^T + mu I in the SVD form of Alg. 1.

    With F = U Sigma V^T (economy SVD),
    P^{-1} z = U [(Sigma^2 + mu I)^{-1} - mu^{-1} I] U^T z + mu^{-1} z.
    """

    def __init__(self, F, mu):
        self.mu = float(mu)
        if F.shape[1] == 0:
            self.U = np.zeros((F.shape[0], 0))
            self.s2 = np.zeros(0)
        else:
            U, s, _ = np.linalg.svd(F, full_matrices=False)
            self.U = U
            self.s2 = s * s

    def apply(self, Z):
        Z = np.asarray(Z, dtype=np.float64)
        squeeze = Z.ndim == 1
        Z2 = Z[:, None] if squeeze else Z
        coef = 1.0 / (self.s2 + self.mu) - 1.0 / self.mu
        out = self.U @ (coef[:, None] * (self.U.T @ Z2)) + Z2 / self.mu
        return out[:, 0] if squeeze else out
