"""Restricted KRR and KRILL preconditioning (Sec. 2.2, Alg. 2), oracle side.

Readings where the paper leaves a choice:

* Centres are sampled uniformly without replacement (Sec. 2.2) as the k
  indices with the smallest keys sm(key(seed,2), i), ties broken by index,
  listed in ascending index order.
* eps_mach in the diagonal shift of Alg. 2 is 2**-52 (FP64 epsilon).
* zeta defaults to ceil(ln(k+1)) (natural log) and the sketch has d = 2k
  rows (Alg. 2 and Sec. 2.2.1).
* Sparse sign embedding (Sec. 2.2.1): column j draws candidate rows
  below(sm(sm(key(seed,3), j), t), d) for t = 0, 1, ... and keeps the first
  zeta distinct ones (rejection on collision, i.e. sampling without
  replacement); the sign of its q-th nonzero is the top bit of
  sm(sm(key(seed,4), j), q) (0 -> +1); values are +-zeta**-0.5.
"""
import math

import numpy as np
import scipy.sparse as sp
from scipy.linalg import solve_triangular

from . import kernels
from .rng import sm, key, below, sm_vec, TAG_CENTER, TAG_SKETCH_ROW, TAG_SKETCH_SIGN

EPS = 2.0 ** -52
MAX_CANDIDATES = 1 << 16


def default_zeta(k):
    return int(math.ceil(math.log(k + 1)))


def sample_centers(N, k, seed):
    """k distinct indices, uniform without replacement, ascending."""
    if not (0 < k <= N):
        raise ValueError("need 0 < k <= N")
    keys = sm_vec(key(seed, TAG_CENTER), np.arange(N, dtype=np.uint64))
    order = np.lexsort((np.arange(N), keys))  # by key, then by index
    return np.sort(order[:k])


def sketch_column(j, d_rows, zeta, seed):
    """(rows, signs) of column j of the sparse sign embedding."""
    kj = sm(key(seed, TAG_SKETCH_ROW), j)
    rows = []
    t = 0
    while len(rows) < zeta:
        if t >= MAX_CANDIDATES:
            raise RuntimeError("sparse sign column did not fill")
        r = below(sm(kj, t), d_rows)
        t += 1
        if r not in rows:
            rows.append(r)
    ks = sm(key(seed, TAG_SKETCH_SIGN), j)
    signs = [(-1.0 if (sm(ks, q) >> 63) else 1.0) for q in range(zeta)]
    return rows, signs


def sketch_columns(N, d_rows, zeta, seed):
    """Rows (N x zeta int) and signs (N x zeta +-1) for all columns.

    The first zeta candidates of every column are drawn at once; columns whose
    first zeta candidates collide are redone one by one with the rejection
    loop of ``sketch_column`` (identical results where there is no collision).
    """
    if not (0 < zeta <= d_rows < 2 ** 31):
        raise ValueError("need 0 < zeta <= d < 2**31")
    j = np.arange(N, dtype=np.uint64)
    kj = sm_vec(key(seed, TAG_SKETCH_ROW), j)
    ks = sm_vec(key(seed, TAG_SKETCH_SIGN), j)
    rows = np.empty((N, zeta), dtype=np.int64)
    signs = np.empty((N, zeta))
    for t in range(zeta):
        x = sm_vec(kj, np.uint64(t))
        # below(x, d) = floor(x * d / 2**64), exactly, in uint64: with
        # x = hi * 2**32 + lo it equals (hi*d + ((lo*d) >> 32)) >> 32 and no
        # intermediate reaches 2**64 while d < 2**31.
        hi = x >> np.uint64(32)
        lo = x & np.uint64(0xFFFFFFFF)
        dd = np.uint64(d_rows)
        rows[:, t] = ((hi * dd + ((lo * dd) >> np.uint64(32))) >> np.uint64(32)).astype(np.int64)
        s = sm_vec(ks, np.uint64(t))
        signs[:, t] = np.where((s >> np.uint64(63)) != 0, -1.0, 1.0)
    srt = np.sort(rows, axis=1)
    bad = np.nonzero(np.any(srt[:, 1:] == srt[:, :-1], axis=1))[0] if zeta > 1 else []
    for jj in bad:
        r, s = sketch_column(int(jj), d_rows, zeta, seed)
        rows[jj] = r
        signs[jj] = s
    return rows, signs


def sketch_matrix(N, d_rows, zeta, seed):
    """Phi as a scipy CSR matrix (d_rows x N)."""
    rows, signs = sketch_columns(N, d_rows, zeta, seed)
    cols = np.repeat(np.arange(N), zeta)
    vals = signs.reshape(-1) / math.sqrt(zeta)
    return sp.csr_matrix((vals, (rows.reshape(-1), cols)), shape=(d_rows, N))


class Krill:
    """KRILL preconditioned restricted KRR (Alg. 2)."""

    def __init__(self, X, kind, sigma, mu, centers, sketch_rows=None, zeta=None, seed=0,
                 phi=None):
        X = np.asarray(X, dtype=np.float64)
        self.X = X
        self.kind, self.sigma, self.mu = kind, float(sigma), float(mu)
        self.S = np.asarray(centers, dtype=np.int64)
        N, k = X.shape[0], self.S.shape[0]
        self.N, self.k = N, k
        Ass = kernels.block(X[self.S], X[self.S], kind, sigma)
        # Alg. 2 steps 1-2: H = mu A_SS + N eps tr(A_SS) I
        self.shift = N * EPS * float(np.trace(Ass))
        self.H = mu * Ass + self.shift * np.eye(k)
        if phi is None:
            d_rows = 2 * k if not sketch_rows else sketch_rows
            z = default_zeta(k) if not zeta else zeta
            phi = sketch_matrix(N, d_rows, z, seed)
        self.Phi = phi
        # A(:, S) held whole: the oracle runs at small N only
        self.AnS = kernels.block(X, X[self.S], kind, sigma)
        self.B = np.asarray(phi @ self.AnS)              # step 5
        self.P = self.B.T @ self.B + self.H              # step 6
        self.C = np.linalg.cholesky(self.P).T            # step 7, P = C^T C

    def rhs(self, y):
        """A(S,:) y (Alg. 2, last step)."""
        return self.AnS.T @ np.asarray(y, dtype=np.float64)

    def product(self, beta):
        """beta -> A(S,:)(A(:,S) beta) + H beta."""
        return self.AnS.T @ (self.AnS @ beta) + self.H @ beta

    def precondition(self, z):
        """z -> C^{-1} (C^{-T} z)."""
        w = solve_triangular(self.C, z, trans="T", lower=False)
        return solve_triangular(self.C, w, lower=False)

    def restricted_matrix(self):
        """M = A(S,:) A(:,S) + H, formed densely (pins only)."""
        return self.AnS.T @ self.AnS + self.H
