"""Seeded synthetic workloads shaped like the paper's experiments.

This module holds only input generation (points, targets, request streams);
none of the method's arithmetic lives here.  Both the FP64 oracle (in tests)
and the GPU library consume these arrays.  The paper's datasets (Table 1,
QM9 and SUSY of Sec. 4) are not available; the shapes below stand in for
them:

* ``c1`` full-data, Gaussian, N=2,000, d=8 (small dense-checkable case);
* ``c2`` full-data, l1 Laplace, N=100,000, d=20 (QM9-sized N, Sec. 4.1);
* ``c3`` full-data, Gaussian, N=1,000,000, d=32, 8 right-hand sides, with
  5% near-duplicate points (an ill-conditioned kernel matrix);
* ``c4`` restricted, Gaussian sigma=4, N=2,000,000, d=16, k=10,000 centres
  (SUSY-like restricted setting of Sec. 4.2);
* ``c5`` a served stream of 256 mixed solves with Poisson arrivals.

Every generator takes an explicit ``n`` so tests can draw the same
distribution at reduced size.  Data seeds are 1000 + config number.
"""
import math
from dataclasses import dataclass, field

import numpy as np

GAUSSIAN = 0
LAPLACE = 1


@dataclass
class Problem:
    name: str
    X: np.ndarray          # N x d, float64
    Y: np.ndarray          # N x m, float64
    kind: int
    sigma: float
    mu: float
    rank: int = 0          # RPCholesky rank r (full-data)
    centers: int = 0       # k (restricted)
    sketch_rows: int = 0
    zeta: int = 0
    tol: float = 1e-6
    algo_seed: int = 0
    extra: dict = field(default_factory=dict)


def c1(n=2000, seed=1001):
    """x ~ N(0, I_8); y = sin(sum x) + 0.1 N(0,1); Gaussian sigma = sqrt(8)."""
    g = np.random.default_rng(seed)
    d = 8
    X = g.standard_normal((n, d))
    y = np.sin(X.sum(axis=1)) + 0.1 * g.standard_normal(n)
    return Problem("c1", X, y[:, None], GAUSSIAN, math.sqrt(d), 1e-3,
                   rank=min(100, n), tol=1e-10, algo_seed=2001)


def c2(n=100_000, seed=1002):
    """10-component Gaussian mixture in d=20 (means ~ N(0, 4I), unit
    covariance, equal weights); y = ||x||_1 mod 3 + 0.05 N(0,1); l1 Laplace
    kernel with sigma = d; mu = 1e-4 N; rank 1000."""
    g = np.random.default_rng(seed)
    d = 20
    means = 2.0 * g.standard_normal((10, d))
    comp = g.integers(0, 10, size=n)
    X = means[comp] + g.standard_normal((n, d))
    y = np.mod(np.abs(X).sum(axis=1), 3.0) + 0.05 * g.standard_normal(n)
    return Problem("c2", X, y[:, None], LAPLACE, float(d), 1e-4 * n,
                   rank=min(1000, n), tol=1e-6, algo_seed=2002)


def c2_test(m=30_000, seed=1002, test_seed=3002):
    """Held-out points of the c2 distribution (the same mixture means, drawn
    from `seed` as c2 does, then m fresh points and targets from
    `test_seed`): the 10^5 / 3 x 10^4 train / test split of Sec. 4.1."""
    means = 2.0 * np.random.default_rng(seed).standard_normal((10, 20))
    g = np.random.default_rng(test_seed)
    comp = g.integers(0, 10, size=m)
    X = means[comp] + g.standard_normal((m, 20))
    y = np.mod(np.abs(X).sum(axis=1), 3.0) + 0.05 * g.standard_normal(m)
    return X, y[:, None]


def c3(n=1_000_000, seed=1003, m=8):
    """Uniform [0,1]^32 with 5% near-duplicates (copies of uniformly chosen
    points plus N(0, 1e-12 I) jitter); m smooth targets
    y_c = sin(w_c . x + phi_c); Gaussian sigma = 1.5; mu = 1e-6 N; rank 2000."""
    g = np.random.default_rng(seed)
    d = 32
    X = g.random((n, d))
    ndup = int(0.05 * n)
    if ndup > 0:
        dst = g.choice(n, size=ndup, replace=False)
        src = g.integers(0, n, size=ndup)
        X[dst] = X[src] + 1e-6 * g.standard_normal((ndup, d))
    W = g.standard_normal((d, m))
    ph = g.random(m) * 2.0 * math.pi
    Y = np.sin(X @ W + ph)
    return Problem("c3", X, Y, GAUSSIAN, 1.5, 1e-6 * n, rank=min(2000, n), tol=1e-6,
                   algo_seed=2003)


def c4(n=2_000_000, seed=1004, k=10_000, d=16):
    """x ~ N(0, I_d) (d = 16) with dimension j scaled by 1/(1+j); labels
    y = sign(sin(sum x)); Gaussian sigma = 4; mu = 1e-5 N; k uniform centres,
    sketch 2k rows, 8 nonzeros per column.  Other d draw the same recipe in
    more dimensions (the stored-block comparison)."""
    g = np.random.default_rng(seed)
    X = g.standard_normal((n, d)) / (1.0 + np.arange(d))[None, :]
    s = np.sin(X.sum(axis=1))
    y = np.where(s >= 0, 1.0, -1.0)
    k = min(k, n)
    return Problem("c4", X, y[:, None], GAUSSIAN, 4.0, 1e-5 * n, centers=k,
                   sketch_rows=2 * k, zeta=8, tol=1e-6, algo_seed=2004)


@dataclass
class Request:
    rid: int
    arrival: float
    n: int
    d: int
    kind: int
    m: int
    rank: int
    seed: int


def c5_stream(count=256, rate=20.0, n_lo=10_000, n_hi=300_000, seed=1005):
    """Served stream: Poisson arrivals (exponential gaps, mean 1/rate),
    N log-uniform in [n_lo, n_hi], d in {8,16,32}, Gaussian or Laplace
    50/50, 1..16 right-hand sides, rank min(1000, N/50)."""
    g = np.random.default_rng(seed)
    t = np.cumsum(g.exponential(1.0 / rate, size=count))
    reqs = []
    for i in range(count):
        n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        d = int(g.choice([8, 16, 32]))
        kind = int(g.integers(0, 2))
        m = int(g.integers(1, 17))
        reqs.append(Request(i, float(t[i]), n, d, kind, m, min(1000, n // 50), 5000 + i))
    return reqs


def c5_problem(req: Request):
    """Points and targets of one served request (mixture features as c2)."""
    g = np.random.default_rng(req.seed)
    means = 2.0 * g.standard_normal((10, req.d))
    comp = g.integers(0, 10, size=req.n)
    X = means[comp] + g.standard_normal((req.n, req.d))
    W = g.standard_normal((req.d, req.m)) / math.sqrt(req.d)
    Y = np.sin(X @ W) + 0.05 * g.standard_normal((req.n, req.m))
    sigma = math.sqrt(req.d) if req.kind == GAUSSIAN else float(req.d)
    return Problem(f"c5-{req.rid}", X, Y, req.kind, sigma, 1e-4 * req.n, rank=req.rank,
                   tol=1e-6, algo_seed=req.seed)
