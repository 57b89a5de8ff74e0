"""Parity of the fused kernel product (krr_kernel_matvec) against the FP64
oracle, element by element, with tolerances derived from the arithmetic:

* FP64 tiles: |W - W_ref| <= 1e-13 * sum_j |K_ij| |V_jc| + 1e-300.
* FP32 Laplace tiles sum |q_x - q_y| exactly over coordinates quantised to
  qbits = min(30, 32 - ceil(log2 dpad)) bits on the common range of both
  point sets, so each entry's exponent is off by at most
  dpad * range / ((2^qbits - 1) sigma) plus FP32 rounding of the sum, scale
  and exp (test_laplace_quantised_wide_range checks this bound directly).
* FP32 Gaussian tiles (f32 MFMA on centred points): each exponent carries at
  most (d + 3) 2^-24 s (max ||x||^2 + max ||y||^2) from the expansion, which
  the tile's routing guard keeps <= 200 * 2^-24 = 1.2e-5 (larger bounds take
  direct differences, |arg| (d + 2) 2^-24), plus 2 ulp of exp; V is rounded
  to FP32 (6e-8 relative) and at most 256 terms are summed in FP32 before
  the FP64 fold (<= 256 * 6e-8 relative to the partial sum of |terms|).
  The bounds used: FP32 Laplace tiles 2e-5 * sum_j |K_ij| |V_jc|; FP32
  Gaussian tiles 3e-5 (1.2e-5 expansion + 1.5e-5 FP32 sums + exp and V
  rounding).
"""
import numpy as np
import pytest
import torch

from oracle import kernels as OK
import synth

pytestmark = pytest.mark.gpu
TOL = {0: 1e-13, 1: 2e-5}
TOL_GAUSS32 = 3e-5


def tol(kind, prec):
    return TOL_GAUSS32 if (kind == 0 and prec == 1) else TOL[prec]


def B():
    from paper_2304_12465_amd import binding
    return binding


def run(kind, prec, Xr, Xc, V, sigma, shift=0.0):
    b = B()
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    Xr_t = t(Xr)
    Xc_t = Xr_t if Xc is Xr else t(Xc)
    W = b.kernel_matvec(kind, sigma, prec, Xr_t, Xc_t, t(V), shift=shift)
    torch.cuda.synchronize()
    return W.cpu().numpy()


def check(kind, prec, Xr, Xc, V, sigma, shift=0.0):
    W = run(kind, prec, Xr, Xc, V, sigma, shift)
    V2 = V if V.ndim == 2 else V[:, None]
    W2 = W if W.ndim == 2 else W[:, None]
    Kb = OK.block(Xr, Xc, kind, sigma)
    ref = Kb @ V2 + shift * V2 if shift else Kb @ V2
    scale = np.abs(Kb) @ np.abs(V2) + abs(shift) * np.abs(V2 if shift else 0)
    err = np.abs(W2 - ref)
    bound = tol(kind, prec) * scale + 1e-300
    worst = float(np.max(err / bound)) if err.size else 0.0
    assert np.all(err <= bound), f"worst err/bound = {worst}"
    return worst


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("d", [1, 3, 8, 12, 17, 20, 23, 32, 33, 64])
def test_square_with_shift(kind, prec, d):
    # padded dimensions 4 to 64; FP32 Gaussian tiles contract three bf16
    # slices per coordinate at 8, 16 (d = 12, four zero coordinates) and 32,
    # and FP32 products at the others
    g = np.random.default_rng(100 + d)
    n = 1337  # several 512-row workgroups and a ragged tail
    X = g.standard_normal((n, d))
    V = g.standard_normal(n)
    check(kind, prec, X, X, V, sigma=np.sqrt(d) * (1.0 if kind == 0 else 1.5), shift=0.37)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 8, 16, 17, 40])
def test_multiple_rhs(m):
    g = np.random.default_rng(7 + m)
    Xr = g.standard_normal((700, 16))
    Xc = g.standard_normal((2100, 16))
    V = g.standard_normal((2100, m))
    for kind in (0, 1):
        for prec in (0, 1):
            check(kind, prec, Xr, Xc, V, sigma=3.0)


@pytest.mark.parametrize("d", [3, 32, 64])
@pytest.mark.parametrize("m", [6, 8])
def test_gaussian_rhs_on_vector_units(d, m):
    # 5..8 right-hand sides: the FP64 Gaussian tile reduces E.V on the vector
    # units, the FP32 one on the matrix cores
    g = np.random.default_rng(300 + d + m)
    Xr = g.standard_normal((1100, d))
    Xc = g.standard_normal((1500, d))
    V = g.standard_normal((1500, m))
    for prec in (0, 1):
        check(0, prec, Xr, Xc, V, sigma=np.sqrt(d))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("sigma", [1e-8, 0.05, 0.4, 3.0, 1e3])
def test_gaussian_exponent_range(prec, sigma):
    # exponents from 0 (coincident points) down past the underflow threshold
    # (FP64: exp(-745) = 0): covers the table-driven exp's whole range, and
    # the small bandwidths route the MFMA jobs to the direct-difference tile
    g = np.random.default_rng(11)
    X = g.standard_normal((900, 6))
    X[100:150] = X[0]  # duplicates: exponent exactly 0 after centring
    V = g.standard_normal((900, 3))
    check(0, prec, X, X, V, sigma=sigma)
    check(0, prec, X, X, V[:, :1], sigma=sigma, shift=0.5)
    check(0, prec, X, X, np.hstack([V, V, V]), sigma=sigma)  # 9 rhs: E.V on the MFMA


def test_rectangular_shapes_and_edges():
    g = np.random.default_rng(3)
    # one row, many columns (many splits); many rows, one column
    for nr, nc in [(1, 5000), (4000, 1), (65, 129), (513, 257)]:
        Xr = g.standard_normal((nr, 5))
        Xc = g.standard_normal((nc, 5))
        V = g.standard_normal((nc, 2))
        for kind in (0, 1):
            check(kind, 0, Xr, Xc, V, sigma=2.0)
            check(kind, 1, Xr, Xc, V, sigma=2.0)


def test_empty_inputs():
    b = B()
    dev = torch.device("cuda:0")
    X = torch.zeros((0, 4), dtype=torch.float64, device=dev)
    Y = torch.randn((5, 4), dtype=torch.float64, device=dev)
    V0 = torch.zeros((0, 1), dtype=torch.float64, device=dev)
    W = b.kernel_matvec(0, 1.0, 0, Y, X, V0)   # nc = 0: W = 0
    torch.cuda.synchronize()
    assert torch.all(W == 0)
    W = b.kernel_matvec(0, 1.0, 0, X, Y, torch.ones((5, 1), dtype=torch.float64, device=dev))
    assert W.shape == (0, 1)


def test_identical_points_and_far_clusters_exact():
    # All-equal points give A = 11^T exactly; two far clusters give the rank-2
    # block matrix of the uniform-sampling failure example (Sec. 3.1).
    X = np.vstack([np.zeros((300, 6)), np.full((40, 6), 1e3)])
    V = np.arange(340.0)[:, None]
    for kind in (0, 1):
        for prec in (0, 1):
            W = run(kind, prec, X, X, V, 1.0)
            np.testing.assert_array_equal(W[:300, 0], np.full(300, V[:300].sum()))
            np.testing.assert_array_equal(W[300:, 0], np.full(40, V[300:].sum()))


def test_invalid_arguments_raise():
    b = B()
    dev = torch.device("cuda:0")
    X = torch.randn((10, 3), dtype=torch.float64, device=dev)
    V = torch.randn((10, 1), dtype=torch.float64, device=dev)
    with pytest.raises(b.KrrError):
        b.kernel_matvec(0, -1.0, 0, X, X, V)
    with pytest.raises(b.KrrError):
        b.kernel_matvec(0, 1.0, 0, X, X[:5].contiguous(), V[:5].contiguous(), shift=1.0)
    with pytest.raises(b.KrrError) as e:
        b.kernel_matvec(0, 1.0, 0, X, X, V, ws=b.workspace(16, dev))
    assert e.value.code == -2


@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_laplace_sampled_rows(prec):
    # The 100,000-point, d = 20 Laplace workload: the product over all columns
    # is checked on 192 sampled rows that the oracle computes one by one.
    p = synth.c2()
    g = np.random.default_rng(11)
    V = g.standard_normal((p.X.shape[0], 1))
    W = run(p.kind, prec, p.X, p.X, V, p.sigma, shift=p.mu)
    rows = np.sort(g.choice(p.X.shape[0], 192, replace=False))
    Kb = OK.block(p.X[rows], p.X, p.kind, p.sigma)
    ref = Kb @ V + p.mu * V[rows]
    scale = np.abs(Kb) @ np.abs(V) + p.mu * np.abs(V[rows])
    assert np.all(np.abs(W[rows] - ref) <= TOL[prec] * scale)


def mixed_tol(Xr, Xc, sigma):
    """Bound on |dW| / sum|K||V| for the bf16-split MFMA tiles.

    With centred points (radius R = max ||x - c||, c = mean of the columns)
    the split dot product misses lo.lo (<= 2^-16 |x||y|) and accumulates in
    FP32 (<= 3 d 2^-24 |x||y|), so each exponent is off by at most
    2 (2^-16 + 3 d 2^-24) R^2 / (2 sigma^2); the exponentiated entry and V
    are split again (2 x 2^-16) and at most 256 terms are summed in FP32.
    """
    c = Xc.mean(axis=0)
    R2 = max(np.max(np.sum((Xr - c) ** 2, axis=1)), np.max(np.sum((Xc - c) ** 2, axis=1)))
    d = Xr.shape[1]
    return 2 * (2 ** -16 + 3 * d * 2 ** -24) * R2 / (2 * sigma ** 2) + 3 * 2 ** -16 + 256 * 2 ** -24


def check_mixed(Xr, Xc, V, sigma, shift=0.0):
    W = run(0, 2, Xr, Xc, V, sigma, shift)
    Kb = OK.block(Xr, Xc, 0, sigma)
    ref = Kb @ V + (shift * V if shift else 0)
    scale = np.abs(Kb) @ np.abs(V) + (abs(shift) * np.abs(V) if shift else 0)
    tol = mixed_tol(Xr, Xc, sigma)
    err = np.abs(W - ref)
    assert np.all(err <= tol * scale + 1e-300), (np.max(err / scale), tol)
    return float(np.max(err / scale))


@pytest.mark.parametrize("d", [3, 8, 16, 20, 32, 33, 64])
def test_mixed_gaussian_square(d):
    g = np.random.default_rng(200 + d)
    n = 1337
    X = g.standard_normal((n, d))
    V = g.standard_normal((n, 1))
    check_mixed(X, X, V, np.sqrt(d), shift=0.37)


@pytest.mark.parametrize("m", [1, 3, 16, 17, 40])
def test_mixed_gaussian_rectangular_rhs(m):
    g = np.random.default_rng(300 + m)
    Xr = g.standard_normal((700, 24)) + 1.0
    Xc = g.standard_normal((2100, 24))
    V = g.standard_normal((2100, m))
    check_mixed(Xr, Xc, V, 4.0)


@pytest.mark.parametrize("d", [4, 20, 33])
def test_mixed_guard_routes_badly_scaled_jobs_to_direct_differences(d):
    # Tight clusters far apart: the centred norms are ~1e3 times s^-1, so the
    # split expansion's exponent error bound s (max||x||^2 + max||y||^2)
    # (3 2^-16 + (3 kp + 2) 2^-24) is far above the guard's 2^-9 and the
    # expansion would miss the within-cluster entries by percents.  The direct
    # tile on FP32 centred points keeps each exponent within
    # |arg| (d + 2) 2^-24 + 2 s ||x - y|| (||x|| + ||y||) 2^-24, V splits to
    # 2^-16 and at most 256 terms are summed in FP32.
    g = np.random.default_rng(400 + d)
    ncl, per = 12, 110
    centres = 40.0 * g.standard_normal((ncl, d))
    X = np.repeat(centres, per, axis=0) + 0.3 * g.standard_normal((ncl * per, d))
    Xc = X[::2].copy()
    V = g.standard_normal((Xc.shape[0], 3))
    sigma = 0.5
    s = 1.0 / (2 * sigma ** 2)
    c = Xc.mean(axis=0)
    R2 = max(np.sum((X - c) ** 2, axis=1).max(), np.sum((Xc - c) ** 2, axis=1).max())
    kp = 32 * ((d + 31) // 32)
    assert s * 2 * R2 * (3 * 2 ** -16 + (3 * kp + 2) * 2 ** -24) > 2 ** -9 * 100
    W = run(0, 2, X, Xc, V, sigma)
    Kb = OK.block(X, Xc, 0, sigma)
    ref = Kb @ V
    scale = np.abs(Kb) @ np.abs(V)
    # within-cluster distances ~ 0.3^2 * 2d, so |arg| <= s * 4 d (generous)
    expo = s * 4 * d * (d + 2) * 2 ** -24 + 2 * s * np.sqrt(4 * d * 0.09) * 2 * np.sqrt(R2) * 2 ** -24
    tol = expo + 4 * 2 ** -24 + 2 * 2 ** -16 + 256 * 2 ** -24
    err = np.abs(W - ref)
    assert np.all(err <= tol * scale + 1e-300), (np.max(err / (scale + 1e-300)), tol)
    # the expansion's own error would be orders larger: the tile did not use it
    assert tol < 1e-3


def test_mixed_laplace_is_fp32_tiles():
    g = np.random.default_rng(9)
    X = g.standard_normal((900, 12))
    V = g.standard_normal((900, 2))
    W2 = run(1, 2, X, X, V, 5.0)
    W1 = run(1, 1, X, X, V, 5.0)
    np.testing.assert_array_equal(W2, W1)


def test_mixed_full_size_uniform_sampled_rows():
    # 1,000,000 points in [0,1]^32 with near-duplicates, 8 right-hand sides:
    # 64 sampled rows against the oracle.
    p = synth.c3()
    g = np.random.default_rng(12)
    V = g.standard_normal((p.X.shape[0], 8))
    W = run(0, 2, p.X, p.X, V, p.sigma, shift=p.mu)
    rows = np.sort(g.choice(p.X.shape[0], 64, replace=False))
    Kb = OK.block(p.X[rows], p.X, 0, p.sigma)
    ref = Kb @ V + p.mu * V[rows]
    scale = np.abs(Kb) @ np.abs(V) + p.mu * np.abs(V[rows])
    tol = mixed_tol(p.X[rows], p.X, p.sigma)
    assert np.all(np.abs(W[rows] - ref) <= tol * scale), np.max(np.abs(W[rows] - ref) / scale)


@pytest.mark.parametrize("prec", [0, 1])
def test_gaussian_full_size_sampled_rows(prec):
    # The 10^12-entry d = 32, m = 8 product on the FP64 / FP32 MFMA tiles:
    # 48 sampled rows against the oracle at the product tolerances.
    p = synth.c3()
    g = np.random.default_rng(13)
    V = g.standard_normal((p.X.shape[0], 8))
    W = run(0, prec, p.X, p.X, V, p.sigma, shift=p.mu)
    rows = np.sort(g.choice(p.X.shape[0], 48, replace=False))
    Kb = OK.block(p.X[rows], p.X, 0, p.sigma)
    ref = Kb @ V + p.mu * V[rows]
    scale = np.abs(Kb) @ np.abs(V) + p.mu * np.abs(V[rows])
    err = np.abs(W[rows] - ref)
    assert np.all(err <= tol(0, prec) * scale), np.max(err / scale)


def test_laplace_quantised_wide_range():
    # Outliers stretch the quantisation range; the bound scales with it.
    g = np.random.default_rng(21)
    d = 20
    Xr = g.standard_normal((900, d))
    Xc = g.standard_normal((1500, d))
    Xc[:3] *= 400.0
    V = g.standard_normal((1500, 2))
    sigma = 30.0
    W = run(1, 1, Xr, Xc, V, sigma)
    Kb = OK.block(Xr, Xc, 1, sigma)
    ref = Kb @ V
    scale = np.abs(Kb) @ np.abs(V)
    rng_ = max(Xr.max(), Xc.max()) - min(Xr.min(), Xc.min())
    dpad, qbits = 20, 27
    delta = dpad * rng_ / ((2 ** qbits - 1) * sigma) + 4 * 2 ** -24
    tol = delta + 257 * 2 ** -24
    assert np.all(np.abs(W - ref) <= tol * scale), (np.max(np.abs(W - ref) / scale), tol)


def test_tile_timing_by_vector_count():
    # krr_timing_read_vectors: every recorded tile launch, and those of the
    # Gaussian matrix-core tile carrying exactly the given number of vectors
    # (the roofline's kernel); the record is cleared by the read
    b = B()
    g = np.random.default_rng(17)
    X = torch.from_numpy(g.standard_normal((3000, 16))).to("cuda:0")
    V1 = torch.from_numpy(g.standard_normal((3000, 1))).to("cuda:0")
    V2 = torch.from_numpy(g.standard_normal((3000, 2))).to("cuda:0")
    b.kernel_matvec(0, 4.0, b.FP64, X, X, V1)
    torch.cuda.synchronize()
    b.timing_read()
    b.timing_enable(True)
    for _ in range(3):
        b.kernel_matvec(0, 4.0, b.FP64, X, X, V1)
    for _ in range(2):
        b.kernel_matvec(0, 4.0, b.FP64, X, X, V2)
    b.kernel_matvec(1, 4.0, b.FP64, X, X, V1)  # Laplace: another tile, no vector tag
    torch.cuda.synchronize()
    b.timing_enable(False)
    ms, n, ms1, n1 = b.timing_read_vectors(1)
    assert n == 6 and n1 == 3, (n, n1)
    assert 0.0 < ms1 < ms
    assert b.timing_read() == (0.0, 0)
    with pytest.raises(b.KrrError):
        b.timing_read_vectors(-1)
