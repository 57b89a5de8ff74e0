"""Out-of-sample prediction (krr_predict) against the oracle's prediction
functions (Sec. 2, Sec. 2.2) on held-out points of the same distributions,
element by element, with the product tolerances of test_gpu_matvec
(FP64 1e-13, FP32 2e-5 Laplace / 3e-5 Gaussian of sum_j |K_ij| |beta_j|); SMAPE (Sec. 4.1) of the
GPU predictions against the oracle's SMAPE on the same coefficients."""
import numpy as np
import pytest
import torch

from oracle import kernels as OK
from oracle import predict as OP
import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL = {0: 1e-13, 1: 2e-5}


def B():
    from paper_2304_12465_amd import binding
    return binding


def T(a, dtype=np.float64):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to(DEV)


def check(got, Xt, Xc, beta, kind, sigma, prec):
    ref = OK.matvec(Xt, Xc, beta, kind, sigma)
    scale = np.abs(OK.block(Xt, Xc, kind, sigma)) @ np.abs(beta)
    err = np.abs(got - ref)
    t = 3e-5 if (kind == 0 and prec == 1) else TOL[prec]  # FP32 Gaussian: MFMA expansion
    assert np.all(err <= t * scale + 1e-300), float(np.max(err / (scale + 1e-300)))
    return ref


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("prec", [0, 1])
def test_full_data_prediction_matches_oracle(kind, prec):
    p = synth.c1(n=2000)
    if kind == 1:
        p.sigma = 8.0
    Xtr, Ytr, Xte, Yte = p.X[:1500], p.Y[:1500], p.X[1500:], p.Y[1500:]
    P = B().rpchol_build(kind, p.sigma, 0, T(Xtr), p.mu, 100, seed=p.algo_seed)
    beta, info = P.solve(T(Ytr), 1e-10, max_iter=600)
    assert info["converged"]
    bh = beta.cpu().numpy()
    got = P.predict(T(Xte), beta, prec=prec).cpu().numpy()
    ref = check(got, Xte, Xtr, bh, kind, p.sigma, prec)
    assert got.shape == (500, 1)
    s_gpu, s_ref = OP.smape(got, Yte), OP.smape(ref, Yte)
    assert abs(s_gpu - s_ref) <= (1e-10 if prec == 0 else 1e-3) * s_ref


def test_restricted_prediction_matches_oracle():
    p = synth.c4(n=3000, k=150)
    Xtr, Ytr, Xte = p.X[:2500], p.Y[:2500], p.X[2500:]
    P = B().krill_build(p.kind, p.sigma, 0, T(Xtr), p.mu, p.centers, sketch_rows=p.sketch_rows,
                        zeta=p.zeta, seed=p.algo_seed)
    beta, info = P.solve(T(Ytr), 1e-8, max_iter=300)
    S = np.array(P.pivots())
    bh = beta.cpu().numpy()
    for prec in (0, 1):
        got = P.predict(T(Xte), beta, prec=prec).cpu().numpy()
        check(got, Xte, Xtr[S], bh, p.kind, p.sigma, prec)
    ref = OP.predict_restricted(Xtr, S, bh, Xte, p.kind, p.sigma)
    np.testing.assert_allclose(P.predict(T(Xte), beta).cpu().numpy(), ref, rtol=1e-12,
                               atol=1e-13 * np.abs(bh).sum())


def test_multiple_rhs_and_empty_test_set():
    p = synth.c1(n=1200)
    g = np.random.default_rng(4)
    Y = np.hstack([p.Y, g.standard_normal((1200, 2))])
    P = B().rpchol_build(p.kind, p.sigma, 0, T(p.X[:1000]), p.mu, 80, seed=1, m_max=3)
    beta, _ = P.solve(T(Y[:1000]), 1e-9, max_iter=600)
    got = P.predict(T(p.X[1000:]), beta).cpu().numpy()
    check(got, p.X[1000:], p.X[:1000], beta.cpu().numpy(), p.kind, p.sigma, 0)
    empty = P.predict(torch.zeros((0, 8), dtype=torch.float64, device=DEV), beta)
    assert empty.shape == (0, 3)


def test_predict_invalid_arguments():
    b = B()
    p = synth.c1(n=400)
    P = b.rpchol_build(p.kind, p.sigma, 0, T(p.X), p.mu, 20, seed=1)
    beta = torch.zeros((400, 1), dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        P.predict(T(p.X[:10, :5]), beta)  # wrong d: refused before any launch
    with pytest.raises(ValueError):
        P.predict(T(p.X[:10]), beta[:300].contiguous())  # wrong number of coefficients
    with pytest.raises(b.KrrError):
        P.predict(T(p.X[:10]), beta, prec=7)
