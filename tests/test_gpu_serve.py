"""Stepped solves and the served stream on the GPU: every request's result
is bitwise identical alone and in the mix (each product keeps its own tile
decomposition whatever shares the launch), a failing request does not
disturb the others, and a small served stream completes."""
import numpy as np
import pytest
import torch

import synth
from oracle import kernels as OK
from paper_2304_12465_amd.serve import Server, GpuBackend, summarize

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def B():
    from paper_2304_12465_amd import binding
    return binding


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def problems():
    out = []
    specs = [(3000, 8, 0, 3, 2), (5200, 16, 1, 1, 1), (4100, 32, 0, 5, 2), (2500, 16, 1, 16, 1)]
    for i, (n, d, kind, m, prec) in enumerate(specs):
        req = synth.Request(i, 0.0, n, d, kind, m, min(200, n // 20), 7000 + i)
        p = synth.c5_problem(req)
        out.append((p, prec))
    return out


def build(p, prec):
    return B().rpchol_build(p.kind, p.sigma, prec, T(p.X), p.mu, p.rank, seed=p.algo_seed,
                            m_max=p.Y.shape[1])


def test_alone_equals_in_the_mix_bitwise():
    probs = problems()
    alone = []
    for p, prec in probs:
        P = build(p, prec)
        beta, info = P.solve(T(p.Y), 1e-8, 400)
        alone.append((beta.cpu().numpy(), info["iters"]))
    Ps = [build(p, prec) for p, prec in probs]
    Ss = [B().Solve(P, T(p.Y), 1e-8, 400) for P, (p, _) in zip(Ps, probs)]
    live = list(Ss)
    while live:
        st = B().solve_step(live)
        live = [s for s, v in zip(live, st) if v == 0]
    for S, (ba, ia) in zip(Ss, alone):
        beta, info = S.end()
        assert info["iters"] == ia
        assert np.array_equal(beta.cpu().numpy(), ba)


def test_fp64_requests_carrying_x_alone_equal_in_the_mix():
    # FP64 requests above the burst size: each carries x beside p in the step
    # predicted to converge (its products then give the exit check), on its
    # own schedule; stepped together their products share launches.  Every
    # request's solution, iteration count, product count and true residual
    # are bitwise those it gets alone.
    specs = [(5000, 8, 0, 1), (6000, 16, 0, 3), (4500, 16, 1, 2)]
    probs = []
    for i, (n, d, kind, m) in enumerate(specs):
        req = synth.Request(i, 0.0, n, d, kind, m, min(200, n // 20), 7100 + i)
        probs.append(synth.c5_problem(req))
    alone = []
    for p in probs:
        P = build(p, 0)
        beta, info = P.solve(T(p.Y), 1e-8, 400)
        assert info["converged"] and info["products"] <= info["iters"] + 1, info
        alone.append((beta.cpu().numpy(), info))
    Ps = [build(p, 0) for p in probs]
    Ss = [B().Solve(P, T(p.Y), 1e-8, 400) for P, p in zip(Ps, probs)]
    live = list(Ss)
    while live:
        st = B().solve_step(live)
        live = [s for s, v in zip(live, st) if v == 0]
    for S, (ba, ia) in zip(Ss, alone):
        beta, info = S.end()
        for key in ("iters", "products", "relres_true", "converged"):
            assert info[key] == ia[key], (key, info, ia)
        assert np.array_equal(beta.cpu().numpy(), ba)


def test_failing_request_is_isolated():
    probs = problems()[:3]
    Ps = [build(p, prec) for p, prec in probs]
    Ys = [p.Y.copy() for p, _ in probs]
    alone = []
    for P, Y in zip(Ps, Ys):
        beta, _ = P.solve(T(Y), 1e-8, 400)
        alone.append(beta.cpu().numpy())
    # request 1 gets an operator that produces NaN mid-solve: poison its targets
    # after begin by solving a NaN right-hand side (detected at begin -> error)
    bad = Ys[1].copy()
    bad[5, 0] = np.nan
    with pytest.raises(B().KrrError):
        B().Solve(Ps[1], T(bad), 1e-8, 400)
    Ss = [B().Solve(Ps[0], T(Ys[0]), 1e-8, 400), B().Solve(Ps[2], T(Ys[2]), 1e-8, 400)]
    live = list(Ss)
    while live:
        st = B().solve_step(live)
        live = [s for s, v in zip(live, st) if v == 0]
    for S, ba in zip(Ss, [alone[0], alone[2]]):
        beta, info = S.end()
        assert np.array_equal(beta.cpu().numpy(), ba)


@pytest.mark.parametrize("workers", [0, 1])
def test_small_served_stream_matches_alone(workers):
    # workers = 1: builds run on a worker thread and its own stream while the
    # admitted solves keep stepping; the results do not depend on that
    reqs = [synth.Request(i, 0.02 * i, n, d, kind, m, min(200, n // 20), 8000 + i)
            for i, (n, d, kind, m) in enumerate([(4000, 8, 0, 2), (6000, 16, 1, 1),
                                                 (3000, 32, 0, 4), (8000, 8, 1, 3),
                                                 (5000, 16, 0, 1), (2000, 32, 1, 2)])]
    be = GpuBackend(2, tol=1e-6, max_iter=400, keep_beta=True)
    srv = Server(be, hbm_budget=4 << 30, max_active=4, build_workers=workers)
    res = srv.run(reqs, synth.c5_problem)
    s = summarize(res)
    assert s["done"] == len(reqs), [r.error for r in res.values()]
    for req in reqs:
        p = synth.c5_problem(req)
        P = B().rpchol_build(p.kind, p.sigma, 2, T(p.X), p.mu, p.rank, seed=p.algo_seed,
                             m_max=p.Y.shape[1])
        beta, info = P.solve(T(p.Y), 1e-6, 400)
        assert np.array_equal(beta.cpu().numpy(), res[req.rid].beta)
        # MIXED solves meet tol on the FP64 true residual; the oracle re-checks
        # it on 128 sampled rows (scaled to all rows, per right-hand side)
        assert res[req.rid].converged and res[req.rid].relres_true <= 1e-6
        bh = res[req.rid].beta
        rows = np.sort(np.random.default_rng(req.rid).choice(p.X.shape[0], 128, replace=False))
        r = p.Y[rows] - (OK.matvec(p.X[rows], p.X, bh, p.kind, p.sigma) + p.mu * bh[rows])
        est = np.sqrt((r ** 2).sum(axis=0) * p.X.shape[0] / 128) / np.linalg.norm(p.Y, axis=0)
        assert np.all(est <= 20e-6), est


def test_active_solve_guards_its_vectors():
    """While a stepped solve is active its precond refuses the calls that
    would overwrite the solve's vectors; the solve then ends with the result
    it has alone, and the precond serves other calls again."""
    p, prec = problems()[0]
    P = build(p, prec)
    ref, _ = P.solve(T(p.Y), 1e-8, 400)
    S = B().Solve(P, T(p.Y), 1e-8, 400)
    Z = torch.ones((p.X.shape[0], 1), dtype=torch.float64, device=DEV)
    for call in (lambda: P.solve(T(p.Y), 1e-8, 400), lambda: P.apply(Z), lambda: P.operator(Z),
                 lambda: B().Solve(P, T(p.Y), 1e-8, 400)):
        with pytest.raises(B().KrrError) as e:
            call()
        assert e.value.code == -1
    live = [S]
    while live:
        live = [s for s, v in zip(live, B().solve_step(live)) if v == 0]
    beta, info = S.end()
    assert np.array_equal(beta.cpu().numpy(), ref.cpu().numpy())
    P.apply(Z)
    S2 = B().Solve(P, T(p.Y), 1e-8, 400)
    S2.free()
    beta2, _ = P.solve(T(p.Y), 1e-8, 400)
    assert np.array_equal(beta2.cpu().numpy(), ref.cpu().numpy())
