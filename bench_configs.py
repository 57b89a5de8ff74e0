"""Measurements beside the headline line of bench.py, and the workloads
other than the headline one:

* the legs bench.py reports as extra keys of its line (functions *_leg):
  the restricted solve with FP32 tiles, the 100,000-point Laplace problem
  (FP32 and FP64 solves, tile rate against the FP32 VALU peak), the
  1,000,000-point Gaussian problem (MIXED, FP32 and FP64 product rates and a
  MIXED solve) and the served stream (batched MIXED against one request at a
  time in MIXED and in FP64);
* c1 -- 2,000-point Gaussian, FP64 tiles, RPCholesky r=100, PCG to 1e-10,
  checked against a dense Cholesky solve;
* c2 -- the 100,000-point Laplace problem alone;
* c3 -- the 1,000,000-point Gaussian problem alone (--product-only for
  counter runs);
* c5 -- the served stream alone (--requests, --order, --no-baseline);
* crossover -- KRILL (FP64 tiles, PCG to 1e-4) against the direct method
  (form A(S,:)A(:,S) + H, factor, solve) on 500,000 points of the restricted
  workload's distribution for k = 250 .. 16,000 centres (Sec. 4.2's
  runtime-against-centres comparison);
* stored -- the restricted operator over a stored A(:,S) (Sec. 4.1) against
  recomputed tiles at d = 16, 32, 64 on the restricted workload's recipe;
* ranks -- pivot rules against the approximation rank on the 100,000-point
  Laplace workload (Sec. 3.1's rules; the iterations-to-1e-3 against rank
  study of Sec. 4.1): build time and PCG iterations to a relative residual
  of 1e-3 for RPCholesky, uniform and greedy pivots at r = 125 .. 4000.

The standalone configurations print one JSON line each.
"""
import json
import sys
import time

import numpy as np

METRIC = ("kernel entries/s in fused matvec; time-to-1e-6 PCG solve; "
          "p50/p99 served solve latency")


def _line(**kw):
    base = {"metric": METRIC, "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "data": "synthetic"}
    base.update(kw)
    print(json.dumps(base), flush=True)


def _product_rate(b, torch, kind, sigma, prec, X, m, launches=3):
    N = X.shape[0]
    V = torch.from_numpy(np.random.default_rng(0).standard_normal((N, m))).to(X.device)
    ws = b.workspace(b.kernel_matvec_ws(prec, N, N, X.shape[1], m), X.device)
    W = torch.empty_like(V)
    b.kernel_matvec(kind, sigma, prec, X, X, V, out=W, ws=ws)
    torch.cuda.synchronize()
    b.timing_read()
    b.timing_enable(True)
    for _ in range(launches):
        b.kernel_matvec(kind, sigma, prec, X, X, V, out=W, ws=ws)
    torch.cuda.synchronize()
    b.timing_enable(False)
    ms, nl = b.timing_read()
    return ms / max(nl, 1)


def c1(a, b, torch, synth):
    from oracle import direct
    p = synth.c1()
    X = torch.from_numpy(p.X).cuda()
    Y = torch.from_numpy(p.Y).cuda()
    ws = b.workspace(b.rpchol_ws(p.kind, b.FP64, 2000, 8, p.rank, 0, 1), X.device)
    times, infos = [], []
    for k in range(a.warmup + a.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P = b.rpchol_build(p.kind, p.sigma, b.FP64, X, p.mu, p.rank, seed=p.algo_seed, ws=ws)
        beta, info = P.solve(Y, p.tol, 1000)
        torch.cuda.synchronize()
        if k >= a.warmup:
            times.append(time.perf_counter() - t0)
            infos.append(info)
    it = infos[-1]["iters"]
    t = float(np.mean(times))
    # cpu_baseline leg: the oracle's dense Cholesky solve, timed; its solution
    # also gives the GPU solve's error
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):  # one host thread, as reported
        t_cpu0 = time.perf_counter()
        xd = direct.full_krr(p.X, p.Y, p.kind, p.sigma, p.mu)
        t_cpu = time.perf_counter() - t_cpu0
    err = float(np.linalg.norm(beta.cpu().numpy() - xd) / np.linalg.norm(xd))
    _line(value=(it + 1) * 2000 * 2000 / t, unit="kernel entries/s", steps=a.steps,
          warmup=a.warmup, ms_per_step=t * 1e3, dtype="f64",
          config={"workload": "full-data KRR, Gaussian, N=2000, d=8, sigma=sqrt(8), mu=1e-3, "
                              "RPCholesky r=100 (B=10), PCG to 1e-10, FP64 tiles"},
          solve={"iters": it, "relres_true": infos[-1]["relres_true"],
                 "rel_error_vs_dense_cholesky": err},
          cpu_baseline={"value": t_cpu, "unit": "s (dense Cholesky solve, scipy)",
                        "kind": "oracle", "cores": 1, "sample": "whole problem"})


F32_PEAK_TFLOPS = 157.3     # MI355X, published FP32 vector / matrix peak
BF16_PEAK_TFLOPS = 2500.0   # MI355X, published dense bf16 matrix peak
FP64_PEAK_TFLOPS = 78.6     # MI355X, published FP64 vector / matrix peak


def c4_fp32_leg(a, b, torch, synth, ctx):
    """The headline restricted solve with FP32 tiles (FP64 refinement rounds)."""
    return c4_prec_leg(b.FP32, b, torch, ctx)


def c4_fp64_leg(a, b, torch, synth, ctx):
    """The headline restricted solve with the sketch on FP64 tiles as well."""
    return c4_prec_leg(b.FP64, b, torch, ctx)


def c4_prec_leg(prec, b, torch, ctx):
    p = ctx["p"]
    X = ctx["X"]
    N, d = p.X.shape
    Y = torch.from_numpy(p.Y).to(X.device)
    ws = b.workspace(b.krill_ws(p.kind, prec, N, d, p.centers, p.sketch_rows, p.zeta, 1),
                     X.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = b.krill_build(p.kind, p.sigma, prec, X, p.mu, p.centers, sketch_rows=p.sketch_rows,
                      zeta=p.zeta, seed=p.algo_seed, ws=ws)
    tb = time.perf_counter() - t0
    beta, info = P.solve(Y, p.tol, 400)
    torch.cuda.synchronize()
    tt = time.perf_counter() - t0
    del P, ws
    return {"build_s": tb, "time_to_solution_s": tt, "iters": info["iters"],
            "products": info["products"], "relres_true": info["relres_true"],
            "converged": info["converged"],
            "entries_per_s": N * p.centers * (1 + 2 * info["products"]) / tt}


def c2_leg(a, b, torch, synth, ctx=None, n=100_000, steps=3):
    """The 100,000-point Laplace problem: FP32-tile and FP64-tile solves
    (RPCholesky r = 1000 + PCG to 1e-6 + the FP64 true residual) and the
    FP32 quantised tile's rate against the published FP32 peak."""
    p = synth.c2(n=n)
    N, d = p.X.shape
    X = torch.from_numpy(p.X).cuda()
    Y = torch.from_numpy(p.Y).cuda()
    out = {}
    for name, prec, reps in (("fp32", b.FP32, steps), ("fp64", b.FP64, 1)):
        ws = b.workspace(b.rpchol_ws(p.kind, prec, N, d, p.rank, 0, 1), X.device)
        P = b.rpchol_build(p.kind, p.sigma, prec, X, p.mu, p.rank, seed=p.algo_seed, ws=ws)
        P.solve(Y, p.tol, 1000)
        del P
        torch.cuda.synchronize()
        infos = []
        t0 = time.perf_counter()
        for _ in range(reps):
            P = b.rpchol_build(p.kind, p.sigma, prec, X, p.mu, p.rank, seed=p.algo_seed, ws=ws)
            beta, info = P.solve(Y, p.tol, 1000)
            infos.append(info)
            del P
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        info = infos[-1]
        out[name] = {"time_to_solution_s": t, "build_s": info["build_seconds"],
                     "iters": info["iters"], "products": info["products"],
                     "relres_true": max(i["relres_true"] for i in infos),
                     "converged": all(i["converged"] for i in infos),
                     "entries_per_s": N * N * info["products"] / t}
        del ws
    ms = _product_rate(b, torch, p.kind, p.sigma, b.FP32, X, 1, launches=5)
    # the method's VALU work per l1 entry: d differences, d absolute-value
    # accumulations, one scale, one exp (4 slots) and m = 1 multiply-add,
    # counted as FP32 operations against the published FP32 peak
    ops = 2 * d + 5 + 1
    out["fp32_tile"] = {"kernel": "tile_lapq<20, 1, 4> (quantised l1, v_sad_u32, FP32 exp)",
                        "launch_ms": ms, "entries_per_launch": N * N, "ops_per_entry": ops,
                        "tops": ops * N * N / (ms * 1e-3) / 1e12,
                        "frac_of_fp32_peak": ops * N * N / (ms * 1e-3) / 1e12 / F32_PEAK_TFLOPS}
    return out


def c2(a, b, torch, synth):
    res = c2_leg(a, b, torch, synth, n=a.n, steps=a.steps)
    _line(value=res["fp32"]["entries_per_s"], unit="kernel entries/s", steps=a.steps, warmup=1,
          ms_per_step=res["fp32"]["time_to_solution_s"] * 1e3, dtype="f32",
          config={"workload": f"full-data KRR, l1 Laplace, N={a.n}, d=20, 10-component Gaussian "
                              "mixture, sigma=20, mu=1e-4 N, RPCholesky r=1000, PCG to 1e-6 "
                              "(FP32 tiles, FP64 CG)"},
          result=res)


def _rounds(h):
    """Refinement rounds of a residual history: a round starts where the
    worst relative recursive residual jumps up (the restart from the FP64
    residual).  Per round: iterations and the last recursive residual."""
    out, start = [], 0
    for i in range(1, len(h) + 1):
        if i == len(h) or h[i] > 3.0 * h[i - 1]:
            out.append({"iters": i - start, "recursive_end": h[i - 1]})
            start = i
    return out


def c3_leg(a, b, torch, synth, ctx=None, solve=True):
    """The 1,000,000-point Gaussian problem (d = 32, 8 right-hand sides):
    product rates of the MIXED, FP32 and FP64 tiles and a MIXED solve to an
    FP64 true residual of 1e-6."""
    p = synth.c3()
    N, d = p.X.shape
    X = torch.from_numpy(p.X).cuda()
    Y = torch.from_numpy(p.Y).cuda()
    m = p.Y.shape[1]
    out = {}
    ms = _product_rate(b, torch, p.kind, p.sigma, b.MIXED, X, m)
    rate = N * N / (ms * 1e-3)
    # executed MFMA work per entry: 3 split products of K = 32 for the
    # distance and 3 of the 16-column V tiles, 2 flops per multiply-add
    mfma_flops = (3 * 2 * 32) + (3 * 2 * 16)
    out["mixed_product"] = {"launch_ms": ms, "entries_per_s": rate,
                            "mfma_tflops_executed": rate * mfma_flops / 1e12,
                            "frac_of_bf16_peak_executed": rate * mfma_flops / 1e12 / BF16_PEAK_TFLOPS}
    ms32 = _product_rate(b, torch, p.kind, p.sigma, b.FP32, X, m, launches=2)
    # FP32 model: distance (K = 32) and E.V (16 columns), 2 flops per
    # multiply-add; executed: the distance as 6 bf16 slice products of K = 32
    # on the bf16 matrix cores, E.V on the FP32 ones (the two are reported as
    # the fraction of the launch their executed work needs at the peaks)
    f32_flops = 2 * 32 + 2 * 16
    t32 = ms32 * 1e-3
    busy = N * N * (6 * 2 * 32 / (BF16_PEAK_TFLOPS * 1e12) + 2 * 16 / (F32_PEAK_TFLOPS * 1e12))
    out["fp32_product"] = {"launch_ms": ms32, "entries_per_s": N * N / t32,
                           "algorithmic_tflops_fp32_model": N * N * f32_flops / t32 / 1e12,
                           "matrix_core_time_frac_executed": busy / t32}
    ms64 = _product_rate(b, torch, p.kind, p.sigma, b.FP64, X, m, launches=2)
    f64_flops = 2 * 32 + 2 + 2 * m  # distance, norms, E.V on the VALU
    out["fp64_product"] = {"launch_ms": ms64, "entries_per_s": N * N / (ms64 * 1e-3),
                           "frac_of_fp64_peak": N * N * f64_flops / (ms64 * 1e-3) / 1e12 /
                           FP64_PEAK_TFLOPS}
    if solve:
        ws = b.workspace(b.rpchol_ws(p.kind, b.MIXED, N, d, p.rank, 0, m), X.device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P = b.rpchol_build(p.kind, p.sigma, b.MIXED, X, p.mu, p.rank, seed=p.algo_seed,
                           m_max=m, ws=ws)
        print(f"c3: build done in {time.perf_counter() - t0:.2f} s", file=sys.stderr, flush=True)
        S = b.Solve(P, Y, p.tol, 2000)
        k = 0
        while b.solve_step([S])[0] == 0:
            k += 1
            if k % 25 == 0:
                print(f"c3: step {k}, {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                      flush=True)
        beta, info = S.end(history=2000)
        torch.cuda.synchronize()
        out["mixed_solve"] = {"time_to_solution_s": time.perf_counter() - t0,
                              "build_s": info["build_seconds"], "iters": info["iters"],
                              "products": info["products"], "relres_true": info["relres_true"],
                              "relres_recursive": info["relres_recursive"],
                              "rank": P.dims()[0], "converged": info["converged"],
                              "rounds": _rounds(info["history"])}
        del P, S, ws
    return out


def c3(a, b, torch, synth):
    if a.product_only:
        p = synth.c3()
        X = torch.from_numpy(p.X).cuda()
        prec = b.FP32 if a.fp32 else b.MIXED
        ms = _product_rate(b, torch, p.kind, p.sigma, prec, X, p.Y.shape[1])
        print(json.dumps({"product_ms": ms, "entries_per_launch": p.X.shape[0] ** 2}), flush=True)
        return
    res = c3_leg(a, b, torch, synth, solve=a.steps > 0)
    sol = res.get("mixed_solve", {})
    _line(value=res["mixed_product"]["entries_per_s"], unit="kernel entries/s",
          steps=1 if sol else 0, warmup=0,
          ms_per_step=sol["time_to_solution_s"] * 1e3 if sol else None, dtype="bf16x3/f32",
          config={"workload": "full-data KRR, Gaussian, N=1e6, d=32, uniform [0,1]^32 with 5% "
                              "near-duplicates, 8 RHS, sigma=1.5, mu=1e-6 N, RPCholesky r=2000, "
                              "bf16-split MFMA tiles, PCG to 1e-6"},
          result=res)


def c5_leg(a, b, torch, synth, ctx=None, requests=None, baselines=True, caps=None):
    """The served stream: batched MIXED (continuous batching, builds on a
    worker thread, admission capped by estimated per-step work), then the
    same arrival trace one request at a time in MIXED and in FP64.  caps: a
    list of work caps to serve the trace with in turn (None = no cap)."""
    from paper_2304_12465_amd.serve import Server, GpuBackend, serve_one_at_a_time, summarize
    count = requests or a.requests
    stream = synth.c5_stream(count=count)
    # the requests' arrays are generated before the clock starts: they stand
    # for data that arrives with each request, not for serving work
    probs = {}
    for i, r in enumerate(stream):
        probs[r.rid] = synth.c5_problem(r)
        if (i + 1) % 32 == 0:
            print(f"c5: generated {i + 1} of {len(stream)} requests", file=sys.stderr, flush=True)
    make = lambda req: probs[req.rid]

    def progress(tag):
        def f(r):
            print(f"c5 {tag}: request {r.rid} {r.status} latency {r.latency:.2f} s",
                  file=sys.stderr, flush=True)
        return f
    be = GpuBackend(b.MIXED, tol=1e-6, max_iter=500)
    out = {"requests": count, "admission_order": a.order}
    for cap in (caps if caps is not None else [a.work_cap]):
        torch.cuda.empty_cache()
        srv = Server(be, hbm_budget=160 << 30, max_active=64, on_finish=progress(f"cap {cap}"),
                     build_workers=a.build_workers, order=a.order, work_cap=cap)
        t0 = time.perf_counter()
        res = srv.run(stream, make)
        s_ = summarize(res)
        s_["work_cap"] = cap
        s_["wall_s"] = time.perf_counter() - t0
        if "batched_mixed" not in out:
            out["batched_mixed"] = s_
            out["batched_wall_s"] = s_["wall_s"]
        else:
            out.setdefault("other_caps", []).append(s_)
    if baselines:
        for tag, prec in (("one_at_a_time_mixed", b.MIXED), ("one_at_a_time_fp64", b.FP64)):
            torch.cuda.empty_cache()
            res1 = serve_one_at_a_time(GpuBackend(prec, tol=1e-6, max_iter=500), stream, make,
                                       on_finish=progress(tag))
            out[tag] = summarize(res1)
    return out


def c5(a, b, torch, synth):
    caps = [a.work_cap, None, 3e10, 3e11, 1e12] if a.sweep else None
    res = c5_leg(a, b, torch, synth, baselines=not a.no_baseline, caps=caps)
    s_mix = res["batched_mixed"]
    _line(value=s_mix["solves_per_s"], unit="solves/s", steps=1, warmup=0,
          ms_per_step=res["batched_wall_s"] * 1e3, dtype="bf16x3/f32 (Gaussian), f32 (Laplace)",
          config={"workload": f"served stream: {a.requests} requests, Poisson 20/s, N log-uniform "
                              "[1e4, 3e5], d in {8,16,32}, Gaussian/Laplace, 1-16 RHS, "
                              "r=min(1000, N/50), PCG to 1e-6"},
          result=res)


def stored_leg(a, b, torch, synth, ctx=None, dims=(16, 32, 64), n=2_000_000):
    """The restricted operator with A(:,S) stored (Sec. 4.1) against
    recomputed tiles, on the restricted workload's recipe at d = 16, 32 and
    64 (N = 2,000,000, k = 10,000): build time, time per operator application
    (two N k products) and one solve to 1e-6, FP64 and FP32."""
    rows = []
    for d in dims:
        p = synth.c4(n=n, d=d)
        N = p.X.shape[0]
        X = torch.from_numpy(p.X).cuda()
        Y = torch.from_numpy(p.Y).cuda()
        V = torch.from_numpy(np.random.default_rng(1).standard_normal((p.centers, 1))).cuda()
        for prec, pname in ((b.FP64, "fp64"), (b.FP32, "fp32")):
            for stored in (False, True):
                # the workspace (160 GB for the stored FP64 block) is
                # allocated before the clock starts: build_s is the build
                q = b.krill_stored_ws if stored else b.krill_ws
                ws = b.workspace(q(p.kind, prec, N, d, p.centers, p.sketch_rows, p.zeta, 1),
                                 X.device)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                P = b.krill_build(p.kind, p.sigma, prec, X, p.mu, p.centers,
                                  sketch_rows=p.sketch_rows, zeta=p.zeta, seed=p.algo_seed,
                                  stored=stored, ws=ws)
                torch.cuda.synchronize()
                tb = time.perf_counter() - t0
                P.operator(V)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                for _ in range(3):
                    P.operator(V)
                torch.cuda.synchronize()
                top = (time.perf_counter() - t1) / 3
                t2 = time.perf_counter()
                beta, info = P.solve(Y, p.tol, 400)
                torch.cuda.synchronize()
                row = {"d": d, "prec": pname, "stored": stored, "build_s": round(tb, 4),
                       "operator_ms": round(top * 1e3, 3), "solve_s": round(time.perf_counter() - t2, 4),
                       "iters": info["iters"], "products": info["products"],
                       "relres_true": info["relres_true"], "converged": info["converged"]}
                if stored:
                    row["stored_gb"] = round(N * ((p.centers + 7) // 8 * 8) *
                                             (8 if prec == b.FP64 else 4) / 1e9, 1)
                    row["stream_tb_per_s"] = round(row["stored_gb"] / 1e3 / top, 3)
                rows.append(row)
                print(json.dumps(row), file=sys.stderr, flush=True)
                del P, beta, ws
                torch.cuda.empty_cache()
        del X, Y, V
        torch.cuda.empty_cache()
    cross = {}
    for pname in ("fp64", "fp32"):
        for d in dims:
            r0 = next(r for r in rows if r["d"] == d and r["prec"] == pname and not r["stored"])
            r1 = next(r for r in rows if r["d"] == d and r["prec"] == pname and r["stored"])
            cross[f"{pname}_d{d}_recomputed_over_stored"] = round(r0["operator_ms"] / r1["operator_ms"], 3)
    return {"table": rows, "operator_time_ratio": cross}


def stored(a, b, torch, synth):
    res = stored_leg(a, b, torch, synth)
    r = next(r for r in res["table"] if r["d"] == 16 and r["prec"] == "fp64" and r["stored"])
    _line(value=2 * 2_000_000 * 10_000 / (r["operator_ms"] * 1e-3), unit="kernel entries/s "
          "(stored FP64 operator, d=16)", steps=3, warmup=1, ms_per_step=r["operator_ms"],
          dtype="f64", config={"workload": "restricted KRR with KRILL, A(:,S) stored vs "
                                           "recomputed: N=2e6, k=1e4, d=16/32/64 (recipe of the "
                                           "restricted workload), FP64 and FP32"},
          result=res)


def ranks(a, b, torch, synth):
    p = synth.c2(n=a.n)
    N, d = p.X.shape
    X = torch.from_numpy(p.X).cuda()
    Y = torch.from_numpy(p.Y).cuda()
    tol = 1e-3
    rules = (("rpcholesky", b.PIVOT_RPCHOL), ("uniform", b.PIVOT_UNIFORM),
             ("greedy", b.PIVOT_GREEDY))
    table = []
    # the workload's ridge and one 100x smaller, where the preconditioner
    # has more of the spectrum to capture
    for mu_n in (1e-4, 1e-6):
        for r in (125, 250, 500, 1000, 2000, 4000):
            ws = b.workspace(b.rpchol_ws(p.kind, b.FP32, N, d, r, 0, 1), X.device)
            for name, rule in rules:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                P = b.nystrom_build(p.kind, p.sigma, b.FP32, X, mu_n * N, r, rule,
                                    seed=p.algo_seed, ws=ws)
                tb = time.perf_counter() - t0
                beta, info = P.solve(Y, tol, 2000)
                torch.cuda.synchronize()
                row = {"mu_over_N": mu_n, "rule": name, "r": r, "rank": P.dims()[0],
                       "build_s": round(tb, 4), "iters": info["iters"],
                       "solve_s": round(time.perf_counter() - t0 - tb, 4),
                       "relres_true": info["relres_true"]}
                table.append(row)
                print(json.dumps(row), file=sys.stderr, flush=True)
                del P
            del ws
            torch.cuda.empty_cache()
    ref = next(t for t in table
               if t["rule"] == "rpcholesky" and t["r"] == 1000 and t["mu_over_N"] == 1e-4)
    _line(value=ref["iters"], unit="PCG iterations to relative residual 1e-3 (RPCholesky, r=1000)",
          steps=1, warmup=0, ms_per_step=(ref["build_s"] + ref["solve_s"]) * 1e3, dtype="f32",
          higher_is_better=False,
          config={"workload": f"pivot rules vs rank: full-data KRR, l1 Laplace, N={N}, d={d}, "
                              "10-component Gaussian mixture, sigma=20, mu=1e-4 N and 1e-6 N, "
                              "FP32 tiles, PCG to 1e-3, r = 125 .. 4000"},
          result={"table": table})


def crossover(a, b, torch, synth):
    n = 500_000
    tol = 1e-4
    rows = []
    for k in (250, 500, 1000, 2000, 4000, 8000, 16000):
        p = synth.c4(n=n, k=k)
        N, d = p.X.shape
        X = torch.from_numpy(p.X).cuda()
        Y = torch.from_numpy(p.Y).cuda()
        ws = b.workspace(b.krill_ws(p.kind, b.FP64, N, d, k, p.sketch_rows, p.zeta, 1), X.device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P = b.krill_build(p.kind, p.sigma, b.FP64, X, p.mu, k, sketch_rows=p.sketch_rows,
                          zeta=p.zeta, seed=p.algo_seed, ws=ws)
        beta_k, info = P.solve(Y, tol, 500)
        torch.cuda.synchronize()
        t_krill = time.perf_counter() - t0
        centres = torch.tensor(P.pivots(), dtype=torch.int64, device=X.device)
        del P, ws
        torch.cuda.empty_cache()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        beta_d = b.restricted_direct(p.kind, p.sigma, X, p.mu, centres, Y)
        torch.cuda.synchronize()
        t_direct = time.perf_counter() - t0
        gap = float(torch.linalg.norm(beta_k - beta_d) / torch.linalg.norm(beta_d))
        row = {"k": k, "krill_s": round(t_krill, 4), "krill_iters": info["iters"],
               "krill_relres_true": info["relres_true"], "direct_s": round(t_direct, 4),
               "coef_gap": gap}
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
        del X, Y, beta_k, beta_d, centres
        torch.cuda.empty_cache()
    cross = next((r["k"] for r in rows if r["krill_s"] < r["direct_s"]), None)
    last = rows[-1]
    _line(value=last["direct_s"] / last["krill_s"], unit="direct time / KRILL time at k=16000",
          steps=1, warmup=0, ms_per_step=last["krill_s"] * 1e3, dtype="f64",
          config={"workload": "restricted KRR, KRILL vs direct: N=500,000 points of the "
                              "restricted workload's distribution (d=16, Gaussian sigma=4, "
                              "mu=1e-5 N), k = 250 .. 16000, FP64 tiles, PCG to 1e-4"},
          result={"table": rows, "krill_faster_from_k": cross})


def run(a):
    import torch
    import synth
    from paper_2304_12465_amd import binding as b
    {"c1": c1, "c2": c2, "c3": c3, "c5": c5, "ranks": ranks, "crossover": crossover,
     "stored": stored}[a.config](a, b, torch, synth)
