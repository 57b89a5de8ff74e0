"""Benchmark of the hot path on one MI355X.

Headline workload (the largest single-GPU configuration): restricted KRR
with KRILL preconditioning (Alg. 2) on N = 2,000,000 points of dimension 16
(standard normal, dimension j scaled by 1/(1+j)), Gaussian kernel sigma = 4,
k = 10,000 centres drawn uniformly, a sparse sign sketch of 2k rows with 8
nonzeros per column, mu = 1e-5 N, PCG to a relative residual of 1e-6: FP64
tiles for the restricted products, the right-hand side and the residual
checks, FP32 tiles for the sketch (KRR_MIXED), FP64 factor and CG.

One step = one whole solve with the inputs resident in HBM: the KRILL build
(centres, H, the sketch, B = Phi A(:,S), B^T B + H, its Cholesky factor and
L^{-1}) plus PCG (two restricted products per iteration, the preconditioner
apply, FP64 recurrences) and the FP64 true residual at exit (carried by the
converging iteration, whose products also multiply x).

`value` is the number of kernel entries the fused restricted products
evaluate (A(S,:) y: N k; each operator application: 2 N k) per second of
timed wall time, everything included.  `roofline` reports the dominant
kernel (the FP64 Gaussian MFMA tile) against the published FP64 MFMA peak,
its launch time measured live with HIP events on its own stream; `issue`
and `traffic` come from rocprofv3 counters in profiles/.  `cpu_baseline`
times the FP64 oracle's restricted product on a bounded row sample on all
host cores.  The other workloads appear beside it as extra keys: the same
solve with FP32 tiles, the restricted operator over a stored A(:,S) against
recomputed tiles at d = 16, 32, 64, the same solve with the sketch on FP64 tiles too, the
1,000,000-point Gaussian problem (MIXED, FP32 and
FP64 product rates and a MIXED solve), the 100,000-point Laplace problem
(FP32 and FP64 solves) and the served stream (p50/p99 latency of 64
requests, batched MIXED against one at a time in MIXED and in FP64).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("kernel entries/s in fused matvec; time-to-1e-6 PCG solve; "
          "p50/p99 served solve latency")
FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X, published dense FP64 matrix peak
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2304_12465_amd", "csrc")
# the dominant tile is built from these sources; counters taken on another
# source are not reported
TILE_SOURCES = ["product_gauss_mfma.hip", "gauss_mfma.h", "exp64.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "tile_gauss_f64_n2e6_k1e4_hbm_traffic.md")
ISSUE_FILE = os.path.join(ROOT, "profiles", "tile_gauss_f64_n2e6_k1e4_sq_counters.md")


def tile_source_sha():
    h = hashlib.sha256()
    for name in TILE_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profile_fields(path):
    """The '- key: value' fields of a counter summary, or None when it was
    taken on another source of the tile."""
    try:
        text = open(path).read()
    except OSError:
        return None
    fields = dict(re.findall(r"^- (\w+): (\S+)$", text, re.M))
    if fields.get("source_sha256") != tile_source_sha():
        return None
    return fields


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--no-extra", action="store_true",
                    help="headline only (no FP32, 1e6-point, Laplace or served legs)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="wall time of the oracle's bounded row sample")
    ap.add_argument("--n", type=int, default=100_000, help="--config c2: number of points")
    ap.add_argument("--config", default="c4",
                    choices=["c1", "c2", "c3", "c4", "c5", "ranks", "crossover", "stored"],
                    help="c4 (default): the headline restricted solve with the other "
                         "workloads as extra keys; c1, c2, c3, c5: one workload each; "
                         "ranks: pivot rules against the approximation rank; crossover: "
                         "KRILL against the direct restricted solve")
    ap.add_argument("--requests", type=int, default=64, help="served stream: number of requests")
    ap.add_argument("--no-baseline", action="store_true",
                    help="--config c5: skip the one-at-a-time runs")
    ap.add_argument("--order", default="fifo", choices=["fifo", "sjf"],
                    help="served stream: admission order (arrival, or smallest estimated work)")
    ap.add_argument("--build-workers", type=int, default=1,
                    help="served stream: preconditioner builds on this many worker threads")
    ap.add_argument("--work-cap", type=float, default=3e11,
                    help="served stream: admit while the admitted requests' estimated "
                         "per-step work (N^2 (d + m) each) stays within this cap; 0: no cap")
    ap.add_argument("--sweep", action="store_true",
                    help="--config c5: serve the trace with several work caps")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (HBM counter calibration)")
    ap.add_argument("--fp32", action="store_true",
                    help="--product-only: FP32 tiles instead of the default precision")
    ap.add_argument("--product-only", action="store_true",
                    help="only run 5 launches of the workload's product (for counter runs)")
    return ap.parse_args()


def headline(a, b, torch, synth, np):
    p = synth.c4()
    N, d = p.X.shape
    k = p.centers
    dev = torch.device("cuda:0")
    X = torch.from_numpy(p.X).to(dev)
    Y = torch.from_numpy(p.Y).to(dev)
    torch.cuda.synchronize()
    ws = b.workspace(b.krill_ws(p.kind, b.MIXED, N, d, k, p.sketch_rows, p.zeta, 1), dev)

    def one():
        P = b.krill_build(p.kind, p.sigma, b.MIXED, X, p.mu, k, sketch_rows=p.sketch_rows,
                          zeta=p.zeta, seed=p.algo_seed, ws=ws)
        beta, info = P.solve(Y, p.tol, 200)
        return P, beta, info

    for _ in range(a.warmup):
        P, _, _ = one()
        del P
    torch.cuda.synchronize()
    b.timing_read()
    b.timing_enable(True)
    infos = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        P, beta, info = one()
        infos.append(info)
        del P
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b.timing_enable(False)
    # every tile launch, and those of the one-vector tile (the roofline's
    # kernel; the iteration that carries x beside p runs the two-vector one)
    tile_ms, launches, one_ms, one_launches = b.timing_read_vectors(1)
    # fused-product entries: A(S,:) y (N k) and 2 N k per operator application
    entries = sum(N * k * (1 + 2 * i["products"]) for i in infos)
    launch_ms = one_ms / max(one_launches, 1)
    # algorithmic FP64 flops of one kernel entry: the distance contraction
    # (d multiply-adds), adding the two squared norms, and the reduction
    # against V (m = 1 multiply-add); the exp is not counted
    flops_entry = 2 * d + 2 + 2 * 1
    achieved = flops_entry * N * k / (launch_ms * 1e-3) / 1e12
    traffic = profile_fields(TRAFFIC_FILE)
    issue = profile_fields(ISSUE_FILE)
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_MFMA_PEAK_TFLOPS, 4),
                "traffic": float(traffic["traffic_bytes_per_launch"]) if traffic else None,
                "traffic_unit": "bytes per launch",
                "kernel": "tile_gauss_mfma<double, 16, 1> (FP64 Gaussian MFMA tile, exp on the VALU)",
                "flops_per_entry": flops_entry, "entries_per_launch": N * k,
                "launch_ms": round(launch_ms, 4), "launches_timed": one_launches,
                "algorithmic_bytes_per_launch": 8 * (N * d + k * d + N + k)}
    if issue:
        # FP64 MFMA and FP64 VALU instructions do not overlap on this tile
        # (co-issue counter 0), so their busy fractions add
        roofline["issue"] = {"valu_busy": float(issue["valu_busy"]),
                             "mfma_busy": float(issue["mfma_busy"]),
                             "valu_plus_mfma": round(float(issue["valu_busy"]) +
                                                     float(issue["mfma_busy"]), 4),
                             "valu_instructions_per_entry": float(issue["valu_per_entry"]),
                             "source": os.path.relpath(ISSUE_FILE, ROOT)}
    solve = {"time_to_solution_s": wall / a.steps,
             "build_s": float(np.mean([i["build_seconds"] for i in infos])),
             "pcg_s": float(np.mean([i["solve_seconds"] for i in infos])),
             "iters": [i["iters"] for i in infos], "products": infos[-1]["products"],
             "relres_true": max(i["relres_true"] for i in infos),
             "converged": all(i["converged"] for i in infos),
             "tile_ms_total": tile_ms, "tile_launches": launches}
    out = {
        "metric": METRIC, "value": entries / wall, "unit": "kernel entries/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": wall / a.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
        "precision": {"restricted_products": "f64", "rhs_and_checks": "f64",
                      "sketch": "f32 (FP32 points as exact bf16 slices, FP32 accumulation, "
                                "FP64 row sums)",
                      "factor": "f64", "cg": "f64"},
        "data": "synthetic",
        "config": {"workload": f"restricted KRR with KRILL: N={N}, d={d} standard normal with "
                               "dimension j scaled by 1/(1+j), Gaussian sigma=4, k=10000 uniform "
                               "centres, sparse sign sketch 20000 rows x 8 nonzeros, mu=1e-5 N, "
                               "PCG to 1e-6, FP64 product tiles, FP32 sketch tiles",
                   "N": N, "d": d, "k": k, "sketch_rows": p.sketch_rows, "zeta": p.zeta,
                   "tol": p.tol},
        "solve": solve,
        "roofline": roofline,
    }
    del ws
    ctx = {"p": p, "X": X, "products": infos[-1]["products"]}
    return out, ctx


def cpu_baseline(a, np, ctx):
    """The FP64 oracle's restricted product K(X, C) v on a bounded sample of
    row blocks, on every host core (one oracle call per 256-row block per
    thread, BLAS held to one thread each), in the fast BLAS-expansion mode
    (pinned against the exact mode in the oracle's tests)."""
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    from oracle import kernels as OK
    from oracle import krill as OKR
    p = ctx["p"]
    N, k = p.X.shape[0], p.centers
    S = OKR.sample_centers(N, k, p.algo_seed)
    C = p.X[S]
    V = np.random.default_rng(0).standard_normal((k, 1))
    cores = len(os.sched_getaffinity(0))
    rows = 256
    deadline = a.cpu_seconds

    def worker(w):
        done = 0
        t_start = time.perf_counter()
        i = w * rows
        while time.perf_counter() - t_start < deadline and i + rows <= N:
            OK.matvec(p.X[i:i + rows], C, V, p.kind, p.sigma, fast=True)
            done += rows
            i += cores * rows
        return done

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        with ThreadPoolExecutor(cores) as ex:
            done = sum(ex.map(worker, range(cores)))
        tc = time.perf_counter() - t0
    rate = done * k / tc
    per_solve = N * k * (1 + 2 * ctx["products"])
    return {"value": rate, "unit": "kernel entries/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle restricted product K(X, X(S,:)) v, fast BLAS-expansion mode, "
                      f"{done} rows x {k} centres ({done * k:.3g} entries) in {tc:.1f} s on "
                      f"{cores} threads",
            "extrapolated_solve_products_s": per_solve / rate,
            "extrapolated_note": f"extrapolated, not run: the {per_solve:.3g} restricted-product "
                                 "entries of one GPU solve at the sampled rate; the KRILL build "
                                 "is not included"}


def product_only(a, b, torch, synth, np):
    """5 launches of the restricted product's first half K(X, X(S,:)) v
    (2e6 x 1e4 entries) for counter runs; --fp32 for the FP32 tile."""
    p = synth.c4()
    N, d = p.X.shape
    dev = torch.device("cuda:0")
    X = torch.from_numpy(p.X).to(dev)
    prec = b.FP32 if a.fp32 else b.FP64
    S = torch.from_numpy(np.sort(np.random.default_rng(2).choice(N, p.centers, replace=False)))
    C = X[S.to(dev)].contiguous()
    V = torch.from_numpy(np.random.default_rng(0).standard_normal((p.centers, 1))).to(dev)
    ws = b.workspace(b.kernel_matvec_ws(prec, N, p.centers, d, 1), dev)
    W = torch.empty((N, 1), dtype=torch.float64, device=dev)
    for _ in range(5):
        b.kernel_matvec(p.kind, p.sigma, prec, X, C, V, out=W, ws=ws)
    torch.cuda.synchronize()
    print(json.dumps({"product_launches": 5, "entries_per_launch": N * p.centers}), flush=True)


def main():
    a = parse()
    if a.work_cap is not None and a.work_cap <= 0:
        a.work_cap = None
    if a.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {a.gpus} is not supported "
              "(sharding over several GPUs is designed, not implemented)", file=sys.stderr)
        sys.exit(2)
    if a.copy_calibration:
        import torch
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8,
                          "launches": 5}))
        return
    if a.config != "c4":
        import bench_configs
        bench_configs.run(a)
        return
    import numpy as np
    import torch
    from paper_2304_12465_amd import binding as b
    import synth
    if a.product_only:
        product_only(a, b, torch, synth, np)
        return
    print("bench: headline solves", file=sys.stderr, flush=True)
    out, ctx = headline(a, b, torch, synth, np)
    if not a.no_extra:
        import bench_configs as BC
        legs = (("c4_fp64", BC.c4_fp64_leg), ("c4_fp32", BC.c4_fp32_leg),
                ("stored_vs_recomputed", BC.stored_leg),
                ("c2", BC.c2_leg), ("c3", BC.c3_leg), ("c5", BC.c5_leg))
        for name, fn in legs:
            print(f"bench: {name}", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
            t0 = time.perf_counter()
            try:
                res = fn(a, b, torch, synth, ctx)
            except Exception as e:  # an extra leg never hides the headline line
                res = {"error": f"{type(e).__name__}: {e}"}
            res["leg_wall_s"] = round(time.perf_counter() - t0, 2)
            out[name] = res
    if not a.no_cpu:
        print("bench: oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(a, np, ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
