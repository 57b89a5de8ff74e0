"""Continuously batched serving of KRR solves.

Requests (points, targets, kernel, rank, right-hand-side count) arrive over
time.  The server admits them in arrival order as long as their HBM
footprint (the library's workspace size plus the request's own arrays) fits
in the budget, keeps every admitted request's points, Nystrom factor and
CG state resident on the device, and advances all admitted solves together:
each tick is one native step (``krr_solve_step``) in which the direction
products of all active requests share kernel launches.  A request leaves as
soon as its solve finishes, freeing memory for the next ones.  Latency is
completion time minus arrival time (queueing included).

With ``build_workers > 0`` a request's preconditioner build (a chain of
small, latency-bound kernels with host synchronisations) runs on a worker
thread while the main loop keeps stepping the admitted solves; the GPU
backend gives each worker thread a stream of its own, so the build's
kernels interleave with the product tiles of the running solves.

The scheduling policy lives here; every numerical step runs in the HIP
library behind a backend object.  ``GpuBackend`` is the product backend;
tests may plug in a fake backend with the same four methods.
"""
import threading
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor, wait, FIRST_COMPLETED
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float = 0.0
    finished: float = 0.0
    status: str = "pending"   # done | failed | rejected
    iters: int = 0
    relres_true: float = float("nan")
    converged: bool = False   # the solve met tol (on the FP64 true residual for FP32 / MIXED)
    error: str = ""
    beta: object = None

    @property
    def latency(self):
        return self.finished - self.arrival


class GpuBackend:
    """Runs requests on the GPU through the C ABI (binding module)."""

    def __init__(self, precision, tol=1e-6, max_iter=500, device="cuda:0", keep_beta=False):
        import torch
        from . import binding
        self.b = binding
        self.torch = torch
        self.prec = precision
        self.tol = tol
        self.max_iter = max_iter
        self.dev = torch.device(device)
        self.keep_beta = keep_beta
        self._local = threading.local()

    def _build_stream(self):
        """The main thread builds on its current stream; every other thread
        on a stream of its own (default priority)."""
        if threading.current_thread() is threading.main_thread():
            return None
        st = getattr(self._local, "stream", None)
        if st is None:
            st = self.torch.cuda.Stream(device=self.dev)
            self._local.stream = st
        return st

    def footprint(self, prob):
        N, d = prob.X.shape
        m = prob.Y.shape[1]
        ws = self.b.rpchol_ws(prob.kind, self.prec, N, d, prob.rank, 0, m)
        return ws + 8 * N * (d + 2 * m) + 4096

    def cost(self, prob):
        """Work estimate for shortest-first admission: one product."""
        N, d = prob.X.shape
        return float(N) * N * (d + prob.Y.shape[1])

    def start(self, prob):
        st = self._build_stream()
        if st is not None:
            with self.torch.cuda.stream(st):
                return self._start(prob)
        return self._start(prob)

    def _start(self, prob):
        # the build and the solve's first step end with a synchronisation of
        # this stream, so the handle is ready for steps on any stream; the
        # request's arrays are freed only after its solve has synchronised
        t = lambda a: self.torch.from_numpy(np.ascontiguousarray(a)).to(self.dev)
        X, Y = t(prob.X), t(prob.Y)
        P = self.b.rpchol_build(prob.kind, prob.sigma, self.prec, X, prob.mu, prob.rank,
                                seed=prob.algo_seed, m_max=Y.shape[1])
        S = self.b.Solve(P, Y, self.tol, self.max_iter)
        return {"P": P, "S": S, "Y": Y}

    def step(self, handles):
        return self.b.solve_step([h["S"] for h in handles], self.dev)

    def finish(self, h):
        beta, info = h["S"].end()
        out = beta.cpu().numpy() if self.keep_beta else None
        h.clear()
        return out, info

    def cancel(self, h):
        h.clear()


class Server:
    def __init__(self, backend, hbm_budget, max_active=64, clock=time.perf_counter,
                 sleep=time.sleep, on_finish=None, order="fifo", build_workers=0,
                 work_cap=None):
        """order: "fifo" admits in arrival order; "sjf" admits the waiting
        request with the smallest estimated work (backend.cost) first.
        build_workers: 0 builds in the loop; n > 0 builds on n worker
        threads while the admitted solves keep stepping.
        work_cap: admit a request only while the estimated per-step work of
        the admitted ones (backend.cost summed) stays within the cap; one
        request is always admitted.  Requests that fill the GPU alone then
        run (nearly) one at a time, with the next build overlapping them,
        while small ones share steps -- instead of every admitted request
        slowing down every other (processor sharing)."""
        self.be = backend
        self.budget = hbm_budget
        self.max_active = max_active
        self.work_cap = work_cap
        self.order = order
        self.clock = clock
        self.sleep = sleep
        self.on_finish = on_finish  # called with each finished Result
        self.build_workers = build_workers

    def run(self, stream, make_problem):
        """Serves ``stream`` (objects with .rid and .arrival in seconds);
        ``make_problem(req)`` gives its arrays.  Returns {rid: Result}."""
        pool = ThreadPoolExecutor(self.build_workers) if self.build_workers > 0 else None
        try:
            return self._run(stream, make_problem, pool)
        finally:
            if pool is not None:
                pool.shutdown(wait=True)

    def _run(self, stream, make_problem, pool):
        pending = deque(sorted(stream, key=lambda r: r.arrival))
        results = {r.rid: Result(r.rid, r.arrival) for r in stream}
        problems = {}
        waiting = deque()
        building = []  # (req, future, bytes): builds on worker threads
        ready = deque()  # (req, handle, bytes): built, waiting for the work cap
        active = []  # (req, handle, bytes): stepping
        used = 0
        work = {}  # rid -> estimated per-step work (backend.cost) of admitted requests
        t0 = self.clock()

        def fail_build(req, need, e):
            nonlocal used
            r = results[req.rid]
            r.status, r.error = "failed", str(e)
            r.finished = self.clock() - t0
            used -= need
            work.pop(req.rid, None)
            problems.pop(req.rid, None)
            if self.on_finish:
                self.on_finish(r)

        def active_work():
            return sum(work[q.rid] for q, _, _ in active)

        while pending or waiting or active or building or ready:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                req = pending.popleft()
                problems[req.rid] = make_problem(req)
                waiting.append(req)
            # finished background builds are ready to step
            still = []
            for req, fut, need in building:
                if not fut.done():
                    still.append((req, fut, need))
                    continue
                try:
                    ready.append((req, fut.result(), need))
                except Exception as e:  # a failed build isolates this request only
                    fail_build(req, need, e)
            building = still
            # admission while the footprint fits: arrival order, or smallest
            # estimated work first.  With a work cap, a request is admitted
            # (and its build started) when the admitted work leaves room for
            # it, or as the one build that runs ahead of the stepping ones.
            if self.order == "sjf" and len(waiting) > 1:
                waiting = deque(sorted(waiting, key=lambda q: self.be.cost(problems[q.rid])))
            while waiting and len(active) + len(building) + len(ready) < self.max_active:
                req = waiting[0]
                prob = problems[req.rid]
                if self.work_cap is not None and (active or building or ready):
                    ahead = pool is not None and not building and not ready
                    if not ahead and sum(work.values()) + self.be.cost(prob) > self.work_cap:
                        break
                need = self.be.footprint(prob)
                if need > self.budget:
                    waiting.popleft()
                    r = results[req.rid]
                    r.status, r.error = "rejected", f"footprint {need} exceeds budget {self.budget}"
                    r.finished = self.clock() - t0
                    continue
                if used + need > self.budget:
                    break
                waiting.popleft()
                r = results[req.rid]
                r.admitted = self.clock() - t0
                used += need
                work[req.rid] = self.be.cost(prob)
                if pool is not None:
                    building.append((req, pool.submit(self.be.start, prob), need))
                    continue
                try:
                    h = self.be.start(prob)
                except Exception as e:  # a failed build isolates this request only
                    fail_build(req, need, e)
                    continue
                ready.append((req, h, need))
            # built requests join the stepped solves within the work cap (the
            # first one always)
            while ready:
                req, h, need = ready[0]
                if (self.work_cap is not None and active and
                        active_work() + work[req.rid] > self.work_cap):
                    break
                ready.popleft()
                active.append((req, h, need))
            if not active:
                if building:
                    wait([f for _, f, _ in building], timeout=0.05, return_when=FIRST_COMPLETED)
                elif pending and not waiting:
                    self.sleep(max(0.0, min(0.05, pending[0].arrival - (self.clock() - t0))))
                continue
            states = self.be.step([h for _, h, _ in active])
            keep = []
            for (req, h, need), st in zip(active, states):
                if st == 0:
                    keep.append((req, h, need))
                    continue
                r = results[req.rid]
                if st < 0:
                    r.status, r.error = "failed", f"solver error {st}"
                    try:
                        self.be.finish(h)
                    except Exception as e:
                        r.error += f" ({e})"
                else:
                    try:
                        beta, info = self.be.finish(h)
                        r.status = "done"
                        r.iters = info["iters"]
                        r.relres_true = info["relres_true"]
                        r.converged = info["converged"]
                        r.beta = beta
                    except Exception as e:
                        r.status, r.error = "failed", str(e)
                r.finished = self.clock() - t0
                used -= need
                work.pop(req.rid, None)
                problems.pop(req.rid, None)
                if self.on_finish:
                    self.on_finish(r)
            active = keep
        return results


def serve_one_at_a_time(backend, stream, make_problem, clock=time.perf_counter,
                        sleep=time.sleep, on_finish=None):
    """Baseline: the same arrival trace served one request at a time (FIFO)."""
    results = {}
    t0 = clock()
    for req in sorted(stream, key=lambda r: r.arrival):
        now = clock() - t0
        if req.arrival > now:
            sleep(req.arrival - now)
        r = Result(req.rid, req.arrival)
        r.admitted = clock() - t0
        prob = make_problem(req)
        try:
            h = backend.start(prob)
            while True:
                st = backend.step([h])[0]
                if st != 0:
                    break
            if st < 0:
                r.status, r.error = "failed", f"solver error {st}"
                backend.finish(h)
            else:
                beta, info = backend.finish(h)
                r.status, r.iters, r.relres_true, r.beta = "done", info["iters"], \
                    info["relres_true"], beta
                r.converged = info["converged"]
        except Exception as e:
            r.status, r.error = "failed", str(e)
        r.finished = clock() - t0
        results[req.rid] = r
        if on_finish:
            on_finish(r)
    return results


def summarize(results):
    lat = np.array([r.latency for r in results.values() if r.status == "done"])
    done = len(lat)
    span = max((r.finished for r in results.values()), default=0.0)
    first = min((r.arrival for r in results.values()), default=0.0)
    return {
        "requests": len(results),
        "done": done,
        "failed": sum(r.status == "failed" for r in results.values()),
        "rejected": sum(r.status == "rejected" for r in results.values()),
        "not_converged": sum(r.status == "done" and not r.converged for r in results.values()),
        "max_relres_true": max((r.relres_true for r in results.values() if r.status == "done"),
                               default=None),
        "p50_s": float(np.percentile(lat, 50)) if done else None,
        "p99_s": float(np.percentile(lat, 99)) if done else None,
        "mean_s": float(lat.mean()) if done else None,
        "solves_per_s": done / max(span - first, 1e-9),
        "makespan_s": span,
    }
