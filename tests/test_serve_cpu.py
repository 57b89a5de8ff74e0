"""Scheduler tests on the CPU with a fake backend (no numerics): admission by
HBM footprint, FIFO order, continuous admission as memory frees, isolation
of failed requests, rejection of requests larger than the budget."""
from dataclasses import dataclass

from paper_2304_12465_amd.serve import Server, serve_one_at_a_time, summarize


@dataclass
class Req:
    rid: int
    arrival: float


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-3)


class FakeBackend:
    """A request needs `steps` ticks of 10 ms; `fail` = 'build' | 'solve'."""

    def __init__(self, clock):
        self.clock = clock
        self.used = 0
        self.max_used = 0
        self.started = []

    def footprint(self, prob):
        return prob["fp"]

    def cost(self, prob):
        return prob["steps"]

    def start(self, prob):
        if prob.get("fail") == "build":
            raise RuntimeError("injected build failure")
        self.used += prob["fp"]
        self.max_used = max(self.max_used, self.used)
        self.started.append(prob["rid"])
        return {"p": prob, "left": prob["steps"]}

    def step(self, handles):
        self.clock.t += 0.01
        out = []
        for h in handles:
            h["left"] -= 1
            if h["p"].get("fail") == "solve" and h["left"] <= 1:
                out.append(-4)
            else:
                out.append(1 if h["left"] <= 0 else 0)
        return out

    def finish(self, h):
        self.used -= h["p"]["fp"]
        return None, {"iters": h["p"]["steps"], "relres_true": 1e-7, "converged": True}

    def cancel(self, h):
        self.used -= h["p"]["fp"]


def run(problems, arrivals, budget, max_active=64, order="fifo", build_workers=0, work_cap=None):
    clk = FakeClock()
    be = FakeBackend(clk)
    reqs = [Req(i, a) for i, a in enumerate(arrivals)]
    srv = Server(be, budget, max_active=max_active, clock=clk, sleep=clk.sleep, order=order,
                 build_workers=build_workers, work_cap=work_cap)
    res = srv.run(reqs, lambda r: dict(problems[r.rid], rid=r.rid))
    return res, be


def test_budget_is_never_exceeded_and_all_finish():
    probs = [dict(fp=30, steps=5 + i % 4) for i in range(12)]
    res, be = run(probs, [0.005 * i for i in range(12)], budget=100)
    assert be.max_used <= 100
    assert all(r.status == "done" for r in res.values())
    assert all(r.latency >= 0 for r in res.values())
    assert be.started == sorted(be.started)  # FIFO admission


def test_continuous_admission_as_memory_frees():
    # 3 fit at once; later arrivals join while earlier ones are still running
    probs = [dict(fp=30, steps=20)] * 3 + [dict(fp=30, steps=2)] * 3
    res, be = run(probs, [0.0, 0.0, 0.0, 0.0, 0.0, 0.001], budget=100)
    first_done = min(res[i].finished for i in range(3))
    assert res[3].admitted < 0.05 + first_done
    assert all(r.status == "done" for r in res.values())
    # request 3 was admitted while requests 0..2 were on the device
    assert res[3].admitted >= min(res[i].admitted for i in range(3))


def test_oversized_request_rejected_not_oom():
    probs = [dict(fp=50, steps=3), dict(fp=500, steps=3), dict(fp=50, steps=3)]
    res, be = run(probs, [0, 0, 0], budget=100)
    assert res[1].status == "rejected"
    assert res[0].status == "done" and res[2].status == "done"
    assert be.max_used <= 100


def test_failures_are_isolated():
    probs = [dict(fp=10, steps=4), dict(fp=10, steps=4, fail="build"),
             dict(fp=10, steps=6, fail="solve"), dict(fp=10, steps=5)]
    res, be = run(probs, [0, 0, 0, 0], budget=100)
    assert res[1].status == "failed" and "build" in res[1].error
    assert res[2].status == "failed"
    assert res[0].status == "done" and res[3].status == "done"
    assert be.used == 0


def test_max_active_limit_and_summary():
    probs = [dict(fp=1, steps=3)] * 10
    res, be = run(probs, [0] * 10, budget=1000, max_active=2)
    assert all(r.status == "done" for r in res.values())
    s = summarize(res)
    assert s["done"] == 10 and s["p50_s"] <= s["p99_s"]


def test_one_at_a_time_baseline():
    clk = FakeClock()
    be = FakeBackend(clk)
    reqs = [Req(i, 0.0) for i in range(4)]
    res = serve_one_at_a_time(be, reqs, lambda r: dict(fp=1, steps=3, rid=r.rid), clock=clk,
                              sleep=clk.sleep)
    lat = sorted(r.latency for r in res.values())
    assert lat == sorted(lat) and lat[-1] > lat[0]


def test_shortest_first_admission_lowers_mean_latency():
    probs = [dict(fp=10, steps=s) for s in (40, 30, 2, 3, 1, 2)]
    fifo, _ = run(probs, [0.0] * 6, budget=1000, max_active=1)
    sjf, be = run(probs, [0.0] * 6, budget=1000, max_active=1, order="sjf")
    mean = lambda res: sum(r.latency for r in res.values()) / len(res)
    assert mean(sjf) < mean(fifo)
    assert be.started[:2] == [4, 2]  # smallest work first


def test_background_builds_keep_budget_and_isolate_failures():
    # builds on a worker thread: admission still counts the footprint at
    # once, the budget and the active limit hold, a failed build is isolated
    probs = [dict(fp=30, steps=4 + i % 3) for i in range(9)]
    probs[4] = dict(fp=30, steps=4, fail="build")
    probs[6] = dict(fp=30, steps=5, fail="solve")
    res, be = run(probs, [0.004 * i for i in range(9)], budget=100, max_active=3,
                  build_workers=1)
    assert be.max_used <= 100
    assert res[4].status == "failed" and "build" in res[4].error
    assert res[6].status == "failed"
    assert all(res[i].status == "done" for i in range(9) if i not in (4, 6))
    assert be.used == 0
    assert be.started == sorted(be.started)  # FIFO admission, one worker


class SharingBackend(FakeBackend):
    """A step of the GPU divides its time among the active requests: each
    request's remaining work falls by 10 ms / (number active) per 10 ms tick
    (processor sharing, the regime of requests that each fill the GPU)."""

    def step(self, handles):
        self.clock.t += 0.01
        out = []
        for h in handles:
            h["left"] -= 1.0 / len(handles)
            out.append(1 if h["left"] <= 1e-9 else 0)
        return out


def test_work_cap_keeps_large_requests_from_sharing():
    # ten requests of equal work arrive at once: with no cap they share the
    # GPU and all finish near the end; with a cap of one request's work they
    # run one after another and the mean latency nearly halves, with the
    # same makespan
    probs = [dict(fp=1, steps=10) for _ in range(10)]

    def go(cap):
        clk = FakeClock()
        be = SharingBackend(clk)
        srv = Server(be, 1000, max_active=64, clock=clk, sleep=clk.sleep, work_cap=cap)
        res = srv.run([Req(i, 0.0) for i in range(10)], lambda r: dict(probs[r.rid], rid=r.rid))
        return res, be
    shared, _ = go(None)
    capped, be = go(10)
    mean = lambda res: sum(r.latency for r in res.values()) / len(res)
    span = lambda res: max(r.finished for r in res.values())
    assert all(r.status == "done" for r in capped.values())
    assert mean(capped) < 0.6 * mean(shared)
    assert abs(span(capped) - span(shared)) < 0.05
    assert be.started == sorted(be.started)


def test_work_cap_batches_small_requests_and_always_admits_one():
    # small requests share steps up to the cap; a request above the cap on
    # its own is still admitted when nothing else runs
    probs = [dict(fp=1, steps=2) for _ in range(6)] + [dict(fp=1, steps=50)]
    res, be = run(probs, [0.0] * 7, budget=1000, work_cap=6)
    assert all(r.status == "done" for r in res.values())
    assert res[6].admitted >= max(res[i].admitted for i in range(6))
    firsts = sorted(res[i].admitted for i in range(6))
    assert firsts[2] == firsts[0]  # three small ones admitted together (3 x 2 <= 6)


def test_work_cap_builds_the_next_request_ahead_but_steps_within_the_cap():
    # with a build worker, the next request is built while the current one
    # steps (its build is started before the current one finishes), but it
    # joins the stepped solves only when the cap leaves room
    probs = [dict(fp=1, steps=10) for _ in range(5)]
    clk = FakeClock()
    be = SharingBackend(clk)
    srv = Server(be, 1000, max_active=64, clock=clk, sleep=clk.sleep, work_cap=10,
                 build_workers=1)
    res = srv.run([Req(i, 0.0) for i in range(5)], lambda r: dict(probs[r.rid], rid=r.rid))
    assert all(r.status == "done" for r in res.values())
    fin = sorted((r.finished, rid) for rid, r in res.items())
    assert [rid for _, rid in fin] == list(range(5))     # one after another
    for i in range(1, 5):
        assert res[i].admitted < res[i - 1].finished     # built ahead
    gaps = [fin[i][0] - fin[i - 1][0] for i in range(1, 5)]
    assert max(gaps) < 0.12                              # ~10 steps of 10 ms each
