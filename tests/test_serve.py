"""The continuous-batching scheduler, driven on the CPU by a stand-in executor
built on the oracle (the GPU executor is exercised in test_gpu_serve.py).

Checks: every request finishes with the result of its system stepped alone;
the HBM budget and the slot limit hold at every admission; requests that
arrive while others run are admitted before those finish (continuous
batching, not a queue); a request that fails fails alone; the one-at-a-time
baseline's FIFO latencies follow the queue recursion.
"""
import numpy as np
import pytest

from oracle.oracle import OracleError, OracleSystem
from paper_1301_1714_amd import serve
from paper_1301_1714_amd import workloads as W


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, d):
        self.t += max(d, 0.0)


class OracleGroup:
    def __init__(self, systems, clock):
        self.sys = [OracleSystem(s["params"], s["x"], s["v"], s["omega"], s["r"], F0=s.get("F"), T0=s.get("T"),
                                 hist_pairs=s.get("hist_pairs"), hist_dt=s.get("hist_dt")) for s in systems]
        self.clock = clock
        self.err = None

    def step(self, steps):
        for s, k in zip(self.sys, steps):
            if self.err is None and k:
                try:
                    s.step(int(k))
                except OracleError as e:
                    self.err = e
        self.clock.t += 1e-3

    def sync(self):
        if self.err is not None:
            raise self.err

    def read_state(self, k):
        return self.sys[k].read_state()

    def read_contacts(self, k):
        return self.sys[k].read_contacts()

    def close(self):
        self.sys = []


class OracleExecutor:
    errors = (OracleError,)

    def __init__(self, clock):
        self.clock = clock
        self.started = []

    def workspace_bytes(self, systems):
        return 4096 + 1000 * sum(len(s["r"]) for s in systems)

    def start(self, systems):
        self.started.append(len(systems))
        return OracleGroup(systems, self.clock)


def make_requests(count=10, seed=7):
    specs = W.serving_requests(seed=seed, count=count, n_lo=20, n_hi=200, steps_lo=3, steps_hi=40)
    arr = W.poisson_arrivals(seed, count, rate=400.0)
    reqs = []
    for k, (d, a) in enumerate(zip(specs, arr)):
        s = W.unit_box_system(d["seed"], d["n"], d["kn"], d["restitution"], d["mu"], d["phi"], precision="fp64")
        reqs.append(serve.Request(k, s, d["steps"], a))
    return reqs


def alone(system, steps):
    o = OracleSystem(system["params"], system["x"], system["v"], system["omega"], system["r"])
    o.step(steps)
    return o.read_state()


def test_results_match_each_request_alone_and_limits_hold():
    clk = Clock()
    ex = OracleExecutor(clk)
    reqs = make_requests()
    budget = 4096 * 3 + 1000 * 450
    srv = serve.Server(ex, hbm_budget=budget, max_slots=4, chunk=7, clock=clk, sleep=clk.sleep)
    done = srv.run(reqs)
    assert sorted(r.rid for r in done) == list(range(len(reqs)))
    assert srv.peak_bytes <= budget and srv.peak_slots <= 4
    for r in done:
        assert r.error is None
        ref = alone(r.system, r.steps)
        for key in ("x", "v", "omega"):
            assert np.array_equal(r.result[key], ref[key]), (r.rid, key)
        assert r.t_done >= r.t_admit >= r.arrival


def test_arrivals_join_while_others_run():
    clk = Clock()
    ex = OracleExecutor(clk)
    reqs = make_requests(count=12, seed=11)
    srv = serve.Server(ex, hbm_budget=10 ** 9, max_slots=64, chunk=5, clock=clk, sleep=clk.sleep)
    done = srv.run(reqs)
    assert len(ex.started) > 1  # more than one admission wave
    overlap = any(b.t_admit > a.t_admit and b.t_admit < a.t_done for a in done for b in done)
    assert overlap, "no request was admitted while another was still running"


def test_a_failing_request_fails_alone():
    clk = Clock()
    ex = OracleExecutor(clk)
    reqs = make_requests(count=6, seed=13)
    bad = reqs[2]
    sysb = dict(bad.system)
    sysb["params"] = dict(sysb["params"], wall_mask=0)
    v = np.array(sysb["v"], copy=True)
    v[0] = (1.0e4, 0.0, 0.0)  # leaves the domain within a few steps, no wall in the way
    sysb["v"] = v
    bad.system = sysb
    bad.steps = 200
    for r in reqs:
        r.arrival = 0.0  # all admitted together in one group
    srv = serve.Server(ex, hbm_budget=10 ** 9, max_slots=64, chunk=50, clock=clk, sleep=clk.sleep)
    done = srv.run(reqs)
    assert len(done) == len(reqs)
    assert ex.started[0] == len(reqs)
    for r in done:
        if r.rid == bad.rid:
            assert r.error is not None and r.result is None
        else:
            assert r.error is None
            ref = alone(r.system, r.steps)
            assert np.array_equal(r.result["x"], ref["x"])


def test_a_finished_member_frees_its_share_for_a_waiting_request():
    """A short request admitted beside a long one: when the short one
    finishes, the group is compacted to the long one alone, its memory goes
    back to the pool and the waiting request is admitted while the long one
    still runs; every result is still bitwise the request stepped alone."""
    clk = Clock()
    ex = OracleExecutor(clk)
    reqs = make_requests(count=3, seed=19)
    long_, short, late = reqs
    long_.steps, short.steps, late.steps = 60, 5, 10
    for r in reqs:
        r.arrival = 0.0
    budget = ex.workspace_bytes([long_.system, short.system])  # the third never fits beside both
    assert budget < ex.workspace_bytes([long_.system, short.system, late.system])
    assert budget >= ex.workspace_bytes([long_.system]) + ex.workspace_bytes([late.system])
    srv = serve.Server(ex, hbm_budget=budget, max_slots=8, chunk=5, clock=clk, sleep=clk.sleep)
    done = {r.rid: r for r in srv.run(reqs)}
    assert srv.compactions >= 1 and srv.peak_bytes <= budget
    assert done[late.rid].t_admit < done[long_.rid].t_done
    for r in done.values():
        assert r.error is None
        ref = alone(r.system, r.steps)
        for key in ("x", "v", "omega"):
            assert np.array_equal(r.result[key], ref[key]), (r.rid, key)


def test_oversized_request_is_rejected_not_stuck():
    clk = Clock()
    ex = OracleExecutor(clk)
    reqs = make_requests(count=3, seed=17)
    srv = serve.Server(ex, hbm_budget=4096 + 1000 * 10, max_slots=8, chunk=5, clock=clk, sleep=clk.sleep)
    done = srv.run(reqs)
    assert len(done) == 3 and all(r.error is not None for r in done)


def test_fifo_latencies():
    a = np.array([0.0, 1.0, 1.5, 10.0])
    s = np.array([2.0, 1.0, 0.5, 1.0])
    # finishes at 2, 3, 3.5, 11
    assert np.allclose(serve.fifo_latencies(a, s), [2.0, 2.0, 2.0, 1.0])
    p = serve.percentiles([1.0, 2.0, 3.0])
    assert p["p50"] == 2.0 and p["mean"] == 2.0


def test_rate_for_load():
    assert serve.rate_for_load(0.5, 1e9, 1e8) == pytest.approx(5.0)
