"""The serving loop and the autotuner on the GPU (needs an MI355X).

Each served request's final state must be bit-identical to its system
stepped alone by the plain single-system path; a request that leaves its
domain fails alone; the autotuner's choice is a function of the system's
class, and a batch built with tuned cells stays bit-identical to its systems
run alone.
"""
import numpy as np
import pytest

from paper_1301_1714_amd import autotune, serve
from paper_1301_1714_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ex():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1301_1714_amd import dem
    dem.lib()
    return serve.GpuExecutor(use_graph=True)


def requests(count, seed, n_hi=6000, steps_hi=60, rate=200.0):
    specs = W.serving_requests(seed=seed, count=count, n_lo=200, n_hi=n_hi, steps_lo=5, steps_hi=steps_hi)
    arr = W.poisson_arrivals(seed, count, rate=rate)
    out = []
    for k, (d, a) in enumerate(zip(specs, arr)):
        s = W.unit_box_system(d["seed"], d["n"], d["kn"], d["restitution"], d["mu"], d["phi"])
        out.append(serve.Request(k, s, d["steps"], a))
    return out


def test_served_results_are_bit_identical_to_alone(ex):
    reqs = requests(16, seed=31)
    srv = serve.Server(ex, hbm_budget=2 << 30, max_slots=8, chunk=16)
    done = srv.run(reqs)
    assert sorted(r.rid for r in done) == list(range(16))
    assert srv.peak_slots <= 8
    for r in done:
        assert r.error is None, r.error
        ref = ex.run_alone(r.system, r.steps)
        for key in ("x", "v", "omega", "F", "T"):
            assert np.array_equal(r.result[key], ref[key]), (r.rid, key)


def test_served_failure_is_isolated(ex):
    reqs = requests(5, seed=37)
    bad = reqs[1]
    s = dict(bad.system)
    s["params"] = dict(s["params"], wall_mask=0)
    v = np.array(s["v"], copy=True)
    v[0] = (1.0e4, 0.0, 0.0)
    s["v"] = v
    bad.system = s
    bad.steps = 300
    for r in reqs:
        r.arrival = 0.0
    srv = serve.Server(ex, hbm_budget=2 << 30, max_slots=8, chunk=100)
    done = srv.run(reqs)
    assert len(done) == 5
    for r in done:
        if r.rid == bad.rid:
            assert r.error is not None
        else:
            assert r.error is None
            ref = ex.run_alone(r.system, r.steps)
            assert np.array_equal(r.result["x"], ref["x"])


def test_autotuned_batch_is_deterministic(ex, tmp_path):
    from paper_1301_1714_amd import dem
    draws = W.batched_draws(seed=41, count=6, n_lo=500, n_hi=3000)
    keys = [autotune.system_class(d["n"], d["phi"]) for d in draws]
    table = autotune.tune(keys, steps=5, factors=(1.0, 1.5), tiles=(0, 4), divisors=(1, 2))
    path = str(tmp_path / "t.json")
    table.save(path)
    t2 = autotune.Table.load(path)
    f1 = autotune.factors_for(draws, table)
    tl = autotune.tiles_for(draws, table)
    dv = autotune.divisors_for(draws, table)
    assert f1 == autotune.factors_for(draws, t2) and tl == autotune.tiles_for(draws, t2)
    assert dv == autotune.divisors_for(draws, t2)
    assert all(f in (1.0, 1.5) for f in f1) and all(t in (0, 4) for t in tl)
    assert all(d == 1 or t == 0 for d, t in zip(dv, tl))
    systems = W.batched_systems(seed=41, count=6, n_lo=500, n_hi=3000, cell_factors=f1, tiles=tl, divisors=dv)
    b = dem.Batch(systems)
    b.use_graph(True)
    b.step([9, 3, 0, 7, 9, 1])
    for k, n in enumerate([9, 3, 0, 7, 9, 1]):
        ref = ex.run_alone(systems[k], n)
        assert np.array_equal(b.read_state(k)["x"], ref["x"])


def test_served_results_track_the_oracle(ex):
    """Requests in FP64 served concurrently with others (admitted while they
    run, compacted when a member finishes): each result agrees with the FP64
    oracle stepping the same request alone, within 1e-12 in x."""
    from oracle.oracle import OracleSystem
    reqs = requests(8, seed=43, n_hi=1500, steps_hi=40)
    for r in reqs:
        r.system = dict(r.system, params=dict(r.system["params"], precision="fp64"))
    srv = serve.Server(ex, hbm_budget=2 << 30, max_slots=4, chunk=8)
    done = srv.run(reqs)
    assert len(done) == 8
    for r in done:
        assert r.error is None, r.error
        s = r.system
        o = OracleSystem(s["params"], s["x"], s["v"], s["omega"], s["r"])
        o.step(r.steps)
        want = o.read_state()
        assert np.max(np.abs(r.result["x"] - want["x"])) < 1e-12, r.rid
        assert np.max(np.abs(r.result["v"] - want["v"])) < 1e-9 * max(np.abs(want["v"]).max(), 1e-12), r.rid
