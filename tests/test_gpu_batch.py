"""Batched systems and graph replay (needs an MI355X).

A system's arithmetic does not depend on the other systems of its batch, on
how its steps are split over calls, or on whether the step is replayed from a
HIP graph: its state, history and diagnostics must be bit-identical to the
same system stepped alone.  Against the oracle each system keeps the
tolerances of the single-system parity tests.
"""
import numpy as np
import pytest

from oracle.oracle import OracleSystem
from paper_1301_1714_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dem():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1301_1714_amd import dem as D
    D.lib()
    return D


def small_system(seed, n, precision="fp64", law="linear", **kw):
    side = ((n * 2.0) ** (1.0 / 3.0) + 1.0) * 0.95 * 2 * 0.01
    c = W.overlapping_cloud(seed, n, box=(side, 0.8 * side, 1.2 * side), r_mean=0.01, r_spread=0.3,
                            law=law, precision=precision, **kw)
    c["params"] = dict(c["params"], mu=kw.get("mu", 0.2), eta_t_ratio=0.5, dt=2e-6)
    return c


def mix(precision="fp64", law="linear"):
    """Systems of uneven size and different materials, boxes and walls."""
    return [
        small_system(11, 1500, precision, law, kn=3e4, restitution=0.6, mu=0.5),
        small_system(12, 37, precision, law, kn=2e5, restitution=0.9, mu=0.1, walls=0x15),
        small_system(13, 4100, precision, law, kn=1e5, restitution=0.8, mu=0.3),
        small_system(14, 1, precision, law),
        small_system(15, 700, precision, law, kn=8e5, restitution=0.95, mu=0.6, walls=0),
    ]


def alone(dem, c, calls, **kw):
    s = dem.System(c["params"], c["x"], c["v"], c["omega"], c["r"], **kw)
    for k in calls:
        s.step(k)
    return s


def same_state(a, b):
    for key in ("x", "v", "omega", "F", "T"):
        assert np.array_equal(a[key], b[key]), key


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_is_bit_identical_to_each_system_alone(dem, precision):
    systems = mix(precision)
    b = dem.Batch(systems)
    plan = [[5, 0, 9, 3, 1], [3, 7, 0, 0, 6], [0, 0, 0, 0, 0], [2, 2, 2, 2, 2]]
    for steps in plan:
        b.step(steps)
    diag = b.diagnostics()
    for k, c in enumerate(systems):
        total = sum(p[k] for p in plan)
        s = alone(dem, c, [total])
        same_state(b.read_state(k), s.read_state())
        pb, db = b.read_contacts(k)
        ps, ds = s.read_contacts()
        assert np.array_equal(pb, ps) and np.array_equal(db, ds)
        assert np.array_equal(diag[k], s.diagnostics())


@pytest.mark.parametrize("law", ["hertz", "simple"])
def test_batch_other_laws_bit_identical(dem, law):
    systems = mix("mixed", law)[:3]
    b = dem.Batch(systems)
    b.step([4, 9, 1])
    for k, (c, n) in enumerate(zip(systems, [4, 9, 1])):
        same_state(b.read_state(k), alone(dem, c, [n]).read_state())


def test_batch_tracks_the_oracle(dem):
    systems = mix("fp64")
    b = dem.Batch(systems)
    steps = [20, 13, 20, 4, 17]
    b.step(steps)
    for k, c in enumerate(systems):
        o = OracleSystem(c["params"], c["x"], c["v"], c["omega"], c["r"])
        o.step(steps[k])
        sg, so = b.read_state(k), o.read_state()
        assert np.max(np.abs(sg["x"] - so["x"])) < 1e-12
        vs = max(np.abs(so["v"]).max(), 1e-300)
        assert np.max(np.abs(sg["v"] - so["v"])) < 1e-9 * vs
        pg, _ = b.read_contacts(k)
        po, _ = o.read_contacts()
        assert np.array_equal(pg, po)


def test_split_calls_are_bit_identical(dem):
    c = small_system(21, 3000, "mixed")
    a = alone(dem, c, [12])
    b = alone(dem, c, [1, 4, 0, 7])
    same_state(a.read_state(), b.read_state())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_is_bit_identical(dem, precision):
    import torch
    c = small_system(22, 3000, precision)
    plain = alone(dem, c, [3, 1, 6])
    st = torch.cuda.Stream()
    g = dem.System(c["params"], c["x"], c["v"], c["omega"], c["r"], stream=st)
    g.use_graph(True)
    for k in (3, 1, 6):
        g.step(k)
    same_state(plain.read_state(), g.read_state())
    pp, dp = plain.read_contacts()
    pg, dg = g.read_contacts()
    assert np.array_equal(pp, pg) and np.array_equal(dp, dg)
    # replays after reads and other work, then back to plain launches
    g.step(2)
    plain.step(2)
    g.use_graph(False)
    g.step(3)
    plain.step(3)
    same_state(plain.read_state(), g.read_state())


def test_batch_graph_replay_is_bit_identical(dem):
    systems = mix("mixed")
    a = dem.Batch(systems)
    g = dem.Batch(systems)
    g.use_graph(True)
    plan = [[5, 0, 9, 3, 1], [3, 7, 0, 0, 6], [1, 1, 1, 1, 1]]
    for steps in plan:
        a.step(steps)
        g.step(steps)
    for k in range(len(systems)):
        same_state(a.read_state(k), g.read_state(k))


def test_graph_needs_a_stream(dem):
    c = small_system(23, 100)
    s = dem.System(c["params"], c["x"], c["v"], c["omega"], c["r"])
    if s.stream.cuda_stream == 0:
        with pytest.raises(dem.DemError):
            s.use_graph(True)


def test_batch_rejects_mixed_laws_and_bad_steps(dem):
    a = small_system(24, 50)
    b = small_system(25, 50, law="hertz")
    with pytest.raises(dem.DemError):
        dem.Batch([a, b])
    bt = dem.Batch([a, small_system(26, 60)])
    with pytest.raises(dem.DemError):
        bt.step([1, -1])
    with pytest.raises((IndexError, dem.DemError)):
        bt.read_state(2)


def test_batch_with_an_empty_system(dem):
    a = small_system(27, 300)
    e = dict(a, x=np.zeros((0, 3)), v=np.zeros((0, 3)), omega=np.zeros((0, 3)), r=np.zeros(0))
    b = dem.Batch([e, a, e])
    b.step([3, 3, 3])
    same_state(b.read_state(1), alone(dem, a, [3]).read_state())
    d = b.diagnostics()
    assert np.all(d[0] == 0) and np.all(d[2] == 0)
