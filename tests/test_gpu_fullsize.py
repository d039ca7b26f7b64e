"""Parity at the full size of the dense-bed benchmark (2^24 spheres), in the
configuration the benchmark times (mixed precision, linear law, one lane per
particle detection), on every output rather than a sample (needs an MI355X).

The state is the benchmark's starting lattice at full radii (neighbouring
large spheres overlap, so most spheres start with contacts) with seeded
random velocities and spins, stepped three times on the GPU so that the
contacts carry tangential history.  On that state, GPU and oracle must give
the same cell ids, sorted order and cell starts and the same contact lists,
bit for bit, and forces and torques within 1e-5 of each particle's
contact-force scale (FP32 forces).  The oracle needs about a minute and a
half of one host core at this size.
"""
import numpy as np
import pytest

from oracle.oracle import OracleSystem
from paper_1301_1714_amd import workloads as W
from parity_util import assert_forces_close

pytestmark = pytest.mark.gpu

N_FULL = 1 << 24
FILL_HEIGHT = 0.93  # as the benchmark's bed


def test_dense_bed_full_size_matches_the_oracle():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1301_1714_amd import dem
    dem.lib()
    w = W.dense_bed_lattice(seed=3000, n=N_FULL, fill_height=FILL_HEIGHT)
    p = w["params"]
    assert p["precision"] == "mixed" and p["law"] == "linear" and p.get("tile_cells", 0) == 0
    rng = np.random.default_rng(77)
    v = rng.normal(0.0, 0.01, (N_FULL, 3))
    om = rng.normal(0.0, 1.0, (N_FULL, 3))
    s = dem.System(p, w["x"], v, om, w["r"])
    s.step(3)
    st = s.read_state()
    pairs, dts = s.read_contacts()
    s.close()
    assert len(pairs) > N_FULL // 2 and np.abs(dts).max() > 0
    kw = dict(F0=st["F"], T0=st["T"], hist_pairs=pairs, hist_dt=dts)
    g = dem.System(p, st["x"], st["v"], st["omega"], w["r"], **kw)
    o = OracleSystem(p, st["x"], st["v"], st["omega"], w["r"], **kw)
    assert g.grid_dims() == o.grid_dims()
    for a, b in zip(g.read_grid(), o.read_grid()):
        assert np.array_equal(a, b)
    assert np.array_equal(g.contacts(), o.contacts())
    F, T, Fa, Ta = o.forces_scale()
    Fg, Tg = g.forces()
    assert_forces_close(Fg, Tg, F, T, Fa, Ta, 1e-5)


def _dem():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1301_1714_amd import dem
    dem.lib()
    return dem


def _same_state_parity(dem, p, st, r, pairs, dts, tol):
    """GPU and oracle on one state (positions, velocities, spins, history)."""
    kw = dict(F0=st["F"], T0=st["T"], hist_pairs=pairs, hist_dt=dts)
    g = dem.System(p, st["x"], st["v"], st["omega"], r, **kw)
    o = OracleSystem(p, st["x"], st["v"], st["omega"], r, **kw)
    if p.get("cell_divisor", 1) == 1:  # finer cells: another grid, the same contacts
        assert g.grid_dims() == o.grid_dims()
        for a, b in zip(g.read_grid(), o.read_grid()):
            assert np.array_equal(a, b)
    assert np.array_equal(g.contacts(), o.contacts())
    F, T, Fa, Ta = o.forces_scale()
    Fg, Tg = g.forces()
    g.close()
    assert_forces_close(Fg, Tg, F, T, Fa, Ta, tol)


@pytest.mark.parametrize("law", ["linear", "simple"])
def test_settling_gas_1M_matches_the_oracle(law):
    # the single-system workload of 2^20 spheres at packing fraction 0.3,
    # practical and simple laws, after 2,000 GPU steps (0.02 time units:
    # long enough for collisions, which last about ten steps, to be under
    # way throughout the gas)
    dem = _dem()
    w = W.gas_mixed(seed=2000, law=law)
    p = w["params"]
    s = dem.System(p, w["x"], w["v"], w["omega"], w["r"])
    s.step(2000)
    st = s.read_state()
    pairs, dts = s.read_contacts()  # the history table (empty for Eq. 1, which keeps none)
    assert np.count_nonzero(s.contacts()[:, 1] >= 0) > 500
    s.close()
    if law == "linear":
        assert np.abs(dts).max() > 0
    _same_state_parity(dem, p, st, w["r"], pairs, dts, 1e-5)


def test_batched_256_systems_full_size():
    # the batched workload at its full size (256 systems, 10.9M spheres),
    # every combination of cell factor and detection launch shape (and the
    # cell divisor 2 with the direct sweep), uneven
    # step counts, graph replay: sampled systems are bit-identical to the
    # same system stepped alone, and the smallest match the oracle on the
    # state the batch reached
    dem = _dem()
    shapes = [(f, t, 1) for f in (1.0, 1.25, 1.5, 2.0) for t in (0, -1, 8, 16)]
    shapes += [(f, 0, 2) for f in (1.0, 1.25, 1.5, 2.0)]
    count = 256
    factors = [shapes[k % len(shapes)][0] for k in range(count)]
    tiles = [shapes[k % len(shapes)][1] for k in range(count)]
    divisors = [shapes[k % len(shapes)][2] for k in range(count)]
    systems = W.batched_systems(seed=4000, count=count, cell_factors=factors, tiles=tiles, divisors=divisors)
    steps = [3 + (k % 5) for k in range(count)]
    b = dem.Batch(systems)
    b.use_graph(True)
    b.step(steps)
    sizes = np.array([len(s["r"]) for s in systems])
    rng = np.random.default_rng(11)
    sample = sorted(set(rng.choice(count, 14, replace=False).tolist()) | set(np.argsort(sizes)[:3].tolist())
                    | set(range(len(shapes))))
    import torch
    stream = torch.cuda.Stream()  # graph capture needs a stream of its own
    for k in sample:
        s = systems[k]
        a = dem.System(s["params"], s["x"], s["v"], s["omega"], s["r"], stream=stream)
        a.use_graph(True)
        a.step(steps[k])
        ra, rb = a.read_state(), b.read_state(k)
        a.close()
        for key in ("x", "v", "omega", "F", "T"):
            assert np.array_equal(ra[key], rb[key]), (k, key)
    for k in np.argsort(sizes)[:3]:
        s = systems[int(k)]
        pairs, dts = b.read_contacts(int(k))
        _same_state_parity(dem, s["params"], b.read_state(int(k)), s["r"], pairs, dts, 1e-5)
    b.close()
