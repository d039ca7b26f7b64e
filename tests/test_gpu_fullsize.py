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
