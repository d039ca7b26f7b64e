"""Optional contact terms on the GPU (cohesion, rolling resistance: force
terms composed with the practical law, Sec. 4's add-or-remove requirement)
against the oracle's, through the C ABI: forces and torques on identical
states within the force tolerance, FP64 trajectories within 1e-12, and a
batch mixing systems with and without terms bitwise equal to each alone."""
import numpy as np
import pytest

from oracle.oracle import OracleSystem
from paper_1301_1714_amd import workloads as W
from parity_util import assert_forces_close

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}


@pytest.fixture(scope="module")
def dem():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1301_1714_amd import dem as D
    D.lib()
    return D


def cloud(seed, n, terms, precision="fp64", law="linear", walls=W.ALL_WALLS):
    side = (n * 1.6) ** (1.0 / 3.0) * 0.95 * 2 * 0.01
    c = W.overlapping_cloud(seed, n, box=(side, 0.8 * side, 1.2 * side), r_mean=0.01, r_spread=0.3,
                            spacing=0.95, law=law, precision=precision, walls=walls)
    # a pull of the order of the typical contact force, a noticeable couple
    fc = 0.2 * c["params"]["kn"] * 0.01 * 0.02 if law == "linear" else 0.5
    c["params"] = dict(c["params"], terms=terms, cohesion=fc, rolling_mu=0.05, mu=0.3, eta_t_ratio=0.5, dt=2e-6)
    return c


CASES = {
    "fp64_linear_both": dict(seed=41, n=2500, terms=("cohesion", "rolling")),
    "mixed_linear_both": dict(seed=42, n=3001, terms=("cohesion", "rolling"), precision="mixed"),
    "fp64_hertz_rolling": dict(seed=43, n=2000, terms=("rolling",), law="hertz"),
    "mixed_hertz_cohesion": dict(seed=44, n=2200, terms=("cohesion",), law="hertz", precision="mixed"),
    "fp64_linear_rolling_nowalls": dict(seed=45, n=1800, terms=("rolling",), walls=0),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_forces_with_terms(dem, name):
    c = cloud(**CASES[name])
    g = dem.System(c["params"], c["x"], c["v"], c["omega"], c["r"])
    o = OracleSystem(c["params"], c["x"], c["v"], c["omega"], c["r"])
    F, T, Fa, Ta = o.forces_scale()
    Fg, Tg = g.forces()
    assert_forces_close(Fg, Tg, F, T, Fa, Ta, TOL[c["params"]["precision"]])
    # the terms matter on this state
    plain = dict(c["params"], terms=())
    Fp, Tp = dem.System(plain, c["x"], c["v"], c["omega"], c["r"]).forces()
    changed = np.abs(Tp - Tg).max() if "rolling" in c["params"]["terms"] else np.abs(Fp - Fg).max()
    assert changed > 1e-3 * max(np.abs(Tg).max(), np.abs(Fg).max() * 1e-3)


@pytest.mark.parametrize("name", ["fp64_linear_both", "fp64_hertz_rolling"])
def test_fp64_steps_with_terms_track_the_oracle(dem, name):
    c = cloud(**CASES[name])
    g = dem.System(c["params"], c["x"], c["v"], c["omega"], c["r"])
    o = OracleSystem(c["params"], c["x"], c["v"], c["omega"], c["r"])
    for _ in range(4):
        g.step(5)
        o.step(5)
    sg, so = g.read_state(), o.read_state()
    assert np.max(np.abs(sg["x"] - so["x"])) < 1e-12
    assert np.max(np.abs(sg["v"] - so["v"])) < 1e-9 * np.abs(so["v"]).max()
    assert np.max(np.abs(sg["omega"] - so["omega"])) < 1e-9 * np.abs(so["omega"]).max()
    pg, dg = g.read_contacts()
    po, do = o.read_contacts()
    assert np.array_equal(pg, po)
    assert np.max(np.abs(dg - do)) <= 1e-9 * max(np.abs(do).max(), 1e-300)


def test_batch_mixing_terms_matches_alone(dem):
    cs = [cloud(51, 1200, ("cohesion", "rolling")), cloud(52, 900, ()), cloud(53, 1000, ("rolling",))]
    systems = [dict(params=c["params"], x=c["x"], v=c["v"], omega=c["omega"], r=c["r"]) for c in cs]
    b = dem.Batch(systems)
    b.step([10, 10, 6])
    for k, (c, steps) in enumerate(zip(cs, [10, 10, 6])):
        g = dem.System(c["params"], c["x"], c["v"], c["omega"], c["r"])
        g.step(steps)
        sa, sb = g.read_state(), b.read_state(k)
        for key in ("x", "v", "omega", "F", "T"):
            assert np.array_equal(sa[key], sb[key]), (k, key)


def test_terms_refused_with_the_simple_law(dem):
    c = cloud(54, 300, ("cohesion",), law="simple")
    with pytest.raises(dem.DemError):
        dem.System(c["params"], c["x"], c["v"], c["omega"], c["r"])
