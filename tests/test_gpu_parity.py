"""GPU-vs-oracle parity through the C ABI (needs an MI355X).

Integer results (cell ids, sorted order, cell starts, contact lists) must be
bit-exact; forces on identical states agree per particle within
tol * (sum of the magnitudes of the contact forces on it), tol = 1e-5 with FP32
forces; a particle without contacts gets exactly 0.  In FP64 the bound is
1e-12 relative plus an absolute floor of 1e-14 times the largest particle
scale: the overlap of a barely touching pair carries an absolute rounding
error of about one ulp of r_i + r_j (S - d on one side, (S^2 - d^2)/(S + d) on
the other), which is large relative to that pair's tiny force.
"""
import math

import numpy as np
import pytest

from oracle.oracle import OracleSystem
from paper_1301_1714_amd import workloads as W
from parity_util import assert_forces_close

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}  # the floor below applies 1e-2 * tol


@pytest.fixture(scope="module")
def dem():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1301_1714_amd import dem as D
    D.lib()
    return D


def cloud(seed, n, precision="fp64", law="linear", walls=W.ALL_WALLS, spread=0.3, spacing=0.95, **kw):
    side = (n * 1.3) ** (1.0 / 3.0) * spacing * 2 * 0.01
    return W.overlapping_cloud(seed, n, box=(side, 0.8 * side, 1.2 * side), r_mean=0.01, r_spread=spread,
                               spacing=spacing, law=law, precision=precision, walls=walls, **kw)


CASES = {
    "fp64_linear_3001": dict(seed=1, n=3001),
    "mixed_linear_3001": dict(seed=2, n=3001, precision="mixed"),
    "fp64_hertz_2500": dict(seed=3, n=2500, law="hertz"),
    "mixed_hertz_2500": dict(seed=4, n=2500, law="hertz", precision="mixed"),
    "fp64_simple_1777": dict(seed=5, n=1777, law="simple"),
    "mixed_simple_1777": dict(seed=6, n=1777, law="simple", precision="mixed"),
    "fp64_partial_walls_5000": dict(seed=7, n=5000, walls=0x15, spread=0.5),
    "mixed_nowalls_poly_4097": dict(seed=8, n=4097, walls=0, spread=0.6, precision="mixed"),
}


def make(dem, c, **kw):
    g = dem.System(c["params"], c["x"], c["v"], c["omega"], c["r"], **kw)
    o = OracleSystem(c["params"], c["x"], c["v"], c["omega"], c["r"], **kw)
    return g, o


@pytest.mark.parametrize("name", sorted(CASES))
def test_grid_and_contacts_bit_exact(dem, name):
    c = cloud(**CASES[name])
    g, o = make(dem, c)
    assert g.grid_dims() == o.grid_dims()
    cg, og, sg = g.read_grid()
    co, oo, so = o.read_grid()
    assert np.array_equal(cg, co)
    assert np.array_equal(og, oo)
    assert np.array_equal(sg, so)
    pg = g.contacts()
    po = o.contacts()
    assert len(po) > len(c["r"]) // 3
    assert np.array_equal(pg, po)


@pytest.mark.parametrize("name", sorted(CASES))
def test_forces_on_identical_state(dem, name):
    c = cloud(**CASES[name])
    g, o = make(dem, c)
    F, T, Fa, Ta = o.forces_scale()
    Fg, Tg = g.forces()
    assert_forces_close(Fg, Tg, F, T, Fa, Ta, TOL[c["params"]["precision"]])
    # the creation-time evaluation is the same evaluation
    st = g.read_state()
    assert_forces_close(st["F"], st["T"], F, T, Fa, Ta, TOL[c["params"]["precision"]])


@pytest.mark.parametrize("name", ["fp64_linear_3001", "mixed_linear_3001", "fp64_hertz_2500",
                                  "fp64_partial_walls_5000"])
def test_forces_with_history(dem, name):
    c = cloud(**CASES[name])
    p = dict(c["params"], mu=0.2, eta_t_ratio=0.5, dt=2e-6)
    o = OracleSystem(p, c["x"], c["v"], c["omega"], c["r"])
    o.step(15)
    st = o.read_state()
    pairs, dts = o.read_contacts()
    assert len(pairs) > 100 and np.abs(dts).max() > 0
    kw = dict(F0=st["F"], T0=st["T"], hist_pairs=pairs, hist_dt=dts)
    g = dem.System(p, st["x"], st["v"], st["omega"], c["r"], **kw)
    o2 = OracleSystem(p, st["x"], st["v"], st["omega"], c["r"], **kw)
    gp, gd = g.read_contacts()
    assert np.array_equal(gp, pairs)
    tol = TOL[p["precision"]]
    assert np.allclose(gd, dts, rtol=0, atol=(1e-15 if tol < 1e-9 else 1e-6) * np.abs(dts).max())
    F, T, Fa, Ta = o2.forces_scale()
    Fg, Tg = g.forces()
    assert_forces_close(Fg, Tg, F, T, Fa, Ta, tol)


@pytest.mark.parametrize("name", ["fp64_linear_3001", "fp64_hertz_2500", "fp64_simple_1777",
                                  "fp64_partial_walls_5000"])
def test_fp64_steps_track_the_oracle(dem, name):
    c = cloud(**CASES[name])
    p = dict(c["params"], mu=0.2, eta_t_ratio=0.5, dt=2e-6)
    c["params"] = p
    g, o = make(dem, c)
    for _ in range(4):
        g.step(5)
        o.step(5)
    sg, so = g.read_state(), o.read_state()
    assert np.max(np.abs(sg["x"] - so["x"])) < 1e-12
    vs = np.abs(so["v"]).max()
    assert np.max(np.abs(sg["v"] - so["v"])) < 1e-9 * vs
    pg, dg = g.read_contacts()
    po, do = o.read_contacts()
    assert np.array_equal(pg, po)
    if len(do):
        assert np.max(np.abs(dg - do)) <= 1e-9 * max(np.abs(do).max(), 1e-300)
    dg_, do_ = g.diagnostics(), o.diagnostics()
    assert np.array_equal(dg_[7:9], do_[7:9])
    assert np.allclose(dg_[[3, 4, 5, 6, 9]], do_[[3, 4, 5, 6, 9]], rtol=1e-9, atol=0)
    assert np.allclose(dg_[:3], do_[:3], rtol=0, atol=1e-9 * np.abs(do_[:3]).max() + 1e-12)


def test_mixed_steps_stay_close(dem):
    c = cloud(**CASES["mixed_linear_3001"])
    p = dict(c["params"], mu=0.2, dt=2e-6)
    c["params"] = p
    g, o = make(dem, c)
    g.step(20)
    o.step(20)
    sg, so = g.read_state(), o.read_state()
    assert np.max(np.abs(sg["x"] - so["x"])) < 1e-9
    assert np.max(np.abs(sg["v"] - so["v"])) < 1e-4 * np.abs(so["v"]).max()


def test_plain_fp64_workload_trajectory(dem):
    w = W.plain_fp64(seed=1000)
    g = dem.System(w["params"], w["x"], w["v"], w["omega"], w["r"])
    o = OracleSystem(w["params"], w["x"], w["v"], w["omega"], w["r"])
    g.step(1000)
    o.step(1000)
    sg, so = g.read_state(), o.read_state()
    err = np.max(np.abs(sg["x"] - so["x"]))
    print(f"plain fp64 4096 x 1000 steps: max |x_gpu - x_oracle| = {err:.3e}")
    assert err <= 1e-9


def test_restart_is_bit_identical(dem):
    c = cloud(**CASES["fp64_linear_3001"])
    p = dict(c["params"], mu=0.3, dt=2e-6)
    a = dem.System(p, c["x"], c["v"], c["omega"], c["r"])
    a.step(20)
    b = dem.System(p, c["x"], c["v"], c["omega"], c["r"])
    b.step(10)
    st = b.read_state()
    pairs, dts = b.read_contacts()
    b2 = dem.System(p, st["x"], st["v"], st["omega"], c["r"], F0=st["F"], T0=st["T"], hist_pairs=pairs,
                    hist_dt=dts)
    b2.step(10)
    sa, sb = a.read_state(), b2.read_state()
    for k in ("x", "v", "omega", "F", "T"):
        assert np.array_equal(sa[k], sb[k]), k


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_runs_are_deterministic(dem, precision):
    c = cloud(**dict(CASES["fp64_partial_walls_5000"], precision=precision))
    out = []
    for _ in range(2):
        g = dem.System(c["params"], c["x"], c["v"], c["omega"], c["r"])
        g.step(25)
        out.append((g.read_state(), g.read_contacts(), g.diagnostics()))
    for k in ("x", "v", "omega", "F", "T"):
        assert np.array_equal(out[0][0][k], out[1][0][k]), k
    assert np.array_equal(out[0][1][0], out[1][1][0]) and np.array_equal(out[0][1][1], out[1][1][1])
    assert np.array_equal(out[0][2], out[1][2])


# ---------------------------------------------------------------- edge cases


def test_single_particle_and_empty(dem):
    p = W.base_params(cell_size=0.1, dt=1e-5)
    g = dem.System(p, [[0.5, 0.5, 0.02]], [[0.1, 0, 0]], [[0, 0, 1.0]], [0.03])
    o = OracleSystem(p, [[0.5, 0.5, 0.02]], [[0.1, 0, 0]], [[0, 0, 1.0]], [0.03])
    g.step(50)
    o.step(50)
    sg, so = g.read_state(), o.read_state()
    assert np.allclose(sg["x"], so["x"], rtol=0, atol=1e-13)
    e = dem.System(p, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0))
    e.step(3)
    assert e.read_state()["x"].shape == (0, 3)
    assert len(e.contacts()) == 0
    assert np.all(e.diagnostics() == 0.0)


def test_one_cell_grid(dem):
    c = W.overlapping_cloud(9, 300, box=(0.3, 0.3, 0.3), r_mean=0.012, spacing=0.95)
    p = dict(c["params"], cell_size=0.3)
    g = dem.System(p, c["x"], c["v"], c["omega"], c["r"])
    o = OracleSystem(p, c["x"], c["v"], c["omega"], c["r"])
    assert g.grid_dims() == (1, 1, 1)
    assert np.array_equal(g.contacts(), o.contacts())
    F, T, Fa, Ta = o.forces_scale()
    Fg, Tg = g.forces()
    assert_forces_close(Fg, Tg, F, T, Fa, Ta, TOL["fp64"])


def test_crowded_cells_keep_the_canonical_order(dem):
    # 2,600 small spheres piled into one cell and 700 spread over the box:
    # cells far above the handful the per-thread insertion sort handles,
    # several workgroup rounds and several LDS rounds of ids per cell
    rng = np.random.default_rng(21)
    spread = rng.uniform(0.05, 0.95, (700, 3))
    pile = rng.uniform(0.21, 0.29, (2600, 3))
    x = np.concatenate([spread, pile])
    r = W.fp32_radii(np.concatenate([rng.uniform(0.01, 0.03, 700), np.full(2600, 0.0012)]))
    p = W.base_params(cell_size=0.1, gravity=(0, 0, 0), contacts_per_particle=64)
    v = rng.normal(0, 0.1, x.shape)
    w = rng.normal(0, 1.0, x.shape)
    g = dem.System(p, x, v, w, r)
    o = OracleSystem(p, x, v, w, r)
    for a, b in zip(g.read_grid(), o.read_grid()):
        assert np.array_equal(a, b)
    assert np.array_equal(g.contacts(), o.contacts())
    g.step(3)
    o.step(3)
    for a, b in zip(g.read_grid(), o.read_grid()):
        assert np.array_equal(a, b)


def test_out_of_domain_is_reported(dem):
    p = W.base_params(cell_size=0.1, wall_mask=0, gravity=(0, 0, 0))
    x = np.array([[0.5, 0.5, 0.5], [1.2, 0.5, 0.5]])
    with pytest.raises(dem.DemError) as e:
        dem.System(p, x, np.zeros((2, 3)), np.zeros((2, 3)), [0.01, 0.01])
    assert e.value.code == dem.DEM_E_OUT_OF_DOMAIN
    # a particle that flies out during the run: sticky error at the next sync
    g = dem.System(p, [[0.5, 0.5, 0.95]], [[0, 0, 50.0]], [[0, 0, 0]], [0.01], )
    g.step(400)
    with pytest.raises(dem.DemError) as e:
        g.read_state()
    assert e.value.code == dem.DEM_E_OUT_OF_DOMAIN
    with pytest.raises(dem.DemError):
        g.step(1)


def test_contact_list_overflow_is_reported(dem):
    c = cloud(**CASES["fp64_linear_3001"])
    o = OracleSystem(c["params"], c["x"], c["v"], c["omega"], c["r"])
    pairs = o.contacts()
    assert len(pairs) > len(c["r"])  # more than one contact per particle
    p = dict(c["params"], contacts_per_particle=1)
    with pytest.raises(dem.DemError) as e:
        g = dem.System(p, c["x"], c["v"], c["omega"], c["r"])
        g.step(1)
        g.sync()
    assert e.value.code == dem.DEM_E_CONTACT_OVERFLOW


@pytest.mark.parametrize("tile,cell_scale", [(1, 1.0), (5, 1.0), (32, 1.0), (32, 4.0), (-1, 1.0), (-1, 4.0)])
@pytest.mark.parametrize("name", ["fp64_partial_walls_5000", "mixed_nowalls_poly_4097", "mixed_hertz_2500"])
def test_tiled_detection_is_bit_identical(dem, name, tile, cell_scale):
    # tile_cells selects the detection launch shape only: the same lists, so
    # the same forces and trajectories to the bit.  cell_scale 4 packs so many
    # particles per cell that the tile's rows overflow LDS and are read from
    # global memory instead, and that the wave shape (-1) sees cells of more
    # than 64 particles and stencils of more than two chunks.
    c = cloud(**CASES[name])
    p = dict(c["params"], mu=0.2, eta_t_ratio=0.5, dt=2e-6, cell_size=cell_scale * c["params"]["cell_size"])
    a = dem.System(p, c["x"], c["v"], c["omega"], c["r"])
    b = dem.System(dict(p, tile_cells=tile), c["x"], c["v"], c["omega"], c["r"])
    assert np.array_equal(a.contacts(), b.contacts())
    Fa, Ta = a.forces()
    Fb, Tb = b.forces()
    assert np.array_equal(Fa, Fb) and np.array_equal(Ta, Tb)
    a.step(6)
    b.step(6)
    sa, sb = a.read_state(), b.read_state()
    for key in ("x", "v", "omega", "F", "T"):
        assert np.array_equal(sa[key], sb[key]), key
    # and the tiled lists are the oracle's on the state reached
    o = OracleSystem(p, sb["x"], sb["v"], sb["omega"], c["r"])
    assert np.array_equal(b.contacts(), o.contacts())


@pytest.mark.parametrize("name", ["fp64_linear_3001", "mixed_nowalls_poly_4097", "fp64_partial_walls_5000",
                                  "mixed_hertz_2500"])
def test_cell_divisor_two_finds_the_same_contacts(dem, name):
    # cells of half the width swept over 5^3 cells cover the same contact
    # distance as the 27-cell sweep: the same contacts, forces within the
    # tolerance (the slot order, and so the summation order, differs), and
    # trajectories that track the oracle's
    c = cloud(**CASES[name])
    p = dict(c["params"], mu=0.2, eta_t_ratio=0.5, dt=2e-6)
    g = dem.System(dict(p, cell_divisor=2), c["x"], c["v"], c["omega"], c["r"])
    o = OracleSystem(p, c["x"], c["v"], c["omega"], c["r"])
    assert all(a >= 2 * b for a, b in zip(g.grid_dims(), o.grid_dims()))
    assert np.array_equal(g.contacts(), o.contacts())
    tol = TOL[p["precision"]]
    F, T, Fa, Ta = o.forces_scale()
    Fg, Tg = g.forces()
    assert_forces_close(Fg, Tg, F, T, Fa, Ta, tol)
    g.step(6)
    o.step(6)
    assert np.array_equal(g.contacts(), o.contacts())
    sg, so = g.read_state(), o.read_state()
    scale = np.abs(so["x"]).max()
    assert np.abs(sg["x"] - so["x"]).max() <= (1e-12 if tol < 1e-9 else 1e-6) * scale


def edge_pairs(seed, k, divisor, precision):
    """k^3 isolated pairs on a lattice, each at a distance a relative 1e-9 to
    1e-3 below or above the sum of its radii (or well inside it), in random
    directions, with seeded FP32 radii between 0.3 and 1 r_max.  With a cell
    of 3 r_max and one grid cell per cell the first spheres reach 0.3 cells
    beyond the box on every side (their partners up to 0.97 cells), where
    the cell ids are clamped; with cells halved every sphere stays inside."""
    rng = np.random.default_rng(seed)
    rmax = 0.01
    cell = 3.0 * rmax
    L = 6.0 * rmax * (k - 1)
    out = 0.3 * cell if divisor == 1 else -2.2 * rmax
    a = np.linspace(-out, L + out, k)
    A = np.stack(np.meshgrid(a, a, a, indexing="ij"), axis=-1).reshape(-1, 3)
    m = len(A)
    r = W.fp32_radii(rng.uniform(0.3, 1.0, 2 * m) * rmax)
    r[0] = rmax  # the largest radius, so that rmax is what the cell was sized for
    rA, rB = r[:m], r[m:]
    f = rng.choice([1 - 1e-9, 1 - 1e-7, 1 - 1e-5, 1 - 1e-3, 1 + 1e-9, 1 + 1e-7, 1 + 1e-5, 1 + 1e-3, 0.7], m)
    d = rng.normal(size=(m, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    B = A + d * ((rA + rB) * f)[:, None]
    x = np.empty((2 * m, 3))
    x[0::2], x[1::2] = A, B
    rr = np.empty(2 * m)
    rr[0::2], rr[1::2] = rA, rB
    p = W.base_params(box_hi=(L, L, L), cell_size=cell, wall_mask=0, precision=precision)
    zero = np.zeros_like(x)
    return p, x, zero, zero, rr, int(np.sum(f < 1))


@pytest.mark.parametrize("divisor,precision", [(1, "mixed"), (1, "fp64"), (2, "mixed")])
def test_pairs_at_the_prefilter_edge(dem, divisor, precision):
    # pairs a relative 1e-9 inside or outside contact, in every direction and
    # across the clamped cells beyond the box: the prefilter passes every true
    # contact, and the exact test decides as the oracle does
    p, x, v, w, r, n_in = edge_pairs(11 + divisor, 12, divisor, precision)
    g = dem.System(dict(p, cell_divisor=divisor), x, v, w, r)
    o = OracleSystem(p, x, v, w, r)
    co = o.contacts()
    assert len(co) == n_in
    assert np.array_equal(g.contacts(), co)


def test_profile_phases_cover_the_step(dem):
    import torch
    c = cloud(seed=9, n=3000, precision="mixed")
    s = dem.System(c["params"], c["x"], c["v"], c["omega"], c["r"])
    s.profile(True)
    torch.cuda.synchronize()
    s.step(10)
    ms, n = s.profile_read()
    assert n == 10 and len(ms) == dem.NUM_PHASES and np.all(ms >= 0) and ms.sum() > 0
    ms2, n2 = s.profile_read()
    assert n2 == 0 and np.all(ms2 == 0)


def crowned_sphere(n_small, seed=0):
    """One large sphere touched by n_small small ones spread over its
    surface, all in one cell, the large one last in id (so every contact is
    one of its backward contacts), with seeded velocities and spins.  The
    small radius shrinks with their number so that they do not touch one
    another (their spacing on the surface is about R sqrt(4 pi / n))."""
    R = 0.05
    r = min(0.01, 0.35 * R * math.sqrt(4 * math.pi / n_small))
    c = np.array([0.1, 0.1, 0.1])
    k = np.arange(n_small) + 0.5
    phi = np.arccos(1 - 2 * k / n_small)
    th = np.pi * (1 + 5 ** 0.5) * k
    d = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], axis=1)
    x = np.concatenate([c + (R + 0.9 * r) * d, c[None]])
    rad = W.fp32_radii(np.concatenate([np.full(n_small, r), [R]]))
    rng = np.random.default_rng(seed)
    v, w = rng.normal(0, 0.05, x.shape), rng.normal(0, 2.0, x.shape)
    p = W.base_params(box_hi=(0.2, 0.2, 0.2), cell_size=0.15, wall_mask=0, gravity=(0, 0, 0), dt=1e-6)
    return p, x, v, w, rad


@pytest.mark.parametrize("n_small,precision", [(6, "fp64"), (20, "fp64"), (20, "mixed"), (32, "mixed")])
def test_long_backward_lists_sum_in_order(dem, n_small, precision):
    # a particle with many lower partners, found in any order: its sums
    # follow the fixed order (ascending owner slot), match the oracle, and
    # stay so over steps
    p, x, v, w, rad = crowned_sphere(n_small, seed=n_small)
    p = dict(p, precision=precision, mu=0.3, eta_t_ratio=0.5)
    g = dem.System(p, x, v, w, rad)
    o = OracleSystem(p, x, v, w, rad)
    assert len(o.contacts()) == n_small
    assert np.array_equal(g.contacts(), o.contacts())
    F, T, Fa, Ta = o.forces_scale()
    Fg, Tg = g.forces()
    assert_forces_close(Fg, Tg, F, T, Fa, Ta, TOL[precision])
    g.step(5)
    o.step(5)
    sg, so = g.read_state(), o.read_state()
    scale = np.abs(so["x"]).max()
    assert np.abs(sg["x"] - so["x"]).max() <= (1e-12 if precision == "fp64" else 1e-6) * scale


@pytest.mark.parametrize("n_small,precision", [(60, "mixed"), (300, "fp64"), (700, "mixed"), (1100, "mixed"),
                                             (1100, "fp64")])
def test_many_backward_contacts(dem, n_small, precision):
    # a particle with more lower partners than a workgroup stages records
    # for (512) or collects at all (1024, beyond which each lane reads its
    # owners' contacts itself): every path sums in the same fixed order and
    # matches the oracle, with no limit on the count
    p, x, v, w, rad = crowned_sphere(n_small, seed=n_small)
    p = dict(p, precision=precision, mu=0.3, eta_t_ratio=0.5)
    g = dem.System(p, x, v, w, rad)
    o = OracleSystem(p, x, v, w, rad)
    assert len(o.contacts()) == n_small
    assert np.array_equal(g.contacts(), o.contacts())
    F, T, Fa, Ta = o.forces_scale()
    Fg, Tg = g.forces()
    assert_forces_close(Fg, Tg, F, T, Fa, Ta, TOL[precision])
