"""Seeded synthetic inputs for the DEM step: positions, radii, velocities and
the parameter dictionaries of the benchmark workloads.

This module is shared by the GPU path's tests and by the oracle's tests, so it
holds no part of the method's arithmetic (no grid, no contact test, no contact
law, no integrator): only random numbers, lattices and the recipe numbers.

The paper's own workload (Sec. 5: 2^17 equal spheres falling from a box
through a slit, run until at rest) gives no geometry, so every workload here
is synthetic.  Sizes are powers of two like the paper's 2^17.

Parameter dictionary keys (each side marshals them into its own structure):
  box_lo, box_hi     domain corners (m)
  wall_mask          bit 2a: wall at box_lo[a]; bit 2a+1: wall at box_hi[a]
  gravity            (m/s^2), added once per particle
  dt, density        time step (s), particle density (kg/m^3)
  law                "linear" (constant kn, kt), "hertz" (Eqs. 8-9: kn, kt are
                     C_kn, C_kt) or "simple" (Eq. 1: simple_k = k_sp, k_da, k_sh)
  kn, kt             normal / tangential spring
  restitution        e, fixes the restitution parameter alpha of Eq. 10
  eta_t_ratio        tangential damping as a fraction of the normal one
  mu                 Coulomb friction coefficient (Eq. 5)
  cell_size          requested cell width of the collision-detection grid
  contacts_per_particle  most contacts one particle may own: partners after it in the
                     sorted order plus walls (GPU only; sizes the contact tables)
  tile_cells         detection launch shape: 0 one lane per particle, -1 one wave
                     per run of cells, 1..32 cells per LDS-staged workgroup
                     (GPU only; speed only)
  cell_divisor       k: grid cells of cell_size / k swept over (2k + 1)^3 cells
                     (GPU only; 1 or 2; speed and summation order only)
  precision          "fp64" or "mixed" (FP32 forces, FP64 positions; GPU only)
  max_materials      most materials of a material-pair table (0: one material)
  terms              optional contact terms, a tuple of "cohesion" and "rolling"
  cohesion, rolling_mu  their constants (pull in N; rolling-resistance coefficient)
  plates             finite walls: dicts axis, at, lo (2), hi (2), at most 4
"""
import math

import numpy as np

RHO = 2500.0
KN = 1.0e5
E_REST = 0.9
MU = 0.3
G = (0.0, 0.0, -9.81)
ALL_WALLS = 0x3F


def base_params(**kw) -> dict:
    p = dict(box_lo=(0.0, 0.0, 0.0), box_hi=(1.0, 1.0, 1.0), wall_mask=ALL_WALLS, gravity=G,
             dt=1.0e-5, density=RHO, law="linear", kn=KN, kt=2.0 / 7.0 * KN, restitution=E_REST,
             eta_t_ratio=0.0, mu=MU, simple_k=(0.0, 0.0, 0.0), cell_size=None,
             contacts_per_particle=16, precision="fp64")
    p.update(kw)
    return p


def linear_contact_time(kn: float, e: float, m_eff: float) -> float:
    """Duration of a linear spring-dashpot contact of restitution e (the
    damped half-period); used only to choose a stable time step."""
    le = math.log(e)
    zeta = -le / math.sqrt(math.pi ** 2 + le * le)
    w0 = math.sqrt(kn / m_eff)
    return math.pi / (w0 * math.sqrt(1.0 - zeta * zeta))


def stable_dt(kn: float, e: float, r_min: float, rho: float = RHO, cap: float = 1.0e-5) -> float:
    """dt = min(cap, t_c / 10) for the contact of the two smallest spheres."""
    m = rho * 4.0 / 3.0 * math.pi * r_min ** 3
    return min(cap, linear_contact_time(kn, e, 0.5 * m) / 10.0)


def fp32_radii(r) -> np.ndarray:
    """Radii as both paths store them (rounded to FP32)."""
    return np.asarray(r, dtype=np.float32).astype(np.float64)


# ---------------------------------------------------------------- placements


def rsa_positions(rng, radii, lo, hi, max_tries=200000):
    """Random sequential addition of non-overlapping spheres inside walls.
    Slow (pure Python loop over particles); for a few thousand spheres."""
    radii = np.asarray(radii, dtype=np.float64)
    n = radii.shape[0]
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    cell = 2.0 * radii.max()
    dims = np.maximum(1, np.floor((hi - lo) / cell).astype(int))
    buckets = {}
    x = np.zeros((n, 3))
    for i in range(n):
        ri = radii[i]
        for _ in range(max_tries):
            p = lo + ri + rng.random(3) * (hi - lo - 2 * ri)
            c = np.minimum(((p - lo) / (hi - lo) * dims).astype(int), dims - 1)
            ok = True
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        for j in buckets.get((c[0] + dx, c[1] + dy, c[2] + dz), ()):
                            if np.sum((x[j] - p) ** 2) <= (radii[j] + ri) ** 2:
                                ok = False
                                break
                        if not ok:
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                x[i] = p
                buckets.setdefault(tuple(c), []).append(i)
                break
        else:
            raise RuntimeError("rsa_positions: box too full")
    return x


def fcc_sites(lo, hi, d_nn, margin):
    """All face-centred-cubic sites with nearest-neighbour distance d_nn whose
    distance to every face of [lo, hi] is at least margin."""
    lo = np.asarray(lo, float) + margin
    hi = np.asarray(hi, float) - margin
    b = d_nn * math.sqrt(2.0)
    counts = np.floor((hi - lo) / b).astype(int) + 1
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    ix = np.arange(counts[0])
    iy = np.arange(counts[1])
    iz = np.arange(counts[2])
    out = []
    for bv in basis:
        X = lo[0] + (ix + bv[0]) * b
        Y = lo[1] + (iy + bv[1]) * b
        Z = lo[2] + (iz + bv[2]) * b
        X = X[X <= hi[0]]
        Y = Y[Y <= hi[1]]
        Z = Z[Z <= hi[2]]
        gz, gy, gx = np.meshgrid(Z, Y, X, indexing="ij")
        out.append(np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1))
    return np.concatenate(out, axis=0)


def fcc_fill(rng, n, lo, hi, margin, jitter_frac=0.0, d_nn=None):
    """n sites of an FCC lattice filling [lo, hi] (minus margin), chosen at
    random when the lattice holds more, each jittered uniformly by up to
    jitter_frac * (d_nn/2 - margin) per axis.  Returns (positions, d_nn)."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    vol = np.prod(hi - lo - 2 * margin)
    if d_nn is None:
        d_nn = (math.sqrt(2.0) * vol / n) ** (1.0 / 3.0)
    while True:
        sites = fcc_sites(lo, hi, d_nn, margin)
        if sites.shape[0] >= n:
            break
        d_nn *= 0.995
    pick = np.sort(rng.choice(sites.shape[0], size=n, replace=False))
    x = sites[pick]
    if jitter_frac > 0.0:
        amp = jitter_frac * max(0.0, 0.5 * d_nn - margin)
        x = x + rng.uniform(-amp, amp, size=x.shape)
    return x, d_nn


def lognormal_radii(rng, n, median, sigma, clip_sigmas=3.0):
    z = np.clip(rng.standard_normal(n), -clip_sigmas, clip_sigmas)
    return median * np.exp(sigma * z)


# ---------------------------------------------------------------- workloads


def plain_fp64(seed=1000, n=4096):
    """4,096 equal spheres (r = 1/64) at random non-overlapping positions in a
    walled unit box, v ~ N(0, 0.1^2) per axis, gravity -9.81 z, linear law
    kn = 1e5, e = 0.9, kt = 2/7 kn, mu = 0.3, dt = 1e-5, FP64."""
    rng = np.random.default_rng(seed)
    r = fp32_radii(np.full(n, 1.0 / 64.0))
    x = rsa_positions(rng, r, (0, 0, 0), (1, 1, 1))
    v = rng.normal(0.0, 0.1, size=(n, 3))
    w = np.zeros((n, 3))
    p = base_params(cell_size=2.0 * r.max(), precision="fp64", dt=1.0e-5)
    return dict(name=f"plain_fp64_{n}", params=p, x=x, v=v, omega=w, r=r)


def gas_mixed(seed=2000, n=1 << 20, law="linear"):
    """2^20 spheres, radii U[0.8, 1.2] / 256, a gas at packing fraction 0.3
    filling the bottom of a walled unit box (jittered FCC), v ~ N(0, 0.1^2),
    settling under gravity; FP32 forces with FP64 positions, dt = 1e-5."""
    rng = np.random.default_rng(seed)
    r0 = 1.0 / 256.0
    r = fp32_radii(rng.uniform(0.8 * r0, 1.2 * r0, size=n))
    vol = float(np.sum(4.0 / 3.0 * math.pi * r ** 3))
    h = min(1.0, vol / 0.3)
    x, _ = fcc_fill(rng, n, (0, 0, 0), (1, 1, h), margin=r.max(), jitter_frac=0.9)
    v = rng.normal(0.0, 0.1, size=(n, 3))
    w = np.zeros((n, 3))
    p = base_params(cell_size=2.0 * r.max(), precision="mixed", dt=1.0e-5, law=law)
    if law == "simple":
        p["simple_k"] = simple_coefficients(r0)
    return dict(name=f"gas_mixed_{n}", params=p, x=x, v=v, omega=w, r=r)


def simple_coefficients(r_med, kn=KN, e=E_REST, rho=RHO):
    """Constant coefficients of Eq. 1 for the comparison run: k_sp = kn and
    k_da = k_sh = the damping of a median-radius linear contact of
    restitution e (critical-damping fraction times 2 sqrt(kn M))."""
    m = rho * 4.0 / 3.0 * math.pi * r_med ** 3
    le = math.log(e)
    zeta = -le / math.sqrt(math.pi ** 2 + le * le)
    eta = 2.0 * zeta * math.sqrt(kn * 0.5 * m)
    return (kn, eta, eta)


def dense_bed_geometry(seed=3000, n=1 << 24, phi=0.55, median=1.0 / 512.0, sigma=0.2):
    """Radii and box of the dense granular bed: log-normal radii (median
    1/512, sigma 0.2, clipped to +-3 sigma), box of aspect 4:1:1 whose volume
    is the total sphere volume / phi, gravity along the short z axis."""
    rng = np.random.default_rng(seed)
    r = fp32_radii(lognormal_radii(rng, n, median, sigma))
    vol = float(np.sum(4.0 / 3.0 * math.pi * r ** 3)) / phi
    ly = (vol / 4.0) ** (1.0 / 3.0)
    hi = (4.0 * ly, ly, ly)
    return rng, r, hi


def dense_bed_params(r, hi, **kw):
    r_min = float(np.min(r))
    p = base_params(box_hi=hi, cell_size=2.0 * float(np.max(r)), precision="mixed",
                    dt=stable_dt(KN, E_REST, r_min), contacts_per_particle=32)
    p.update(kw)
    return p


def dense_bed_lattice(seed=3000, n=1 << 24, phi=0.55, fill_height=1.0):
    """Starting point of the dense bed: every sphere on an FCC site of the
    4:1:1 box (its lower fill_height fraction), at rest.  With full radii
    neighbouring large spheres overlap; the bed is prepared by growing the
    radii from the lattice's touching scale (see ``lattice_scale``) to full
    size with strong damping."""
    rng, r, hi = dense_bed_geometry(seed, n, phi)
    top = (hi[0], hi[1], hi[2] * fill_height)
    x, d_nn = fcc_fill(rng, n, (0, 0, 0), top, margin=float(r.max()), jitter_frac=0.0)
    # the lattice is filled in a fixed order; shuffle which radius sits where
    perm = rng.permutation(n)
    r = r[perm]
    p = dense_bed_params(r, hi)
    z = np.zeros((n, 3))
    return dict(name=f"dense_bed_{n}", params=p, x=x, v=z, omega=z.copy(), r=r, d_nn=d_nn,
                fill_height=fill_height)


def lattice_scale(r, d_nn):
    """Largest common radius scale at which no two lattice neighbours overlap."""
    return min(1.0, d_nn / (2.0 * float(np.max(r))))


def overlapping_cloud(seed, n, box=(1.0, 1.0, 1.0), r_mean=0.03, r_spread=0.2, spacing=0.95,
                      v_sigma=0.1, w_sigma=10.0, law="linear", precision="fp64", walls=ALL_WALLS,
                      jitter=0.3, **kw):
    """A small, crowded test state: spheres on a jittered simple-cubic lattice
    whose spacing is `spacing` times the mean diameter, so that many pairs and
    the walls overlap; random velocities and spins.  For parity tests."""
    rng = np.random.default_rng(seed)
    r = fp32_radii(r_mean * (1.0 + r_spread * rng.uniform(-1, 1, size=n)))
    a = spacing * 2.0 * r_mean
    box = np.asarray(box, float)
    dims = np.maximum(1, np.floor(box / a).astype(int))
    if np.prod(dims) < n:
        raise ValueError("overlapping_cloud: box too small for n")
    idx = np.sort(rng.choice(int(np.prod(dims)), size=n, replace=False))
    ijk = np.stack([idx % dims[0], (idx // dims[0]) % dims[1], idx // (dims[0] * dims[1])], axis=1)
    x = (ijk + 0.5) * a + rng.uniform(-jitter * a, jitter * a, size=(n, 3))
    x = np.clip(x, 0.5 * r_mean, box - 0.5 * r_mean)
    v = rng.normal(0.0, v_sigma, size=(n, 3))
    w = rng.normal(0.0, w_sigma, size=(n, 3))
    p = base_params(box_hi=tuple(box), cell_size=2.0 * float(r.max()), law=law, precision=precision,
                    wall_mask=walls, **kw)
    if law == "simple":
        p["simple_k"] = simple_coefficients(r_mean)
    if law == "hertz":
        p["kn"] = kw.get("kn", 1.0e7)
        p["kt"] = kw.get("kt", 2.0 / 7.0 * p["kn"])
    return dict(name=f"cloud_{n}_{seed}", params=p, x=x, v=v, omega=w, r=r)


# ------------------------------------------------- many independent systems

E_U3 = (1.2 ** 4 - 0.8 ** 4) / (4.0 * 0.4)  # E[u^3] for u ~ U[0.8, 1.2]


def system_draw(rng, n_lo, n_hi):
    """Size and material of one independent system: n log-uniform in
    [n_lo, n_hi], kn log-uniform in [1e4, 1e6], e ~ U[0.5, 0.95],
    mu ~ U[0.1, 0.6], packing fraction phi ~ U[0.2, 0.55]."""
    n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
    kn = math.exp(rng.uniform(math.log(1.0e4), math.log(1.0e6)))
    e = rng.uniform(0.5, 0.95)
    mu = rng.uniform(0.1, 0.6)
    phi = rng.uniform(0.2, 0.55)
    return dict(n=n, kn=kn, restitution=e, mu=mu, phi=phi)


def unit_box_system(seed, n, kn, restitution, mu, phi, precision="mixed", law="linear", cell_factor=1.0,
                    contacts_per_particle=16, tile_cells=0, cell_divisor=1):
    """One system of the batched and serving workloads: n spheres with radii
    U[0.8, 1.2] r_s in a walled unit box, r_s set so that the spheres fill the
    packing fraction phi, on a jittered FCC lattice, v ~ N(0, 0.1^2) per axis,
    omega = 0, gravity -9.81 z, kt = 2/7 kn, dt = t_c,min / 10 (at most
    1e-5), cell = cell_factor x the largest diameter.

    Where the lattice cannot hold the spheres at phi without overlaps (above
    a packing fraction of about 0.44 for these radii), the spheres start at
    the largest common scale of their drawn radii that the lattice holds: `r`
    is then that starting size and `r_target` the drawn radii, which
    ``prepare.grow_systems`` reaches by growing the packing; phi_start is the
    packing fraction of `r`.  The parameters (cell, dt) are those of the
    drawn radii."""
    rng = np.random.default_rng(seed)
    r_s = (phi / (n * 4.0 / 3.0 * math.pi * E_U3)) ** (1.0 / 3.0)
    r_draw = rng.uniform(0.8 * r_s, 1.2 * r_s, size=n)
    r_max = float(r_draw.max()) if n else r_s
    x, d_nn = fcc_fill(rng, n, (0, 0, 0), (1, 1, 1), margin=r_max, jitter_frac=0.9)
    lam = lattice_scale(r_draw, d_nn) if n else 1.0
    r_full = fp32_radii(r_draw)
    r = fp32_radii(r_draw * lam) if lam < 1.0 else r_full
    v = rng.normal(0.0, 0.1, size=(n, 3))
    w = np.zeros((n, 3))
    r_min = float(r_full.min()) if n else r_s
    dmax = 2.0 * (float(r_full.max()) if n else r_s)
    p = base_params(kn=kn, kt=2.0 / 7.0 * kn, restitution=restitution, mu=mu, law=law, precision=precision,
                    dt=stable_dt(kn, restitution, r_min), cell_size=min(1.0, cell_factor * dmax),
                    contacts_per_particle=contacts_per_particle, tile_cells=tile_cells,
                    cell_divisor=cell_divisor)
    phi_start = float(np.sum(4.0 / 3.0 * math.pi * r ** 3))
    return dict(name=f"system_{n}_{seed}", params=p, x=x, v=v, omega=w, r=r, phi=phi, phi_start=phi_start,
                r_target=r_full if lam < 1.0 else None)


def batched_draws(seed=4000, count=256, n_lo=1024, n_hi=262144):
    """Sizes and materials of the batched workload's systems."""
    rng = np.random.default_rng(seed)
    return [system_draw(rng, n_lo, n_hi) for _ in range(count)]


def batched_systems(seed=4000, count=256, n_lo=1024, n_hi=262144, precision="mixed", law="linear",
                    cell_factors=None, tiles=None, divisors=None):
    """The batched workload: `count` independent systems, each drawn by
    ``system_draw`` and built by ``unit_box_system`` with seed seed + 1 + k.
    cell_factors, tiles and divisors (one per system) come from the
    autotuner; default 1, 0 and 1."""
    out = []
    for k, d in enumerate(batched_draws(seed, count, n_lo, n_hi)):
        cf = 1.0 if cell_factors is None else float(cell_factors[k])
        tc = 0 if tiles is None else int(tiles[k])
        cd = 1 if divisors is None else int(divisors[k])
        out.append(unit_box_system(seed + 1 + k, d["n"], d["kn"], d["restitution"], d["mu"], d["phi"],
                                   precision=precision, law=law, cell_factor=cf, tile_cells=tc,
                                   cell_divisor=cd))
    return out


def serving_requests(seed=5000, count=512, n_lo=1024, n_hi=1 << 20, steps_lo=100, steps_hi=10000):
    """Request specifications of the serving workload (built lazily with
    ``unit_box_system``): size log-uniform in [n_lo, n_hi], step count
    log-uniform in [steps_lo, steps_hi], materials as the batched systems."""
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(count):
        d = system_draw(rng, n_lo, n_hi)
        d["steps"] = int(round(math.exp(rng.uniform(math.log(steps_lo), math.log(steps_hi)))))
        d["seed"] = seed + 1 + k
        reqs.append(d)
    return reqs


# ------------------------------------------------- the paper's sample problem

def slit_plates(z, x0, x1, box_lo, box_hi):
    """Two finite walls at height z that close the box's cross-section except
    for the slit x0 < x < x1 (across the whole y range)."""
    return [dict(axis=2, at=float(z), lo=(float(box_lo[0]), float(box_lo[1])), hi=(float(x0), float(box_hi[1]))),
            dict(axis=2, at=float(z), lo=(float(x1), float(box_lo[1])), hi=(float(box_hi[0]), float(box_hi[1])))]


def slit_hopper(seed=6000, n=1 << 17, r=1.0e-3, nx=64, ny=16, slit_diameters=10.0, low_cells=64,
                precision="mixed", law="linear", rest_fraction=1.0e-5):
    """Sec. 5's sample problem: n equal spheres that fall from a box through a
    slit in its bottom onto a floor, run until every particle's step is below
    a set displacement.  The paper gives no sizes; here the spheres (radius r)
    start at rest on a jittered cubic lattice of spacing 2.2 r, nx x ny x
    n / (nx ny) sites, filling the upper chamber of a walled box whose
    bottom is a pair of plates at height z_s = low_cells x 2.2 r with a slit
    of slit_diameters diameters across the middle of x; the floor is the box's
    lower z wall.  Materials as the other workloads (k_n 1e5, e 0.9,
    k_t 2/7 k_n, mu 0.3), dt = t_c / 10, cell = 2 r.  `rest_displacement` is
    the stopping threshold rest_fraction x r per step."""
    rng = np.random.default_rng(seed)
    nz = n // (nx * ny)
    if nx * ny * nz != n:
        raise ValueError("n must be a multiple of nx * ny")
    a = 2.2 * r
    Lx, Ly = nx * a, ny * a
    zs = low_cells * a
    hi = (Lx, Ly, zs + (nz + 1) * a)
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    sites = np.stack([(i.ravel() + 0.5) * a, (j.ravel() + 0.5) * a, zs + (k.ravel() + 0.5) * a], axis=1)
    x = sites + rng.uniform(-0.04 * a, 0.04 * a, size=sites.shape)
    rr = fp32_radii(np.full(n, r))
    w = slit_diameters * 2.0 * r
    plates = slit_plates(zs, 0.5 * Lx - 0.5 * w, 0.5 * Lx + 0.5 * w, (0.0, 0.0, 0.0), hi)
    p = base_params(box_hi=hi, cell_size=2.0 * float(rr.max()), dt=stable_dt(KN, E_REST, float(rr.min())),
                    precision=precision, law=law, contacts_per_particle=12, plates=plates)
    return dict(name=f"slit_hopper_{n}", params=p, x=x, v=np.zeros((n, 3)), omega=np.zeros((n, 3)), r=rr,
                slit=(0.5 * Lx - 0.5 * w, 0.5 * Lx + 0.5 * w), z_slit=zs, rest_displacement=rest_fraction * r)


def poisson_arrivals(seed, count, rate):
    """Arrival times (s) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
