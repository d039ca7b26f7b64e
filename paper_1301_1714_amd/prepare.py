"""Preparation of the dense granular bed (untimed, seeded, deterministic).

A random dense packing of polydisperse spheres at packing fraction 0.55 with
sustained contacts cannot be placed directly: it is grown.  The spheres start
on the FCC lattice of the bed's box at the largest common radius scale with
no overlap, and their radii are raised to full size in stages with strongly
damped contacts (restitution 0.1), no gravity and friction on, so that they
push each other into a jammed arrangement; the bed then settles under
gravity.  The growth runs through this library's own step (the GPU path);
it produces the benchmark's starting state only, never an expected value.

A bed filling the box evenly at packing fraction 0.55 is below jamming and
would need a long fall under gravity to compact; instead the lattice fills
the lower part of the box (the ``fill_height`` of the lattice), so that the
spheres jam while growing, without gravity, at the local packing fraction
0.55 / fill_height.  The box, and so its mean packing fraction, is the
workload's; the top of the box stays empty.  The grown bed is then relaxed
under gravity by quenching: 16 times, the system restarts at rest and runs
500 steps, which brings it to a static packing (about 3.5-4 contacts per
sphere at a fill height of 0.93).  Growth: 60 stages of 60 steps, friction
0.5; restitution 0.1 throughout.
"""
import sys
import time

import numpy as np

from . import dem
from . import workloads as W


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def grow_dense_bed(w, stages=60, steps_per_stage=60, settle_steps=0, grow_mu=0.5, settle_g=1.0,
                   relax_steps=0, quench_cycles=16, quench_steps=500, device="cuda", verbose=True):
    """w: the dict of ``workloads.dense_bed_lattice``.  Returns (x, v, omega,
    info) of the prepared bed (original particle order).  grow_mu: friction
    while growing; settle_g: gravity multiple while settling (then relax_steps
    at normal gravity)."""
    import torch

    t0 = time.time()
    r_full = np.asarray(w["r"], dtype=np.float64)
    lam0 = W.lattice_scale(r_full, w["d_nn"])
    n = r_full.shape[0]
    zero = np.zeros((n, 3))
    hi = tuple(w["params"]["box_hi"])
    grow_box = (hi[0], hi[1], hi[2] * w.get("fill_height", 1.0))
    grow_p = dict(w["params"], restitution=0.1, mu=grow_mu, eta_t_ratio=1.0, gravity=(0.0, 0.0, 0.0),
                  box_hi=grow_box)
    s = dem.System(grow_p, w["x"], zero, zero, r_full * lam0, device=device)
    for k in range(1, stages + 1):
        lam = lam0 + (1.0 - lam0) * k / stages
        s.set_radii(r_full * lam)
        s.step(steps_per_stage)
        if verbose and (k % 10 == 0 or k == stages):
            d = s.diagnostics()
            _log(f"[prep] growth stage {k}/{stages} scale {lam:.3f}: pairs {int(d[7])} "
                 f"Z {2 * d[7] / n:.2f} max overlap {d[9]:.2e} ({time.time() - t0:.1f}s)")
    st = s.read_state()
    s.close()
    del s
    torch.cuda.empty_cache()
    g = tuple(settle_g * t for t in w["params"]["gravity"])
    settle_p = dict(w["params"], restitution=0.1, mu=0.3, eta_t_ratio=1.0, gravity=g)
    s = dem.System(settle_p, st["x"], st["v"], st["omega"], r_full, device=device)
    if settle_steps > 0:
        s.step(settle_steps)
    relax_p = dict(w["params"], restitution=0.1, mu=0.3, eta_t_ratio=1.0)
    if relax_steps > 0:
        st = s.read_state()
        s.close()
        del s
        s = dem.System(relax_p, st["x"], st["v"], st["omega"], r_full, device=device)
        s.step(relax_steps)
    # quench: restart at rest (no history) and let the bed find its static
    # equilibrium under gravity again, several times
    for q in range(quench_cycles):
        st = s.read_state()
        s.close()
        del s
        s = dem.System(relax_p, st["x"], zero, zero, r_full, device=device)
        s.step(quench_steps)
        if verbose and (q % 4 == 3 or q == quench_cycles - 1):
            d = s.diagnostics()
            _log(f"[prep] quench {q + 1}/{quench_cycles}: Z {(2 * d[7] + d[8]) / n:.2f} KE {d[3]:.3e} J "
                 f"max overlap {d[9]:.2e} ({time.time() - t0:.1f}s)")
    d = s.diagnostics()
    st = s.read_state()
    s.close()
    del s
    torch.cuda.empty_cache()
    info = dict(lattice_scale=lam0, fill_height=w.get("fill_height", 1.0), stages=stages,
                steps_per_stage=steps_per_stage, settle_steps=settle_steps,
                grow_mu=grow_mu, settle_g=settle_g, relax_steps=relax_steps, quench_cycles=quench_cycles,
                quench_steps=quench_steps,
                pairs=int(d[7]), walls=int(d[8]), Z=float(2 * d[7] + d[8]) / n, max_overlap=float(d[9]),
                kinetic_energy=float(d[3]), seconds=time.time() - t0)
    if verbose:
        _log(f"[prep] settled: Z {info['Z']:.2f} (pairs {info['pairs']}, walls {info['walls']}), "
             f"max overlap {info['max_overlap']:.2e}, KE {info['kinetic_energy']:.3e} J, {info['seconds']:.1f}s")
    return st["x"], st["v"], st["omega"], info


def grow_systems(systems, stages=40, steps_per_stage=50, grow_mu=0.5, verbose=False, max_batch=1 << 23):
    """``grow_one_batch`` over groups of at most max_batch spheres."""
    out = [dict(s) for s in systems]
    group, size = [], 0
    todo = [k for k, s in enumerate(systems) if s.get("r_target") is not None]
    t0 = time.time()
    for k in todo + [None]:
        n = 0 if k is None else len(systems[k]["r"])
        if group and (k is None or size + n > max_batch):
            grown = grow_one_batch([systems[j] for j in group], stages, steps_per_stage, grow_mu)
            for j, g in zip(group, grown):
                out[j] = g
            group, size = [], 0
        if k is not None:
            group.append(k)
            size += n
    if verbose and todo:
        _log(f"[prep] grew {len(todo)} systems to their packing fractions in {time.time() - t0:.1f}s")
    return out


def grow_one_batch(systems, stages=40, steps_per_stage=50, grow_mu=0.5, verbose=False):
    """Bring the systems of the batched and serving workloads that start
    below their drawn packing fraction (``r_target`` set by
    ``workloads.unit_box_system``: the lattice cannot hold the drawn radii
    without overlaps) to their drawn radii: all of them in one batch, radii
    raised in `stages` equal steps of the scale with strongly damped contacts
    (restitution 0.1, friction grow_mu), no gravity, `steps_per_stage` steps
    each.  Untimed preparation through this library; it makes starting states
    only.  Returns new system dicts (the others unchanged) whose x are the
    grown positions, r the drawn radii, v, omega the workload's initial ones,
    and phi_start the packing fraction reached."""
    grow = [k for k, s in enumerate(systems) if s.get("r_target") is not None]
    out = [dict(s) for s in systems]
    if not grow:
        return out
    t0 = time.time()
    sub = []
    for k in grow:
        s = systems[k]
        p = dict(s["params"], restitution=0.1, mu=grow_mu, eta_t_ratio=1.0, gravity=(0.0, 0.0, 0.0),
                 tile_cells=0, cell_divisor=1)
        z = np.zeros_like(s["x"])
        sub.append(dict(params=p, x=s["x"], v=z, omega=z, r=s["r"]))
    b = dem.Batch(sub)
    r0 = [np.asarray(systems[k]["r"], dtype=np.float64) for k in grow]
    r1 = [np.asarray(systems[k]["r_target"], dtype=np.float64) for k in grow]
    for stage in range(1, stages + 1):
        f = stage / stages
        b.set_radii([a + (c - a) * f for a, c in zip(r0, r1)])
        b.step(steps_per_stage)
    for j, k in enumerate(grow):
        st = b.read_state(j)
        s = out[k]
        s["x"] = st["x"]
        s["r"] = systems[k]["r_target"]
        s["r_target"] = None
        s["phi_start"] = float(np.sum(4.0 / 3.0 * np.pi * np.asarray(s["r"], dtype=np.float64) ** 3))
    b.close()
    if verbose:
        _log(f"[prep] grew {len(grow)} systems to their packing fractions in {time.time() - t0:.1f}s")
    return out
