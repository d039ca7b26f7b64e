#!/usr/bin/env python3
"""Benchmark of the DEM step (practical contact model, linear law) on one GPU.

Headline workload: the dense granular bed -- 2^24 = 16,777,216 spheres with
log-normal radii (median 1/512, sigma 0.2, clipped to +-3 sigma) at packing
fraction 0.55 in a walled 4:1:1 box, gravity along the short axis, FP32 forces
with FP64 positions, dt = t_c,min / 10.  The bed is prepared untimed (radius
growth in the lower 93% of the box, then quenched relaxation under gravity;
see paper_1301_1714_amd/prepare.py); the timed steps run with kn = 1e5,
e = 0.9, kt = 2/7 kn, mu = 0.3.

Also measured (unless skipped):
  configs  the other single-system workloads, each as specified: 4,096 equal
           spheres in FP64 (1,000 steps) and the 2^20-sphere settling gas
           under the practical (linear) law and under the simple law of Eq. 1
           (10,000 steps each), with graph replay; the practical/simple time
           ratio is reported next to the paper's (about 7 on its GPU).
  batched  256 independent systems (sizes log-uniform in [1k, 256k], materials
           and packing fractions drawn per system), cells from the autotuner,
           all stepped together with graph replay, 1,000 steps each; against
           the same systems run one at a time through the plain path.
  serving  requests (sizes log-uniform in [1k, 1M], steps in [100, 1e4]) with
           Poisson arrivals at 70% of the one-at-a-time server's capacity,
           served by the continuous-batching loop; p50/p99 completion latency
           and throughput against the one-at-a-time FIFO baseline on the same
           arrivals, and a check that every served result is bit-identical.

Prints one JSON line: particle-steps/s of the dense bed, the roofline of its
dominant kernel (timed live with HIP events on the library's stream), the
per-phase times, the batched and serving results, and the FP64 CPU oracle
timed on a bounded sample of the dense-bed recipe.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (practical model) at 16M"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
FILL_HEIGHT = 0.93     # the prepared bed fills the lower 93% of the box
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "hbm_traffic_dense_bed_16M.json")
VALU_JSON = os.path.join(ROOT, "profiles", "sq_counters_dense_bed_16M.json")
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    """sha256 of the kernel source: HBM traffic counted for an older version
    of the kernels is not reported for this one."""
    import hashlib

    path = os.path.join(ROOT, "paper_1301_1714_amd", "csrc", "dem_kernels.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc
    summary (FETCH_SIZE and WRITE_SIZE scaled by what the same counters read
    for a plain copy of known size), or None when there is none for the
    current kernel source."""
    path = TRAFFIC_JSON
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else float(k["bytes_per_launch"])


def measured_valu(kernel):
    """FP32 VALU utilisation of `kernel` from the committed rocprofv3 --pmc
    summary (SQ_INSTS_VALU per busy CU cycle against the 2 wave64
    instructions per CU cycle of the 157.3 TFLOP/s peak, times the share of
    lanes active), or None when there is none for the current kernel
    source."""
    path = VALU_JSON
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if k is None:
        return None
    return {"frac": float(k["valu_utilisation"]), "issue_frac": float(k["valu_issue"]),
            "lane_use": float(k["lane_use"]), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "address_unit_busy": float(k["ta_busy"])}


def copy_probe(mib, reps):
    """A plain device-to-device copy of known size, for scaling the HBM
    counters of the profiler (run under rocprofv3 --pmc)."""
    import torch

    n = mib << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n, "copy_probe_bytes_written": n, "reps": reps}), flush=True)


# ------------------------------------------------------------ byte models
# Algorithmic bytes: what a kernel must move at least, each item once per
# launch; neighbour data reused from LDS or cache is not counted.  R is the
# size of a Real (4 with FP32 forces, 8 in FP64).

def contacts_bytes(n, ncell, P, R):
    """k_contacts_direct (detection and the contact law in one pass): per
    particle its 8-byte fixed-point candidate record, its packed state (x
    24 B, v and w 6R, r, id, previous slot and history count 16 B) and cell
    (4 B) read, its contact count, history count and first contact index
    (4 B each) written; per owned contact (P of them, pairs once plus walls)
    the list entry (4 B), the committed history entry read (key 4 B, delta_t
    3R), the new one written (4 + 3R), the force record written (6R), the
    partner slot (4 B) and the entry filed with the partner's workgroup (8 B;
    its count's atomic is one per group of a wave's contacts and not
    counted); the cell starts read once.  Partner records and neighbouring
    candidate records are reuse."""
    return n * (64 + 6 * R) + P * (24 + 12 * R) + 4 * (ncell + 1)


def gather_bytes(n, P, R):
    """k_gather: per particle its packed state (40 + 6R), contact count and
    first contact index (4 B each), the state written back (x 24 B, r 4, id
    4, v and w 6R, cell 4); per contact the force record read by the owner
    and by the partner (2 x 6R) and the filed entry (8 B)."""
    return n * (84 + 12 * R) + P * (8 + 12 * R)


def step_algorithmic_bytes(n, z, R):
    """Minimum HBM bytes of a whole step per the method: the particle state
    read and written once (x 24 B, v and w 6R, r 4, id 4), cell id and
    permutation written and read (16 B), cell starts (about 3 B), and the
    tangential history of the Z/2 pairs of each particle read and written
    (Z/2 x (4 + 3R) x 2)."""
    state = 24 + 6 * R + 4 + 4
    return n * (2 * state + 16 + 3 + z * (4 + 3 * R))


# ------------------------------------------------------------ CPU oracle

CPU_SAMPLE_N = 1 << 15


def oracle_sample(seed, seconds):
    """The FP64 oracle, single-threaded, on 2^15 spheres of the dense-bed
    recipe (same radius distribution, number density, box aspect and cell
    width) on its FCC lattice at 1.05x the largest non-overlapping radius
    scale, stepped for about `seconds`; returns (particle-steps, elapsed s,
    steps, lattice scale)."""
    from oracle.oracle import OracleSystem
    from paper_1301_1714_amd import workloads as W

    w = W.dense_bed_lattice(seed=seed, n=CPU_SAMPLE_N)
    lam = 1.05 * W.lattice_scale(w["r"], w["d_nn"])
    o = OracleSystem(w["params"], w["x"], w["v"], w["omega"], w["r"] * lam)
    t0 = time.perf_counter()
    o.step(2)
    per = (time.perf_counter() - t0) / 2
    k = max(2, int(seconds / max(per, 1e-6)))
    t0 = time.perf_counter()
    o.step(k)
    dt = time.perf_counter() - t0
    return CPU_SAMPLE_N * k, dt, k, lam


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    share = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"model": model, "nproc": os.cpu_count(), "usable": share}


def cpu_baseline(target_seconds):
    """The FP64 oracle on the host: one thread on a bounded sample of the
    dense-bed recipe (the paper's CPU baseline is one core), and the same on
    every usable core at once -- independent oracle processes, each on its own
    seeded sample, their particle-steps summed (the oracle's arithmetic and
    order are untouched; the host's cores are used the way independent runs
    would use them).  At most 16 processes (the host share of one GPU)."""
    from oracle import build as oracle_build
    from oracle.oracle import OracleSystem
    from paper_1301_1714_amd import workloads as W

    oracle_build.build()  # -O3, as the tests use it
    info = cpu_info()
    work, dt, k, lam = oracle_sample(3000, 0.5 * target_seconds)
    single = {"value": work / dt, "unit": "particle-steps/s", "cores": 1,
              "sample": f"{CPU_SAMPLE_N} spheres of the dense-bed recipe (lattice at {lam:.3f} of full radii), "
                        f"{k} steps, {dt:.1f} s, FP64, one thread"}
    procs = max(1, min(16, int(info["usable"] or 1)))
    import subprocess

    cmd = [sys.executable, os.path.abspath(__file__), "--oracle-worker"]
    kids = [subprocess.Popen(cmd + [str(3000 + 17 * j), str(0.5 * target_seconds)], stdout=subprocess.PIPE,
                             text=True) for j in range(procs)]
    t0 = time.perf_counter()
    outs = [json.loads(kid.communicate()[0].strip().splitlines()[-1]) for kid in kids]
    wall = time.perf_counter() - t0
    total = sum(o["work"] for o in outs)
    span = max(o["seconds"] for o in outs)
    out = {"value": total / span, "unit": "particle-steps/s", "cores": procs, "kind": "oracle",
           "sample": f"{procs} independent single-thread oracle processes, each {CPU_SAMPLE_N} spheres of the "
                     f"dense-bed recipe on its own seeded lattice, about {0.5 * target_seconds:.0f} s each "
                     f"({wall:.1f} s wall); FP64, built -O3",
           "cpu": info, "single_core": single}
    # the 4,096-sphere FP64 configuration in full (1,000 steps), for the
    # GPU/CPU ratio of the paper's kind (one core)
    wp = W.plain_fp64(seed=1000)
    o = OracleSystem(wp["params"], wp["x"], wp["v"], wp["omega"], wp["r"])
    t0 = time.perf_counter()
    o.step(1000)
    dt = time.perf_counter() - t0
    out["plain_fp64_4096"] = {"value": 4096 * 1000 / dt, "unit": "particle-steps/s", "cores": 1,
                              "sample": f"4096 spheres, 1000 steps, {dt:.1f} s"}
    return out


# ------------------------------------------------------------ dense bed

_DENSE = {}  # the prepared bed, for the law comparison of bench_configs


def bench_dense(args):
    import torch

    from paper_1301_1714_amd import dem, prepare
    from paper_1301_1714_amd import workloads as W

    t0 = time.time()
    w = W.dense_bed_lattice(seed=args.seed, n=args.n, fill_height=FILL_HEIGHT)
    log(f"[bench] generated {args.n} spheres in {time.time() - t0:.1f}s; box {w['params']['box_hi']}")
    if args.cache and os.path.exists(args.cache):
        z = np.load(args.cache)
        x, v, om = z["x"], z["v"], z["omega"]
        prep = json.loads(str(z["info"]))
        log(f"[bench] prepared bed loaded from {args.cache}")
    else:
        x, v, om, prep = prepare.grow_dense_bed(w)
        if args.cache:
            np.savez(args.cache, x=x, v=v, omega=om, info=json.dumps(prep))
    p = w["params"]
    _DENSE.update(w=w, x=x, v=v, omega=om)
    s = dem.System(p, x, v, om, w["r"])
    dims = s.grid_dims()
    ncell = dims[0] * dims[1] * dims[2]
    s.step(args.warmup)
    s.sync()
    d0 = s.diagnostics()
    s.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    s.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms, timed = s.profile_read()
    d1 = s.diagnostics()
    s.close()
    n = args.n
    value = n * args.steps / elapsed
    ms_per_step = elapsed * 1e3 / args.steps
    phase_ms = {ph: float(ms[i] / max(timed, 1)) for i, ph in enumerate(dem.PHASES)}
    # contacts owned per particle (pairs once, walls) and coordination number
    pairs = 0.5 * (d0[7] + d1[7])
    walls = 0.5 * (d0[8] + d1[8])
    P = pairs + walls
    Z = 2.0 * pairs / n
    R = 4 if p["precision"] == "mixed" else 8
    kernels = {
        "k_contacts_direct": ("contacts", contacts_bytes(n, ncell, P, R)),
        "k_gather": ("gather", gather_bytes(n, P, R)),
    }
    name = max(kernels, key=lambda k: phase_ms[kernels[k][0]])
    ph, nbytes = kernels[name]
    avg = phase_ms[ph]
    roof = {"kernel": name, "bound": "hbm", "achieved": nbytes / (avg * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "traffic": measured_traffic(name), "bytes_per_launch": nbytes, "avg_ms": avg,
            "valu": measured_valu(name)}
    roof["frac"] = roof["achieved"] / roof["peak"]
    others = {k: {"avg_ms": phase_ms[v[0]], "bytes_per_launch": v[1],
                  "achieved_GBs": v[1] / (phase_ms[v[0]] * 1e-3) / 1e9} for k, v in kernels.items()}
    sb = step_algorithmic_bytes(n, Z, R)
    out = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 forces, f64 positions", "data": "synthetic",
        "config": {"workload": f"dense_bed_{n}", "n_particles": n, "law": p["law"], "precision": p["precision"],
                   "phi": 0.55, "box": list(p["box_hi"]), "dt": p["dt"], "cell": p["cell_size"],
                   "grid": list(dims), "Z": Z, "contacts_per_particle": P / n, "prep": prep},
        "roofline": roof,
        "kernels": others,
        "phases_ms": phase_ms,
        "step_hbm": {"algorithmic_bytes_per_step": sb, "achieved_GBs": sb / (ms_per_step * 1e-3) / 1e9,
                     "frac": sb / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS},
    }
    return out


# ------------------------------------------------------------ precision

def _force_errors(F, T, Fo, To, Fa, Ta, mask):
    """Per-particle force and torque errors against the oracle, relative to
    each particle's contact-force scale (the sum of the magnitudes of its
    contact forces / torques); particles with contacts in `mask`."""
    m = mask & (Fa > 0)
    ef = np.linalg.norm(F - Fo, axis=1)[m] / Fa[m]
    mt = mask & (Ta > 0)
    et = np.linalg.norm(T - To, axis=1)[mt] / Ta[mt]
    q = lambda a, p: float(np.percentile(a, p)) if a.size else None
    return {"particles": int(m.sum()), "force_max": q(ef, 100), "force_p50": q(ef, 50), "force_p99": q(ef, 99),
            "torque_max": q(et, 100), "torque_p50": q(et, 50)}


def precision_errors(name, w, x, v, om, checkpoints, window=None):
    """The error of mixed precision (FP32 v, w, forces and history, FP64
    positions and reductions) stated per result for one workload:
      trajectory  the same initial state stepped in mixed precision and in FP64
                  (both on the GPU; the FP64 path tracks the FP64 oracle to
                  1e-9 in the tests) -- largest position difference, relative
                  to the largest radius, at each checkpoint
      diagnostics the FP64 reductions (momentum, kinetic, rotational,
                  potential and elastic energy) of both runs, their relative
                  difference at each checkpoint
      forces      at the last checkpoint, the mixed-precision forces on the
                  mixed run's own state (positions, velocities, spins and
                  committed history) against the FP64 oracle's on that same
                  state, per particle relative to its contact-force scale;
                  window=(axis, lo, hi, margin): only the particles with
                  lo <= x_axis < hi go to the oracle, and those at least
                  `margin` inside the window are compared (all their contacts
                  lie in it)."""
    from oracle.oracle import OracleSystem
    from paper_1301_1714_amd import dem

    r = np.asarray(w["r"])
    rmax = float(r.max())
    pm = dict(w["params"], precision="mixed")
    pf = dict(w["params"], precision="fp64")
    t0 = time.time()
    sm = dem.System(pm, x, v, om, r)
    sf = dem.System(pf, x, v, om, r)
    traj, diag = [], []
    done = 0
    keys = ("momentum", "kinetic", "rotational", "potential", "elastic")
    for c in checkpoints:
        sm.step(c - done)
        sf.step(c - done)
        done = c
        a, b = sm.read_state(), sf.read_state()
        dm, df = sm.diagnostics(), sf.diagnostics()
        traj.append({"step": c, "x_max_diff_over_rmax": float(np.abs(a["x"] - b["x"]).max() / rmax),
                     "v_max_diff": float(np.abs(a["v"] - b["v"]).max()), "v_max": float(np.abs(b["v"]).max())})
        mom = float(np.linalg.norm(dm[:3] - df[:3]) / max(np.linalg.norm(df[:3]), 1e-300))
        rel = lambda i: float(abs(dm[i] - df[i]) / max(abs(df[i]), 1e-300))
        diag.append({"step": c, **dict(zip(keys, [mom] + [rel(i) for i in (3, 4, 5, 6)])),
                     "pairs_mixed": int(dm[7]), "pairs_fp64": int(df[7])})
    sf.close()
    del sf
    st = sm.read_state()
    pairs, dts = sm.read_contacts()
    F, T = sm.forces()
    sm.close()
    del sm
    if window is None:
        sel = np.arange(len(r))
        inner = np.ones(len(r), bool)
    else:
        ax, lo, hi, margin = window
        sel = np.nonzero((st["x"][:, ax] >= lo) & (st["x"][:, ax] < hi))[0]
        xa = st["x"][sel, ax]
        inner = (xa >= lo + margin) & (xa < hi - margin)
    local = -np.ones(len(r), np.int64)
    local[sel] = np.arange(len(sel))
    keep = (local[pairs[:, 0]] >= 0) & ((pairs[:, 1] < 0) | (local[np.maximum(pairs[:, 1], 0)] >= 0))
    hp = pairs[keep].copy()
    hp[:, 0] = local[hp[:, 0]]
    hp[:, 1] = np.where(hp[:, 1] >= 0, local[np.maximum(hp[:, 1], 0)], hp[:, 1])
    o = OracleSystem(pf, st["x"][sel], st["v"][sel], st["omega"][sel], r[sel], F0=np.zeros((len(sel), 3)),
                     T0=np.zeros((len(sel), 3)), hist_pairs=hp, hist_dt=dts[keep])
    Fo, To, Fa, Ta = o.forces_scale()
    del o
    out = {"workload": name, "trajectory": traj, "diagnostics": diag,
           "forces": {"step": done, **_force_errors(F[sel], T[sel], Fo, To, Fa, Ta, inner),
                      "compared": "all particles" if window is None else
                      f"{int(inner.sum())} particles at least {window[3]:.4g} m inside a window of {len(sel)}"},
           "seconds": time.time() - t0}
    log(f"[bench] precision {name}: forces max {out['forces']['force_max']:.2e}, x diff "
        f"{traj[-1]['x_max_diff_over_rmax']:.2e} r_max after {done} steps ({out['seconds']:.0f}s)")
    return out


def bench_precision(args):
    """Mixed precision's error on the 2^20 settling gas (from its seeded start,
    over 3,000 steps; the oracle takes the whole system) and on the prepared
    2^24 bed (100 steps; the oracle takes a window of the bed)."""
    from paper_1301_1714_amd import workloads as W

    out = {}
    g = W.gas_mixed(seed=2000)
    out["gas_2^20"] = precision_errors("gas_2^20", g, g["x"], g["v"], g["omega"], (10, 100, 1000, 3000))
    if _DENSE:
        w = _DENSE["w"]
        cell = float(w["params"]["cell_size"])
        mid = 0.5 * float(w["params"]["box_hi"][0])
        out["dense_2^24"] = precision_errors("dense_2^24", w, _DENSE["x"], _DENSE["v"], _DENSE["omega"], (10, 100),
                                             window=(0, mid - 0.03, mid + 0.03, 1.5 * cell))
    return out


# ------------------------------------------------------------ other configs

PAPER_SIMPLE_RATIO = 21266.0 / 2960.0  # Table 3: simple vs practical model, OpenCL on its GPU
PAPER_GPU_VS_CPU = 2960.0 / 474.0       # Table 3: practical model, its GPU vs one core of its CPU


def time_system(w, steps, warmup):
    """Particle-steps/s of one system stepped alone with graph replay."""
    import torch

    from paper_1301_1714_amd import dem

    st = torch.cuda.Stream()
    s = dem.System(w["params"], w["x"], w["v"], w["omega"], w["r"], stream=st)
    try:
        s.use_graph(True)
        s.step(warmup)
        s.sync()
        t0 = time.perf_counter()
        s.step(steps)
        s.sync()
        el = time.perf_counter() - t0
        d = s.diagnostics()
    finally:
        s.close()
    n = len(w["r"])
    return {"value": n * steps / el, "unit": "particle-steps/s", "ms_per_step": 1e3 * el / steps, "n": n,
            "steps": steps, "Z": 2.0 * float(d[7]) / max(n, 1)}


def bench_configs(args):
    from paper_1301_1714_amd import workloads as W

    out = {"plain_fp64_4096": time_system(W.plain_fp64(seed=1000), 1000, 20)}
    log(f"[bench] plain FP64 4096: {out['plain_fp64_4096']['value']:.4g} particle-steps/s")
    # both laws from the same seeded gas, over the configuration's 10,000 steps
    for law in ("linear", "simple"):
        w = W.gas_mixed(seed=2000, law=law)
        out[f"gas_2^20_{law}"] = time_system(w, args.gas_steps, 20)
        log(f"[bench] gas 2^20 {law}: {out[f'gas_2^20_{law}']['value']:.4g} particle-steps/s")
    lin, sim = out["gas_2^20_linear"], out["gas_2^20_simple"]
    out["practical_vs_simple_time_ratio"] = lin["ms_per_step"] / sim["ms_per_step"]
    out["paper_practical_vs_simple_time_ratio"] = PAPER_SIMPLE_RATIO
    # the same comparison where contacts abound: the prepared 2^24 bed under
    # both laws (simple-law coefficients for its median radius)
    if _DENSE:
        w = _DENSE["w"]
        base = dict(w, x=_DENSE["x"], v=_DENSE["v"], omega=_DENSE["omega"])
        r_med = float(np.median(w["r"]))
        runs = {}
        for law in ("linear", "simple"):
            p = dict(w["params"], law=law)
            if law == "simple":
                p["simple_k"] = W.simple_coefficients(r_med)
            runs[law] = time_system(dict(base, params=p), args.dense_law_steps, 10)
            log(f"[bench] dense 2^24 {law} (graph replay): {runs[law]['ms_per_step']:.3f} ms/step")
        out["dense_2^24_linear"], out["dense_2^24_simple"] = runs["linear"], runs["simple"]
        out["dense_practical_vs_simple_time_ratio"] = runs["linear"]["ms_per_step"] / runs["simple"]["ms_per_step"]
    out["slit_hopper_131072"] = bench_hopper(args)
    return out


def bench_hopper(args):
    """The paper's sample problem (Sec. 5): 2^17 equal spheres falling from a
    box through a slit onto a floor.  Timed: the first hopper_steps steps
    from rest with graph replay (the fall, the first impacts on the plates
    and the first spheres through the slit).  With --hopper-rest the run then
    goes on until every sphere's step dt |v| is below the workload's threshold
    (checked every 2,000 steps), and the steps to rest are reported."""
    import torch

    from paper_1301_1714_amd import dem
    from paper_1301_1714_amd import workloads as W

    w = W.slit_hopper()
    st = torch.cuda.Stream()
    s = dem.System(w["params"], w["x"], w["v"], w["omega"], w["r"], stream=st)
    try:
        s.use_graph(True)
        s.step(20)
        s.sync()
        t0 = time.perf_counter()
        s.step(args.hopper_steps)
        s.sync()
        el = time.perf_counter() - t0
        d = s.diagnostics()
        n = len(w["r"])
        out = {"value": n * args.hopper_steps / el, "unit": "particle-steps/s",
               "ms_per_step": 1e3 * el / args.hopper_steps, "n": n, "steps": args.hopper_steps,
               "Z": (2.0 * float(d[7]) + float(d[8])) / n, "slit": list(w["slit"]), "z_slit": w["z_slit"],
               "box": list(w["params"]["box_hi"]), "dt": w["params"]["dt"]}
        if args.hopper_rest:
            t0 = time.perf_counter()
            k = s.run_to_rest(w["rest_displacement"], 2000, args.hopper_rest_max)
            el = time.perf_counter() - t0
            x = s.read_state()["x"]
            out["to_rest"] = {"steps": 20 + args.hopper_steps + k, "reached": bool(k < args.hopper_rest_max),
                              "seconds": el, "particle_steps_per_s": n * k / el,
                              "fraction_below_slit": float(np.mean(x[:, 2] < w["z_slit"])),
                              "threshold_m_per_step": w["rest_displacement"]}
    finally:
        s.close()
    log(f"[bench] slit hopper 2^17: {out['value']:.4g} particle-steps/s")
    return out


# ------------------------------------------------------------ batched

def bench_batched(args):
    import torch

    from paper_1301_1714_amd import autotune, dem, prepare
    from paper_1301_1714_amd import workloads as W

    draws = W.batched_draws(seed=args.batch_seed, count=args.batch_systems)
    t0 = time.time()
    table = autotune.Table.load(args.tune_cache)
    keys = [autotune.system_class(d["n"], d["phi"]) for d in draws]
    table = autotune.tune(keys, table, steps=20, log=log)
    table.save(args.tune_cache)
    t_tune = time.time() - t0
    factors = autotune.factors_for(draws, table)
    tiles = autotune.tiles_for(draws, table)
    divisors = autotune.divisors_for(draws, table)
    t0 = time.time()
    systems = W.batched_systems(seed=args.batch_seed, count=args.batch_systems, cell_factors=factors, tiles=tiles,
                                divisors=divisors)
    # systems drawn denser than their lattice holds are grown to their drawn
    # packing fraction first (untimed)
    systems = prepare.grow_systems(systems, verbose=True)
    ns = np.array([len(s["r"]) for s in systems])
    log(f"[bench] batched: {len(systems)} systems, {ns.sum()} spheres, generated in {time.time() - t0:.1f}s, "
        f"tuned in {t_tune:.1f}s")
    b = dem.Batch(systems)
    d0 = b.diagnostics()
    z_start = (2.0 * d0[:, 7] + d0[:, 8]) / np.maximum(ns, 1)
    b.use_graph(True)
    b.step(10)
    b.sync()
    b.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(args.batch_steps)
    b.sync()
    elapsed = time.perf_counter() - t0
    ms, timed = b.profile_read()
    diag = b.diagnostics()
    b.close()
    del b
    work = float(ns.sum()) * args.batch_steps
    batched_rate = work / elapsed
    # the same systems one at a time through the plain single-system path
    # (skipped with --plain-steps 0, e.g. for a profile of the batch alone)
    t_plain = 0.0
    for s in systems if args.plain_steps > 0 else []:
        one = dem.System(s["params"], s["x"], s["v"], s["omega"], s["r"])
        one.step(2)
        one.sync()
        t0 = time.perf_counter()
        one.step(args.plain_steps)
        one.sync()
        t_plain += time.perf_counter() - t0
        one.close()
    plain_rate = float(ns.sum()) * args.plain_steps / t_plain if t_plain > 0 else None
    fac, cnt = np.unique(factors, return_counts=True)
    til, tcnt = np.unique(tiles, return_counts=True)
    return {
        "workload": f"batched_{len(systems)}_systems", "systems": len(systems), "n_total": int(ns.sum()),
        "n_min": int(ns.min()), "n_max": int(ns.max()), "steps": args.batch_steps,
        "value": batched_rate, "unit": "particle-steps/s", "ms_per_step": elapsed * 1e3 / args.batch_steps,
        "graph": True, "plain_one_at_a_time": {"value": plain_rate, "unit": "particle-steps/s",
                                              "steps_per_system": args.plain_steps},
        "speedup_vs_plain": batched_rate / plain_rate if plain_rate else None,
        "cell_factors": {str(f): int(c) for f, c in zip(fac, cnt)},
        "detect_tiles": {str(t): int(c) for t, c in zip(til, tcnt)},
        "cell_divisors": {str(int(d)): int(c) for d, c in zip(*np.unique(divisors, return_counts=True))},
        "Z_mean": float(2.0 * diag[:, 7].sum() / ns.sum()),
        "Z_mean_start": float(np.sum(z_start * ns) / ns.sum()),
        "per_system": {"n": ns.tolist(), "phi": [round(float(s["phi"]), 4) for s in systems],
                       "phi_start": [round(float(s["phi_start"]), 4) for s in systems],
                       "Z_start": [round(float(z), 3) for z in z_start]},
        "phi_start_minus_phi_max_abs": float(max(abs(s["phi_start"] - s["phi"]) for s in systems)),
        "tune_seconds": t_tune,
    }


# ------------------------------------------------------------ serving

def bench_serving(args):
    import torch

    from paper_1301_1714_amd import prepare, serve
    from paper_1301_1714_amd import workloads as W

    specs = W.serving_requests(seed=args.serve_seed, count=args.serve_requests)
    t0 = time.time()
    systems = [W.unit_box_system(d["seed"], d["n"], d["kn"], d["restitution"], d["mu"], d["phi"]) for d in specs]
    # a request's initial state is the client's: requests drawn denser than
    # their lattice holds arrive grown to their packing fraction (untimed)
    systems = prepare.grow_systems(systems, verbose=True)
    log(f"[bench] serving: {len(specs)} requests, {sum(d['n'] for d in specs)} spheres, "
        f"{sum(d['n'] * d['steps'] for d in specs):.3e} particle-steps, generated in {time.time() - t0:.1f}s")
    ex = serve.GpuExecutor(use_graph=True)
    # one at a time, plain path: measured service times (create, step, read back)
    ex.run_alone(systems[0], 5)  # warm the code paths
    ref = []
    service = []
    for d, s in zip(specs, systems):
        t0 = time.perf_counter()
        st = ex.run_alone(s, d["steps"])
        service.append(time.perf_counter() - t0)
        ref.append(st["x"])
    service = np.array(service)
    work = np.array([d["n"] * d["steps"] for d in specs], dtype=float)
    plain_rate = work.sum() / service.sum()
    rate = serve.rate_for_load(args.serve_load, plain_rate, work.mean())
    arrivals = W.poisson_arrivals(args.serve_seed, len(specs), rate)
    base_lat = serve.fifo_latencies(arrivals, service)
    base_span = max(arrivals[k] + base_lat[k] for k in range(len(specs))) - arrivals[0]
    log(f"[bench] serving: one-at-a-time busy {service.sum():.1f}s; arrival rate {rate:.3f}/s")
    reqs = [serve.Request(k, s, d["steps"], a) for k, (d, s, a) in enumerate(zip(specs, systems, arrivals))]
    torch.cuda.empty_cache()
    budget = int(args.serve_hbm_frac * ex.free_bytes())
    srv = serve.Server(ex, hbm_budget=budget, max_slots=args.serve_slots, chunk=args.serve_chunk)
    done = srv.run(reqs)
    by_id = {r.rid: r for r in done}
    identical = all(by_id[k].error is None and np.array_equal(by_id[k].result["x"], ref[k])
                    for k in range(len(specs)))
    lat = np.array([by_id[k].latency for k in range(len(specs))])
    span = max(by_id[k].t_done for k in range(len(specs))) - arrivals[0]
    return {
        "workload": f"serving_{len(specs)}_requests", "requests": len(specs),
        "arrival_rate_per_s": rate, "load_vs_one_at_a_time": args.serve_load,
        "served": {**serve.percentiles(lat), "throughput": work.sum() / span, "unit_latency": "s",
                   "unit_throughput": "particle-steps/s", "peak_slots": srv.peak_slots,
                   "peak_bytes": srv.peak_bytes, "iterations": srv.iterations, "chunk_steps": args.serve_chunk},
        "one_at_a_time": {**serve.percentiles(base_lat), "throughput": work.sum() / base_span,
                          "busy_throughput": plain_rate, "unit_latency": "s"},
        "results_bit_identical_to_alone": bool(identical),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=1 << 24, help="particles of the dense bed (default 2^24)")
    ap.add_argument("--seed", type=int, default=3000)
    ap.add_argument("--cache", default=None, help="npz file holding the prepared bed (written if missing)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the FP64 4,096 and the 2^20 gas runs")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the mixed-precision error statement (gas and bed against FP64 and the oracle)")
    ap.add_argument("--gas-steps", type=int, default=10000)
    ap.add_argument("--dense-law-steps", type=int, default=100)
    ap.add_argument("--hopper-steps", type=int, default=2000)
    ap.add_argument("--hopper-rest", action="store_true",
                    help="also run the slit hopper until every sphere is at rest (long)")
    ap.add_argument("--hopper-rest-max", type=int, default=3000000)
    ap.add_argument("--batch-systems", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--batch-seed", type=int, default=4000)
    ap.add_argument("--plain-steps", type=int, default=50)
    ap.add_argument("--tune-cache", default=os.path.join(os.path.expanduser("~"), ".cache",
                                                         "paper_1301_1714_amd", "autotune.json"))
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests served (the recipe's stream is 512; 200 keep the default run within minutes)")
    ap.add_argument("--serve-seed", type=int, default=5000)
    ap.add_argument("--serve-load", type=float, default=0.7)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-chunk", type=int, default=100)
    ap.add_argument("--serve-hbm-frac", type=float, default=0.8)
    ap.add_argument("--only-dense", action="store_true", help="skip the other configs, batched, serving and the CPU baseline")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the batched workload and print its record (a profile of the batch)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this size (profiler counter calibration)")
    if len(sys.argv) == 4 and sys.argv[1] == "--oracle-worker":
        work, dt, k, _ = oracle_sample(int(sys.argv[2]), float(sys.argv[3]))
        print(json.dumps({"work": work, "seconds": dt, "steps": k}), flush=True)
        return
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only: multi-GPU runs are a design, not "
                                   "built (run with --gpus 1)"}))
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe:
        copy_probe(args.copy_probe, 5)
        return
    from paper_1301_1714_amd import dem
    dem.lib()
    if args.only_batched:
        print(json.dumps({"batched": bench_batched(args)}), flush=True)
        return
    out = bench_dense(args)
    log(f"[bench] dense bed: {out['value']:.4g} particle-steps/s, {out['ms_per_step']:.3f} ms/step")
    if not (args.no_configs or args.only_dense):
        out["configs"] = bench_configs(args)
    if not (args.no_precision or args.only_dense):
        out["precision_errors"] = bench_precision(args)
    if not (args.no_batched or args.only_dense):
        out["batched"] = bench_batched(args)
        log(f"[bench] batched: {out['batched']['value']:.4g} particle-steps/s "
            f"({out['batched']['speedup_vs_plain'] or 0:.2f}x plain)")
    if not (args.no_serve or args.only_dense):
        out["serving"] = bench_serving(args)
        sv = out["serving"]
        log(f"[bench] serving: p50 {sv['served']['p50']:.3f}s p99 {sv['served']['p99']:.3f}s vs one at a time "
            f"p50 {sv['one_at_a_time']['p50']:.3f}s p99 {sv['one_at_a_time']['p99']:.3f}s")
    if not (args.no_cpu_baseline or args.only_dense):
        log("[bench] timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        if "configs" in out:
            g, c = out["configs"]["plain_fp64_4096"], out["cpu_baseline"]["plain_fp64_4096"]
            g["vs_oracle_1core"] = g["value"] / c["value"]
            g["paper_gpu_vs_cpu"] = PAPER_GPU_VS_CPU
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
