"""Autotuner of the per-system launch shape of the DEM step.

The knob is the cell width of the detection grid (Sec. 4.1 requires only that
a cell holds the largest contact distance, so any width >= 2 r_max gives the
same contacts): a wider cell means fewer, fuller cells -- fewer empty cells
to count and scan in a dilute system, more candidate pairs to reject in a
dense one.  The tuner times short runs of a representative system of each
class (size octave x packing-fraction band) for every candidate width and
keeps the fastest.  The choice for a system is then a pure function of its
class and the table, so the same system always gets the same grid, alone or
in a batch, and its results do not depend on what it runs with.
"""
import json
import math
import os
import time

CANDIDATES = (1.0, 1.25, 1.5, 2.0)  # cell width / largest diameter
PHI_BANDS = (0.3, 0.42)              # band edges of the packing fraction
DEFAULT_PATH = os.path.join(os.path.expanduser("~"), ".cache", "paper_1301_1714_amd", "autotune.json")


def system_class(n: int, phi: float) -> str:
    """Class key: the size octave and the packing-fraction band."""
    octave = int(round(math.log2(max(int(n), 1))))
    band = sum(phi > b for b in PHI_BANDS)
    return f"n{octave}_phi{band}"


def representative(key: str):
    """Size, packing fraction and median material of a class."""
    octave, band = key[1:].split("_phi")
    octave, band = int(octave), int(band)
    edges = (0.2,) + PHI_BANDS + (0.55,)
    phi = 0.5 * (edges[band] + edges[band + 1])
    return dict(n=1 << octave, kn=1.0e5, restitution=0.725, mu=0.35, phi=phi)


class Table:
    """Class -> cell factor, with the trial times that chose it."""

    def __init__(self, entries=None):
        self.entries = dict(entries or {})

    def factor(self, n: int, phi: float, default: float = 1.0) -> float:
        e = self.entries.get(system_class(n, phi))
        return float(e["factor"]) if e else default

    def save(self, path=DEFAULT_PATH):
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)

    @classmethod
    def load(cls, path=DEFAULT_PATH):
        if not os.path.exists(path):
            return cls()
        with open(path) as f:
            return cls(json.load(f))


def time_candidate(spec, factor, steps, precision="mixed", seed=1):
    """Seconds per step of one system alone (graph replay, after warm-up)."""
    import torch

    from . import dem
    from . import workloads as W

    s = W.unit_box_system(seed, spec["n"], spec["kn"], spec["restitution"], spec["mu"], spec["phi"],
                          precision=precision, cell_factor=factor)
    st = torch.cuda.Stream()
    sysm = dem.System(s["params"], s["x"], s["v"], s["omega"], s["r"], stream=st)
    try:
        sysm.use_graph(True)
        sysm.step(3)
        sysm.sync()
        t0 = time.perf_counter()
        sysm.step(steps)
        sysm.sync()
        return (time.perf_counter() - t0) / steps
    finally:
        sysm.close()


def tune(keys, table=None, steps=20, precision="mixed", log=None):
    """Time every candidate for each class not yet in the table; the fastest
    wins (the smaller factor on a tie within 2%)."""
    table = table or Table()
    for key in sorted(set(keys)):
        if key in table.entries:
            continue
        spec = representative(key)
        times = {}
        for f in CANDIDATES:
            times[f] = time_candidate(spec, f, steps, precision)
        best = min(times.values())
        choice = min(f for f in CANDIDATES if times[f] <= 1.02 * best)
        table.entries[key] = {"factor": choice, "ms_per_step": {str(f): 1e3 * t for f, t in times.items()}}
        if log:
            log(f"[autotune] {key}: factor {choice} ({', '.join(f'{f}: {1e3 * t:.3f} ms' for f, t in times.items())})")
    return table


def factors_for(draws, table):
    """Cell factor of each system drawn by workloads.system_draw."""
    return [table.factor(d["n"], d["phi"]) for d in draws]
