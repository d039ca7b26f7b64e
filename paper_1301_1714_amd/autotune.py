"""Autotuner of the per-system launch shape of the DEM step.

Three knobs, none of which changes the contacts found:
  cell width  Sec. 4.1 requires only that a cell holds the largest contact
              distance, so any width >= 2 r_max gives the same contacts: a
              wider cell means fewer, fuller cells -- fewer empty cells to
              count and scan in a dilute system, more candidates to reject
              in a dense one;
  tile        the detection launch shape: one lane per particle reading its
              neighbours through the caches (0), one wave per run of cells
              with the candidates in the lanes and survivors compacted by
              ballot (-1), or workgroups over runs of that many cells staging
              the neighbouring rows in LDS (8, 16);
  divisor     cells of the width divided by 2 swept over 5^3 cells (one lane
              per particle only): fewer candidates, eight times the cells.
The tuner times short runs of a representative system of each class (size
octave x packing-fraction band) for every candidate pair and keeps the
fastest.  The choice for a system is then a pure function of its class and
the table, so the same system always gets the same grid and launch shape,
alone or in a batch.  (The cell width and the divisor do change the slot
order and so the rounding of the sums; the tile never changes a bit.)
"""
import json
import math
import os
import time

CANDIDATES = (1.0, 1.25, 1.5, 2.0)  # cell width / largest diameter
TILES = (0, -1, 8, 16)               # detection launch shape (tile_cells)
DIVISORS = (1, 2)                    # cell divisor (with tile 0 only)
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

    def tile(self, n: int, phi: float, default: int = 0) -> int:
        e = self.entries.get(system_class(n, phi))
        return int(e.get("tile", default)) if e else default

    def divisor(self, n: int, phi: float, default: int = 1) -> int:
        e = self.entries.get(system_class(n, phi))
        return int(e.get("divisor", default)) if e else default

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


def time_candidate(spec, factor, steps, precision="mixed", seed=1, tile=0, divisor=1):
    """Seconds per step of one system alone (graph replay, after warm-up)."""
    import torch

    from . import dem
    from . import workloads as W

    s = W.unit_box_system(seed, spec["n"], spec["kn"], spec["restitution"], spec["mu"], spec["phi"],
                          precision=precision, cell_factor=factor, tile_cells=tile, cell_divisor=divisor)
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


def tune(keys, table=None, steps=20, precision="mixed", log=None, factors=CANDIDATES, tiles=TILES,
         divisors=DIVISORS):
    """Time every candidate (cell factor, tile, divisor) for each class not
    yet in the table (divisors above 1 with tile 0 only); the fastest wins
    (on a tie within 2%, the first in the order of the candidate lists)."""
    table = table or Table()
    for key in sorted(set(keys)):
        if key in table.entries:
            continue
        spec = representative(key)
        cands = [(f, t, d) for d in divisors for f in factors for t in tiles if d == 1 or t == 0]
        times = {c: time_candidate(spec, c[0], steps, precision, tile=c[1], divisor=c[2]) for c in cands}
        best = min(times.values())
        choice = next(c for c in cands if times[c] <= 1.02 * best)
        table.entries[key] = {"factor": choice[0], "tile": choice[1], "divisor": choice[2],
                              "ms_per_step": {f"{f}/{t}/{d}": 1e3 * v for (f, t, d), v in times.items()}}
        if log:
            log(f"[autotune] {key}: cell x{choice[0]} tile {choice[1]} divisor {choice[2]} "
                f"({1e3 * times[choice]:.3f} ms/step; "
                f"worst {1e3 * max(times.values()):.3f})")
    return table


def factors_for(draws, table):
    """Cell factor of each system drawn by workloads.system_draw."""
    return [table.factor(d["n"], d["phi"]) for d in draws]


def tiles_for(draws, table):
    """Detection launch shape of each system drawn by workloads.system_draw."""
    return [table.tile(d["n"], d["phi"]) for d in draws]


def divisors_for(draws, table):
    """Cell divisor of each system drawn by workloads.system_draw."""
    return [table.divisor(d["n"], d["phi"]) for d in draws]
