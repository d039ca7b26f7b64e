"""ctypes wrapper of the FP64 CPU oracle (``dem_oracle.c``) -- TEST INFRASTRUCTURE ONLY.

Parameters come in as the plain workload dictionary (the keys the seeded
input generators produce); this module marshals them into the oracle's own
structure.  All arrays are in input (id) order.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None

LAWS = {"linear": 0, "hertz": 1, "simple": 2}
TERMS = {"cohesion": 1, "rolling": 2}  # optional contact terms (params["terms"]: a tuple of names)
STATUS = {0: "ok", -1: "invalid argument", -4: "particle out of domain", -5: "non-finite value",
          -8: "out of host memory", -9: "output capacity too small"}


class OracleError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"oracle {where}: {STATUS.get(code, code)} ({code})")
        self.code = code


class OrcPlate(C.Structure):
    _fields_ = [("axis", C.c_int32), ("pad_", C.c_int32), ("at", C.c_double),
                ("lo", C.c_double * 2), ("hi", C.c_double * 2)]


MAX_PLATES = 4


class OrcParams(C.Structure):
    _fields_ = [
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("wall_mask", C.c_int32), ("law", C.c_int32),
        ("g", C.c_double * 3),
        ("dt", C.c_double), ("rho", C.c_double),
        ("kn", C.c_double), ("kt", C.c_double),
        ("e", C.c_double), ("eta_t_ratio", C.c_double), ("mu", C.c_double),
        ("k_sp", C.c_double), ("k_da", C.c_double), ("k_sh", C.c_double),
        ("cell", C.c_double),
        ("terms", C.c_int32), ("pad_", C.c_int32),
        ("cohesion", C.c_double), ("rolling_mu", C.c_double),
        ("nplates", C.c_int32), ("pad2_", C.c_int32),
        ("plates", OrcPlate * MAX_PLATES),
    ]


def lib():
    global _LIB
    if _LIB is None:
        path = os.environ.get("DEM_ORACLE_LIB", _build.LIB)  # a planted-mistake build, for pin checks
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        P, I64, D, I32 = C.c_void_p, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_int32)
        L.orc_create.argtypes = [C.POINTER(OrcParams), I64, P, P, P, P, P, P, I64, P, P, C.POINTER(P)]
        L.orc_create.restype = C.c_int
        L.orc_step.argtypes = [P, I64]
        L.orc_step.restype = C.c_int
        L.orc_forces.argtypes = [P, P, P]
        L.orc_forces.restype = C.c_int
        L.orc_forces_scale.argtypes = [P, P, P, P, P]
        L.orc_forces_scale.restype = C.c_int
        L.orc_read_state.argtypes = [P, P, P, P, P, P]
        L.orc_read_state.restype = C.c_int
        L.orc_read_contacts.argtypes = [P, I64, C.POINTER(I64), P, P]
        L.orc_read_contacts.restype = C.c_int
        L.orc_contacts.argtypes = [P, I64, C.POINTER(I64), P]
        L.orc_contacts.restype = C.c_int
        L.orc_read_grid.argtypes = [P, P, P, P]
        L.orc_read_grid.restype = C.c_int
        L.orc_grid_dims.argtypes = [P, I32]
        L.orc_grid_dims.restype = C.c_int
        L.orc_diagnostics.argtypes = [P, D]
        L.orc_diagnostics.restype = C.c_int
        L.orc_num_cells.argtypes = [P]
        L.orc_num_cells.restype = C.c_int64
        L.orc_set_materials.argtypes = [P, C.c_int32, P, P, C.c_int32]
        L.orc_set_materials.restype = C.c_int
        L.orc_max_speed.argtypes = [P, D]
        L.orc_max_speed.restype = C.c_int
        L.orc_destroy.argtypes = [P]
        L.orc_destroy.restype = None
        _LIB = L
    return _LIB


def make_params(p: dict) -> OrcParams:
    o = OrcParams()
    o.lo[:] = [float(t) for t in p["box_lo"]]
    o.hi[:] = [float(t) for t in p["box_hi"]]
    o.wall_mask = int(p.get("wall_mask", 0x3F))
    o.law = LAWS[p.get("law", "linear")]
    o.g[:] = [float(t) for t in p.get("gravity", (0.0, 0.0, -9.81))]
    o.dt = float(p["dt"])
    o.rho = float(p.get("density", 2500.0))
    o.kn = float(p["kn"])
    o.kt = float(p.get("kt", 0.0))
    o.e = float(p.get("restitution", 1.0))
    o.eta_t_ratio = float(p.get("eta_t_ratio", 0.0))
    o.mu = float(p.get("mu", 0.0))
    sk = p.get("simple_k", (0.0, 0.0, 0.0))
    o.k_sp, o.k_da, o.k_sh = float(sk[0]), float(sk[1]), float(sk[2])
    o.cell = float(p["cell_size"])
    o.terms = (TERMS["cohesion"] if "cohesion" in p.get("terms", ()) else 0) | \
        (TERMS["rolling"] if "rolling" in p.get("terms", ()) else 0)
    o.cohesion = float(p.get("cohesion", 0.0))
    o.rolling_mu = float(p.get("rolling_mu", 0.0))
    plates = p.get("plates", ())
    if len(plates) > MAX_PLATES:
        raise ValueError("at most 4 plates")
    o.nplates = len(plates)
    for k, q in enumerate(plates):
        o.plates[k].axis = int(q["axis"])
        o.plates[k].at = float(q["at"])
        o.plates[k].lo[:] = [float(t) for t in q["lo"]]
        o.plates[k].hi[:] = [float(t) for t in q["hi"]]
    return o


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _d3(a, n):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(n, 3))
    return a


class OracleSystem:
    """One DEM system held by the oracle (arrays in id order)."""

    def __init__(self, params: dict, x, v, omega, r, F0=None, T0=None, hist_pairs=None, hist_dt=None):
        L = lib()
        r = np.ascontiguousarray(np.asarray(r, dtype=np.float64).reshape(-1))
        n = r.shape[0]
        self.n = n
        self.params = dict(params)
        self._p = make_params(params)
        x, v, omega = _d3(x, n), _d3(v, n), _d3(omega, n)
        F0 = None if F0 is None else _d3(F0, n)
        T0 = None if T0 is None else _d3(T0, n)
        nh = 0
        if hist_pairs is not None and len(hist_pairs) > 0:
            hist_pairs = np.ascontiguousarray(np.asarray(hist_pairs, dtype=np.int64).reshape(-1, 2))
            hist_dt = np.ascontiguousarray(np.asarray(hist_dt, dtype=np.float64).reshape(-1, 3))
            nh = hist_pairs.shape[0]
        else:
            hist_pairs = hist_dt = None
        h = C.c_void_p()
        st = L.orc_create(C.byref(self._p), n, _ptr(x), _ptr(v), _ptr(omega), _ptr(r), _ptr(F0), _ptr(T0),
                          nh, _ptr(hist_pairs), _ptr(hist_dt), C.byref(h))
        if st != 0:
            raise OracleError(st, "create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _LIB is not None:
            _LIB.orc_destroy(h)
            self._h = None

    def _check(self, st, where):
        if st != 0:
            raise OracleError(st, where)

    def step(self, nsteps: int = 1):
        self._check(lib().orc_step(self._h, int(nsteps)), "step")

    def max_speed(self):
        out = C.c_double()
        self._check(lib().orc_max_speed(self._h, C.byref(out)), "max_speed")
        return out.value

    def run_to_rest(self, threshold, check_every, max_steps):
        """Step in chunks of check_every until dt * max |v_i| < threshold
        (Sec. 5's run until every displacement is below a set value) or
        max_steps are done; returns the steps done."""
        done = 0
        dt = self.params["dt"]
        while done < max_steps:
            k = min(check_every, max_steps - done)
            self.step(k)
            done += k
            if dt * self.max_speed() < threshold:
                break
        return done

    def forces(self):
        F = np.zeros((self.n, 3))
        T = np.zeros((self.n, 3))
        self._check(lib().orc_forces(self._h, _ptr(F), _ptr(T)), "forces")
        return F, T

    def forces_scale(self):
        """Forces, torques and their per-particle error scales (sum of the
        magnitudes of the contact forces / torques on each particle)."""
        F = np.zeros((self.n, 3))
        T = np.zeros((self.n, 3))
        Fa = np.zeros(self.n)
        Ta = np.zeros(self.n)
        self._check(lib().orc_forces_scale(self._h, _ptr(F), _ptr(T), _ptr(Fa), _ptr(Ta)), "forces_scale")
        return F, T, Fa, Ta

    def read_state(self):
        out = [np.zeros((self.n, 3)) for _ in range(5)]
        self._check(lib().orc_read_state(self._h, *[_ptr(a) for a in out]), "read_state")
        x, v, w, F, T = out
        return {"x": x, "v": v, "omega": w, "F": F, "T": T}

    def read_contacts(self):
        n = C.c_int64()
        lib().orc_read_contacts(self._h, 0, C.byref(n), None, None)
        pairs = np.zeros((max(n.value, 1), 2), dtype=np.int64)
        dt = np.zeros((max(n.value, 1), 3))
        self._check(lib().orc_read_contacts(self._h, n.value, C.byref(n), _ptr(pairs), _ptr(dt)), "read_contacts")
        return pairs[: n.value], dt[: n.value]

    def contacts(self):
        n = C.c_int64()
        st = lib().orc_contacts(self._h, 0, C.byref(n), None)
        if st not in (0, -9):
            self._check(st, "contacts")
        pairs = np.zeros((max(n.value, 1), 2), dtype=np.int64)
        self._check(lib().orc_contacts(self._h, n.value, C.byref(n), _ptr(pairs)), "contacts")
        return pairs[: n.value]

    def grid_dims(self):
        d = (C.c_int32 * 3)()
        self._check(lib().orc_grid_dims(self._h, d), "grid_dims")
        return tuple(int(t) for t in d)

    def read_grid(self):
        nc = lib().orc_num_cells(self._h)
        cell = np.zeros(self.n, dtype=np.int32)
        order = np.zeros(self.n, dtype=np.int32)
        start = np.zeros(nc + 1, dtype=np.int32)
        self._check(lib().orc_read_grid(self._h, _ptr(cell), _ptr(order), _ptr(start)), "read_grid")
        return cell, order, start

    def diagnostics(self):
        out = (C.c_double * 10)()
        self._check(lib().orc_diagnostics(self._h, out), "diagnostics")
        return np.array(out[:])

    def set_materials(self, types, table, wall_type=0):
        """Material-pair table: table[t, u] = (kn, kt, restitution, mu) of a
        particle of material t touching one of material u (symmetric),
        types[i] the material of particle i (input order), walls of material
        wall_type.  types=None goes back to the parameters' one material."""
        if types is None:
            self._check(lib().orc_set_materials(self._h, 0, None, None, 0), "set_materials")
            return
        tab = np.ascontiguousarray(np.asarray(table, dtype=np.float64))
        nt = tab.shape[0]
        if tab.shape != (nt, nt, 4):
            raise ValueError("table must be ntypes x ntypes x 4")
        ty = np.ascontiguousarray(np.asarray(types, dtype=np.int32).reshape(-1))
        if ty.shape[0] != self.n:
            raise ValueError("one material per particle")
        self._check(lib().orc_set_materials(self._h, nt, _ptr(tab), _ptr(ty), int(wall_type)), "set_materials")
