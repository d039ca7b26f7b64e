"""Python binding of libdem.so: argument marshalling only.

Every step of the DEM path runs in the HIP kernels behind the C ABI of
``include/dem.h``; PyTorch provides the device workspace and the stream.  The
functions keep the C names (``dem_create``, ``dem_step``, ...); ``System`` is
a thin owner of one handle and its workspace.  There is no CPU fallback: if
the library is missing or no GPU is present the calls raise.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

LAWS = {"linear": 0, "hertz": 1, "simple": 2}
PRECISIONS = {"fp64": 0, "mixed": 1}
TERMS = {"cohesion": 1, "rolling": 2}  # optional contact terms: params["terms"] is a tuple of these names

DEM_OK = 0
DEM_E_INVALID = -1
DEM_E_WORKSPACE = -2
DEM_E_CONTACT_OVERFLOW = -3
DEM_E_OUT_OF_DOMAIN = -4
DEM_E_NONFINITE = -5
DEM_E_HIP = -6
DEM_E_STATE = -7
DEM_E_CAPACITY = -9

NUM_PHASES = 6
PHASES = ("kick_drift_hash", "sort", "reorder", "contacts", "law_pass", "gather")

_LIB = None


class DemError(RuntimeError):
    def __init__(self, code, where):
        msg = lib().dem_status_string(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{where}: {msg} ({code})")
        self.code = code


MAX_PLATES = 4


class DemPlate(C.Structure):
    _fields_ = [("axis", C.c_int32), ("reserved", C.c_int32), ("at", C.c_double),
                ("lo", C.c_double * 2), ("hi", C.c_double * 2)]


class DemParams(C.Structure):
    _fields_ = [
        ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
        ("wall_mask", C.c_uint32), ("law", C.c_int32),
        ("gravity", C.c_double * 3),
        ("dt", C.c_double), ("density", C.c_double),
        ("kn", C.c_double), ("kt", C.c_double),
        ("restitution", C.c_double), ("eta_t_ratio", C.c_double), ("mu", C.c_double),
        ("simple_k", C.c_double * 3),
        ("cell_size", C.c_double),
        ("contacts_per_particle", C.c_int32), ("precision", C.c_int32),
        ("tile_cells", C.c_int32), ("cell_divisor", C.c_int32),
        ("max_materials", C.c_int32), ("terms", C.c_uint32),
        ("cohesion", C.c_double), ("rolling_mu", C.c_double),
        ("nplates", C.c_int32), ("reserved", C.c_int32),
        ("plates", DemPlate * MAX_PLATES),
    ]


def lib():
    """Load libdem.so (built in-tree by ``__graft_entry__.build()``)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            raise RuntimeError(f"libdem.so not built at {_build.LIB}; run __graft_entry__.build() first")
        L = C.CDLL(_build.LIB)
        P, I64, S = C.c_void_p, C.c_int64, C.c_size_t
        st = C.c_int
        sig = {
            "dem_workspace_bytes": ([C.POINTER(DemParams), I64, C.POINTER(S)], st),
            "dem_create": ([C.POINTER(DemParams), I64, P, P, P, P, P, P, I64, P, P, P, S, P, C.POINTER(P)], st),
            "dem_create_static": ([C.POINTER(DemParams), I64, P, P, P, P, P, P, I64, P, P, P, C.POINTER(P)], st),
            "dem_static_workspace_capacity": ([], S),
            "dem_step": ([P, I64], st),
            "dem_forces": ([P, P, P], st),
            "dem_read_state": ([P, P, P, P, P, P], st),
            "dem_read_contacts": ([P, I64, C.POINTER(I64), P, P], st),
            "dem_contacts": ([P, I64, C.POINTER(I64), P], st),
            "dem_read_grid": ([P, P, P, P], st),
            "dem_grid_dims": ([P, C.POINTER(C.c_int32)], st),
            "dem_diagnostics": ([P, C.POINTER(C.c_double)], st),
            "dem_sync": ([P], st),
            "dem_set_radii": ([P, P], st),
            "dem_set_materials": ([P, C.c_int32, P, P, C.c_int32], st),
            "dem_max_speed": ([P, C.POINTER(C.c_double)], st),
            "dem_run_to_rest": ([P, C.c_double, I64, I64, C.POINTER(I64)], st),
            "dem_batch_max_speed": ([P, P], st),
            "dem_profile": ([P, C.c_int], st),
            "dem_profile_read": ([P, C.POINTER(C.c_double), C.POINTER(I64)], st),
            "dem_use_graph": ([P, C.c_int], st),
            "dem_destroy": ([P], st),
            "dem_status_string": ([st], C.c_char_p),
            "dem_batch_workspace_bytes": ([C.c_int32, P, P, C.POINTER(S)], st),
            "dem_batch_create": ([C.c_int32, P, P, P, P, P, P, P, P, P, P, P, P, S, P, C.POINTER(P)], st),
            "dem_batch_set_radii": ([P, P], st),
            "dem_batch_set_materials": ([P, C.c_int32, C.c_int32, P, P, C.c_int32], st),
            "dem_batch_step": ([P, P], st),
            "dem_batch_read_state": ([P, C.c_int32, P, P, P, P, P], st),
            "dem_batch_read_contacts": ([P, C.c_int32, I64, C.POINTER(I64), P, P], st),
            "dem_batch_diagnostics": ([P, P], st),
            "dem_batch_use_graph": ([P, C.c_int], st),
            "dem_batch_profile": ([P, C.c_int], st),
            "dem_batch_profile_read": ([P, C.POINTER(C.c_double), C.POINTER(I64)], st),
            "dem_batch_sync": ([P], st),
            "dem_batch_destroy": ([P], st),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _LIB = L
    return _LIB


def make_params(p: dict) -> DemParams:
    o = DemParams()
    o.box_lo[:] = [float(t) for t in p["box_lo"]]
    o.box_hi[:] = [float(t) for t in p["box_hi"]]
    o.wall_mask = int(p.get("wall_mask", 0x3F))
    o.law = LAWS[p.get("law", "linear")]
    o.gravity[:] = [float(t) for t in p.get("gravity", (0.0, 0.0, -9.81))]
    o.dt = float(p["dt"])
    o.density = float(p.get("density", 2500.0))
    o.kn = float(p["kn"])
    o.kt = float(p.get("kt", 0.0))
    o.restitution = float(p.get("restitution", 1.0))
    o.eta_t_ratio = float(p.get("eta_t_ratio", 0.0))
    o.mu = float(p.get("mu", 0.0))
    o.simple_k[:] = [float(t) for t in p.get("simple_k", (0.0, 0.0, 0.0))]
    o.cell_size = float(p["cell_size"])
    o.contacts_per_particle = int(p.get("contacts_per_particle", 16))
    o.precision = PRECISIONS[p.get("precision", "fp64")]
    o.tile_cells = int(p.get("tile_cells", 0))
    o.cell_divisor = int(p.get("cell_divisor", 1))
    o.max_materials = int(p.get("max_materials", 0))
    o.terms = sum(TERMS[t] for t in p.get("terms", ()))
    o.cohesion = float(p.get("cohesion", 0.0))
    o.rolling_mu = float(p.get("rolling_mu", 0.0))
    plates = p.get("plates", ())
    if len(plates) > MAX_PLATES:
        raise ValueError(f"at most {MAX_PLATES} plates")
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
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(n, 3))


def _check(code, where):
    if code != DEM_OK:
        raise DemError(code, where)


def dem_workspace_bytes(params: dict, n: int) -> int:
    b = C.c_size_t()
    _check(lib().dem_workspace_bytes(C.byref(make_params(params)), int(n), C.byref(b)), "dem_workspace_bytes")
    return b.value


def dem_static_workspace_capacity() -> int:
    """Bytes of the per-device array behind ``dem_create_static``."""
    return int(lib().dem_static_workspace_capacity())


class System:
    """One DEM system on the GPU: the handle of ``dem_create`` plus the torch
    workspace that backs it, or with static=True the handle of
    ``dem_create_static``, whose workspace is the library's per-device array
    (no device memory is allocated for it; one such system per device at a
    time)."""

    def __init__(self, params: dict, x, v, omega, r, F0=None, T0=None, hist_pairs=None, hist_dt=None,
                 device="cuda", stream=None, static=False):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("libdem needs a GPU: torch.cuda.is_available() is False")
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
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        if static:
            self.workspace = None
            with torch.cuda.device(self.device):
                _check(L.dem_create_static(C.byref(self._p), n, _ptr(x), _ptr(v), _ptr(omega), _ptr(r), _ptr(F0),
                                           _ptr(T0), nh, _ptr(hist_pairs), _ptr(hist_dt),
                                           C.c_void_p(self.stream.cuda_stream), C.byref(h)), "dem_create_static")
            self._h = h
            return
        nbytes = dem_workspace_bytes(params, n)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        _check(L.dem_create(C.byref(self._p), n, _ptr(x), _ptr(v), _ptr(omega), _ptr(r), _ptr(F0), _ptr(T0),
                            nh, _ptr(hist_pairs), _ptr(hist_dt), C.c_void_p(self.workspace.data_ptr()), nbytes,
                            C.c_void_p(self.stream.cuda_stream), C.byref(h)), "dem_create")
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and _LIB is not None:
            self._h = None
            _LIB.dem_destroy(h)

    __del__ = close

    @property
    def handle(self):
        if self._h is None:
            raise DemError(DEM_E_STATE, "system")
        return self._h

    def step(self, nsteps: int = 1):
        _check(lib().dem_step(self.handle, int(nsteps)), "dem_step")

    def sync(self):
        _check(lib().dem_sync(self.handle), "dem_sync")

    def forces(self):
        F = np.zeros((self.n, 3))
        T = np.zeros((self.n, 3))
        _check(lib().dem_forces(self.handle, _ptr(F), _ptr(T)), "dem_forces")
        return F, T

    def read_state(self):
        out = [np.zeros((self.n, 3)) for _ in range(5)]
        _check(lib().dem_read_state(self.handle, *[_ptr(a) for a in out]), "dem_read_state")
        x, v, w, F, T = out
        return {"x": x, "v": v, "omega": w, "F": F, "T": T}

    def read_contacts(self):
        n = C.c_int64()
        st = lib().dem_read_contacts(self.handle, 0, C.byref(n), None, None)
        if st not in (DEM_OK, DEM_E_CAPACITY):
            _check(st, "dem_read_contacts")
        pairs = np.zeros((max(n.value, 1), 2), dtype=np.int64)
        dt = np.zeros((max(n.value, 1), 3))
        _check(lib().dem_read_contacts(self.handle, n.value, C.byref(n), _ptr(pairs), _ptr(dt)), "dem_read_contacts")
        return pairs[: n.value], dt[: n.value]

    def contacts(self):
        n = C.c_int64()
        st = lib().dem_contacts(self.handle, 0, C.byref(n), None)
        if st not in (DEM_OK, DEM_E_CAPACITY):
            _check(st, "dem_contacts")
        pairs = np.zeros((max(n.value, 1), 2), dtype=np.int64)
        _check(lib().dem_contacts(self.handle, n.value, C.byref(n), _ptr(pairs)), "dem_contacts")
        return pairs[: n.value]

    def grid_dims(self):
        d = (C.c_int32 * 3)()
        _check(lib().dem_grid_dims(self.handle, d), "dem_grid_dims")
        return tuple(int(t) for t in d)

    def read_grid(self):
        dims = self.grid_dims()
        nc = dims[0] * dims[1] * dims[2]
        cell = np.zeros(self.n, dtype=np.int32)
        order = np.zeros(self.n, dtype=np.int32)
        start = np.zeros(nc + 1, dtype=np.int32)
        _check(lib().dem_read_grid(self.handle, _ptr(cell), _ptr(order), _ptr(start)), "dem_read_grid")
        return cell, order, start

    def diagnostics(self):
        out = (C.c_double * 10)()
        _check(lib().dem_diagnostics(self.handle, out), "dem_diagnostics")
        return np.array(out[:])

    def set_radii(self, r):
        r = np.ascontiguousarray(np.asarray(r, dtype=np.float64).reshape(-1))
        if r.shape[0] != self.n:
            raise ValueError("set_radii: one radius per particle")
        _check(lib().dem_set_radii(self.handle, _ptr(r)), "dem_set_radii")

    def max_speed(self):
        out = C.c_double()
        _check(lib().dem_max_speed(self.handle, C.byref(out)), "dem_max_speed")
        return out.value

    def run_to_rest(self, threshold, check_every, max_steps):
        """Step in chunks of check_every until dt * max |v_i| < threshold or
        max_steps are done; returns the steps done."""
        done = C.c_int64()
        _check(lib().dem_run_to_rest(self.handle, float(threshold), int(check_every), int(max_steps),
                                     C.byref(done)), "dem_run_to_rest")
        return done.value

    def set_materials(self, types, table, wall_type=0):
        """Material-pair table: table[t, u] = (kn, kt, restitution, mu) of a
        particle of material t touching one of material u (symmetric),
        types[i] the material of particle i (original order), walls of
        material wall_type; types=None goes back to the parameters' one
        material."""
        nt, tab, ty = _material_args(types, table, self.n)
        _check(lib().dem_set_materials(self.handle, nt, _ptr(tab), _ptr(ty), int(wall_type)), "dem_set_materials")

    def use_graph(self, enable: bool = True):
        """Replay each time step from a HIP graph (needs a non-default stream)."""
        _check(lib().dem_use_graph(self.handle, int(bool(enable))), "dem_use_graph")

    def profile(self, enable: bool = True):
        _check(lib().dem_profile(self.handle, int(bool(enable))), "dem_profile")

    def profile_read(self):
        """(milliseconds per phase summed over the timed steps, number of
        timed steps); phases as ``PHASES``."""
        ms = (C.c_double * NUM_PHASES)()
        n = C.c_int64()
        _check(lib().dem_profile_read(self.handle, ms, C.byref(n)), "dem_profile_read")
        return np.array(ms[:]), n.value


def _material_args(types, table, n):
    if types is None:
        return 0, None, None
    tab = np.ascontiguousarray(np.asarray(table, dtype=np.float64))
    nt = tab.shape[0]
    if tab.shape != (nt, nt, 4):
        raise ValueError("table must be ntypes x ntypes x 4")
    ty = np.ascontiguousarray(np.asarray(types, dtype=np.int32).reshape(-1))
    if ty.shape[0] != n:
        raise ValueError("one material per particle")
    return nt, tab, ty


def _params_array(params_list):
    arr = (DemParams * len(params_list))()
    for k, p in enumerate(params_list):
        arr[k] = make_params(p)
    return arr


def dem_batch_workspace_bytes(params_list, ns) -> int:
    b = C.c_size_t()
    n = np.ascontiguousarray(np.asarray(ns, dtype=np.int64).reshape(-1))
    if n.shape[0] != len(params_list):
        raise ValueError("one particle count per system")
    _check(lib().dem_batch_workspace_bytes(len(params_list), _params_array(params_list), _ptr(n), C.byref(b)),
           "dem_batch_workspace_bytes")
    return b.value


class Batch:
    """Several independent systems stepped by one launch sequence: the handle
    of ``dem_batch_create`` plus its torch workspace and its own stream.

    ``systems`` is a list of dicts with keys params, x, v, omega, r (one
    system each; ids are local to the system) and, to restart a system
    exactly, F, T (its last forces) and hist_pairs, hist_dt (its committed
    tangential history, as ``read_contacts`` returns it).  All systems share
    the contact law and the precision."""

    def __init__(self, systems, device="cuda", stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("libdem needs a GPU: torch.cuda.is_available() is False")
        L = lib()
        if len(systems) == 0:
            raise ValueError("a batch holds at least one system")
        rs = [np.ascontiguousarray(np.asarray(s["r"], dtype=np.float64).reshape(-1)) for s in systems]
        self.ns = [int(r.shape[0]) for r in rs]
        self.S = len(systems)
        self.params = [dict(s["params"]) for s in systems]
        cat3 = lambda key: np.ascontiguousarray(np.concatenate(
            [_d3(s[key], n) for s, n in zip(systems, self.ns)]) if sum(self.ns) else np.zeros((0, 3)))
        x, v, w = cat3("x"), cat3("v"), cat3("omega")
        r = np.ascontiguousarray(np.concatenate(rs))
        n = np.asarray(self.ns, dtype=np.int64)
        F0 = T0 = None
        if any("F" in s for s in systems):
            if not all("F" in s and "T" in s for s in systems):
                raise ValueError("restart forces F, T are given for every system or for none")
            F0, T0 = cat3("F"), cat3("T")
        n_hist = hp = hd = None
        if any(s.get("hist_pairs") is not None for s in systems):
            pairs = [np.asarray(s.get("hist_pairs", np.zeros((0, 2))), dtype=np.int64).reshape(-1, 2) for s in systems]
            dts = [np.asarray(s.get("hist_dt", np.zeros((0, 3))), dtype=np.float64).reshape(-1, 3) for s in systems]
            n_hist = np.ascontiguousarray([len(q) for q in pairs], dtype=np.int64)
            hp = np.ascontiguousarray(np.concatenate(pairs) if n_hist.sum() else np.zeros((1, 2), np.int64))
            hd = np.ascontiguousarray(np.concatenate(dts) if n_hist.sum() else np.zeros((1, 3)))
        self.device = torch.device(device)
        nbytes = dem_batch_workspace_bytes(self.params, n)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if stream is None:
            stream = torch.cuda.Stream(self.device)
            stream.wait_stream(torch.cuda.current_stream(self.device))
        self.stream = stream
        h = C.c_void_p()
        _check(L.dem_batch_create(self.S, _params_array(self.params), _ptr(n), _ptr(x), _ptr(v), _ptr(w), _ptr(r),
                                  _ptr(F0), _ptr(T0), _ptr(n_hist), _ptr(hp), _ptr(hd),
                                  C.c_void_p(self.workspace.data_ptr()), nbytes, C.c_void_p(stream.cuda_stream),
                                  C.byref(h)), "dem_batch_create")
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and _LIB is not None:
            self._h = None
            _LIB.dem_batch_destroy(h)

    __del__ = close

    @property
    def handle(self):
        if self._h is None:
            raise DemError(DEM_E_STATE, "batch")
        return self._h

    def step(self, steps):
        """Advance system k by steps[k] (an int applies to every system)."""
        if np.isscalar(steps):
            steps = [int(steps)] * self.S
        s = np.ascontiguousarray(np.asarray(steps, dtype=np.int64).reshape(-1))
        if s.shape[0] != self.S:
            raise ValueError("one step count per system")
        _check(lib().dem_batch_step(self.handle, _ptr(s)), "dem_batch_step")

    def sync(self):
        _check(lib().dem_batch_sync(self.handle), "dem_batch_sync")

    def set_radii(self, radii):
        """New radii for every system (a list of per-system arrays)."""
        r = np.ascontiguousarray(np.concatenate([np.asarray(q, dtype=np.float64).reshape(-1) for q in radii]))
        if [len(np.asarray(q).reshape(-1)) for q in radii] != self.ns:
            raise ValueError("set_radii: one radius per particle of every system")
        _check(lib().dem_batch_set_radii(self.handle, _ptr(r)), "dem_batch_set_radii")

    def max_speed(self):
        out = np.zeros(self.S)
        _check(lib().dem_batch_max_speed(self.handle, _ptr(out)), "dem_batch_max_speed")
        return out

    def set_materials(self, k: int, types, table, wall_type=0):
        """``System.set_materials`` for system k (types in its own order)."""
        nt, tab, ty = _material_args(types, table, self.ns[k])
        _check(lib().dem_batch_set_materials(self.handle, int(k), nt, _ptr(tab), _ptr(ty), int(wall_type)),
               "dem_batch_set_materials")

    def use_graph(self, enable: bool = True):
        _check(lib().dem_batch_use_graph(self.handle, int(bool(enable))), "dem_batch_use_graph")

    def read_state(self, k: int):
        n = self.ns[k]
        out = [np.zeros((n, 3)) for _ in range(5)]
        _check(lib().dem_batch_read_state(self.handle, int(k), *[_ptr(a) for a in out]), "dem_batch_read_state")
        x, v, w, F, T = out
        return {"x": x, "v": v, "omega": w, "F": F, "T": T}

    def read_contacts(self, k: int):
        n = C.c_int64()
        st = lib().dem_batch_read_contacts(self.handle, int(k), 0, C.byref(n), None, None)
        if st not in (DEM_OK, DEM_E_CAPACITY):
            _check(st, "dem_batch_read_contacts")
        pairs = np.zeros((max(n.value, 1), 2), dtype=np.int64)
        dt = np.zeros((max(n.value, 1), 3))
        _check(lib().dem_batch_read_contacts(self.handle, int(k), n.value, C.byref(n), _ptr(pairs), _ptr(dt)),
               "dem_batch_read_contacts")
        return pairs[: n.value], dt[: n.value]

    def diagnostics(self):
        out = np.zeros((self.S, 10))
        _check(lib().dem_batch_diagnostics(self.handle, _ptr(out)), "dem_batch_diagnostics")
        return out

    def profile(self, enable: bool = True):
        _check(lib().dem_batch_profile(self.handle, int(bool(enable))), "dem_batch_profile")

    def profile_read(self):
        ms = (C.c_double * NUM_PHASES)()
        n = C.c_int64()
        _check(lib().dem_batch_profile_read(self.handle, ms, C.byref(n)), "dem_batch_profile_read")
        return np.array(ms[:]), n.value


def dem_create(params, x, v, omega, r, **kw) -> System:
    return System(params, x, v, omega, r, **kw)


def dem_step(system: System, nsteps: int = 1):
    system.step(nsteps)


def dem_forces(system: System):
    return system.forces()


def dem_read_state(system: System):
    return system.read_state()


def dem_read_contacts(system: System):
    return system.read_contacts()


def dem_contacts(system: System):
    return system.contacts()


def dem_read_grid(system: System):
    return system.read_grid()


def dem_diagnostics(system: System):
    return system.diagnostics()


def dem_destroy(system: System):
    system.close()
