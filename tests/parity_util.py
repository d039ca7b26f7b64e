"""Shared check of GPU forces against the oracle's (imported by the parity tests)."""
import numpy as np


def assert_forces_close(Fg, Tg, F, T, Fa, Ta, tol, floor_abs=0.0, torque_floor_abs=0.0):
    """floor_abs: an absolute force floor for states whose overlaps are so
    small that one ulp of a radius in the oracle's plain S - d is not small
    against them (spheres at rest); torque_floor_abs likewise."""
    dF = np.linalg.norm(Fg - F, axis=1)
    dT = np.linalg.norm(Tg - T, axis=1)
    free = Fa == 0
    assert np.all(Fg[free] == 0.0) and np.all(Tg[Ta == 0] == 0.0)
    floor = 1e-2 * tol  # only matters in FP64 (see the module docstring)
    if np.any(~free):
        bound = tol * Fa[~free] + floor * Fa.max() + floor_abs
        worst = np.max(dF[~free] / bound)
        assert worst <= 1.0, f"force error {worst:.3f} x the bound (tol {tol:.1e})"
    has_t = Ta > 0
    if np.any(has_t):
        bound = tol * Ta[has_t] + floor * Ta.max() + torque_floor_abs
        wt = np.max(dT[has_t] / bound)
        assert wt <= 1.0, f"torque error {wt:.3f} x the bound (tol {tol:.1e})"
