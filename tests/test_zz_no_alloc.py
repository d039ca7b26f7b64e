"""dem_create_static (no device allocation: the workspace is the library's
per-device static array) against dem_create (the caller's workspace): the
same kernels on the same inputs, so every result must be bitwise the same.
Two systems in a row on one device, the second smaller than the first, so
the second runs on what the first left in the array."""
import numpy as np
import pytest

from paper_1301_1714_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dem():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1301_1714_amd import dem as D
    D.lib()
    return D


def cloud(seed, n, **kw):
    side = (n * 1.3) ** (1.0 / 3.0) * 0.95 * 2 * 0.01
    return W.overlapping_cloud(seed, n, box=(side, 0.8 * side, 1.2 * side), r_mean=0.01, r_spread=0.3,
                               spacing=0.95, **kw)


def run(dem, c, steps, static):
    g = dem.System(dict(c["params"], mu=0.3), c["x"], c["v"], c["omega"], c["r"], static=static)
    F0, T0 = g.forces()
    g.step(steps)
    out = dict(g.read_state())
    out["F0"], out["T0"] = F0, T0
    out["contacts"] = g.contacts()
    out["hist_pairs"], out["hist_dt"] = g.read_contacts()
    out["diag"] = g.diagnostics()
    g.close()
    return out


@pytest.mark.parametrize("seed,n,precision,law", [(11, 3000, "mixed", "linear"), (12, 1200, "fp64", "hertz")])
def test_static_matches_workspace(dem, seed, n, precision, law):
    c = cloud(seed, n, precision=precision, law=law)
    a = run(dem, c, 25, static=False)
    b = run(dem, c, 25, static=True)
    for key in a:
        assert a[key].shape == b[key].shape, key
        assert np.array_equal(a[key], b[key]), f"{key} differs between dem_create and dem_create_static"
    assert len(a["contacts"]) > n // 2  # a crowded state: the law and the history are exercised


def test_static_limits(dem):
    cap = dem.dem_static_workspace_capacity()
    assert cap == 64 << 20
    c = cloud(13, 600)
    g = dem.System(c["params"], c["x"], c["v"], c["omega"], c["r"], static=True)
    try:
        # the device's array is in use: a second static system is refused
        with pytest.raises(dem.DemError) as e:
            dem.System(c["params"], c["x"], c["v"], c["omega"], c["r"], static=True)
        assert e.value.code == dem.DEM_E_STATE
    finally:
        g.close()
    # a size whose workspace exceeds the array is refused before any device work
    big = W.overlapping_cloud(14, 200, box=(1.0, 1.0, 1.0), r_mean=0.01)
    n_big = 1 << 20
    assert dem.dem_workspace_bytes(big["params"], n_big) > cap
    r = np.full(n_big, 0.001)
    x = np.random.default_rng(0).uniform(0.1, 0.9, size=(n_big, 3))
    with pytest.raises(dem.DemError) as e:
        dem.System(big["params"], x, np.zeros_like(x), np.zeros_like(x), r, static=True)
    assert e.value.code == dem.DEM_E_WORKSPACE
    # after the refusals the array is free again
    g = dem.System(c["params"], c["x"], c["v"], c["omega"], c["r"], static=True)
    g.step(3)
    g.close()
