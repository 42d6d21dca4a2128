"""The step without allocation (rmhd_imex_step_noalloc) against the context's step
(rmhd_imex_step): same kernels, so the states after a few steps must be equal bit for bit.
Two calls in a row share the library's scratch array, the second on a smaller grid (and
the other model), so leftovers of the first cannot leak into the second.  Requests the
array cannot hold, and per-cell conductivities, are refused before any GPU work."""
import numpy as np
import pytest

from paper_1808_09721_amd import workloads as WL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1808_09721_amd import rmhd
    rmhd.lib()
    return rmhd


def run_pair(R, wl, steps, integrator=0):
    """(context step result, no-alloc step result) after `steps` steps from the same state."""
    import torch
    print(f"\n[gpu-case] no-alloc step vs context step: {wl.name} {wl.nx}x{wl.ny} "
          f"integrator {integrator}, {steps} steps", flush=True)
    p = R.params_from(wl, integrator=integrator)
    assert 0 < R.rmhd_noalloc_scratch_bytes(p) <= (64 << 20)
    s = R.Solver(p)
    cons, prims = s.initial_state(wl.prims, wl.EB)
    cons_b, prims_b = cons.clone(), prims.clone()
    dt = s.dt()
    for _ in range(steps):
        s.step(dt, cons, prims)
    for _ in range(steps):
        R.rmhd_imex_step_noalloc(p, dt, cons_b, prims_b)
    torch.cuda.synchronize()
    out = (s.grid.download_all(cons), s.grid.download_all(prims),
           s.grid.download_all(cons_b), s.grid.download_all(prims_b))
    s.close()
    return out


def test_noalloc_step_equals_context_step_twice():
    import torch  # noqa: F401
    from paper_1808_09721_amd import rmhd as R
    R.lib()
    # first call: the largest benchmark grid the array holds (256 x 512, single fluid)
    c, w, cb, wb = run_pair(R, WL.kelvin_helmholtz_2d(steps=3), 3)
    assert np.all(np.isfinite(cb)) and np.array_equal(c, cb) and np.array_equal(w, wb)
    # second call, smaller and ragged, other model: stale scratch from the first must not matter
    c, w, cb, wb = run_pair(R, WL.two_fluid_sheet_2d(40, 28, steps=3, seed=9), 3)
    assert np.all(np.isfinite(cb)) and np.array_equal(c, cb) and np.array_equal(w, wb)


def test_noalloc_step_ssp3_and_1d(R):
    c, w, cb, wb = run_pair(R, WL.brio_wu_1d(400), 5, integrator=R.SSP3_332)
    assert np.array_equal(c, cb) and np.array_equal(w, wb)
    c, w, cb, wb = run_pair(R, WL.as_ideal(WL.kelvin_helmholtz_2d(64, 36, steps=2)), 2)
    assert np.array_equal(c, cb) and np.array_equal(w, wb)


def test_noalloc_refuses_what_it_cannot_hold(R):
    import torch
    wl = WL.two_fluid_sheet_2d(512, 512, steps=1)
    p = R.params_from(wl)
    assert R.rmhd_noalloc_scratch_bytes(p) > (64 << 20)
    g = R.Grid(p)
    cons, prims = g.alloc(18), g.alloc(10)
    with pytest.raises(R.RmhdError, match="scratch"):
        R.rmhd_imex_step_noalloc(p, 1e-3, cons, prims)
    wl = WL.learned_guess_sheet(32, steps=1)
    sig = R.Grid(R.params_from(wl)).sigma_plane(wl.sigma_cell)
    p = R.params_from(wl, sigma_cell=sig)
    g = R.Grid(p)
    with pytest.raises(R.RmhdError, match="per-cell conductivity"):
        R.rmhd_imex_step_noalloc(p, 1e-3, g.alloc(18), g.alloc(10))
    torch.cuda.synchronize()
    del cons, prims
