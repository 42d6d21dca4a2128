"""Failure handling on the GPU, forced from the host: every kernel still runs to completion
and reports per-cell status codes (0 ok, 1 recovery not converged, 2 unphysical, 3 Newton
not converged, 4 line search failed) and failure counts; nothing faults or hangs, since every
iteration in the kernels has a fixed cap and NaN fails every comparison that admits a state."""
import numpy as np
import pytest

from paper_1808_09721_amd import workloads as WL
from tests.oracle_runs import grid_of, initial_state
from tests.test_gpu_parity import gpu_solver, rel_linf, upload_all

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1808_09721_amd import rmhd
    rmhd.lib()
    return rmhd


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def banner(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def status_plane(R, s, fill=9):
    import torch
    L = s.grid.layout
    return torch.full((1, L.nyg, L.pitch), fill, dtype=torch.int8, device="cuda")


@pytest.mark.parametrize("case", ["khi", "sheet"])
def test_recovery_flags_unphysical_and_nan_cells(R, O, case):
    """Cells whose energy cannot carry their momentum (Gamma (tau~ + D) <= |S~|), a negative
    density and a NaN density come back with status 2; every other cell recovers as the
    oracle does."""
    banner(f"recovery failures {case}")
    wl = WL.kelvin_helmholtz_2d(40, 24, steps=1) if case == "khi" else WL.two_fluid_sheet_2d(40, 24, steps=1)
    s = gpu_solver(R, wl)
    g, ocons, oprims = initial_state(wl)
    bad = ocons.copy()
    tau = 4
    bad[tau, 10, 10] = -bad[0, 10, 10] + 1e-3            # tau~ + D tiny against |S~|
    bad[1, 10, 10] = 5.0
    bad[0, 12, 20] = -1.0                                 # negative density
    bad[0, 15, 30] = float("nan")                         # NaN density
    cons = upload_all(R, s.grid, bad)
    prims = upload_all(R, s.grid, oprims)
    st = status_plane(R, s)
    R.rmhd_cons2prim(s.ctx, cons, prims, st)
    import torch
    torch.cuda.synchronize()
    stv = s.grid.all_view(st).cpu().numpy()[0]
    for (j, i) in ((10, 10), (12, 20), (15, 30)):
        assert stv[j, i] == 2, (j, i, stv[j, i])
        # the oracle flags the same cells
        w = oprims[:, j, i].copy()
        assert O.cons2prim_cell(g, bad[:, j, i], w)[1] == 2
    mask = np.ones_like(stv, dtype=bool)
    mask[10, 10] = mask[12, 20] = mask[15, 30] = False
    assert (stv[mask] == 0).all()
    gp = s.grid.download_all(prims)
    assert np.all(np.abs(gp[:, mask] - oprims[:, mask]) <= 1e-12 * np.abs(oprims).max(axis=(1, 2))[:, None])
    s.close()


def test_newton_cap_of_one_reports_unconverged_cells(R, O):
    """With max_newton_iter = 1 a stiff stage cannot converge in most cells: they end with
    status 3 (4 where the single step's line search fails), the statistics count exactly the
    interior ones, and the oracle (same cap, same start) agrees cell by cell."""
    banner("max_newton_iter = 1")
    import torch
    wl = WL.kelvin_helmholtz_2d(40, 24, steps=1, sigma=1e6)
    s = gpu_solver(R, wl, max_newton_iter=1)
    s.set_newton_cap(1 << 20)
    g, ocons, oprims = initial_state(wl)
    cons = upload_all(R, s.grid, ocons)
    prims = upload_all(R, s.grid, oprims)
    Q = s.grid.alloc(g.ncons)
    st = status_plane(R, s)
    a = 0.3 * s.dt()
    s.stats(reset=True)
    R.rmhd_implicit_stage(s.ctx, a, cons, None, Q, prims, st)
    torch.cuda.synchronize()
    stats = s.stats(reset=True)
    stv = s.grid.interior_view(st).cpu().numpy()[0]
    assert set(np.unique(stv)) <= {0, 3, 4}
    assert (stv == 3).sum() > 0.5 * stv.size
    assert stats["failures"] == int((stv != 0).sum())
    assert stats["stage_cells"] == wl.cells and stats["newton_max"] == 1
    go = grid_of(wl, max_newton_iter=1)
    agree = 0
    for jj in range(stv.shape[0]):
        for ii in range(stv.shape[1]):
            _, _, sto, _ = O.implicit_cell(go, a, ocons[:, jj + 2, ii + 2], w_guess=oprims[:, jj + 2, ii + 2])
            agree += int(sto == stv[jj, ii])
    assert agree >= 0.99 * stv.size
    s.close()


@pytest.mark.parametrize("model", [0, 1])
def test_nan_cell_in_a_stage_stays_local(R, O, model):
    """A NaN in one cell's right-hand side fails that cell (status 2, counted once) and leaves
    every other cell's solution equal to the clean run."""
    banner(f"NaN in the stage right-hand side model={model}")
    import torch
    wl = WL.kelvin_helmholtz_2d(40, 24, steps=1) if model == 0 else WL.two_fluid_sheet_2d(40, 24, steps=1)
    s = gpu_solver(R, wl)
    g, ocons, oprims = initial_state(wl)
    a = 0.3 * s.dt()
    out = []
    for poison in (False, True):
        c = ocons.copy()
        if poison:
            c[0, 9, 17] = float("nan")
        cons = upload_all(R, s.grid, c)
        prims = upload_all(R, s.grid, oprims)
        Q = s.grid.alloc(g.ncons)
        st = status_plane(R, s)
        s.stats(reset=True)
        R.rmhd_implicit_stage(s.ctx, a, cons, None, Q, prims, st)
        torch.cuda.synchronize()
        out.append((s.grid.download_all(Q), s.grid.all_view(st).cpu().numpy()[0], s.stats(reset=True)))
    (q0, st0, s0), (q1, st1, s1) = out
    assert (st0 == 0).all() and s0["failures"] == 0
    assert st1[9, 17] == 2 and s1["failures"] == 1
    mask = np.ones(st1.shape, dtype=bool)
    mask[9, 17] = False
    assert (st1[mask] == 0).all()
    np.testing.assert_array_equal(q1[:, mask], q0[:, mask])
    s.close()


def test_ideal_recovery_flags_unphysical_and_nan_cells(R, O):
    """Ideal model: a cell whose energy cannot carry its momentum, a negative density and a
    NaN density come back with status 2 (no physical primitives), as the oracle flags them;
    every other cell recovers as the oracle does."""
    banner("ideal recovery failures")
    import torch
    wl = WL.as_ideal(WL.kelvin_helmholtz_2d(40, 24, steps=1))
    s = gpu_solver(R, wl)
    g, ocons, oprims = initial_state(wl)
    bad = ocons.copy()
    bad[4, 10, 10] = -bad[0, 10, 10] + 1e-3              # tau + D tiny against |S|
    bad[1, 10, 10] = 5.0
    bad[0, 12, 20] = -1.0                                 # negative density
    bad[0, 15, 30] = float("nan")                         # NaN density
    cons = upload_all(R, s.grid, bad)
    prims = upload_all(R, s.grid, oprims)
    st = status_plane(R, s)
    R.rmhd_cons2prim(s.ctx, cons, prims, st)
    torch.cuda.synchronize()
    stv = s.grid.all_view(st).cpu().numpy()[0]
    for (j, i) in ((10, 10), (12, 20), (15, 30)):
        assert stv[j, i] == 2, (j, i, stv[j, i])
        assert O.cons2prim_cell(g, bad[:, j, i], oprims[:, j, i].copy())[1] == 2
    mask = np.ones_like(stv, dtype=bool)
    mask[10, 10] = mask[12, 20] = mask[15, 30] = False
    assert (stv[mask] == 0).all()
    gp = s.grid.download_all(prims)
    assert np.all(np.abs(gp[:, mask] - oprims[:, mask]) <= 1e-12 * np.abs(oprims).max(axis=(1, 2))[:, None])
    s.close()
