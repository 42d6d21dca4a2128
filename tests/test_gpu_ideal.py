"""The ideal RMHD model (explicit steps, two-dimensional recovery) on the GPU against the
oracle: initial data and recovery, L(q), whole explicit SSP2 / SSP3 steps in 1-D, 2-D (ragged
tiles and the full 256 x 512 grid) and 3-D, graph replays, and the recovery's fallback."""
import numpy as np
import pytest

from paper_1808_09721_amd import workloads as WL
from tests.oracle_runs import advance, initial_state
from tests.test_gpu_parity import gpu_solver, rel_linf, run_both, upload_all

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


def khi(nx=70, ny=37, steps=1):
    return WL.as_ideal(WL.kelvin_helmholtz_2d(nx, ny, steps=steps))


@pytest.mark.parametrize("case", ["brio_wu", "khi", "khi3"])
def test_ideal_init_and_cons2prim_match_oracle(R, O, case):
    banner(f"ideal init/cons2prim {case}")
    wl = {"brio_wu": WL.as_ideal(WL.brio_wu_1d()), "khi": khi(),
          "khi3": WL.as_ideal(WL.kelvin_helmholtz_3d(20, 14, 13))}[case]
    s = gpu_solver(R, wl)
    cons, prims = s.initial_state(wl.prims, wl.EB)
    g, ocons, oprims = initial_state(wl)
    assert np.all(rel_linf(s.grid.download_all(cons), ocons) < 1e-14)
    assert np.all(rel_linf(s.grid.download_all(prims), oprims) < 1e-12)
    s.close()


def test_ideal_cons2prim_random_states(R, O):
    """Random magnetised states (W <= 3, |B| <= 1, p/rho in [0.1, 10], rho in [0.1, 10]): the
    two-dimensional Newton recovers the generating primitives to 1e-11 (the oracle's own bar
    on these states) from its default start (the guesses are -1, so Newton starts at
    Z = tau + D, v^2 = 0)."""
    banner("ideal cons2prim random states")
    import torch
    n = 4000
    og = O.Grid(model=2, ndim=1, nx=n, ny=1, dx=1.0 / n, dy=1.0, gamma=4.0 / 3.0, sigma=1.0, bc=0)
    prims, EB = WL.random_states(n, 0, seed=211, w_max=3.0, field_max=1.0, log_rho=(-1, 1), log_p_over_rho=(-1, 1))
    q = np.stack([O.prim2cons_cell(og, prims[k], EB[k]) for k in range(n)], axis=1)
    wl = WL.as_ideal(WL.brio_wu_1d(n))
    wl.gamma = 4.0 / 3.0
    s = gpu_solver(R, wl)
    full_q = np.zeros((9, 1, n + 4))
    full_q[:, 0, 2:-2] = q
    full_q[:, 0, :2] = q[:, :1]
    full_q[:, 0, -2:] = q[:, -1:]
    cons = upload_all(R, s.grid, full_q)
    pr = s.grid.alloc(5, fill=-1.0)
    status = torch.zeros((1, s.grid.layout.nyg, s.grid.layout.pitch), dtype=torch.int8, device="cuda")
    R.rmhd_cons2prim(s.ctx, cons, pr, status)
    torch.cuda.synchronize()
    w = s.grid.download_interior(pr)[:, 0]
    assert int(s.grid.interior_view(status).abs().max()) == 0
    np.testing.assert_allclose(w[0], prims[:, 0], rtol=1e-11)
    np.testing.assert_allclose(w[4], prims[:, 4], rtol=1e-11)
    np.testing.assert_allclose(w[1:4], prims[:, 1:4].T, rtol=0, atol=1e-11)
    s.close()


def test_ideal_flux_divergence_matches_oracle(R, O):
    banner("ideal flux divergence")
    import torch
    wl = khi()
    g, ocons, oprims = initial_state(wl)
    advance(g, ocons, oprims, O.dt(g, 0.5), steps=3)
    oL = O.rhs(g, ocons, oprims)
    s = gpu_solver(R, wl)
    cons = upload_all(R, s.grid, ocons)
    prims = upload_all(R, s.grid, oprims)
    L = s.grid.alloc(9, fill=float("nan"))
    R.rmhd_F(s.ctx, cons, prims, L)
    torch.cuda.synchronize()
    gL = s.grid.download_interior(L)
    ref = g.interior(oL)
    fmax = np.zeros(9)
    qi, wi = g.interior(ocons).reshape(9, -1), g.interior(oprims).reshape(5, -1)
    for k in range(0, qi.shape[1], max(1, qi.shape[1] // 200)):
        for d in range(2):
            fmax = np.maximum(fmax, np.abs(O.flux_cell(g, qi[:, k], wi[:, k], d)))
    scale = np.maximum(np.abs(ref).reshape(9, -1).max(axis=1), fmax / min(g.dx, g.dy))
    scale = np.where(scale > 0, scale, 1.0)   # S_z and B_z carry no flux in this 2-D set-up
    err = np.abs(gL - ref).reshape(9, -1).max(axis=1) / scale
    print("rel err per variable", err)
    assert np.all(err < 1e-12)
    s.close()


@pytest.mark.parametrize("scheme", ["ssp2", "ssp3"])
@pytest.mark.parametrize("steps,t_end", [(100, None), (None, 0.4)])
def test_ideal_brio_wu_matches_oracle(R, O, scheme, steps, t_end):
    banner(f"ideal Brio-Wu {scheme} steps={steps} t_end={t_end}")
    wl = WL.as_ideal(WL.brio_wu_1d())
    g, oc, op, gc, gp, st = run_both(R, O, wl, steps, t_end, scheme=scheme)
    assert np.all(rel_linf(g.interior(gc), g.interior(oc)) < 1e-9)
    assert np.all(rel_linf(g.interior(gp), g.interior(op)) < 1e-9)


@pytest.mark.parametrize("case,scheme,steps", [("khi", "ssp2", 100), ("khi", "ssp3", 50), ("khi3", "ssp2", 30),
                                               ("khi3", "ssp3", 30)])
def test_ideal_steps_match_oracle(R, O, case, scheme, steps):
    """Ragged 2-D (70 x 37) and 3-D (20 x 14 x 13) tilings: 1e-9 relative per variable."""
    banner(f"ideal {case} {scheme} {steps} steps")
    wl = khi(steps=steps) if case == "khi" else WL.as_ideal(WL.kelvin_helmholtz_3d(20, 14, 13, steps=steps))
    g, oc, op, gc, gp, st = run_both(R, O, wl, steps, scheme=scheme)
    err = rel_linf(g.interior(gc), g.interior(oc))
    print("rel Linf per variable", err)
    assert np.all(err < 1e-9)
    assert np.all(rel_linf(g.interior(gp), g.interior(op)) < 1e-9)
    assert st["stage_cells"] == 0


def test_ideal_khi_full_size_100_steps(R, O):
    """The Kelvin-Helmholtz benchmark grid (256 x 512) with the ideal model, 100 SSP2 steps."""
    banner("ideal KHI 256x512 100 steps")
    wl = WL.as_ideal(WL.kelvin_helmholtz_2d())
    g, oc, op, gc, gp, st = run_both(R, O, wl, 100)
    err = rel_linf(g.interior(gc), g.interior(oc))
    print("rel Linf per variable", err)
    assert np.all(err < 1e-9)


@pytest.mark.parametrize("integrator", [0, 1])
def test_ideal_graph_replays_match_eager_steps(R, O, integrator):
    """Three graph replays (eager work and synchronisations in between) against eager steps."""
    banner(f"ideal graph replays integrator={integrator}")
    import torch
    wl = khi()
    s1 = gpu_solver(R, wl, integrator=integrator)
    s2 = gpu_solver(R, wl, integrator=integrator)
    c1, p1 = s1.initial_state(wl.prims, wl.EB)
    c2, p2 = s2.initial_state(wl.prims, wl.EB)
    s2.set_graph(True)
    dt = s1.dt()
    for _ in range(3):
        s1.step(dt, c1, p1)
        s2.step(dt, c2, p2)
        torch.cuda.synchronize()
        junk = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        del junk
        np.testing.assert_array_equal(s2.grid.download_all(c2), s1.grid.download_all(c1))
        np.testing.assert_array_equal(s2.grid.download_all(p2), s1.grid.download_all(p1))
    s1.close()
    s2.close()


def test_ideal_context_has_no_implicit_stage(R, O):
    wl = khi()
    s = gpu_solver(R, wl)
    cons, prims = s.initial_state(wl.prims, wl.EB)
    Q = s.grid.alloc(9)
    with pytest.raises(R.RmhdError, match="no implicit stage"):
        R.rmhd_implicit_stage(s.ctx, 0.1, cons, None, Q, prims)
    s.close()


def test_ideal_recovery_fallback_takes_over(R, O):
    """With the two-dimensional Newton capped at 2 iterations most cells stop unconverged
    (status 1); with the one-dimensional bracketed route as fallback every cell recovers
    the oracle's primitives (1e-12)."""
    banner("ideal recovery fallback")
    import torch
    wl = khi()
    g, ocons, oprims = initial_state(wl)
    advance(g, ocons, oprims, O.dt(g, 0.5), steps=3)
    out = {}
    for primary_only in (1, 0):
        s = gpu_solver(R, wl, max_c2p_iter=2, c2p_primary_only=primary_only)
        cons = upload_all(R, s.grid, ocons)
        pr = s.grid.alloc(5, fill=-1.0)
        status = torch.zeros((1, s.grid.layout.nyg, s.grid.layout.pitch), dtype=torch.int8, device="cuda")
        R.rmhd_cons2prim(s.ctx, cons, pr, status)
        torch.cuda.synchronize()
        out[primary_only] = (s.grid.download_interior(pr), s.grid.interior_view(status).cpu().numpy())
        s.close()
    (w1, st1), (w0, st0) = out[1], out[0]
    assert (st1 == 1).mean() > 0.5
    assert (st0 == 0).all()
    assert np.all(rel_linf(w0, g.interior(oprims)) < 1e-12)


@pytest.mark.parametrize("case", ["khi", "khi3"])
def test_ideal_32x32_tiles_match_oracle(R, O, case):
    """The 32 x 32 tile form (both stencils through LDS, the recovery in every pass), which the
    library picks for narrow grids, on the ragged 2-D (70 x 37) and 3-D (20 x 14 x 13)
    tilings: 30 SSP2 steps against the oracle to 1e-9 relative per variable."""
    banner(f"ideal {case} 32x32 tiles 30 steps")
    steps = 30
    wl = khi(steps=steps) if case == "khi" else WL.as_ideal(WL.kelvin_helmholtz_3d(20, 14, 13, steps=steps))
    g, oc, op = initial_state(wl)
    dt = O.dt(g, wl.cfl)
    advance(g, oc, op, dt, steps=steps)
    s = gpu_solver(R, wl)
    s.set_flux_rows(32)
    cons, prims = s.initial_state(wl.prims, wl.EB)
    for _ in range(steps):
        s.step(dt, cons, prims)
    gc, gp = s.grid.download_all(cons), s.grid.download_all(prims)
    s.close()
    err = rel_linf(g.interior(gc), g.interior(oc))
    print("rel Linf per variable", err)
    assert np.all(err < 1e-9)
    assert np.all(rel_linf(g.interior(gp), g.interior(op)) < 1e-9)
