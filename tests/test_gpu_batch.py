"""Batched form on the GPU: every domain advanced by the batched step must match the
single-grid step of the same domain (same per-cell method), under every launch shape, and
the oracle; graph replays are checked one by one against eager steps."""
import numpy as np
import pytest

from paper_1808_09721_amd import workloads as WL
from tests.oracle_runs import advance, initial_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available()
    from paper_1808_09721_amd import rmhd
    rmhd.lib()
    return rmhd


def banner(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def small_batch():
    doms = [WL.brio_wu_1d(130, sigma=1e5, seed=11), WL.brio_wu_1d(257, sigma=30.0, seed=12),
            WL.brio_wu_1d(300, sigma=1e3, seed=13),
            WL.kelvin_helmholtz_2d(64, 70, sigma=1e6, seed=14), WL.kelvin_helmholtz_2d(97, 64, sigma=15.0, seed=15),
            WL.kelvin_helmholtz_2d(65, 66, sigma=1e3, seed=16)]
    return doms


def rel(a, b):
    a, b = a.reshape(a.shape[0], -1), b.reshape(b.shape[0], -1)
    s = np.maximum(np.abs(b).max(axis=1), 1e-8 * np.abs(b).max())
    s = np.where(s > 0, s, 1.0)
    return float((np.abs(a - b).max(axis=1) / s).max())


def plain_run(R, wl, steps):
    s = R.Solver(R.params_from(wl))
    s.set_newton_cap(1000)    # the uninterrupted solve, no queue
    c, p = s.initial_state(wl.prims, wl.EB)
    for _ in range(steps):
        s.step(s.dt(), c, p)
    out = s.grid.download_all(c), s.grid.download_all(p)
    s.close()
    return out


@pytest.fixture(scope="module")
def plain_results(R):
    return [plain_run(R, wl, 12) for wl in small_batch()]


@pytest.mark.parametrize("shape", [dict(persistent=0, newton_cap=50, flux_rows=16, use_graph=0),
                                   dict(persistent=1, newton_cap=2, flux_rows=8, use_graph=0),
                                   dict(persistent=0, newton_cap=1, flux_rows=16, use_graph=1),
                                   dict(persistent=1, newton_cap=3, flux_rows=16, use_graph=1, chunks_per_item=3)])
def test_batch_matches_single_grid(R, plain_results, shape):
    banner(f"batch vs single grid {shape}")
    doms = small_batch()
    B = R.Batch(doms)
    B.tune(**shape)
    for _ in range(12):
        B.step()
    st = B.stats()
    assert st["failures"] == 0
    assert st["stage_cells"] == 2 * 12 * sum(w.cells for w in doms)
    # Without a Newton cap every cell runs the single-grid arithmetic: bit for bit.  A cell
    # moved to the queue resumes from its saved unknowns and pressure with a fresh Jacobian,
    # which agrees with the uninterrupted solve to the Newton tolerance, not bit for bit.
    capped = shape["newton_cap"] < 50
    for d, (c_ref, p_ref) in enumerate(plain_results):
        g = B.grids[d]
        if capped:
            assert rel(g.download_all(B.cons[d]), c_ref) < 1e-9, d
            assert rel(g.download_all(B.prims[d]), p_ref) < 1e-9, d
        else:
            np.testing.assert_array_equal(g.download_all(B.cons[d]), c_ref)
            np.testing.assert_array_equal(g.download_all(B.prims[d]), p_ref)
    B.close()


def test_batch_graph_replays_match_eager(R):
    """Each replay of the captured step, with eager work and synchronisation between the
    replays, equals the eager step."""
    banner("batch graph replays")
    import torch
    doms = small_batch()
    Bg, Be = R.Batch(doms), R.Batch(doms)
    Bg.tune(use_graph=1)
    Be.tune(use_graph=0)
    for k in range(4):
        Bg.step()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()   # unrelated eager work between replays
        Be.step()
        torch.cuda.synchronize()
        for d in range(len(doms)):
            g = Bg.grids[d]
            np.testing.assert_array_equal(g.download_all(Bg.cons[d]), g.download_all(Be.cons[d]))
    Bg.close()
    Be.close()


def test_batch_autotune_leaves_state_untouched(R):
    banner("batch autotune")
    doms = small_batch()
    B = R.Batch(doms)
    before = [B.grids[d].download_all(B.cons[d]) for d in range(len(doms))]
    t = B.autotune()
    assert t["step_ms"] > 0 and t["flux_rows"] in (8, 16)
    for d in range(len(doms)):
        np.testing.assert_array_equal(B.grids[d].download_all(B.cons[d]), before[d])
    B.step()
    assert B.stats()["failures"] == 0
    B.close()


def test_batch_matches_oracle_100_steps(R, oracle_lib):
    banner("batch vs oracle 100 steps")
    O = oracle_lib
    doms = [WL.brio_wu_1d(128, sigma=1e5, seed=21), WL.kelvin_helmholtz_2d(64, 64, sigma=50.0, seed=22)]
    B = R.Batch(doms)
    B.tune(newton_cap=2, persistent=1)
    for _ in range(100):
        B.step()
    assert B.stats()["failures"] == 0
    for d, wl in enumerate(doms):
        g, oc, op = initial_state(wl)
        advance(g, oc, op, O.dt(g, wl.cfl), steps=100)
        gc = B.grids[d].download_all(B.cons[d])
        assert rel(g.interior(gc), g.interior(oc)) < 1e-9, wl.name
    B.close()


def test_full_batched_workload_runs(R):
    """The 64-domain batched workload (2.7 M cells): autotune, 5 graph steps, no failures,
    and the batched stage counts every interior cell twice per step."""
    banner("64-domain batch")
    doms = WL.batched_domains(seed=4)
    B = R.Batch(doms)
    B.autotune()
    B.stats(reset=True)
    for _ in range(5):
        B.step()
    st = B.stats()
    assert st["failures"] == 0
    assert st["stage_cells"] == 2 * 5 * sum(w.cells for w in doms)
    for d in range(len(doms)):
        assert np.all(np.isfinite(B.grids[d].download_interior(B.cons[d])))
    B.close()
