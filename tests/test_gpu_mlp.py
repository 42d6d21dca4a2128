"""Learned starting guess on the GPU, through the C ABI, against the FP64 reference.

Tolerances.  FP32-activation forward and the gradient: 1e-4 of the largest magnitude (FP32
accumulation of sums of at most 64 products, and of 64 per-block partial gradients).
Inference on the matrix cores: both sides round the layer inputs to bfloat16, so they differ
by FP32 accumulation order plus the rare hidden value whose FP32 and FP64 forms round to
neighbouring bfloat16 numbers; one such flip moves a standardised output by at most
2^-8 max|W3| ~ 1e-3, hence 5e-3 for the worst sample and 1e-4 for the median.  Whole steps
with the learned guess: 1e-9 relative L-infinity against the oracle, as for the plain guess,
since the FP64 Newton stops at the same tolerance."""
import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_1808_09721_amd import workloads as WL
from tests.oracle_runs import advance, grid_of, initial_state
from tests.test_gpu_parity import gpu_solver, rel_linf

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


def cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def random_net(seed, scale=0.05):
    rng = np.random.default_rng(seed)
    theta = WL.mlp_initial_params(seed).astype(np.float64) + scale * rng.normal(size=M.N_PARAMS)
    theta = theta.astype(np.float32)
    norm = np.concatenate([rng.normal(size=19), rng.uniform(0.5, 2.0, 19), rng.normal(size=7) * 0.1,
                           rng.uniform(0.1, 1.0, 7)]).astype(np.float32)
    return theta, norm


def split_norm(norm):
    n = norm.astype(np.float64)
    return n[:19], n[19:38], n[38:45], n[45:52]


def oracle_predict(theta, norm, X, act_bf16):
    fm, fs, tm, ts = split_norm(norm)
    return M.predict(theta.astype(np.float64), fm, fs, tm, ts, X.astype(np.float64), act_bf16)


@pytest.mark.parametrize("n", [1, 100, 1000])
def test_fp32_forward_matches_reference(R, n):
    banner(f"mlp fp32 forward n={n}")
    theta, norm = random_net(1)
    X = np.random.default_rng(2).normal(size=(n, 19)).astype(np.float32) * 2.0
    net = R.Mlp(theta)
    net.set_norm(norm)
    Y = net.forward(cuda(X), precision=0).cpu().numpy()
    ref = oracle_predict(theta, norm, X, act_bf16=False)
    assert np.abs(Y - ref).max() <= 1e-4 * np.abs(ref).max()
    net.close()


@pytest.mark.parametrize("n", [5, 16, 1003, 70000])
def test_matrix_core_inference_matches_reference(R, n):
    banner(f"mlp bf16 inference n={n}")
    theta, norm = random_net(3)
    X = np.random.default_rng(4).normal(size=(n, 19)).astype(np.float32)
    net = R.Mlp(theta)
    net.set_norm(norm)
    Y = net.forward(cuda(X), precision=1).cpu().numpy()
    ref = oracle_predict(theta, norm, X, act_bf16=True)
    ts = split_norm(norm)[3]
    err = np.abs(Y - ref).max(axis=1) / ts.max()     # in standardised output units
    assert err.max() <= 5e-3, err.max()
    assert np.median(err) <= 1e-4, np.median(err)
    # and it is the bfloat16 arithmetic that is modelled: the FP64 forward differs more
    ref64 = oracle_predict(theta, norm, X, act_bf16=False)
    assert np.abs(Y - ref64).max() > np.abs(Y - ref).max()
    net.close()


@pytest.mark.parametrize("n", [64, 1000])
def test_gradient_matches_reference(R, n):
    banner(f"mlp gradient n={n}")
    theta, norm = random_net(5)
    rng = np.random.default_rng(6)
    X = rng.normal(size=(n, 19)).astype(np.float32)
    T = rng.normal(size=(n, 7)).astype(np.float32)
    net = R.Mlp(theta)
    net.set_norm(norm)
    loss, g = net.loss_grad(cuda(X), cuda(T))
    fm, fs, tm, ts = split_norm(norm)
    U = (X.astype(np.float64) - fm) / fs
    Ts = (T.astype(np.float64) - tm) / ts
    ref_loss, ref_g = M.loss_and_grad(theta.astype(np.float64), U, Ts)
    g = g.cpu().numpy()
    assert abs(loss - ref_loss) <= 1e-4 * ref_loss
    assert np.abs(g - ref_g).max() <= 1e-4 * np.abs(ref_g).max()
    net.close()


def test_adam_steps_match_reference(R):
    banner("mlp adam")
    theta, norm = random_net(7)
    rng = np.random.default_rng(8)
    n = 777
    X = rng.normal(size=(n, 19)).astype(np.float32)
    T = rng.normal(size=(n, 7)).astype(np.float32)
    net = R.Mlp(theta)
    net.set_norm(norm)
    fm, fs, tm, ts = split_norm(norm)
    U = (X.astype(np.float64) - fm) / fs
    Ts = (T.astype(np.float64) - tm) / ts
    lr = 1e-3
    th = theta.astype(np.float64)
    m = np.zeros(M.N_PARAMS)
    v = np.zeros(M.N_PARAMS)
    for t in range(1, 4):
        cur = net.params().astype(np.float64)
        _, grad = M.loss_and_grad(cur, U, Ts)
        net.train_step(cuda(X), cuda(T), lr=lr)
        th_ref, m, v = M.adam_step(cur, m, v, grad, t, lr)
        new = net.params().astype(np.float64)
        # weights whose gradient the FP32 sums resolve to 0.3 % move as the reference says,
        # to 1 % of a step; no weight moves by much more than lr
        ok = np.abs(grad) > 3e-2 * np.abs(grad).max()
        assert np.abs(new - th_ref)[ok].max() <= 1e-2 * lr
        assert np.abs(new - cur).max() <= 3.0 * lr
    assert net.steps() == 3
    net.close()


def test_fit_norm_matches_reference(R):
    banner("mlp fit_norm")
    rng = np.random.default_rng(9)
    n = 5001
    X = (rng.normal(size=(n, 19)) * 10.0 ** rng.uniform(-3, 3, 19) + rng.normal(size=19)).astype(np.float32)
    X[:, 4] = 0.25
    T = (rng.normal(size=(n, 7)) * 1e-4).astype(np.float32)
    net = R.Mlp(WL.mlp_initial_params(0))
    net.fit_norm(cuda(X), cuda(T))
    got = net.norm().astype(np.float64)
    fm, fs = M.norm_stats(X)
    tm, ts = M.norm_stats(T)
    ref = np.concatenate([fm, fs, tm, ts])
    np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-12)
    assert got[19 + 4] == 1.0
    net.close()


def test_training_fits_a_smooth_map(R):
    banner("mlp training")
    rng = np.random.default_rng(10)
    n = 20000
    X = rng.uniform(-1, 1, size=(n, 19)).astype(np.float32)
    T = np.stack([np.sin(2 * X[:, k]) * X[:, (k + 3) % 19] for k in range(7)], axis=1).astype(np.float32)
    net = R.Mlp(WL.mlp_initial_params(10))
    Xg, Tg = cuda(X), cuda(T)
    net.fit_norm(Xg, Tg)
    hist = net.train(Xg, Tg, batch=1024, epochs=15, lr0=3e-3, lr1=3e-4, seed=1)
    assert hist[-1] < 0.1 * hist[0], hist
    net.close()


# ------------------------------------------------------------------------------------------
# harvest and the learned guess inside the two-fluid stage
# ------------------------------------------------------------------------------------------
def sheet(nx, ny, seed, steps=3):
    return WL.two_fluid_sheet_2d(nx, ny, steps=steps, seed=seed, sigma_range=(1e2, 1e6))


def test_harvest_matches_reference_stage(R, O):
    banner("harvest vs oracle stage")
    import torch
    wl = sheet(24, 20, seed=31)
    s = gpu_solver(R, wl)
    cons, prims = s.initial_state(wl.prims, wl.EB)
    n = wl.nx * wl.ny
    X = torch.zeros((n + 5, 19), dtype=torch.float32, device="cuda")
    T = torch.zeros((n + 5, 7), dtype=torch.float32, device="cuda")
    s.set_harvest(X, T)
    a = 0.3 * s.dt()
    Q = s.grid.alloc(18)
    pr = prims.clone()
    R.rmhd_implicit_stage(s.ctx, a, cons, None, Q, pr)
    assert s.harvest_count() == n
    R.rmhd_implicit_stage(s.ctx, a, cons, None, Q, pr)     # no room for a second stage
    assert s.harvest_count() == n
    g, ocons, oprims = initial_state(wl)
    Xh, Th = X.cpu().numpy()[:n], T.cpu().numpy()[:n]
    assert not X[n:].any()
    k = 0
    for j in range(2, wl.ny + 2):
        for i in range(2, wl.nx + 2):
            Rc = ocons[:, j, i]
            sig = g.sigma_cell[j, i]
            Qo, _, st, _ = O.implicit_cell(g, a, Rc, w_guess=oprims[:, j, i], sigma=sig)
            assert st == 0
            f = M.features(Rc, a, sig, wl.mu1)
            # Dbar / D is formed by cancellation between the species: its FP64 round-off is
            # 1e-16 |mu1| in absolute terms
            np.testing.assert_allclose(Xh[k], f, rtol=2e-7, atol=1e-11)
            t = M.targets(Rc, Qo, wl.mu1)
            # both Newton solutions meet |G| <= 1e-12 max(1, |R_x|): they agree to ~1e-11 of that
            scale = max(1.0, np.abs(M.unknowns(Rc, wl.mu1)).max()) / Rc[0]
            assert np.abs(Th[k] - t).max() <= 2e-7 * np.abs(t).max() + 1e-10 * scale
            k += 1
    s.close()


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_learned_guess_planes_match_reference(R, O, case):
    """rmhd_learned_guess on an evolved two-fluid state: y = (x0 - R_x) / D at every cell of
    the padded grid, ghosts included, against the reference network on the FP64 features of
    the same R (bfloat16 layer inputs), at the inference test's tolerance; the other planes
    and the row padding are left untouched."""
    banner(f"learned guess planes {case}")
    import torch
    theta, norm = random_net(7)
    net = R.Mlp(theta)
    net.set_norm(norm)
    wl = sheet(70, 37, seed=5, steps=1) if case == "2d" else WL.two_fluid_sheet_3d(16, 12, 10, steps=1)
    s = gpu_solver(R, wl)
    cons, prims = s.initial_state(wl.prims, wl.EB)
    s.step(s.dt(), cons, prims)
    a = 0.3 * s.dt()
    guess = torch.full_like(cons, float("nan"))
    R.rmhd_learned_guess(s.ctx, net, a, cons, guess)
    torch.cuda.synchronize()
    g = grid_of(wl)
    Rc = s.grid.download_all(cons).reshape(18, -1).T
    Gc = s.grid.download_all(guess).reshape(18, -1).T
    sig = g.sigma_cell.reshape(-1) if g.sigma_cell is not None else wl.sigma
    src = [6, 7, 8, 9, 13, 14, 15]
    assert np.isfinite(Gc[:, src]).all()
    assert np.isnan(np.delete(Gc, src, axis=1)).all()
    # every plane's row padding is left as it was
    assert torch.isnan(guess[..., s.grid.layout.nxg:]).all()
    Rg = Rc.copy()
    Rg[:, src] = Gc[:, src]
    y = (M.unknowns(Rg, wl.mu1) - M.unknowns(Rc, wl.mu1)) / Rc[:, 0:1]
    ref = oracle_predict(theta, norm, M.features(Rc, a, sig, wl.mu1), act_bf16=True)
    ts = split_norm(norm)[3]
    err = np.abs(y - ref).max(axis=1) / ts.max()
    print("worst / median error (standardised units)", err.max(), np.median(err))
    assert err.max() <= 5e-3 and np.median(err) <= 1e-4
    s.close()
    net.close()


@pytest.fixture(scope="module")
def trained(R):
    X, T = R.harvest_stages([sheet(64, 64, seed=sd, steps=4) for sd in (41, 42)], 4, (1.0, 0.5, 0.25))
    net = R.Mlp(WL.mlp_initial_params(43))
    net.fit_norm(X, T)
    hist = net.train(X, T, batch=2048, epochs=40, lr0=3e-3, lr1=2e-4, seed=44)
    assert hist[-1] < 0.5 * hist[0], hist
    yield net
    net.close()


def run_sheet(R, wl, net):
    s = gpu_solver(R, wl)
    s.set_stats_detail(True)
    cons, prims = s.initial_state(wl.prims, wl.EB)
    s.set_guess_model(net)
    for _ in range(wl.steps):
        s.step(s.dt(), cons, prims)
    st = s.stats()
    out = s.grid.download_all(cons)
    s.close()
    return out, st


def test_learned_guess_steps_match_oracle(R, O, trained):
    banner("learned guess steps vs oracle")
    wl = sheet(40, 28, seed=5, steps=4)
    gc, st = run_sheet(R, wl, trained)
    assert st["failures"] == 0
    g, oc, op = initial_state(wl)
    advance(g, oc, op, O.dt(g, wl.cfl), steps=wl.steps)
    assert rel_linf(gc, oc).max() < 1e-9


def test_bad_network_falls_back_to_plain_guess(R, O):
    banner("learned guess fallback")
    theta = (WL.mlp_initial_params(50) * 50.0).astype(np.float32)
    net = R.Mlp(theta)
    net.set_norm(np.concatenate([np.zeros(19), np.ones(19), np.zeros(7), np.full(7, 1e3)]))
    wl = sheet(24, 20, seed=51, steps=2)
    gc, st = run_sheet(R, wl, net)
    assert st["failures"] == 0
    g, oc, op = initial_state(wl)
    advance(g, oc, op, O.dt(g, wl.cfl), steps=wl.steps)
    assert rel_linf(gc, oc).max() < 1e-9
    net.close()


def test_default_stage_queue_is_off(R):
    """Without an explicit Newton cap, a two-fluid stage runs as one uncapped pass from the
    plain and from the learned guess: each default run equals the run with a cap above the
    iteration limit set explicitly, bit for bit."""
    banner("default stage queue")
    theta, norm = random_net(9, scale=0.01)
    net = R.Mlp(theta)
    net.set_norm(norm)
    wl = sheet(40, 28, seed=6, steps=3)

    def run(cap, model):
        s = gpu_solver(R, wl)
        if cap is not None:
            s.set_newton_cap(cap)
        cons, prims = s.initial_state(wl.prims, wl.EB)
        if model is not None:
            s.set_guess_model(model)
        for _ in range(wl.steps):
            s.step(s.dt(), cons, prims)
        out = (s.grid.download_all(cons), s.grid.download_all(prims), s.stats())
        s.close()
        return out

    for model, cap in ((None, 1000), (net, 1000)):
        a, b = run(None, model), run(cap, model)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])
        assert a[2]["newton_iters"] == b[2]["newton_iters"] and a[2]["failures"] == 0
    net.close()


def test_learned_guess_gain(R, trained):
    """Newton iterations per cell and stage with and without the network, at the same final
    residual tolerance, on a held-out seed."""
    banner("learned guess gain")
    wl = sheet(128, 128, seed=5, steps=3)
    plain, sp = run_sheet(R, wl, None)
    learned, sl = run_sheet(R, wl, trained)
    ip = sp["newton_iters"] / sp["stage_cells"]
    il = sl["newton_iters"] / sl["stage_cells"]
    print(f"newton iterations per cell and stage: plain {ip:.3f}, learned {il:.3f}; Jacobians "
          f"{sp['jacobian_evals'] / sp['stage_cells']:.3f} / {sl['jacobian_evals'] / sl['stage_cells']:.3f}", flush=True)
    assert sp["failures"] == 0 and sl["failures"] == 0
    # equal final residual: both end every cell below the same stopping tolerance
    assert 0.0 < sp["residual_max"] <= 1e-12 and 0.0 < sl["residual_max"] <= 1e-12
    assert rel_linf(learned, plain).max() < 1e-9
    # a network trained on two 64^2 sheets gains a little on this 128^2 one; the trained
    # network of the benchmark, on its held-out 1024^2 sheet, must gain at least 10 %
    # (test_gpu_fullsize)
    assert il < ip


def test_learned_guess_and_harvest_on_a_3d_grid(R, O, trained):
    """3-D two-fluid grid: the learned guess (trained on 2-D sheets) leaves whole steps equal
    to the oracle's to 1e-9, and harvesting writes one row per interior cell and stage."""
    banner("learned guess on a 3-D grid")
    import torch
    wl = WL.two_fluid_sheet_3d(16, 12, 10, steps=3)
    s = gpu_solver(R, wl)
    cons, prims = s.initial_state(wl.prims, wl.EB)
    n = wl.cells
    X = torch.zeros((2 * n + 3, 19), dtype=torch.float32, device="cuda")
    T = torch.zeros((2 * n + 3, 7), dtype=torch.float32, device="cuda")
    s.set_harvest(X, T)
    s.step(s.dt(), cons, prims)
    assert s.harvest_count() == 2 * n
    s.set_harvest(None, None)
    s.set_guess_model(trained)
    for _ in range(wl.steps - 1):
        s.step(s.dt(), cons, prims)
    st = s.stats()
    gc = s.grid.download_all(cons)
    s.close()
    assert st["failures"] == 0
    g, oc, op = initial_state(wl)
    advance(g, oc, op, O.dt(g, wl.cfl), steps=wl.steps)
    assert rel_linf(gc, oc).max() < 1e-9
    # the harvested features of the first stage: f_k = R_k / D of the initial state
    x = X[:n].cpu().numpy()
    qi = g.interior(initial_state(wl)[1]).reshape(18, -1)
    np.testing.assert_allclose(x[:, 1], (qi[1] / qi[0]).astype(np.float32), rtol=1e-5, atol=1e-7)


def test_learned_start_matches_caller_guess_planes(R, trained):
    """The learned start a context with the network set takes (inference kernel, then the
    stage from its planes) against the same planes handed to rmhd_implicit_stage as the
    caller's guess (which starts at the better of that guess and R_x): on an evolved state
    both converge every cell to the same solution within the Newton tolerance, and the Newton
    step counts agree wherever the caller-guess path kept the learned start (nearly
    everywhere)."""
    banner("learned start vs caller guess planes")
    import torch
    wl = sheet(70, 37, seed=5, steps=2)
    s = gpu_solver(R, wl)
    cons, prims = s.initial_state(wl.prims, wl.EB)
    for _ in range(wl.steps):
        s.step(s.dt(), cons, prims)
    a = 0.29 * s.dt()
    out = {}
    for mode in ("fused", "planes"):
        Q = torch.full_like(cons, float("nan"))
        w = prims.clone()
        st = torch.zeros(s.grid.cell_shape, dtype=torch.int8, device="cuda")
        it = torch.zeros(s.grid.cell_shape, dtype=torch.int32, device="cuda")
        if mode == "fused":
            s.set_guess_model(trained)
            R.rmhd_implicit_stage(s.ctx, a, cons, None, Q, w, st, it)
            s.set_guess_model(None)
        else:
            guess = torch.full_like(cons, float("nan"))
            R.rmhd_learned_guess(s.ctx, trained, a, cons, guess)
            R.rmhd_implicit_stage(s.ctx, a, cons, guess, Q, w, st, it)
        torch.cuda.synchronize()
        out[mode] = (s.grid.download_all(Q), s.grid.download_all(st[None])[0], s.grid.download_all(it[None])[0])
    s.close()
    (qf, sf, itf), (qp, sp, itp) = out["fused"], out["planes"]
    assert (sf == 0).all() and (sp == 0).all()
    scale = np.maximum(np.abs(qp).max(axis=(1, 2)), 1e-300)[:, None, None]
    assert np.all(np.abs(qf - qp) <= 1e-10 * scale + 1e-300)
    same = float((itf == itp).mean())
    print(f"cells with equal Newton counts: {same:.4f}", flush=True)
    assert same >= 0.9
