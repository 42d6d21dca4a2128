"""Pins of the FP64 reference of the learned Newton guess (CPU only).

The network reference is checked against things other than itself: central finite
differences, a library network and its automatic differentiation, a library optimizer, a
library bfloat16 conversion, closed forms of Adam, and the exact round trip of the feature,
target and guess definitions through the two-fluid implicit-stage solution of the oracle."""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as M
from paper_1808_09721_amd import workloads as WL


def _data(n, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, M.N_IN)), rng.normal(size=(n, M.N_OUT))


def _torch_net(theta):
    P = M.unpack(theta)
    net = torch.nn.Sequential(torch.nn.Linear(19, 64), torch.nn.Tanh(), torch.nn.Linear(64, 64), torch.nn.Tanh(),
                              torch.nn.Linear(64, 7)).double()
    with torch.no_grad():
        for k, lyr in zip((1, 2, 3), (net[0], net[2], net[4])):
            lyr.weight.copy_(torch.tensor(P[f"W{k}"]))
            lyr.bias.copy_(torch.tensor(P[f"b{k}"]))
    return net


def test_parameter_count_and_layout():
    assert M.N_PARAMS == 64 * 19 + 64 + 64 * 64 + 64 + 7 * 64 + 7 == 5895
    theta = WL.mlp_initial_params(3)
    assert theta.shape == (M.N_PARAMS,) and theta.dtype == np.float32
    P = M.unpack(theta.astype(np.float64))
    assert np.abs(P["W1"]).max() <= 1 / np.sqrt(19) and np.abs(P["W2"]).max() <= 1 / 8
    assert not P["b1"].any() and not P["b3"].any()


def test_bf16_rounding_matches_library_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.uniform(-6, 6, 4000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -(1.0 + 2 ** -8)]])
    x32 = x.astype(np.float32)
    ref = torch.tensor(x32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16_round(x32), ref)
    # ties go to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert M.bf16_round(np.float32(1.0 + 2 ** -8)) == 1.0
    assert M.bf16_round(np.float32(1.0 + 3 * 2 ** -8)) == 1.0 + 2 ** -6


def test_forward_matches_library_network():
    theta = WL.mlp_initial_params(5).astype(np.float64)
    theta[64 * 19:64 * 20] = np.random.default_rng(1).normal(size=64) * 0.1   # non-zero b1
    U, _ = _data(50, 2)
    V, _ = M.forward(theta, U)
    ref = _torch_net(M.bf16_round(theta))(torch.tensor(U)).detach().numpy()
    np.testing.assert_allclose(V, ref, rtol=0, atol=1e-13)


def test_bf16_activation_forward_is_close_but_not_identical():
    theta = WL.mlp_initial_params(6).astype(np.float64)
    U, _ = _data(200, 3)
    V64, _ = M.forward(theta, U)
    V16, _ = M.forward(theta, U, act_bf16=True)
    d = np.abs(V16 - V64).max()
    assert 0 < d < 2e-2 * np.abs(V64).max()
    # rounding the activations is the only difference: bf16-exact inputs to a network whose
    # second and third layers see bf16-exact hidden values agree with the FP64 forward
    V1, (_, H1, _, _) = M.forward(theta, M.bf16_round(U))
    Va, _ = M.forward(theta, M.bf16_round(U), act_bf16=True)
    assert np.abs(Va - V1).max() <= d * 1.5 + 1e-12


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(7)
    theta = WL.mlp_initial_params(7).astype(np.float64) + 0.05 * rng.normal(size=M.N_PARAMS)
    U, T = _data(16, 8)
    loss, g = M.loss_and_grad(theta, U, T, quantize=False)
    idx = rng.choice(M.N_PARAMS, 60, replace=False)
    idx = np.concatenate([idx, [0, 64 * 19, 64 * 20, M.N_PARAMS - 8, M.N_PARAMS - 1]])
    for p in idx:
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        fd = (M.loss_and_grad(tp, U, T, quantize=False)[0] - M.loss_and_grad(tm, U, T, quantize=False)[0]) / (2 * h)
        assert abs(fd - g[p]) <= 1e-6 * max(abs(g[p]), 1e-3), (p, fd, g[p])


def test_gradient_matches_library_autograd_on_rounded_weights():
    theta = WL.mlp_initial_params(9).astype(np.float64)
    U, T = _data(33, 10)
    loss, g = M.loss_and_grad(theta, U, T)
    net = _torch_net(M.bf16_round(theta))
    out = net(torch.tensor(U))
    ref_loss = ((out - torch.tensor(T)) ** 2).sum(dim=1).mean()
    ref_loss.backward()
    ref = torch.cat([p.grad.reshape(-1) for p in net.parameters()]).numpy()
    assert abs(loss - ref_loss.item()) <= 1e-13 * ref_loss.item()
    np.testing.assert_allclose(g, ref, rtol=1e-11, atol=1e-14)


def test_adam_first_step_closed_form_and_library_optimizer():
    rng = np.random.default_rng(11)
    theta = rng.normal(size=40)
    g = rng.normal(size=40)
    lr = 1e-3
    t1, m, v = M.adam_step(theta, np.zeros(40), np.zeros(40), g, 1, lr)
    # first step: m_hat = g, v_hat = g^2, so each weight moves by lr g / (|g| + eps)
    np.testing.assert_allclose(t1, theta - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # a constant gradient keeps m_hat = g and v_hat = g^2 at every step
    t2, _, _ = M.adam_step(t1, m, v, g, 2, lr)
    np.testing.assert_allclose(t2 - t1, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-16)
    # five steps with changing gradients against the library optimizer
    w = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.Adam([w], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    th, m, v = theta.copy(), np.zeros(40), np.zeros(40)
    for t in range(1, 6):
        gt = rng.normal(size=40)
        w.grad = torch.tensor(gt)
        opt.step()
        th, m, v = M.adam_step(th, m, v, gt, t, lr)
    np.testing.assert_allclose(th, w.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_norm_stats_two_pass_and_constant_columns():
    rng = np.random.default_rng(12)
    X = rng.normal(3.0, 2.0, size=(500, 4))
    X[:, 2] = 7.25
    mean, std = M.norm_stats(X)
    np.testing.assert_allclose(mean, X.mean(axis=0), rtol=1e-14)
    np.testing.assert_allclose(std[[0, 1, 3]], X[:, [0, 1, 3]].std(axis=0), rtol=1e-12)
    assert std[2] == 1.0


def test_training_lowers_the_loss_on_a_smooth_map():
    rng = np.random.default_rng(13)
    U = rng.uniform(-1, 1, size=(256, M.N_IN))
    T = np.stack([np.sin(U[:, k]) * U[:, (k + 1) % 19] for k in range(7)], axis=1)
    theta = WL.mlp_initial_params(13).astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = M.loss_and_grad(theta, U, T)[0]
    for t in range(1, 301):
        loss, g = M.loss_and_grad(theta, U, T)
        theta, m, v = M.adam_step(theta, m, v, g, t, 3e-3)
    assert M.loss_and_grad(theta, U, T)[0] < 0.2 * l0


def test_features_targets_and_guess_round_trip_through_the_stage(oracle_lib):
    from oracle import oracle as O
    from oracle_runs import grid_of
    wl = WL.two_fluid_sheet_2d(8, 8, steps=1, seed=21)
    g = grid_of(wl)
    prims, EB = WL.random_states(6, WL.TWO_FLUID, seed=22, w_max=1.5, field_max=1.0, drift=1e-3)
    a, sig, mu = 2e-4, 3e3, wl.mu1
    for k in range(len(prims)):
        R = O.prim2cons_cell(g, prims[k], EB[k])
        Q, w, st, it = O.implicit_cell(g, a, R, w_guess=prims[k], sigma=sig)
        assert st == 0
        f = M.features(R, a, sig, mu)
        assert f[0] == pytest.approx(np.log10(a * mu * mu * R[0]), rel=1e-15)
        assert f[18] == pytest.approx(np.log10(a * sig), rel=1e-15)
        np.testing.assert_allclose(f[1:18] * R[0], R[1:18], rtol=1e-15)
        y = M.targets(R, Q, mu)
        x_star = M.guess(R, y, mu)
        np.testing.assert_allclose(x_star, M.unknowns(Q, mu), rtol=1e-14, atol=1e-300)
        # starting the stage at the learned guess built from the exact target converges at once
        Qs = R.copy()
        Qs[6:10] = x_star[:4] * abs(mu)
        Qs[13:16] = x_star[4:]
        Q2, _, st2, it2 = O.implicit_cell(g, a, R, w_guess=prims[k], sigma=sig, Q_start=Qs)
        assert st2 == 0 and it2 <= 1
        np.testing.assert_allclose(Q2, Q, rtol=1e-11, atol=1e-12 * np.abs(Q).max())
