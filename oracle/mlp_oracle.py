"""Plain FP64 reference of the learned Newton guess for the two-fluid implicit stage.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module; the product path never does.

The implicit stage of Sec. 2.2.1 (Eq. 10) solves, per cell, for the seven source-carrying
unknowns x = (Sbar/|mu1|, taubar/|mu1|, E) of the two-fluid model (Sec. 3, Eqs. 27-30) by
Newton iteration from a starting point.  The paper only says that a guess is made; the plain
guess is x0 = R_x, the unknowns of the stage's right-hand side R.  The learned guess replaces
it by x0 = R_x + D * y, where y is the output of a small network evaluated on per-cell
features of R:

  features (19):  f0 = log10(a mu1^2 D)   (stiffness of the plasma-frequency terms, a = gamma dt)
                  f_k = R_k / D, k = 1..17 (the other conserved variables per unit density)
                  f18 = log10(a sigma)     (stiffness of the resistive terms, sigma = 1/eta)
  target (7):     (x* - R_x) / D, x* the converged solution of the stage.

Network: standardised inputs u = (f - mean_f) / std_f, two hidden layers of 64 tanh units and a
linear output, v = W3 tanh(W2 tanh(W1 u + b1) + b2) + b3, and y = mean_t + std_t * v.  Weights
are used in bfloat16-rounded form (nearest, ties to even, of the FP32 master value).  Training
minimises the mean over samples of the squared error summed over the 7 standardised outputs,
with Adam (Kingma & Ba, 2015) on the FP32 master weights.

parity unpinned: nothing in the paper fixes these numbers; the network is an accelerator whose
result is always polished by the FP64 Newton of the stage.  The functions below are pinned
against finite differences, a library network of the same shape, and closed forms.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 19, 64, 7
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)

# two-fluid conserved-variable order: D, S(3), tau, Dbar, Sbar(3), taubar, B(3), E(3), psi, phi
_SBAR, _TAUBAR, _E = slice(6, 9), 9, slice(13, 16)


def unpack(theta: np.ndarray) -> dict:
    out, k = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[k:k + n], dtype=np.float64).reshape(shape)
        k += n
    return out


def bf16_round(x) -> np.ndarray:
    """Round to float32, then to bfloat16 (nearest, ties to even); returned as float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ----------------------------------------------------------------------------------------
# features and targets of one stage (definition above)
# ----------------------------------------------------------------------------------------
def unknowns(Q: np.ndarray, mu1: float) -> np.ndarray:
    """x = (Sbar/|mu1|, taubar/|mu1|, E) of conserved states Q[..., 18]."""
    Q = np.asarray(Q, dtype=np.float64)
    m = abs(mu1)
    return np.concatenate([Q[..., _SBAR] / m, Q[..., _TAUBAR:_TAUBAR + 1] / m, Q[..., _E]], axis=-1)


def features(R: np.ndarray, a: float, sigma, mu1: float) -> np.ndarray:
    """Features [..., 19] of stage right-hand sides R[..., 18] (FP64)."""
    R = np.asarray(R, dtype=np.float64)
    D = R[..., 0]
    f = np.empty(R.shape[:-1] + (N_IN,))
    f[..., 0] = np.log10(a * mu1 * mu1 * D)
    f[..., 1:18] = R[..., 1:18] / D[..., None]
    f[..., 18] = np.log10(a * np.asarray(sigma, dtype=np.float64))
    return f


def targets(R: np.ndarray, Q: np.ndarray, mu1: float) -> np.ndarray:
    """(x* - R_x) / D for stage right-hand sides R and solutions Q."""
    R = np.asarray(R, dtype=np.float64)
    return (unknowns(Q, mu1) - unknowns(R, mu1)) / R[..., 0:1]


def guess(R: np.ndarray, y: np.ndarray, mu1: float) -> np.ndarray:
    """Learned starting point x0 = R_x + D * y."""
    R = np.asarray(R, dtype=np.float64)
    return unknowns(R, mu1) + R[..., 0:1] * np.asarray(y, dtype=np.float64)


# ----------------------------------------------------------------------------------------
# standardisation
# ----------------------------------------------------------------------------------------
def norm_stats(X: np.ndarray):
    """Column means and standard deviations (two-pass, population); a column whose spread is
    below 1e-12 (1 + |mean|) gets std = 1."""
    X = np.asarray(X, dtype=np.float64)
    mean = X.mean(axis=0)
    std = np.sqrt(((X - mean) ** 2).mean(axis=0))
    std = np.where(std > 1e-12 * (1.0 + np.abs(mean)), std, 1.0)
    return mean, std


# ----------------------------------------------------------------------------------------
# network
# ----------------------------------------------------------------------------------------
def forward(theta: np.ndarray, U: np.ndarray, act_bf16: bool = False, quantize: bool = True):
    """Standardised outputs v for standardised inputs U[n, 19], with bf16-rounded weights
    (quantize=False uses theta as given).  act_bf16 also rounds each layer's input (U, H1, H2)
    to bfloat16: the inference arithmetic of the device, which multiplies bfloat16 operands
    and accumulates in FP32."""
    P = unpack(bf16_round(theta) if quantize else theta)
    q = bf16_round if act_bf16 else (lambda z: z)
    U = np.asarray(U, dtype=np.float64)
    H1 = np.tanh(q(U) @ P["W1"].T + P["b1"])
    H2 = np.tanh(q(H1) @ P["W2"].T + P["b2"])
    V = q(H2) @ P["W3"].T + P["b3"]
    return V, (U, H1, H2, P)


def predict(theta, fmean, fstd, tmean, tstd, F, act_bf16: bool = False) -> np.ndarray:
    """Network outputs in target units for raw features F[n, 19]."""
    V, _ = forward(theta, (np.asarray(F, dtype=np.float64) - fmean) / fstd, act_bf16)
    return tmean + tstd * V


def loss_and_grad(theta: np.ndarray, U: np.ndarray, T: np.ndarray, quantize: bool = True):
    """Loss mean_n sum_k (v - T)^2 on standardised data and its gradient with respect to the
    (bf16-rounded, unless quantize=False) weights, by the chain rule, layer by layer."""
    V, (U, H1, H2, P) = forward(theta, U, quantize=quantize)
    n = U.shape[0]
    Rr = V - np.asarray(T, dtype=np.float64)
    loss = float(np.sum(Rr * Rr) / n)
    dV = 2.0 * Rr / n
    g = {"W3": dV.T @ H2, "b3": dV.sum(axis=0)}
    dZ2 = (dV @ P["W3"]) * (1.0 - H2 * H2)
    g["W2"] = dZ2.T @ H1
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ P["W2"]) * (1.0 - H1 * H1)
    g["W1"] = dZ1.T @ U
    g["b1"] = dZ1.sum(axis=0)
    return loss, np.concatenate([g[name].ravel() for name, _ in SHAPES])


def adam_step(theta, m, v, grad, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam update of the master weights (step count t starts at 1)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
