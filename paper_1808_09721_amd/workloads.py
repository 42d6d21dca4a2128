"""Seeded synthetic initial data for the resistive / two-fluid SRMHD workloads.

This module holds no arithmetic of the numerical method: it only lays out initial
primitive fields (density, velocity, pressure, B, E) on a grid from closed-form profiles
and ``numpy.random.default_rng(seed)`` draws.  Conversion to conserved variables is done
by whoever consumes the data.

Every generator returns a :class:`Workload`: grid and physics parameters plus interior
arrays ``prims[var][ny][nx]`` and ``EB[6][ny][nx]`` (Bx, By, Bz, Ex, Ey, Ez), float64,
with ``ny = 1`` in 1-D, and ``prims[var][nz][ny][nx]``, ``EB[6][nz][ny][nx]`` in 3-D.  Primitive order: single fluid (rho, vx, vy, vz, p); two fluid
(rho1, v1x, v1y, v1z, p1, rho2, v2x, v2y, v2z, p2).

Set-ups follow the paper's Sec. 4 (Brio-Wu shock tube, self-similar current sheet,
Kelvin-Helmholtz instability) with the concrete sizes of the benchmark workloads.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SINGLE_FLUID, TWO_FLUID, IDEAL = 0, 1, 2
BC_OUTFLOW, BC_PERIODIC = 0, 1


@dataclass
class Workload:
    name: str
    model: int
    ndim: int
    nx: int
    ny: int
    x0: float
    x1: float
    y0: float
    y1: float
    gamma: float
    sigma: float
    bc: int
    cfl: float = 0.5
    mu1: float = 0.0
    mu2: float = 0.0
    kappa: float = 1.0
    steps: int = 100
    t_end: float | None = None
    prims: np.ndarray = field(default=None, repr=False)
    EB: np.ndarray = field(default=None, repr=False)
    sigma_cell: np.ndarray | None = field(default=None, repr=False)  # interior cell shape or None
    nz: int = 1
    z0: float = 0.0
    z1: float = 1.0

    @property
    def dx(self) -> float:
        return (self.x1 - self.x0) / self.nx

    @property
    def dy(self) -> float:
        return (self.y1 - self.y0) / self.ny if self.ndim >= 2 else 1.0

    @property
    def dz(self) -> float:
        return (self.z1 - self.z0) / self.nz if self.ndim == 3 else 1.0

    @property
    def ncons(self) -> int:
        return {SINGLE_FLUID: 14, TWO_FLUID: 18, IDEAL: 9}[self.model]

    @property
    def nprim(self) -> int:
        return 10 if self.model == TWO_FLUID else 5

    @property
    def cells(self) -> int:
        return self.nx * (self.ny if self.ndim >= 2 else 1) * (self.nz if self.ndim == 3 else 1)


def _centres(n: int, lo: float, hi: float) -> np.ndarray:
    return lo + (np.arange(n) + 0.5) * (hi - lo) / n


def brio_wu_1d(nx: int = 400, sigma: float = 100.0, seed: int = 1, noise: float = 1e-6) -> Workload:
    """1-D resistive Brio-Wu shock tube on [0, 1] (Sec. 4.1): left state (rho, p, By, Bx) =
    (1, 1, 1, 0.5), right (0.125, 0.1, -1, 0.5), v = E = 0, Gamma = 2, outflow boundaries,
    split at x = 1/2, seeded uniform noise of amplitude ``noise`` on rho, t_end = 0.4."""
    rng = np.random.default_rng(seed)
    x = _centres(nx, 0.0, 1.0)
    left = x < 0.5
    prims = np.zeros((5, 1, nx))
    EB = np.zeros((6, 1, nx))
    prims[0, 0] = np.where(left, 1.0, 0.125) + noise * rng.uniform(-1.0, 1.0, nx)
    prims[4, 0] = np.where(left, 1.0, 0.1)
    EB[0, 0] = 0.5
    EB[1, 0] = np.where(left, 1.0, -1.0)
    return Workload("brio_wu_1d", SINGLE_FLUID, 1, nx, 1, 0.0, 1.0, 0.0, 1.0, gamma=2.0, sigma=sigma,
                    bc=BC_OUTFLOW, steps=320, t_end=0.4, prims=prims, EB=EB)


def kelvin_helmholtz_2d(nx: int = 256, ny: int = 512, sigma: float = 1e3, seed: int = 2,
                        steps: int = 100) -> Workload:
    """2-D resistive Kelvin-Helmholtz set-up on [-1/2, 1/2] x [-1, 1], periodic (Sec. 4.4):
    shear layers at |y| = 1/2 of width a = 0.01 with v_x = 0.5 tanh((|y| - 1/2)/a),
    rho = 0.55 - 0.45 tanh((|y| - 1/2)/a) (1 between the layers, 0.1 outside), p = 1,
    B_z = 0.1, E = 0, Gamma = 4/3, and a seeded random v_y = 0.01 xi exp(-(|y| - 1/2)^2/l^2)
    with xi ~ U(-1, 1) per cell and l = 0.1."""
    rng = np.random.default_rng(seed)
    x = _centres(nx, -0.5, 0.5)
    y = _centres(ny, -1.0, 1.0)
    Y = np.broadcast_to(y[:, None], (ny, nx))
    a, l = 0.01, 0.1
    t = np.tanh((np.abs(Y) - 0.5) / a)
    prims = np.zeros((5, ny, nx))
    EB = np.zeros((6, ny, nx))
    prims[0] = 0.55 - 0.45 * t
    prims[1] = 0.5 * t
    prims[2] = 0.01 * rng.uniform(-1.0, 1.0, (ny, nx)) * np.exp(-((np.abs(Y) - 0.5) ** 2) / l ** 2)
    prims[4] = 1.0
    EB[2] = 0.1
    del x
    return Workload("kelvin_helmholtz_2d", SINGLE_FLUID, 2, nx, ny, -0.5, 0.5, -1.0, 1.0, gamma=4.0 / 3.0,
                    sigma=sigma, bc=BC_PERIODIC, steps=steps, prims=prims, EB=EB)


def kelvin_helmholtz_3d(nx: int = 128, ny: int = 256, nz: int = 128, sigma: float = 1e3, seed: int = 6,
                        steps: int = 100) -> Workload:
    """3-D version of :func:`kelvin_helmholtz_2d` on [-1/2, 1/2] x [-1, 1] x [-1/2, 1/2],
    periodic: the same shear-layer profile in y, uniform in z, with seeded perturbations
    v_y = 0.01 xi exp(-(|y| - 1/2)^2/l^2) and v_z = 0.01 zeta exp(-(|y| - 1/2)^2/l^2),
    xi, zeta ~ U(-1, 1) independently per cell."""
    rng = np.random.default_rng(seed)
    y = _centres(ny, -1.0, 1.0)
    Y = np.broadcast_to(y[None, :, None], (nz, ny, nx))
    a, l = 0.01, 0.1
    t = np.tanh((np.abs(Y) - 0.5) / a)
    env = np.exp(-((np.abs(Y) - 0.5) ** 2) / l ** 2)
    prims = np.zeros((5, nz, ny, nx))
    EB = np.zeros((6, nz, ny, nx))
    prims[0] = 0.55 - 0.45 * t
    prims[1] = 0.5 * t
    prims[2] = 0.01 * rng.uniform(-1.0, 1.0, (nz, ny, nx)) * env
    prims[3] = 0.01 * rng.uniform(-1.0, 1.0, (nz, ny, nx)) * env
    prims[4] = 1.0
    EB[2] = 0.1
    return Workload("kelvin_helmholtz_3d", SINGLE_FLUID, 3, nx, ny, -0.5, 0.5, -1.0, 1.0, gamma=4.0 / 3.0,
                    sigma=sigma, bc=BC_PERIODIC, steps=steps, prims=prims, EB=EB, nz=nz, z0=-0.5, z1=0.5)


def two_fluid_sheet_3d(nx: int = 64, ny: int = 64, nz: int = 64, sigma: float = 1e4, mu: float = 1000.0,
                       seed: int = 7, noise: float = 1e-3, delta: float = 0.05, steps: int = 100) -> Workload:
    """3-D version of :func:`two_fluid_sheet_2d` on [-1/2, 1/2)^3, periodic: the same B_y(x)
    sheets, uniform in y and z, with seeded velocity noise per component, species and cell."""
    rng = np.random.default_rng(seed)
    x = _centres(nx, -0.5, 0.5)
    X = np.broadcast_to(x[None, None, :], (nz, ny, nx))
    prims = np.zeros((10, nz, ny, nx))
    EB = np.zeros((6, nz, ny, nx))
    for s in range(2):
        prims[5 * s + 0] = 1.0
        prims[5 * s + 4] = 1.0
        for c in range(3):
            prims[5 * s + 1 + c] = noise * rng.uniform(-1.0, 1.0, (nz, ny, nx))
    EB[1] = np.tanh(X / delta) - np.tanh((X - 0.5) / delta) - np.tanh((X + 0.5) / delta)
    return Workload("two_fluid_sheet_3d", TWO_FLUID, 3, nx, ny, -0.5, 0.5, -0.5, 0.5, gamma=4.0 / 3.0,
                    sigma=sigma, bc=BC_PERIODIC, mu1=mu, mu2=-mu, steps=steps, prims=prims, EB=EB,
                    nz=nz, z0=-0.5, z1=0.5)


def as_ideal(wl: Workload) -> Workload:
    """The same single-fluid set-up for the ideal model: the same primitives and B (the ideal
    model's electric field is -v x B, so the given E is not used)."""
    assert wl.model == SINGLE_FLUID
    return Workload(wl.name + "_ideal", IDEAL, wl.ndim, wl.nx, wl.ny, wl.x0, wl.x1, wl.y0, wl.y1, gamma=wl.gamma,
                    sigma=wl.sigma, bc=wl.bc, cfl=wl.cfl, kappa=wl.kappa, steps=wl.steps, t_end=wl.t_end,
                    prims=wl.prims, EB=wl.EB, nz=wl.nz, z0=wl.z0, z1=wl.z1)


def _vector_slots(model: int) -> list[tuple[int, int, int]]:
    """Indices of the (x, y, z) components of each velocity in a primitive array."""
    return [(1, 2, 3), (6, 7, 8)] if model == TWO_FLUID else [(1, 2, 3)]


def _rotate_components(arr: np.ndarray, slots) -> np.ndarray:
    """Cyclic rotation of vector components, (a_x, a_y, a_z) -> (a_z, a_x, a_y)."""
    out = arr.copy()
    for (ix, iy, iz) in slots:
        out[ix], out[iy], out[iz] = arr[iz], arr[ix], arr[iy]
    return out


def extrude_z(wl: Workload, nz: int, z0: float = -0.5, z1: float = 0.5) -> Workload:
    """A 2-D workload copied onto every plane of a 3-D grid with nz planes (z-independent)."""
    assert wl.ndim == 2
    rep = lambda a: np.ascontiguousarray(np.repeat(a[:, None], nz, axis=1))
    return Workload(wl.name + "_z", wl.model, 3, wl.nx, wl.ny, wl.x0, wl.x1, wl.y0, wl.y1, gamma=wl.gamma,
                    sigma=wl.sigma, bc=wl.bc, cfl=wl.cfl, mu1=wl.mu1, mu2=wl.mu2, kappa=wl.kappa, steps=wl.steps,
                    t_end=wl.t_end, prims=rep(wl.prims), EB=rep(wl.EB),
                    sigma_cell=None if wl.sigma_cell is None else np.repeat(wl.sigma_cell[None], nz, axis=0),
                    nz=nz, z0=z0, z1=z1)


def rotate_axes(wl: Workload) -> Workload:
    """The same physical set-up turned by the cyclic rotation of the axes that takes x to y,
    y to z and z to x; vector components turn with the grid, (a_x, a_y, a_z) ->
    (a_z, a_x, a_y).  A 1-D or 2-D workload is first embedded in 3-D (uniform copies: 4 along
    each missing axis, spaced as x), so a 1-D set-up along x comes out along y, and rotated
    twice along z."""
    if wl.ndim < 3:
        ny = wl.ny if wl.ndim == 2 else 4
        pr = wl.prims if wl.ndim == 2 else np.repeat(wl.prims, ny, axis=1)
        eb = wl.EB if wl.ndim == 2 else np.repeat(wl.EB, ny, axis=1)
        y0, y1 = (wl.y0, wl.y1) if wl.ndim == 2 else (0.0, ny * wl.dx)
        wl = Workload(wl.name, wl.model, 3, wl.nx, ny, wl.x0, wl.x1, y0, y1, gamma=wl.gamma, sigma=wl.sigma,
                      bc=wl.bc, cfl=wl.cfl, mu1=wl.mu1, mu2=wl.mu2, kappa=wl.kappa, steps=wl.steps,
                      t_end=wl.t_end, prims=np.repeat(pr[:, None], 4, axis=1),
                      EB=np.repeat(eb[:, None], 4, axis=1), nz=4, z0=0.0, z1=4 * wl.dx)
    # arrays are [var][z][y][x]; new x = old z, new y = old x, new z = old y
    move = lambda a: np.ascontiguousarray(np.transpose(a, (0, 2, 3, 1)))
    prims = _rotate_components(move(wl.prims), _vector_slots(wl.model))
    EB = _rotate_components(move(wl.EB), [(0, 1, 2), (3, 4, 5)])
    sc = None if wl.sigma_cell is None else np.ascontiguousarray(np.transpose(wl.sigma_cell, (1, 2, 0)))
    return Workload(wl.name + "_rot", wl.model, 3, wl.nz, wl.nx, wl.z0, wl.z1, wl.x0, wl.x1, gamma=wl.gamma,
                    sigma=wl.sigma, bc=wl.bc, cfl=wl.cfl, mu1=wl.mu1, mu2=wl.mu2, kappa=wl.kappa,
                    steps=wl.steps, t_end=wl.t_end, prims=prims, EB=EB, sigma_cell=sc, nz=wl.ny, z0=wl.y0,
                    z1=wl.y1)


def two_fluid_sheet_2d(nx: int = 512, ny: int = 512, sigma: float = 1e4, mu: float = 1000.0, seed: int = 3,
                       noise: float = 1e-3, delta: float = 0.05, steps: int = 100,
                       sigma_range: tuple[float, float] | None = None) -> Workload:
    """2-D two-fluid current sheet on [-1/2, 1/2)^2, periodic: two species with charge-to-
    mass ratios +mu and -mu, rho_s = p_s = 1, Gamma = 4/3, B_y = tanh(x/d) - tanh((x - 1/2)/d)
    - tanh((x + 1/2)/d) (the sheet at x = 0 plus its periodic return sheet at x = +-1/2),
    E = 0, and seeded uniform velocity noise of amplitude ``noise`` per component, species
    and cell.  With ``sigma_range`` the conductivity is drawn per cell, log-uniform."""
    rng = np.random.default_rng(seed)
    x = _centres(nx, -0.5, 0.5)
    X = np.broadcast_to(x[None, :], (ny, nx))
    prims = np.zeros((10, ny, nx))
    EB = np.zeros((6, ny, nx))
    for s in range(2):
        prims[5 * s + 0] = 1.0
        prims[5 * s + 4] = 1.0
        for c in range(3):
            prims[5 * s + 1 + c] = noise * rng.uniform(-1.0, 1.0, (ny, nx))
    EB[1] = np.tanh(X / delta) - np.tanh((X - 0.5) / delta) - np.tanh((X + 0.5) / delta)
    sigma_cell = None
    if sigma_range is not None:
        lo, hi = np.log10(sigma_range[0]), np.log10(sigma_range[1])
        sigma_cell = 10.0 ** rng.uniform(lo, hi, (ny, nx))
    return Workload("two_fluid_sheet_2d", TWO_FLUID, 2, nx, ny, -0.5, 0.5, -0.5, 0.5, gamma=4.0 / 3.0,
                    sigma=sigma, bc=BC_PERIODIC, mu1=mu, mu2=-mu, steps=steps, prims=prims, EB=EB,
                    sigma_cell=sigma_cell)


def entropy_wave_1d(nx: int, sigma: float = 1e6, model: int = SINGLE_FLUID, mu: float = 1000.0,
                    amplitude: float = 0.5, vx: float = 0.5, t_end: float = 2.0) -> Workload:
    """Smooth advected density wave on the periodic unit interval: rho = 1 + A sin(2 pi x),
    v = (vx, 0, 0), p = 1, B = (0, 0, 0.1) and E = -v x B = (0, vx B_z, 0), so the fluid is
    force free and current free and the exact solution is rho(x - vx t).  Two fluid: both
    species carry the same density profile and velocity (rho_s = rho/2, p_s = 1/2)."""
    x = _centres(nx, 0.0, 1.0)
    Bz = 0.1
    EB = np.zeros((6, 1, nx))
    EB[2] = Bz
    EB[4] = vx * Bz
    rho = 1.0 + amplitude * np.sin(2.0 * np.pi * x)
    if model == SINGLE_FLUID:
        prims = np.zeros((5, 1, nx))
        prims[0, 0] = rho
        prims[1, 0] = vx
        prims[4, 0] = 1.0
        return Workload("entropy_wave_1d", SINGLE_FLUID, 1, nx, 1, 0.0, 1.0, 0.0, 1.0, gamma=4.0 / 3.0,
                        sigma=sigma, bc=BC_PERIODIC, t_end=t_end, steps=0, prims=prims, EB=EB)
    prims = np.zeros((10, 1, nx))
    for s in range(2):
        prims[5 * s + 0, 0] = 0.5 * rho
        prims[5 * s + 1, 0] = vx
        prims[5 * s + 4, 0] = 0.5
    return Workload("entropy_wave_1d_tf", TWO_FLUID, 1, nx, 1, 0.0, 1.0, 0.0, 1.0, gamma=4.0 / 3.0,
                    sigma=sigma, bc=BC_PERIODIC, mu1=mu, mu2=-mu, t_end=t_end, steps=0, prims=prims, EB=EB)


def current_sheet_1d(nx: int = 50, sigma: float = 100.0, model: int = SINGLE_FLUID, mu: float = 1000.0,
                     t0: float = 1.0, half_width: float = 1.5) -> Workload:
    """Self-similar current sheet (Sec. 4.2): rho = 1, p = 50, v = 0, E = 0 and
    B_y = erf(x sqrt(sigma / t0) / 2) at the start time t0 = 1, on [-1.5, 1.5] with outflow
    boundaries (the domain is not printed).  Two fluid: a pair plasma with rho_s = 1/2,
    p_s = 25 and charge-to-mass ratios +-mu."""
    from math import erf
    x = _centres(nx, -half_width, half_width)
    EB = np.zeros((6, 1, nx))
    EB[1, 0] = [erf(0.5 * xi * np.sqrt(sigma / t0)) for xi in x]
    if model == SINGLE_FLUID:
        prims = np.zeros((5, 1, nx))
        prims[0, 0] = 1.0
        prims[4, 0] = 50.0
        return Workload("current_sheet_1d", SINGLE_FLUID, 1, nx, 1, -half_width, half_width, 0.0, 1.0,
                        gamma=4.0 / 3.0, sigma=sigma, bc=BC_OUTFLOW, prims=prims, EB=EB, steps=0)
    prims = np.zeros((10, 1, nx))
    for s in range(2):
        prims[5 * s + 0, 0] = 0.5
        prims[5 * s + 4, 0] = 25.0
    return Workload("current_sheet_1d_tf", TWO_FLUID, 1, nx, 1, -half_width, half_width, 0.0, 1.0,
                    gamma=4.0 / 3.0, sigma=sigma, bc=BC_OUTFLOW, mu1=mu, mu2=-mu, prims=prims, EB=EB, steps=0)


def random_states(n: int, model: int, seed: int, w_max: float = 10.0, field_max: float = 10.0,
                  log_rho: tuple[float, float] = (-2.0, 2.0), log_p_over_rho: tuple[float, float] = (-3.0, 3.0),
                  drift: float | None = None):
    """Random physical cell states for per-cell tests: Lorentz factor uniform in [1, w_max]
    with isotropic direction, rho log-uniform over ``log_rho`` (decades), p/rho log-uniform
    over ``log_p_over_rho``, E and B components uniform in [-field_max, field_max].  Two
    fluid: each species drawn independently, or, with ``drift``, species 2 copies species 1's
    density and pressure up to a relative perturbation in [-drift, drift] and its velocity up
    to an absolute drift in [-drift, drift] per component (a quasi-neutral plasma carrying a
    current).  Returns (prims[n][nprim], EB[n][6])."""
    rng = np.random.default_rng(seed)
    nsp = 1 if model == SINGLE_FLUID else 2
    prims = np.zeros((n, 5 * nsp))
    for s in range(nsp):
        W = rng.uniform(1.0, w_max, n)
        vmag = np.sqrt(1.0 - 1.0 / W ** 2)
        d = rng.normal(size=(n, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        rho = 10.0 ** rng.uniform(log_rho[0], log_rho[1], n)
        prims[:, 5 * s + 0] = rho
        prims[:, 5 * s + 1:5 * s + 4] = vmag[:, None] * d
        prims[:, 5 * s + 4] = rho * 10.0 ** rng.uniform(log_p_over_rho[0], log_p_over_rho[1], n)
    if nsp == 2 and drift is not None:
        prims[:, 5] = prims[:, 0] * (1.0 + drift * rng.uniform(-1.0, 1.0, n))
        prims[:, 9] = prims[:, 4] * (1.0 + drift * rng.uniform(-1.0, 1.0, n))
        v2 = prims[:, 1:4] + drift * rng.uniform(-1.0, 1.0, (n, 3))
        speed = np.linalg.norm(v2, axis=1, keepdims=True)
        prims[:, 6:9] = np.where(speed < 0.999, v2, v2 * 0.999 / speed)
    EB = rng.uniform(-field_max, field_max, (n, 6))
    return prims, EB


def batched_domains(seed: int = 4, n1: int = 32, n2: int = 32, n1_range=(128, 4096), side_range=(64, 512),
                    log_sigma=(1.0, 6.0)) -> list[Workload]:
    """Many independent single-fluid domains of uneven size and stiffness: ``n1`` 1-D Brio-Wu
    shock tubes with N ~ U[128, 4096] and ``n2`` 2-D Kelvin-Helmholtz set-ups with
    nx, ny ~ U[64, 512] independently, each with sigma ~ 10^U[1, 6].  Drawn in a fixed order
    from ``seed``: all 1-D sizes, all 2-D sizes, all sigmas, then one initial-data seed per
    domain."""
    rng = np.random.default_rng(seed)
    n1s = rng.integers(n1_range[0], n1_range[1] + 1, n1)
    sides = rng.integers(side_range[0], side_range[1] + 1, (n2, 2))
    sigmas = 10.0 ** rng.uniform(log_sigma[0], log_sigma[1], n1 + n2)
    seeds = rng.integers(0, 2 ** 31 - 1, n1 + n2)
    out = []
    for k in range(n1):
        out.append(brio_wu_1d(int(n1s[k]), sigma=float(sigmas[k]), seed=int(seeds[k])))
    for k in range(n2):
        wl = kelvin_helmholtz_2d(int(sides[k, 0]), int(sides[k, 1]), sigma=float(sigmas[n1 + k]),
                                 seed=int(seeds[n1 + k]))
        out.append(wl)
    return out


# ----------------------------------------------------------------------------------------
# learned Newton guess: seeded inputs
# ----------------------------------------------------------------------------------------
MLP_SHAPES = [(64, 19), (64,), (64, 64), (64,), (7, 64), (7,)]   # W1, b1, W2, b2, W3, b3


def mlp_initial_params(seed: int) -> np.ndarray:
    """Initial FP32 master weights of the 19-64-64-7 guess network, flattened in the order
    W1, b1, W2, b2, W3, b3 (row-major): weights uniform in +-1/sqrt(fan_in), biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in MLP_SHAPES:
        if len(shape) == 2:
            lim = 1.0 / np.sqrt(shape[1])
            parts.append(rng.uniform(-lim, lim, shape).astype(np.float32).ravel())
        else:
            parts.append(np.zeros(shape, dtype=np.float32))
    return np.concatenate(parts)


def learned_guess_sheet(n: int = 1024, seed: int = 5, steps: int = 10) -> Workload:
    """Two-fluid current sheet with a per-cell conductivity sigma ~ 10^U[2, 6] (eta from 1e-6
    to 1e-2), the workload of the learned starting guess.  Training data come from the same
    set-up at other seeds (the evaluation seed 5 is held out)."""
    return two_fluid_sheet_2d(n, n, seed=seed, steps=steps, sigma_range=(1e2, 1e6))


def charged_field(ndim: int, n: int = 32, bc: int = BC_PERIODIC, seed: int = 8, sigma: float = 10.0,
                  ny: int | None = None, nz: int | None = None) -> Workload:
    """Single-fluid plasma at rest (rho = 1, p = 1, seeded velocity noise 1e-3 per component)
    on the unit square / cube with an electric field of nonzero divergence, for the initial
    charge density of Gauss's law: E_x = sin(2 pi x) cos(2 pi y), E_y = 1/2 cos(2 pi x)
    sin(4 pi y), E_z = 1/4 sin(2 pi z) (only the components along simulated directions vary
    along them), B = (0.3, 0, 0.2).  Its divergence is
    2 pi cos(2 pi x)[cos(2 pi y) + cos(4 pi y)] + pi/2 cos(2 pi z) in 3-D (drop the terms of
    directions not simulated)."""
    rng = np.random.default_rng(seed)
    nx = n
    ny = (ny or n) if ndim >= 2 else 1
    nz = (nz or n) if ndim == 3 else 1
    x = _centres(nx, 0.0, 1.0)
    y = _centres(ny, 0.0, 1.0) if ndim >= 2 else np.zeros(1)
    z = _centres(nz, 0.0, 1.0) if ndim == 3 else np.zeros(1)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    EB = np.zeros((6, nz, ny, nx))
    EB[0] = 0.3
    EB[2] = 0.2
    EB[3] = np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    EB[4] = 0.5 * np.cos(2 * np.pi * X) * np.sin(4 * np.pi * Y)
    EB[5] = 0.25 * np.sin(2 * np.pi * Z)
    prims = np.zeros((5, nz, ny, nx))
    prims[0] = 1.0
    prims[4] = 1.0
    prims[1:4] = 1e-3 * rng.uniform(-1.0, 1.0, (3, nz, ny, nx))
    if ndim < 3:
        prims, EB = prims[:, 0], EB[:, 0]
    return Workload(f"charged_field_{ndim}d", SINGLE_FLUID, ndim, nx, ny, 0.0, 1.0, 0.0, 1.0, gamma=4.0 / 3.0,
                    sigma=sigma, bc=bc, steps=0, prims=prims, EB=EB, nz=nz if ndim == 3 else 1, z0=0.0, z1=1.0)
