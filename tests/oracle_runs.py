"""Test-side glue: run the CPU oracle on a seeded workload.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use this module.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


# (x, y, z) component triples of the vectors in each array, by model: conserved (S, [Sbar,]
# B, E), primitive (the velocity of each fluid)
CONS_VECTORS = {0: [(1, 2, 3), (5, 6, 7), (8, 9, 10)], 1: [(1, 2, 3), (6, 7, 8), (10, 11, 12), (13, 14, 15)],
                2: [(1, 2, 3), (5, 6, 7)]}
PRIM_VECTORS = {0: [(1, 2, 3)], 1: [(1, 2, 3), (6, 7, 8)], 2: [(1, 2, 3)]}


def rotate_state(arr: np.ndarray, slots) -> np.ndarray:
    """A [var][NZ][NY][NX] field turned like workloads.rotate_axes: x -> y, y -> z, z -> x,
    (a_x, a_y, a_z) -> (a_z, a_x, a_y)."""
    moved = np.ascontiguousarray(np.transpose(arr, (0, 2, 3, 1)))
    out = moved.copy()
    for (ix, iy, iz) in slots:
        out[ix], out[iy], out[iz] = moved[iz], moved[ix], moved[iy]
    return out


def grid_of(wl, **overrides) -> O.Grid:
    g = O.Grid(model=wl.model, ndim=wl.ndim, nx=wl.nx, ny=wl.ny, dx=wl.dx, dy=wl.dy, gamma=wl.gamma,
               sigma=wl.sigma, bc=wl.bc, mu1=wl.mu1, mu2=wl.mu2, kappa=wl.kappa,
               nz=wl.nz if wl.ndim == 3 else 1, dz=wl.dz)
    if wl.sigma_cell is not None:
        sc = g.embed(wl.sigma_cell[None])[0]
        O.bc_fill(g, sc[None])
        g.sigma_cell = np.ascontiguousarray(sc)
    for k, v in overrides.items():
        setattr(g, k, v)
    return g


def initial_state(wl, g: O.Grid | None = None):
    """Conserved and primitive fields (oracle layout, ghosts filled) of a workload."""
    g = g or grid_of(wl)
    prims = g.embed(wl.prims)
    EB = g.embed(wl.EB)
    cons = O.init_state(g, prims, EB)
    O.bc_fill(g, prims)
    prims, status, _ = O.cons2prim(g, cons, prims)
    assert (status == 0).all(), "initial data not recoverable"
    return g, cons, prims


def advance(g: O.Grid, cons, prims, dt: float, steps: int | None = None, t0: float = 0.0,
            t_end: float | None = None, scheme: str = "ssp2"):
    """SSP2(222) (or, scheme="ssp3", SSP3(332)) steps of size dt (the last one truncated to
    hit t_end)."""
    step = O.ssp2_step if scheme == "ssp2" else O.ssp3_step
    t, n, nit, mx = t0, 0, 0, 0
    while True:
        if steps is not None and n >= steps:
            break
        if t_end is not None and t >= t_end - 1e-12:
            break
        h = dt if t_end is None else min(dt, t_end - t)
        bad, ni, m = step(g, h, cons, prims)
        assert bad == 0, f"oracle step {n}: {bad} cells failed"
        t += h
        n += 1
        nit += ni
        mx = max(mx, m)
    return t, n, nit, mx
