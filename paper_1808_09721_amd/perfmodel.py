"""Algorithmic work of the hot-path kernels, for roofline reporting.

FLOPs are counted from the kernel source with +, -, *, /, sqrt each one FLOP and a fused
multiply-add two (divisions and square roots are therefore undercounted relative to their
hardware cost, which only lowers the reported fraction).

A Jacobian evaluation is counted as its derivative work alone, the primal values being those
of the residual evaluation at the same iterate.  Single fluid (forward-mode dual numbers): the
tangent propagation of its 3 columns at the tangent-only cost of every elementary operation
(add/sub 1, product with a constant 1, product of two varying values 3, reciprocal 3, square
root 2), plus the inverse.  Two fluid (the chain rule written out): the tangent set-up shared
by the 7 columns, each column's tangents, and the factorisation.  The kernels recompute the
primal values the Jacobian needs instead of keeping them from the residual evaluation, so
they execute somewhat more than this; the counted figure stays below the FP64 operations the
hardware counters report for the same dispatch.

Single-fluid implicit stage, per cell (stage.hpp, physics.hpp):
  primitive-recovery Newton iteration (fluid_root loop body)          22
  residual evaluation without the recovery iterations
    (split 26 + recovery set-up/final 7 + finish 54)                  87
  Jacobian evaluation: 3 tangent columns of
    (split 62 + root tangent 19 + finish 143 as dual arithmetic, 224,
     less the primal split 26 and finish 54) = 3 x 144 = 432,
    inverse by the adjugate 42                                        474
  Newton step (applying the inverse 15, step update 6)                21
  per-cell set-up, closed forms of psi and phi, final primitives      41
Two-fluid implicit stage, per cell:
  primitive-recovery Newton iteration                                 22
  residual evaluation without the recovery iterations
    (split 62 + two recovery set-ups/finals 14 + finish 148)          224
  Jacobian evaluation by the chain rule (stage.hpp, tf_jacobian):
    shared set-up: root partials 2 x 18, d rho / d(v.dv) 2 x 2,
      species signs 2 x 2, S_s x B 2 x 9, mu_s^2 2, a/|mu1| 1        65
    columns: species tangents 2 x (17, 17, 17, 13, 22, 22, 22)
      + source tangents (89, 89, 89, 89, 91, 91, 91)                  889
    7x7 LU factorisation with pivoting                                210
                                                                      1164
  Newton step (LU solve 91, step update 15)                           106
  per-cell set-up, closed forms and final primitives                  110
A Newton step counts every step a cell takes, the polishing step after convergence
included; Jacobian evaluations are counted apart (rmhd_stats.jacobian_evals): the
polishing step and chord steps reuse the last one.

Flux kernel, algorithmic HBM bytes per interior cell (each value read or written once):
  first pass  q^n (ncons) + Q1 source parts (nsrc) + w1 (nprim) in, R2 + ACC (2 ncons) out
  second pass ACC (ncons) + Q2 (ncons) + w2 (nprim) in, q^{n+1} (ncons) + its primitives
              (nprim, recovered in the same kernel) out
  F(U) alone  q (ncons) + w (nprim) in, L (ncons) out
"""
from __future__ import annotations

STAGE_FLOPS = {
    0: {"c2p_iter": 22, "residual": 87, "jacobian": 474, "newton": 21, "cell": 41},
    1: {"c2p_iter": 22, "residual": 224, "jacobian": 1164, "newton": 106, "cell": 110},
}

NCONS = {0: 14, 1: 18}
NPRIM = {0: 5, 1: 10}
NSRC = {0: 5, 1: 9}

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_VECTOR_TFLOPS = 78.6


def stage_flops(model: int, stage_cells: int, residual_evals: int, newton_iters: int, c2p_iters: int,
                jacobian_evals: int) -> float:
    k = STAGE_FLOPS[model]
    return (k["cell"] * stage_cells + k["residual"] * residual_evals + k["jacobian"] * jacobian_evals
            + k["newton"] * newton_iters + k["c2p_iter"] * c2p_iters)


def stage_flops_of(model: int, stats: dict) -> float:
    """Algorithmic FLOPs of the stage solves counted in a statistics record."""
    return stage_flops(model, stats["stage_cells"], stats["residual_evals"], stats["newton_iters"],
                       stats["c2p_iters"], stats["jacobian_evals"])


def flux_bytes_per_cell(model: int, which: str) -> int:
    nc, npr, ns = NCONS[model], NPRIM[model], NSRC[model]
    if which == "first":
        return 8 * (nc + ns + npr + 2 * nc)
    if which == "second":
        return 8 * (nc + nc + npr + nc + npr)
    return 8 * (nc + npr + nc)
