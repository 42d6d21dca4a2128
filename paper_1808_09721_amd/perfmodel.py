"""Algorithmic work of the hot-path kernels, for roofline reporting.

FLOPs are counted from the kernel source with +, -, *, /, sqrt each one FLOP and a fused
multiply-add two (divisions and square roots are therefore undercounted relative to their
hardware cost, which only lowers the reported fraction).  Dual-number operations count
their value and tangent parts: add/sub 2, dual*double 2, dual*dual 4, reciprocal 4,
square root 3.

Single-fluid implicit stage, per cell (stage.hpp, physics.hpp):
  primitive-recovery Newton iteration (fluid_root loop body)          22
  residual evaluation without the recovery iterations
    (split 26 + recovery set-up/final 7 + finish 54)                  87
  Newton iteration: exact Jacobian, 3 dual columns of
    (split 62 + root tangent 19 + finish 143)                         672
    3x3 elimination with pivoting                                     31
    step update                                                       8   -> 711
  per-cell set-up, closed forms of psi and phi, final primitives      41
Two-fluid implicit stage, per cell:
  primitive-recovery Newton iteration                                 22
  residual evaluation without the recovery iterations
    (split 62 + two recovery set-ups/finals 14 + finish 148)          224
  Newton iteration: 7 dual columns of
    (split 137 + two root tangents 38 + finish 371) = 3822,
    7x7 elimination with pivoting 301, step update 15                 4138
  per-cell set-up, closed forms and final primitives                  110

Flux kernel, algorithmic HBM bytes per interior cell (each value read or written once):
  first pass  q^n (ncons) + Q1 source parts (nsrc) + w1 (nprim) in, R2 + ACC (2 ncons) out
  second pass ACC (ncons) + Q2 (ncons) + w2 (nprim) in, q^{n+1} (ncons) + its primitives
              (nprim, recovered in the same kernel) out
  F(U) alone  q (ncons) + w (nprim) in, L (ncons) out
"""
from __future__ import annotations

STAGE_FLOPS = {
    0: {"c2p_iter": 22, "residual": 87, "newton": 711, "cell": 41},
    1: {"c2p_iter": 22, "residual": 224, "newton": 4138, "cell": 110},
}

NCONS = {0: 14, 1: 18}
NPRIM = {0: 5, 1: 10}
NSRC = {0: 5, 1: 9}

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_VECTOR_TFLOPS = 78.6


def stage_flops(model: int, stage_cells: int, residual_evals: int, newton_iters: int, c2p_iters: int) -> float:
    k = STAGE_FLOPS[model]
    return (k["cell"] * stage_cells + k["residual"] * residual_evals + k["newton"] * newton_iters
            + k["c2p_iter"] * c2p_iters)


def flux_bytes_per_cell(model: int, which: str) -> int:
    nc, npr, ns = NCONS[model], NPRIM[model], NSRC[model]
    if which == "first":
        return 8 * (nc + ns + npr + 2 * nc)
    if which == "second":
        return 8 * (nc + nc + npr + nc + npr)
    return 8 * (nc + npr + nc)
