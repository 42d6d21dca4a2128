// mlp.hpp -- interface between the solver context (rmhd.hip) and the learned-guess network
// (mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/rmhd_mlp.h"
#include "kernels.hpp"

namespace rmhd {
// Enqueue the learned starting point of a two-fluid implicit stage with right-hand side R
// and coefficient a: the seven source-carrying planes of guess (Sbar, taubar, E) receive
// x0 = R_x + D y in conserved units for every cell of the padded grid.  0 on success.
int mlp_launch_guess(const rmhd_mlp *m, hipStream_t stream, const CPlanes &R, const Planes &guess, const Geo &g,
                     const Phys &P, double a);
}  // namespace rmhd
