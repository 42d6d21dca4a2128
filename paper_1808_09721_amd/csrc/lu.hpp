// lu.hpp -- LU factorisation with partial pivoting and the matching solve for the small
// dense Newton systems of the implicit stage (7x7 two-fluid), held entirely in registers.
// Plain arithmetic on double arrays with compile-time sizes: host-callable as well, so that
// the routine can be checked on the host against a library solve.
#pragma once

#include <cmath>

namespace rmhd {

// LU factorisation of a small dense A held in registers, partial pivoting.  Pivot rows are
// bubbled into place with compile-time indices (conditional swaps, recorded bit k*N+r of
// *swaps*), so nothing is indexed dynamically.  The
// multipliers are kept below the diagonal so the factors can be reused for a new right-hand
// side.  lu_solve replays the swaps and eliminations in the order they were made, so a
// multiplier must stay where it was formed: the swaps of step k move columns k..N-1 only,
// never the multipliers of earlier steps in columns 0..k-1.  The diagonal keeps the
// reciprocals of the pivots, so that the solve multiplies instead of dividing.
template <int N>
__host__ __device__ __forceinline__ bool lu_factor(double (&A)[N][N], unsigned long long &swaps)
{
    swaps = 0ull;
#pragma unroll
    for (int k = 0; k < N; ++k) {
#pragma unroll
        for (int r = k + 1; r < N; ++r) {
            const bool sw = std::fabs(A[r][k]) > std::fabs(A[k][k]);
            swaps |= (unsigned long long)sw << (k * N + r);
            // a branch rather than selects: most wavefronts swap the same rows or none, and a
            // skipped swap costs nothing (two-fluid stage 319 -> 312 us on the 1024^2 sheet)
            if (sw) {
#pragma unroll
                for (int c = k; c < N; ++c) {
                    const double t = A[k][c];
                    A[k][c] = A[r][c];
                    A[r][c] = t;
                }
            }
        }
        if (!(A[k][k] != 0.0) || !std::isfinite(A[k][k])) return false;
        const double inv = 1.0 / A[k][k];
        A[k][k] = inv;
#pragma unroll
        for (int r = k + 1; r < N; ++r) {
            const double m = A[r][k] * inv;
            A[r][k] = m;
#pragma unroll
            for (int c = k + 1; c < N; ++c) A[r][c] -= m * A[k][c];
        }
    }
    return true;
}

template <int N>
__host__ __device__ __forceinline__ void lu_solve(const double (&A)[N][N], unsigned long long swaps, double (&b)[N])
{
#pragma unroll
    for (int k = 0; k < N; ++k) {
#pragma unroll
        for (int r = k + 1; r < N; ++r) {
            const bool sw = (swaps >> (k * N + r)) & 1ull;
            const double t = b[k];
            b[k] = sw ? b[r] : t;
            b[r] = sw ? t : b[r];
        }
#pragma unroll
        for (int r = k + 1; r < N; ++r) b[r] -= A[r][k] * b[k];
    }
#pragma unroll
    for (int r = N - 1; r >= 0; --r) {
        double acc = b[r];
#pragma unroll
        for (int c = r + 1; c < N; ++c) acc -= A[r][c] * b[c];
        b[r] = acc * A[r][r];
    }
}

}  // namespace rmhd
