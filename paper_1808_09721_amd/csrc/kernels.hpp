// kernels.hpp -- gfx950 kernels shared by the single-grid path (rmhd.hip) and the batched
// path (batch.hip): ghost fill, initial data, primitive recovery, the per-cell implicit stage
// and the FVS + WENO3 flux tile, for the resistive single-fluid and two-fluid SRMHD model of
// Wright & Hawke (arXiv:1808.09721).
//
//   k_init    prim -> cons on the interior, rho_e = div E (Sec. 2.1.1 Eq. 2; Sec. 2.1.2 Eq. 6)
//   k_bc      ghost fill (outflow copy / periodic wrap) of any set of planes
//   k_c2p     primitive recovery on every cell (Sec. 2.1.3)
//   k_stage   implicit-stage Newton solve per cell, ghosts included (Sec. 2.2.1 Eq. 10)
//   k_flux    FVS + WENO3 flux divergence L (Sec. 2.2.2 Eq. 12), fused with the SSP2 stage
//             combiners (Eqs. 10-11, Table 2), with the ghost fill of its first output and
//             the recovery of that output's primitives; on 3-D grids k_flux_z forms the z
//             term first and the x-y tiles of k_flux add it and do the rest
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/rmhd.h"
#include "physics.hpp"
#include "stage.hpp"

namespace rmhd {

// ---------------------------------------------------------------------------------------
// kernel argument blocks
// ---------------------------------------------------------------------------------------
struct Planes {
    double *p[18];
};
struct CPlanes {
    const double *p[18];
};

// Cell (i, j, k) of a variable lives at k * slab + j * pitch + i; r = k * nyg + j numbers the
// rows of all z planes together (rows = nyg * nzg), so pointwise kernels see one 2-D array.
struct Geo {
    int nx, ny, nxg, nyg;
    int pitch, ndim, bc, nz;
    long plane;
    double idx, idy;  // 1/dx, 1/dy
    int nzg, rows;
    long slab;
    double idz;       // 1/dz
};

template <int M>
struct Model;
template <>
struct Model<0> {
    static constexpr int NC = 14, NP = 5, NX = 3;
};
template <>
struct Model<1> {
    static constexpr int NC = 18, NP = 10, NX = 7;
};
template <>
struct Model<2> {   // ideal: no implicit stage
    static constexpr int NC = 9, NP = 5, NX = 0;
};

// Per-model recovery and fluxes (model 0 single fluid, 1 two fluid, 2 ideal).
template <int M>
__device__ __forceinline__ int cons2prim_m(const double *q, double *w, const Phys &P, int &it)
{
    if constexpr (M == 0) return sf_cons2prim(q, w, P, it);
    else if constexpr (M == 1) return tf_cons2prim(q, w, P, it);
    else return id_cons2prim(q, w, P, it);
}
template <int M>
__device__ __forceinline__ void flux_source_m(const double *q, const double *w, double sig, const Phys &P, double *fx,
                                              double *fy, double *src, bool need_src = true)
{
    if constexpr (M == 0) sf_flux_source(q, w, sig, P, fx, fy, src);
    else if constexpr (M == 1) tf_flux_source(q, w, sig, P, fx, fy, src, need_src);
    else id_flux_source(q, w, P, fx, fy, src);
}
template <int M>
__device__ __forceinline__ void flux_z_m(const double *q, const double *w, double sig, const Phys &P, double *fz)
{
    if constexpr (M == 0) sf_flux_z(q, w, sig, P, fz);
    else if constexpr (M == 1) tf_flux_z(q, w, P, fz);
    else id_flux_z(q, w, P, fz);
}

// components that carry a source term
__host__ __device__ constexpr bool has_source(int M, int v)
{
    return M == 0   ? (v == sf::EX || v == sf::EY || v == sf::EZ || v == sf::PSI || v == sf::PHI)
           : M == 1 ? (v == tf::SBX || v == tf::SBY || v == tf::SBZ || v == tf::TAUB || v == tf::EX ||
                       v == tf::EY || v == tf::EZ || v == tf::PSI || v == tf::PHI)
                    : v == id::PHI;
}

// Whether cell i of row r (= k * nyg + j) is an interior cell.
__device__ __forceinline__ bool is_interior(const Geo &g, int i, int r)
{
    if (!(i >= 2 && i < g.nx + 2)) return false;
    if (g.ndim == 1) return true;
    if (g.ndim == 2) return r >= 2 && r < g.ny + 2;
    const int j = r % g.nyg, k = r / g.nyg;
    return j >= 2 && j < g.ny + 2 && k >= 2 && k < g.nz + 2;
}

// Row-major rank of an interior cell among the interior cells (x fastest, then y, then z).
__device__ __forceinline__ long interior_rank(const Geo &g, int i, int r)
{
    if (g.ndim == 1) return i - 2;
    if (g.ndim == 2) return (long)(r - 2) * g.nx + (i - 2);
    const int j = r % g.nyg, k = r / g.nyg;
    return ((long)(k - 2) * g.ny + (j - 2)) * g.nx + (i - 2);
}

// padded index of the interior cell that a ghost (or interior) index copies
__device__ __forceinline__ int bc_src(int i, int n, int bc)
{
    if (i >= 2 && i < n + 2) return i;
    if (bc == RMHD_BC_PERIODIC) return i < 2 ? i + n : i - n;
    return i < 2 ? 2 : n + 1;
}

// Ghost images along one direction of n interior cells: v[0] is the padded index of the
// cell with interior coordinate c, and v[1], v[2] become the ghost indices that copy it under
// the boundary condition (-1: none).  n >= 4, so a cell has images on one side at most.
__device__ __forceinline__ void images_1d(int bc, int n, int c, int (&v)[3])
{
    if (bc == RMHD_BC_PERIODIC) {
        if (c < 2) v[1] = v[0] + n;
        if (c >= n - 2) v[2] = v[0] - n;
    } else {
        if (c == 0) { v[1] = 0; v[2] = 1; }
        if (c == n - 1) { v[1] = n + 2; v[2] = n + 3; }
    }
}

// Ghost images of interior cell (ii, jj) (interior coordinates) in x and, with ydir, in y:
// images_1d in both directions, written with one branch on the boundary condition (the form
// the 2-D flux kernels compile best with).
__device__ __forceinline__ void ghost_images(const Geo &g, int ii, int jj, bool ydir, int (&xi)[3], int (&yj)[3])
{
    if (g.bc == RMHD_BC_PERIODIC) {
        if (ii < 2) xi[1] = xi[0] + g.nx;
        if (ii >= g.nx - 2) xi[2] = xi[0] - g.nx;
        if (ydir) {
            if (jj < 2) yj[1] = yj[0] + g.ny;
            if (jj >= g.ny - 2) yj[2] = yj[0] - g.ny;
        }
    } else {
        if (ii == 0) { xi[1] = 0; xi[2] = 1; }
        if (ii == g.nx - 1) { xi[1] = g.nx + 2; xi[2] = g.nx + 3; }
        if (ydir) {
            if (jj == 0) { yj[1] = 0; yj[2] = 1; }
            if (jj == g.ny - 1) { yj[1] = g.ny + 2; yj[2] = g.ny + 3; }
        }
    }
}

// ---------------------------------------------------------------------------------------
// ghost fill
// ---------------------------------------------------------------------------------------
static __global__ __launch_bounds__(256) void k_bc(Planes a, int nvar, Geo g)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t % g.pitch), r = (int)(t / g.pitch);
    if (i >= g.nxg || r >= g.rows || is_interior(g, i, r)) return;
    const int j = r % g.nyg, k = r / g.nyg;
    const int si = bc_src(i, g.nx, g.bc);
    const int sj = g.ndim >= 2 ? bc_src(j, g.ny, g.bc) : 0;
    const int sk = g.ndim == 3 ? bc_src(k, g.nz, g.bc) : 0;
    const long d = (long)r * g.pitch + i, s = (long)sk * g.slab + (long)sj * g.pitch + si;
    for (int v = 0; v < nvar; ++v) a.p[v][d] = a.p[v][s];
}

// ---------------------------------------------------------------------------------------
// initial data
// ---------------------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(256) void k_init(CPlanes prims, CPlanes EB, Planes cons, Geo g, Phys P)
{
    constexpr int NC = Model<M>::NC, NP = Model<M>::NP;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t % g.pitch), r = (int)(t / g.pitch);
    if (i >= g.nxg || r >= g.rows || !is_interior(g, i, r)) return;
    const long idx = (long)r * g.pitch + i;
    const int j = r % g.nyg, k = r / g.nyg;
    const long zo = (long)k * g.slab;
    double w[NP], eb[6], q[NC];
#pragma unroll
    for (int v = 0; v < NP; ++v) w[v] = prims.p[v][idx];
#pragma unroll
    for (int v = 0; v < 6; ++v) eb[v] = EB.p[v][idx];
    if constexpr (M == 0) {
        // Gauss's law rho_e = div E, central differences; neighbours through the boundary map
        const long xm = zo + (long)j * g.pitch + bc_src(i - 1, g.nx, g.bc);
        const long xp = zo + (long)j * g.pitch + bc_src(i + 1, g.nx, g.bc);
        double div = (EB.p[3][xp] - EB.p[3][xm]) * (0.5 * g.idx);
        if (g.ndim >= 2) {
            const long ym = zo + (long)bc_src(j - 1, g.ny, g.bc) * g.pitch + i;
            const long yp = zo + (long)bc_src(j + 1, g.ny, g.bc) * g.pitch + i;
            div += (EB.p[4][yp] - EB.p[4][ym]) * (0.5 * g.idy);
        }
        if (g.ndim == 3) {
            const long zm = (long)bc_src(k - 1, g.nz, g.bc) * g.slab + (long)j * g.pitch + i;
            const long zp = (long)bc_src(k + 1, g.nz, g.bc) * g.slab + (long)j * g.pitch + i;
            div += (EB.p[5][zp] - EB.p[5][zm]) * (0.5 * g.idz);
        }
        sf_prim2cons(w, eb, div, P, q);
    } else if constexpr (M == 1) {
        tf_prim2cons(w, eb, P, q);
    } else {
        id_prim2cons(w, eb, P, q);
    }
#pragma unroll
    for (int v = 0; v < NC; ++v) cons.p[v][idx] = q[v];
}

// ---------------------------------------------------------------------------------------
// primitive recovery
// ---------------------------------------------------------------------------------------
// Recovery of every cell, starting from the primitives prims holds (updated in place).
template <int M>
__global__ __launch_bounds__(256) void k_c2p(CPlanes cons, Planes prims, int8_t *status, int32_t *iters, Geo g,
                                             Phys P)
{
    constexpr int NC = Model<M>::NC, NP = Model<M>::NP;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t % g.pitch), r = (int)(t / g.pitch);
    if (i >= g.nxg || r >= g.rows) return;
    const long idx = (long)r * g.pitch + i;
    double q[NC], w[NP];
#pragma unroll
    for (int v = 0; v < NC; ++v) q[v] = cons.p[v][idx];
#pragma unroll
    for (int v = 0; v < NP; ++v) w[v] = prims.p[v][idx];
    int it = 0;
    const int st = cons2prim_m<M>(q, w, P, it);
#pragma unroll
    for (int v = 0; v < NP; ++v) prims.p[v][idx] = w[v];
    if (status) status[idx] = (int8_t)st;
    if (iters) iters[idx] = it;
}

// ---------------------------------------------------------------------------------------
// implicit stage
// ---------------------------------------------------------------------------------------
// SSP2(222) coefficient gamma = 1 - 1/sqrt(2) (Table 2), correctly rounded; every path that
// advances a grid uses this one value so that they agree bit for bit
constexpr double SSP2_GAMMA = 0.29289321881345247559915563789515;

// statistics counters: STATS_SLOTS slots of STATS_STRIDE (256 bytes) each, summed on read;
// per slot [0] cells [1] Newton steps [2] recovery iterations [3] failures [4] Newton maximum
// [5] residual evaluations [6..21] histogram of per-cell Newton steps (last bucket: >= 15)
constexpr int STATS_SLOTS = 64;
constexpr int STATS_STRIDE = 32;
constexpr int STATS_HIST = 6, STATS_NHIST = 16, STATS_RES = 22;   // [22]: largest final relative residual (bits)
constexpr int STATS_JAC = 23;   // Jacobian evaluations

struct StageArgs {
    CPlanes R, guess, win;
    Planes Q, wout;
    int8_t *status;
    int32_t *iters;
    unsigned long long *stats;  // [0] cells [1] newton [2] c2p [3] failures [4] newton max [5] residuals
    unsigned long long *wstats; // per-wavefront slots of the basic counters (detail off), or nullptr
    double a;
    Geo g;
    Phys P;
    int write_all;
    int stats_detail; // also the Newton-step histogram and the largest final residual
    int use_guess;    // start Newton from guess (plain guess R_x again for a cell that fails)
    int compare_start;   // with use_guess, two fluid: start at whichever of guess and R_x has
                         // the smaller residual (one more residual per cell)
    // optional harvest of (features, target) rows of the learned guess, two fluid only:
    // interior cell (i, j) writes row hbase + (j - 2) nx + (i - 2)
    float *hx, *ht;
    long hbase;
    // convergence-compacted queue: a cell still unconverged after cap Newton steps is
    // appended (cell index, unknowns, pressure guesses, steps taken) and finished by k_drain
    int cap;          // >= P.max_newton: no queue
    int qcap;
    int *qidx, *qit;
    double *qx;       // [NX][qcap]
    double *qp;       // [2][qcap]
    unsigned *qcount;
};

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_maxd(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Add per-thread contributions to the statistics: wave shuffles, then LDS, then one atomic
// per counter per block, spread over STATS_SLOTS padded slots so blocks rarely share an
// address.  Every thread of the block must call it.
//   cells: cells counted (0/1); nit: Newton iterations added to the sum; nmax: value for the
//   maximum; cit: recovery iterations; fail: failed cells (0/1); rit: residual evaluations;
//   hbin: final Newton step count of a finished counted cell, for the histogram (-1: none);
//   gres: its final relative residual (>= 0), for the maximum.
__device__ __forceinline__ void stats_block_add(unsigned long long *stats, unsigned cells, unsigned nit, unsigned nmax,
                                                unsigned cit, unsigned fail, unsigned rit, int hbin, double gres,
                                                bool detail, unsigned jac)
{
    __shared__ unsigned long long red[16][7];
    __shared__ unsigned hist[16][STATS_NHIST];
    __shared__ double gmax[16];
    unsigned long long v[7] = {cells, nit, cit, fail, nmax, rit, jac};
#pragma unroll
    for (int k = 0; k < 7; ++k) v[k] = k == 4 ? (unsigned long long)wave_max((int)nmax) : wave_sum(v[k]);
    const int tid = threadIdx.x + blockDim.x * threadIdx.y, wave = tid >> 6;
    if ((tid & 63) == 0)
#pragma unroll
        for (int k = 0; k < 7; ++k) red[wave][k] = v[k];
    if (detail) {   // block-uniform
        const int bin = hbin < 0 ? -1 : min(hbin, STATS_NHIST - 1);
        unsigned hc[STATS_NHIST];
#pragma unroll
        for (int b = 0; b < STATS_NHIST; ++b) hc[b] = (unsigned)__popcll(__ballot(bin == b));
        const double gw = wave_maxd(hbin < 0 || !(gres >= 0.0) ? 0.0 : gres);
        if ((tid & 63) == 0) {
#pragma unroll
            for (int b = 0; b < STATS_NHIST; ++b) hist[wave][b] = hc[b];
            gmax[wave] = gw;
        }
    }
    __syncthreads();
    if (detail && tid == STATS_NHIST) {
        // non-negative doubles order like their bit patterns
        double g = 0.0;
        const int nw = (int)((blockDim.x * blockDim.y + 63) >> 6);
        for (int wv = 0; wv < nw; ++wv) g = fmax(g, gmax[wv]);
        if (g > 0.0)
            atomicMax(&stats[((blockIdx.x + gridDim.x * blockIdx.y) % STATS_SLOTS) * STATS_STRIDE + STATS_RES],
                      (unsigned long long)__double_as_longlong(g));
    }
    if (detail && tid < STATS_NHIST) {
        unsigned long long t = 0;
        const int nw = (int)((blockDim.x * blockDim.y + 63) >> 6);
        for (int wv = 0; wv < nw; ++wv) t += hist[wv][tid];
        if (t) atomicAdd(&stats[((blockIdx.x + gridDim.x * blockIdx.y) % STATS_SLOTS) * STATS_STRIDE + STATS_HIST + tid], t);
    }
    if (tid == 0) {
        unsigned long long t[7] = {0, 0, 0, 0, 0, 0, 0};
        const int nw = (int)((blockDim.x * blockDim.y + 63) >> 6);
        for (int wv = 0; wv < nw; ++wv)
#pragma unroll
            for (int k = 0; k < 7; ++k) t[k] = k == 4 ? max(t[k], red[wv][k]) : t[k] + red[wv][k];
        if (t[0] || t[1] || t[3]) {
            unsigned long long *slot = stats + ((blockIdx.x + gridDim.x * blockIdx.y) % STATS_SLOTS) * STATS_STRIDE;
            if (t[0]) atomicAdd(&slot[0], t[0]);
            if (t[1]) atomicAdd(&slot[1], t[1]);
            if (t[2]) atomicAdd(&slot[2], t[2]);
            if (t[3]) atomicAdd(&slot[3], t[3]);
            atomicMax(&slot[4], t[4]);
            if (t[5]) atomicAdd(&slot[5], t[5]);
            if (t[6]) atomicAdd(&slot[STATS_JAC], t[6]);
        }
    }
    __syncthreads();  // red[] may be reused by a following call in the same block
}

// The basic counters without block barriers or atomics (used while the detailed statistics
// are off): every wavefront of a launch owns one slot of STATS_WAVE counters in wstats, at
// its index in the launch.  It reads its slot when it starts, so the load is long done by
// its end, when its first lane writes back the slot plus the wavefront's totals.  Launches
// on one stream run one after another, so a slot never has two writers at once;
// rmhd_get_stats folds the slots into the counters.  Measured: the block reduction and
// atomics of stats_block_add cost ~3 us per stage launch on the 256 x 512 grid, where every
// block ends at about the same time.
constexpr int STATS_WAVE = 8;   // [0] cells [1] newton [2] c2p [3] failures [4] newton max [5] residuals
                                // [6] Jacobian evaluations
}  // namespace rmhd
// wavefront sum of the device library (its 32-bit and max forms are declared by HIP itself)
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_add_u64(unsigned long long);
namespace rmhd {
struct WaveStats {
    unsigned long long *slot;
    unsigned long long old[7];
};
__device__ __forceinline__ void wave_stats_begin(unsigned long long *wstats, WaveStats &ws)
{
    ws.slot = wstats + ((long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * STATS_WAVE;
#pragma unroll
    for (int k = 0; k < 7; ++k) ws.old[k] = ws.slot[k];
}
__device__ __forceinline__ void wave_stats_end(const WaveStats &ws, unsigned cells, unsigned nit, unsigned nmax,
                                               unsigned cit, unsigned fail, unsigned rit, unsigned jac)
{
    // the device library's wavefront reductions (cross-lane data-parallel moves, much shorter
    // than a shuffle tree); a wavefront's totals fit 32 bits except the recovery iterations
    const unsigned long long v[7] = {__ockl_wfred_add_u32(cells), __ockl_wfred_add_u32(nit),
                                     __ockl_wfred_add_u64(cit), __ockl_wfred_add_u32(fail),
                                     (unsigned long long)__ockl_wfred_max_i32((int)nmax), __ockl_wfred_add_u32(rit),
                                     __ockl_wfred_add_u32(jac)};
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < 7; ++k) ws.slot[k] = k == 4 ? max(ws.old[k], v[k]) : ws.old[k] + v[k];
    }
}

// Fold the wavefront slots into slot 0 of the counters and clear them.  Each block folds a
// strided share of the slots (blocks of 256 threads) and adds its totals with device atomics:
// integer sums and one maximum, so the result does not depend on the order of the blocks.
static __global__ __launch_bounds__(256) void k_wave_stats_fold(unsigned long long *wstats, long nslots,
                                                                unsigned long long *stats)
{
    __shared__ unsigned long long red[7][256];
    unsigned long long t[7] = {0, 0, 0, 0, 0, 0, 0};
    for (long sl = (long)blockIdx.x * blockDim.x + threadIdx.x; sl < nslots; sl += (long)gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            const unsigned long long x = wstats[sl * STATS_WAVE + k];
            t[k] = k == 4 ? max(t[k], x) : t[k] + x;
            wstats[sl * STATS_WAVE + k] = 0;
        }
    }
#pragma unroll
    for (int k = 0; k < 7; ++k) red[k][threadIdx.x] = t[k];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                const unsigned long long a = red[k][threadIdx.x], b = red[k][threadIdx.x + h];
                red[k][threadIdx.x] = k == 4 ? max(a, b) : a + b;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 7) {
        if (threadIdx.x == 4) atomicMax(&stats[4], red[4][0]);
        else if (threadIdx.x == 6) atomicAdd(&stats[STATS_JAC], red[6][0]);
        else atomicAdd(&stats[threadIdx.x], red[threadIdx.x][0]);
    }
}
// Blocks for a fold of nslots slots (at least one, at most 256).
static inline unsigned wave_stats_fold_blocks(long nslots)
{
    const long b = (nslots + 255) / 256;
    return (unsigned)(b < 1 ? 1 : b > 256 ? 256 : b);
}

// Starting unknowns of a cell: the caller's guess planes, or the plain guess R_x.
template <int M>
__device__ __forceinline__ void stage_start(const StageArgs &A, long idx, bool guess, double (&x)[Model<M>::NX])
{
    const CPlanes &X0 = guess ? A.guess : A.R;
    if constexpr (M == 0) {
        x[0] = X0.p[sf::EX][idx]; x[1] = X0.p[sf::EY][idx]; x[2] = X0.p[sf::EZ][idx];
    } else {
        const double isc = frcp(fabs(A.P.mu1));
        x[0] = X0.p[tf::SBX][idx] * isc; x[1] = X0.p[tf::SBY][idx] * isc; x[2] = X0.p[tf::SBZ][idx] * isc;
        x[3] = X0.p[tf::TAUB][idx] * isc;
        x[4] = X0.p[tf::EX][idx]; x[5] = X0.p[tf::EY][idx]; x[6] = X0.p[tf::EZ][idx];
    }
}

// One solve attempt of a cell from x (TF: with R_x as the alternative start when alt).
template <int M>
__device__ __forceinline__ int stage_solve(const double *R, const StageArgs &A, double sig, const Phys &P,
                                          double (&x)[Model<M>::NX], double *w, int &nit, int &cit, int &rit,
                                          bool alt, int cap, double &gres, int &jit)
{
    int n = 0, c = 0, r = 0, st;
    if constexpr (M == 0) {
        (void)alt;
        st = sf_stage(R, A.a, sig, P, x, w, n, c, r, cap, &gres, &jit);
    } else {
        const double isc = frcp(fabs(P.mu1));
        const double rx[7] = {R[tf::SBX] * isc, R[tf::SBY] * isc, R[tf::SBZ] * isc, R[tf::TAUB] * isc,
                              R[tf::EX], R[tf::EY], R[tf::EZ]};
        st = tf_stage(R, A.a, sig, P, x, w, n, c, r, alt ? rx : nullptr, cap, &gres, &jit);
    }
    nit += n;
    cit += c;
    rit += r;
    return st;
}

// Outputs of a finished cell: the source-carrying components of Q (psi and phi in closed
// form), the other components when Q != R, primitives, status, iterations, harvest row.
template <int M>
__device__ __forceinline__ void stage_write(const StageArgs &A, long idx, int i, int j, const double *R,
                                           const double (&x)[Model<M>::NX], const double *w, int st, int nit,
                                           double sig)
{
    constexpr int NC = Model<M>::NC, NP = Model<M>::NP;
    const Geo &g = A.g;
    const double aK = frcp(1.0 + A.a * A.P.kappa);
    if constexpr (M == 0) {
        A.Q.p[sf::EX][idx] = x[0]; A.Q.p[sf::EY][idx] = x[1]; A.Q.p[sf::EZ][idx] = x[2];
        A.Q.p[sf::PHI][idx] = R[sf::PHI] * aK;
        A.Q.p[sf::PSI][idx] = (R[sf::PSI] + A.a * R[sf::RHOE]) * aK;
    } else {
        const double sc = fabs(A.P.mu1), isc = frcp(sc);
        A.Q.p[tf::SBX][idx] = x[0] * sc; A.Q.p[tf::SBY][idx] = x[1] * sc; A.Q.p[tf::SBZ][idx] = x[2] * sc;
        A.Q.p[tf::TAUB][idx] = x[3] * sc;
        A.Q.p[tf::EX][idx] = x[4]; A.Q.p[tf::EY][idx] = x[5]; A.Q.p[tf::EZ][idx] = x[6];
        A.Q.p[tf::PHI][idx] = R[tf::PHI] * aK;
        A.Q.p[tf::PSI][idx] = (R[tf::PSI] + A.a * R[tf::DB]) * aK;
        if (A.hx && is_interior(g, i, j)) {
            // features of R and target (x* - R_x) / D of the learned guess
            const long row = A.hbase + interior_rank(g, i, j);
            const double iD = 1.0 / R[tf::D];
            float *f = A.hx + row * 19;
            f[0] = (float)log10(A.a * A.P.mu1 * A.P.mu1 * R[tf::D]);
#pragma unroll
            for (int v = 1; v < 18; ++v) f[v] = (float)(R[v] * iD);
            f[18] = (float)log10(A.a * sig);
            const double rx[7] = {R[tf::SBX] * isc, R[tf::SBY] * isc, R[tf::SBZ] * isc, R[tf::TAUB] * isc,
                                  R[tf::EX], R[tf::EY], R[tf::EZ]};
            float *tg = A.ht + row * 7;
#pragma unroll
            for (int k = 0; k < 7; ++k) tg[k] = st == CELL_OK ? (float)((x[k] - rx[k]) * iD) : 0.0f;
        }
    }
    if (A.write_all) {
#pragma unroll
        for (int v = 0; v < NC; ++v)
            if (!has_source(M, v)) A.Q.p[v][idx] = R[v];
    }
#pragma unroll
    for (int v = 0; v < NP; ++v) A.wout.p[v][idx] = w[v];
    if (A.status) A.status[idx] = (int8_t)st;
    if (A.iters) A.iters[idx] = nit;
}

// Implicit stage over every cell, ghosts included.  With a guess the cell starts there (TF
// with compare_start: at the better of guess and R_x); a failed cell is solved again from
// R_x.  A cell still unconverged after A.cap steps is appended to the queue (one atomic per
// block).
template <int M>
__global__ __launch_bounds__(256) void k_stage(StageArgs A)
{
    constexpr int NC = Model<M>::NC, NP = Model<M>::NP, NX = Model<M>::NX;
    const Geo &g = A.g;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t % g.pitch), j = (int)(t / g.pitch);
    const bool live = i < g.nxg && j < g.rows;   // j: row of all z planes
    const long idx = (long)j * g.pitch + i;
    int nit = 0, cit = 0, rit = 0, jit = 0, st = CELL_OK;
    bool push = false;
    double x[NX], w[NP], gres = 0.0;
    const bool wave_stats = A.stats && A.wstats && !A.stats_detail;
    WaveStats ws{};
    if (wave_stats) wave_stats_begin(A.wstats, ws);
    if (live) {
        const double sig = cell_sigma(A.P, idx);
        double R[NC];
#pragma unroll
        for (int v = 0; v < NC; ++v) R[v] = A.R.p[v][idx];
#pragma unroll
        for (int v = 0; v < NP; ++v) w[v] = A.win.p[v][idx];
        for (int attempt = A.use_guess ? 0 : 1;; ++attempt) {
            stage_start<M>(A, idx, attempt == 0, x);
            if (attempt == 1 && A.use_guess)
#pragma unroll
                for (int v = 0; v < NP; ++v) w[v] = A.win.p[v][idx];
            st = stage_solve<M>(R, A, sig, A.P, x, w, nit, cit, rit, attempt == 0 && A.compare_start, A.cap, gres,
                                jit);
            if (st == CELL_OK || st == CELL_QUEUED || attempt == 1) break;
        }
        push = st == CELL_QUEUED;
        if (!push) stage_write<M>(A, idx, i, j, R, x, w, st, nit, sig);
    }
    if (A.cap < A.P.max_newton) {
        // block-aggregated append: wave ballots, per-wave counts in LDS, one atomic
        __shared__ int s_wc[4];
        __shared__ int s_base;
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        const unsigned long long mask = __ballot(push);
        if (lane == 0) s_wc[wave] = __popcll(mask);
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) tot += s_wc[wv];
            s_base = tot ? (int)atomicAdd(A.qcount, (unsigned)tot) : 0;
        }
        __syncthreads();
        if (push) {
            int e = s_base;
            for (int wv = 0; wv < wave; ++wv) e += s_wc[wv];
            e += __popcll(mask & ((1ull << lane) - 1ull));
            // the queue holds every cell of the grid, so e < qcap
            A.qidx[e] = (int)idx;
            A.qit[e] = nit;
#pragma unroll
            for (int k = 0; k < NX; ++k) A.qx[(long)k * A.qcap + e] = x[k];
            A.qp[e] = w[4];
            if constexpr (M == 1) A.qp[(long)A.qcap + e] = w[9];
        }
    }
    if (A.stats) {
        const bool c = live && is_interior(g, i, j);
        if (wave_stats)
            wave_stats_end(ws, c, c ? nit : 0, c && !push ? nit : 0, c ? cit : 0, c && !push && st != CELL_OK,
                           c ? rit : 0, c ? jit : 0);
        else
            stats_block_add(A.stats, c, c ? nit : 0, c && !push ? nit : 0, c ? cit : 0, c && !push && st != CELL_OK,
                            c ? rit : 0, c && !push ? nit : -1, gres, A.stats_detail != 0, c ? jit : 0);
    }
}

// Finish the queued cells in full wavefronts: each thread resumes one entry from its saved
// unknowns and pressures with the Newton steps it has left.  Sized for the largest queue;
// blocks past the tail exit at once.
template <int M>
__global__ __launch_bounds__(256) void k_drain(StageArgs A)
{
    constexpr int NC = Model<M>::NC, NP = Model<M>::NP, NX = Model<M>::NX;
    const int tail = (int)min(*A.qcount, (unsigned)A.qcap);
    if ((int)(blockIdx.x * blockDim.x) >= tail) return;   // whole block past the tail
    const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const Geo &g = A.g;
    int nit = 0, cit = 0, rit = 0, jit = 0, st = CELL_OK, done = 0;
    bool interior = false;
    double gres = 0.0;
    const bool wave_stats = A.stats && A.wstats && !A.stats_detail;
    WaveStats ws{};
    if (wave_stats) wave_stats_begin(A.wstats, ws);
    if (e < tail) {
        const long idx = A.qidx[e];
        const int i = (int)(idx % g.pitch), j = (int)(idx / g.pitch);
        interior = is_interior(g, i, j);
        done = A.qit[e];
        const double sig = cell_sigma(A.P, idx);
        double R[NC], x[NX], w[NP];
#pragma unroll
        for (int v = 0; v < NC; ++v) R[v] = A.R.p[v][idx];
#pragma unroll
        for (int v = 0; v < NP; ++v) w[v] = A.win.p[v][idx];
#pragma unroll
        for (int k = 0; k < NX; ++k) x[k] = A.qx[(long)k * A.qcap + e];
        w[4] = A.qp[e];
        if constexpr (M == 1) w[9] = A.qp[(long)A.qcap + e];
        Phys P = A.P;
        P.max_newton = max(1, A.P.max_newton - done);
        for (int attempt = 0;; ++attempt) {
            if (attempt == 1) {
                // a guessed start led nowhere: the plain guess with the full step budget
                stage_start<M>(A, idx, false, x);
#pragma unroll
                for (int v = 0; v < NP; ++v) w[v] = A.win.p[v][idx];
                P.max_newton = A.P.max_newton;
            }
            st = stage_solve<M>(R, A, sig, P, x, w, nit, cit, rit, false, 1 << 30, gres, jit);
            if (st == CELL_OK || !A.use_guess || attempt == 1) break;
        }
        stage_write<M>(A, idx, i, j, R, x, w, st, done + nit, sig);
    }
    // the cell was counted by k_stage; iterations, the maximum and failures are added here
    if (A.stats) {
        const bool c = e < tail && interior;
        if (wave_stats)
            wave_stats_end(ws, 0u, c ? nit : 0, c ? done + nit : 0, c ? cit : 0, c && st != CELL_OK, c ? rit : 0,
                           c ? jit : 0);
        else
            stats_block_add(A.stats, 0u, c ? nit : 0, c ? done + nit : 0, c ? cit : 0, c && st != CELL_OK, c ? rit : 0,
                            c ? done + nit : -1, gres, A.stats_detail != 0, c ? jit : 0);
    }
}

static __global__ void k_qreset(unsigned *count)
{
    if (threadIdx.x == 0) *count = 0u;
}

// ---------------------------------------------------------------------------------------
// flux pass: FVS + WENO3 and the fused stage combiners
// ---------------------------------------------------------------------------------------
// One output of the flux pass: out = base + cL L + cS Psi, per interior cell (base.p[0] ==
// nullptr: no base term; out may alias base).
struct FluxOut {
    CPlanes base;
    Planes out;
    double cL, cS;
};
constexpr int FLUX_MAXOUT = 3;

// Apart from q, every set of planes here lies g.plane doubles apart from its first plane (the
// tile kernels read only p[0] of them).
struct FluxArgs {
    CPlanes q, w;
    FluxOut o[FLUX_MAXOUT];   // outputs 0 .. n-1 used (the launch fixes n), the rest ignored
    Geo g;
    Phys P;
    int fuse_bc;          // also write the ghost images of output 0
    // wnew.p[0] != nullptr (single fluid and ideal): also recover the primitives of output 0
    // (guess: w) and write them, with their ghost images, to wnew, which must not alias w
    // (halo cells of other tiles still read w)
    Planes wnew;
    // 3-D: the z term L_z of every variable at the interior cells, formed by k_flux_z before
    // the x-y tiles, which add it and complete the outputs
    Planes lz;
};

// Plane v of a set whose planes lie g.plane doubles apart, as the outputs, bases and
// primitives of every flux pass do (only q mixes planes of several arrays): one pointer per
// set rather than one per variable keeps the tile kernels within their scalar registers.
template <typename P>
__device__ __forceinline__ auto plane_at(const P &s, int v, const Geo &g)
{
    return s.p[0] + (long)v * g.plane;
}

// The base terms of component v for the NO outputs at this cell (zero away from the interior).
// BQ: every output has the same base, whose source-free planes are q's (the first pass of a
// step, which reads q^n both as its state's source-free part and as the base): the base of a
// source-free component is the cell's own q[v], and one value serves every output.  The
// values are those a load would give.
// (Loading the two-fluid source components' base values with the state instead, so that no
// round of the first pass waits for a load, measured slower: 227 against 223 us per pass on
// the 1024^2 sheet.)
template <int M, int NO, bool BQ, int NC>
__device__ __forceinline__ void base_terms(const FluxArgs &A, const double (&q)[NC], int v, bool interior, long idx,
                                           double (&b)[NO])
{
    const int vc = v < NC ? v : NC - 1;
    if constexpr (BQ) {
        b[0] = (v < NC && interior) ? (has_source(M, vc) ? plane_at(A.o[0].base, vc, A.g)[idx] : q[vc]) : 0.0;
#pragma unroll
        for (int k = 1; k < NO; ++k) b[k] = b[0];
    } else {
#pragma unroll
        for (int k = 0; k < NO; ++k)
            b[k] = (v < NC && interior && A.o[k].base.p[0]) ? plane_at(A.o[k].base, vc, A.g)[idx] : 0.0;
    }
}

// Store a cell's value and, where the cell has ghost images (img), the images too: the
// image loop sits behind one branch, which whole wavefronts away from the boundary skip.
__device__ __forceinline__ void store_with_images(double *plane, long zoff, int pitch, const int (&xi)[3],
                                                  const int (&yj)[3], int ny_img, bool img, double val)
{
    plane[zoff + (long)yj[0] * pitch + xi[0]] = val;
    if (img) {
#pragma unroll
        for (int aa = 0; aa < 3; ++aa)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb)
                if ((aa || bb) && bb < ny_img && xi[aa] >= 0 && yj[bb] >= 0)
                    plane[zoff + (long)yj[bb] * pitch + xi[aa]] = val;
    }
}

// The same on a 3-D grid: the cell and its x-y images on its own z plane and on each z image
// plane zk[1], zk[2] (img_xy: the cell has x or y images; img: it has any).
__device__ __forceinline__ void store_with_images3(double *plane, const Geo &g, const int (&xi)[3],
                                                   const int (&yj)[3], const int (&zk)[3], bool img_xy, bool img,
                                                   double val)
{
    store_with_images(plane, (long)zk[0] * g.slab, g.pitch, xi, yj, 3, img_xy, val);
    if (img) {
#pragma unroll
        for (int cc = 1; cc < 3; ++cc)
            if (zk[cc] >= 0) store_with_images(plane, (long)zk[cc] * g.slab, g.pitch, xi, yj, 3, img_xy, val);
    }
}

// Primitives of a cell's new state q (guess w), written with the ghost images of the cell.
template <int M>
__device__ __forceinline__ void flux_recover(const FluxArgs &A, const double *q, const double *w,
                                            const int (&xi)[3], const int (&yj)[3], const int (&zk)[3], bool img_xy,
                                            bool img)
{
    constexpr int NP = Model<M>::NP;
    double wn[NP];
#pragma unroll
    for (int v = 0; v < NP; ++v) wn[v] = w[v];
    int it = 0;
    cons2prim_m<M>(q, wn, A.P, it);
#pragma unroll
    for (int v = 0; v < NP; ++v) store_with_images3(plane_at(A.wnew, v, A.g), A.g, xi, yj, zk, img_xy, img, wn[v]);
}

// WENO3 value at the downwind face of b from the upwind-ordered stencil (a, b, c):
// candidates b + (b - a)/2 and b + (c - b)/2 with linear weights 1/3, 2/3 and
// alpha_k = d_k / (1e-6 + beta_k)^2 (Jiang-Shu), written with one division:
// w0 = t1^2 / (t1^2 + 2 t0^2), t_k = 1e-6 + beta_k.
// Two reconstructions (f+ on one side, f- on the other, of the same cell) share one
// reciprocal: 1/n1 = n2 / (n1 n2) and 1/n2 = n1 / (n1 n2); n_k >= 3e-12, so the product
// neither underflows nor overflows for any representable flux.
__device__ __forceinline__ void weno3_pair(double ap, double bp, double cp, double am, double bm, double cm,
                                           double &vp, double &vm)
{
    const double d0p = bp - ap, d1p = cp - bp, d0m = bm - am, d1m = cm - bm;
    const double t0p = 1e-6 + d0p * d0p, t1p = 1e-6 + d1p * d1p;
    const double t0m = 1e-6 + d0m * d0m, t1m = 1e-6 + d1m * d1m;
    const double t1ps = t1p * t1p, t1ms = t1m * t1m;
    const double np = t1ps + 2.0 * (t0p * t0p), nm = t1ms + 2.0 * (t0m * t0m);
    const double r = frcp(np * nm);
    const double w0p = t1ps * nm * r, w0m = t1ms * np * r;
    vp = bp + 0.5 * (d1p + w0p * (d0p - d1p));
    vm = bm + 0.5 * (d1m + w0m * (d0m - d1m));
}

// One tile of the flux pass, both directions staged through LDS (used for 1-D blocks, whose
// rows span several wavefronts); every thread of the block must call it (it holds
// barriers).  (bx, by) is the tile position in units of interior tiles; zoff is the offset of
// the z plane (0 below 3-D, where a 2-D tile forms the x and y terms of one plane).
template <int M, int NDIM, int BX, int BY, int NO, int GV = 1, bool RECOVER = true, bool Z3 = false, bool BQ = false>
__device__ __forceinline__ void flux_tile_lds(const FluxArgs &A, int bx, int by, long zoff)
{
    constexpr int NC = Model<M>::NC, NP = Model<M>::NP;
    constexpr int TX = BX - 4, TY = NDIM == 2 ? BY - 4 : 1;
    // split fluxes f+ / f- per direction, then the half reconstructions: cell i holds
    // f+ at its right face (i+1/2) and f- at its left face (i-1/2); GV variables per round
    __shared__ double sfp[GV][NDIM][BY][BX], sfm[GV][NDIM][BY][BX];
    __shared__ double shp[GV][NDIM][BY][BX], shm[GV][NDIM][BY][BX];
    const Geo &g = A.g;
    const int tx = threadIdx.x, ty = NDIM == 2 ? threadIdx.y : 0;
    const int ii = bx * TX + tx - 2;
    const int jj = NDIM == 2 ? by * TY + ty - 2 : 0;
    const int i = min(max(ii + 2, 0), g.nxg - 1);
    const int j = NDIM == 2 ? min(max(jj + 2, 0), g.nyg - 1) : 0;
    const long idx = zoff + (long)j * g.pitch + i;

    double q[NC], w[NP], fx[NC], fy[NC], src[NC];
#pragma unroll
    for (int v = 0; v < NC; ++v) q[v] = A.q.p[v][idx];
#pragma unroll
    for (int v = 0; v < NP; ++v) w[v] = plane_at(A.w, v, g)[idx];
    const double sig = cell_sigma(A.P, idx);
    // the halo rows' cells (whole wavefronts when a wavefront holds one or two tile rows) need
    // no source
    flux_source_m<M>(q, w, sig, A.P, fx, fy, src,
                     NDIM == 1 || (BX != 64 && BX != 32) || (ty >= 2 && ty < BY - 2));

    const bool interior = tx >= 2 && tx < BX - 2 && ii < g.nx &&
                          (NDIM == 1 || (ty >= 2 && ty < BY - 2 && jj < g.ny));
    const bool do_x = tx >= 1 && tx <= BX - 2 && (NDIM == 1 || (ty >= 2 && ty <= BY - 3));
    const bool do_y = NDIM == 2 && ty >= 1 && ty <= BY - 2 && tx >= 2 && tx <= BX - 3;

    // ghost images of this interior cell (fused boundary fill of output 0; on a 3-D grid in z
    // as well, the tile completing the outputs there)
    int xi[3] = {i, -1, -1}, yj[3] = {j, -1, -1}, zk[3] = {Z3 ? (int)(zoff / g.slab) : 0, -1, -1};
    if (A.fuse_bc && interior) {
        ghost_images(g, ii, jj, NDIM == 2, xi, yj);
        if constexpr (Z3) images_1d(g.bc, g.nz, zk[0] - 2, zk);
    }
    const bool img_xy = xi[1] >= 0 || xi[2] >= 0 || yj[1] >= 0 || yj[2] >= 0;
    const bool img = img_xy || zk[1] >= 0 || zk[2] >= 0;

#pragma unroll
    for (int v0 = 0; v0 < NC; v0 += GV) {
        // base terms (and the z term) first, so that their loads overlap the reconstruction
        double bv[GV][NO], lzv[GV];
#pragma unroll
        for (int gv = 0; gv < GV; ++gv) {
            base_terms<M, NO, BQ>(A, q, v0 + gv, interior, idx, bv[gv]);
            lzv[gv] = (Z3 && v0 + gv < NC && interior) ? plane_at(A.lz, v0 + gv, g)[idx] : 0.0;
        }
#pragma unroll
        for (int gv = 0; gv < GV; ++gv) {
            const int v = v0 + gv;
            if (v >= NC) break;
            sfp[gv][0][ty][tx] = 0.5 * (fx[v] + q[v]);
            sfm[gv][0][ty][tx] = 0.5 * (fx[v] - q[v]);
            if constexpr (NDIM == 2) {
                sfp[gv][NDIM - 1][ty][tx] = 0.5 * (fy[v] + q[v]);
                sfm[gv][NDIM - 1][ty][tx] = 0.5 * (fy[v] - q[v]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int gv = 0; gv < GV; ++gv) {
            if (v0 + gv >= NC) break;
            if (do_x) {
                double vp, vm;
                weno3_pair(sfp[gv][0][ty][tx - 1], sfp[gv][0][ty][tx], sfp[gv][0][ty][tx + 1], sfm[gv][0][ty][tx + 1],
                           sfm[gv][0][ty][tx], sfm[gv][0][ty][tx - 1], vp, vm);
                shp[gv][0][ty][tx] = vp;
                shm[gv][0][ty][tx] = vm;
            }
            if constexpr (NDIM == 2) {
                if (do_y) {
                    double vp, vm;
                    weno3_pair(sfp[gv][NDIM - 1][ty - 1][tx], sfp[gv][NDIM - 1][ty][tx], sfp[gv][NDIM - 1][ty + 1][tx],
                               sfm[gv][NDIM - 1][ty + 1][tx], sfm[gv][NDIM - 1][ty][tx], sfm[gv][NDIM - 1][ty - 1][tx],
                               vp, vm);
                    shp[gv][NDIM - 1][ty][tx] = vp;
                    shm[gv][NDIM - 1][ty][tx] = vm;
                }
            }
        }
        __syncthreads();
        if (interior) {
#pragma unroll
            for (int gv = 0; gv < GV; ++gv) {
                const int v = v0 + gv;
                if (v >= NC) break;
                double L = -((shp[gv][0][ty][tx] + shm[gv][0][ty][tx + 1]) - (shp[gv][0][ty][tx - 1] + shm[gv][0][ty][tx])) *
                           g.idx;
                if constexpr (NDIM == 2)
                    L -= ((shp[gv][NDIM - 1][ty][tx] + shm[gv][NDIM - 1][ty + 1][tx]) -
                          (shp[gv][NDIM - 1][ty - 1][tx] + shm[gv][NDIM - 1][ty][tx])) * g.idy;
                if constexpr (Z3) L += lzv[gv];
                const double S = has_source(M, v) ? src[v] : 0.0;
                double o0 = 0.0;
#pragma unroll
                for (int k = 0; k < NO; ++k) {
                    const FluxOut &F = A.o[k];
                    const double o = bv[gv][k] + F.cL * L + F.cS * S;
                    if (k == 0) {
                        o0 = o;
                        store_with_images3(plane_at(F.out, v, g), g, xi, yj, zk, img_xy, img, o);
                    } else {
                        plane_at(F.out, v, g)[idx] = o;
                    }
                }
                q[v] = o0;   // this thread's own q[v] is not read again
            }
        }
    }
    if constexpr (RECOVER)
        if (A.wnew.p[0] && interior) flux_recover<M>(A, q, w, xi, yj, zk, img_xy, img);
}

// Row-form flux components per model (single fluid and ideal; the two-fluid model uses the
// LDS form).
template <int M>
__device__ __forceinline__ auto row_quantities(const double *q, const double *w, double sig, const Phys &P)
{
    if constexpr (M == 0) return sf_row(q, w, sig, P);
    else return id_row(q, w);
}
template <int M, int K, typename T>
__device__ __forceinline__ double row_flux(int c, const double *q, const T &I)
{
    if constexpr (M == 0) return sf_row_flux<K>(c, q, I);
    else return id_row_flux<K>(c, q, I);
}
template <int M, typename T>
__device__ __forceinline__ double row_source(int c, const double *q, const T &I, const Phys &P)
{
    if constexpr (M == 0) return sf_row_src(c, q, I, P);
    else return c == id::PHI ? -P.kappa * q[id::PHI] : 0.0;
}

// Values of the lanes to the left and right in the same wavefront (a lane at the edge gets
// its own value back; edge lanes are halo cells whose results are not used).
// Whole-wavefront shifts by one lane on the VALU's data-parallel move (DPP wave_shr:1 /
// wave_shl:1, two 32-bit moves per double), instead of the LDS crossbar permute a generic
// shuffle compiles to: single-fluid 256x512 pass 28.0 -> 26.7 us.  A lane with no source
// lane (0 for the right shift, 63 for the left) keeps its own value.
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_left(double v) { return dpp_shift<0x138>(v); }
__device__ __forceinline__ double from_right(double v) { return dpp_shift<0x130>(v); }

// One tile of a 2-D flux pass with 64-wide rows: each row of the block is one wavefront, so
// the x stencil is read from neighbouring lanes (no LDS, no barrier) and only the y stencil
// goes through LDS, G variables per pair of barriers.  The arithmetic per face and cell is
// that of flux_tile_lds.  Every thread of the block must call it.
template <int M, int BY, int NO, bool RECOVER = true, bool Z3 = false, bool BQ = false>
__device__ __forceinline__ void flux_tile_rows(const FluxArgs &A, int bx, int by, long zoff)
{
    constexpr int NC = Model<M>::NC, NP = Model<M>::NP;
    constexpr int BX = 64, TX = BX - 4, TY = BY - 4;
    constexpr int G = 2;   // variables per LDS round: G x 4 x BY x 64 doubles (measured best)
    __shared__ double sfp[G][BY][BX], sfm[G][BY][BX], shp[G][BY][BX], shm[G][BY][BX];
    const Geo &g = A.g;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int ii = bx * TX + tx - 2;
    const int jj = by * TY + ty - 2;
    const int i = min(max(ii + 2, 0), g.nxg - 1);
    const int j = min(max(jj + 2, 0), g.nyg - 1);
    const long idx = zoff + (long)j * g.pitch + i;

    double q[NC], w[NP];
#pragma unroll
    for (int v = 0; v < NC; ++v) q[v] = A.q.p[v][idx];
#pragma unroll
    for (int v = 0; v < NP; ++v) w[v] = plane_at(A.w, v, g)[idx];
    // quantities shared by the flux components; each round forms only its own components
    const auto I = row_quantities<M>(q, w, cell_sigma(A.P, idx), A.P);

    const bool interior = tx >= 2 && tx < BX - 2 && ii < g.nx && ty >= 2 && ty < BY - 2 && jj < g.ny;
    const bool do_y = ty >= 1 && ty <= BY - 2 && tx >= 2 && tx <= BX - 3;

    // ghost images of this interior cell (fused boundary fill of output 0; on a 3-D grid in z
    // as well, the tile completing the outputs there)
    int xi[3] = {i, -1, -1}, yj[3] = {j, -1, -1}, zk[3] = {Z3 ? (int)(zoff / g.slab) : 0, -1, -1};
    if (A.fuse_bc && interior) {
        ghost_images(g, ii, jj, true, xi, yj);
        if constexpr (Z3) images_1d(g.bc, g.nz, zk[0] - 2, zk);
    }
    const bool img_xy = xi[1] >= 0 || xi[2] >= 0 || yj[1] >= 0 || yj[2] >= 0;
    const bool img = img_xy || zk[1] >= 0 || zk[2] >= 0;

#pragma unroll
    for (int v0 = 0; v0 < NC; v0 += G) {
        // the base terms of this round's outputs, loaded first so that their latency is
        // spent on the x reconstructions below (base is read only at interior cells, ghost
        // images are written only at ghost cells, so no store of this pass can change them)
        double bv[G][NO], lzv[G];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            base_terms<M, NO, BQ>(A, q, v0 + k, interior, idx, bv[k]);
            lzv[k] = (Z3 && v0 + k < NC && interior) ? plane_at(A.lz, v0 + k, g)[idx] : 0.0;
        }
        double Lx[G];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const int v = v0 + k;
            if (v >= NC) break;
            // x: split fluxes and both half reconstructions from the neighbouring lanes
            const double fxv = row_flux<M, 0>(v, q, I);
            const double fp = 0.5 * (fxv + q[v]), fm = 0.5 * (fxv - q[v]);
            double vp, vm;
            weno3_pair(from_left(fp), fp, from_right(fp), from_right(fm), fm, from_left(fm), vp, vm);
            Lx[k] = -((vp + from_right(vm)) - (from_left(vp) + vm)) * g.idx;
            // y: split fluxes to LDS
            const double fyv = row_flux<M, 1>(v, q, I);
            sfp[k][ty][tx] = 0.5 * (fyv + q[v]);
            sfm[k][ty][tx] = 0.5 * (fyv - q[v]);
        }
        __syncthreads();
        if (do_y) {
#pragma unroll
            for (int k = 0; k < G; ++k) {
                if (v0 + k >= NC) break;
                double vp, vm;
                weno3_pair(sfp[k][ty - 1][tx], sfp[k][ty][tx], sfp[k][ty + 1][tx], sfm[k][ty + 1][tx], sfm[k][ty][tx],
                           sfm[k][ty - 1][tx], vp, vm);
                shp[k][ty][tx] = vp;
                shm[k][ty][tx] = vm;
            }
        }
        __syncthreads();
        if (interior) {
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const int v = v0 + k;
                if (v >= NC) break;
                double L = Lx[k];
                L -= ((shp[k][ty][tx] + shm[k][ty + 1][tx]) - (shp[k][ty - 1][tx] + shm[k][ty][tx])) * g.idy;
                if constexpr (Z3) L += lzv[k];
                const double S = row_source<M>(v, q, I, A.P);
#pragma unroll
                for (int kk = 0; kk < NO; ++kk) {
                    const FluxOut &F = A.o[kk];
                    const double o = bv[k][kk] + F.cL * L + F.cS * S;
                    if (kk == 0) {
                        store_with_images3(plane_at(F.out, v, g), g, xi, yj, zk, img_xy, img, o);
                    } else {
                        plane_at(F.out, v, g)[idx] = o;
                    }
                }
            }
        }
        // the next round rewrites sfp/sfm only after every thread has passed the barrier
        // above, and shp/shm only after the next round's first barrier
    }
    if constexpr (RECOVER)
        if (A.wnew.p[0] && interior) {
            // the new state, read back from output 0 (written above by this thread)
            double qn[NC];
#pragma unroll
            for (int v = 0; v < NC; ++v) qn[v] = plane_at(A.o[0].out, v, g)[idx];
            flux_recover<M>(A, qn, w, xi, yj, zk, img_xy, img);
        }
}

// One tile of the flux pass: single-fluid and ideal 2-D tiles with 64-wide rows use the
// wavefront-row form, everything else the LDS form (measured: for the two-fluid model the
// row form's extra live registers cost more than its saved LDS traffic: with the whole flux
// vectors formed up front and the x stencil read from neighbouring lanes, the 1024^2 sheet's
// pass took 238-257 us against 227 us, spilling 76-240 bytes per lane at 16 rows).  The
// two-fluid 2-D tile stages two variables per pair of barriers (239 against 253 us per pass
// on the 1024^2 sheet at 16 rows, 221 against 245 us at 12 rows; 64 against 67 us on 512^2),
// three in the 12-row tile, whose three rounds' arrays (147 KB) still fit the CU's LDS
// (1024^2 sheet 226 against 232 us per pass); measured no better in the two-fluid row form
// either (x stencil from neighbouring lanes, flux components formed per round: 236 us).
// NO: outputs used (o[0..NO-1]), fixed at compile time so unused ones cost no registers.
// RECOVER = false: the tile never recovers primitives (every pass but a step's last, except in
// the ideal model's explicit steps), so the recovery's registers are not reserved.  BQ: see
// base_terms.
template <int M, int NDIM, int BX, int BY, int NO, bool RECOVER = true, bool Z3 = false, bool BQ = false>
__device__ __forceinline__ void flux_tile(const FluxArgs &A, int bx, int by, long zoff = 0)
{
    static_assert(NO >= 1 && NO <= FLUX_MAXOUT, "outputs");
    if constexpr (M != 1 && NDIM == 2 && BX == 64) flux_tile_rows<M, BY, NO, RECOVER, Z3, BQ>(A, bx, by, zoff);
    else
        flux_tile_lds<M, NDIM, BX, BY, NO, (M == 1 && NDIM == 2) ? (BX * BY <= 768 ? 3 : 2) : (NDIM == 2 && BX == 32 ? 2 : 1), RECOVER, Z3,
                      BQ>(A, bx, by, zoff);
}

// Workgroups are dealt to the 8 XCDs in turn (linear id mod 8), each XCD with its own L2.
// Renumbering so that each XCD receives one contiguous run of tiles (row-major) keeps the
// halo rows that vertically adjacent tiles share inside one L2.  A bijection of the tiles.
__device__ __forceinline__ int xcd_order(int lin, int n)
{
    const int q = n >> 3, r = n & 7, x = lin & 7, slot = lin >> 3;
    return x * q + min(x, r) + slot;
}
// (Column-major tile order, which keeps vertically adjacent tiles and their shared halo rows
// together, measured slower: 265 against 232 us per pass on the two-fluid 1024^2 sheet.)
__device__ __forceinline__ void xcd_tile(int &bx, int &by)
{
    const int t = xcd_order(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    bx = t % gridDim.x;
    by = t / gridDim.x;
}

// The same over a 3-D grid of blocks (x fastest, then y, then z).
__device__ __forceinline__ void xcd_tile3(int &bx, int &by, int &bz)
{
    const int gxy = gridDim.x * gridDim.y;
    const int t = xcd_order((blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x, gxy * gridDim.z);
    bx = t % gridDim.x;
    by = (t % gxy) / gridDim.x;
    bz = t / gxy;
}

// Flux pass.  NDIM = 3: one 2-D tile of an interior z plane (blockIdx.z), forming
// out_k = base_k + c_kL (Lx + Ly + Lz) + c_kS Psi with Lz from k_flux_z (launched first).
template <int M, int NDIM, int BX, int BY, int NO, bool BQ = false>
__global__ __launch_bounds__(BX *BY) void k_flux(FluxArgs A)
{
    int bx = blockIdx.x, by = blockIdx.y;
    if constexpr (NDIM == 3) {
        int bz;
        xcd_tile3(bx, by, bz);
        flux_tile<M, 2, BX, BY, NO, NO == 1 || M == 2, true, BQ>(A, bx, by, (long)(bz + 2) * A.g.slab);
    } else {
        if constexpr (NDIM == 2) xcd_tile(bx, by);
        // only a step's last pass (one output) recovers primitives, except in the ideal
        // model's explicit steps, whose every pass does; the others reserve no registers for it
        flux_tile<M, NDIM, BX, BY, NO, NO == 1 || M == 2, false, BQ>(A, bx, by);
    }
}

// z term of a 3-D flux pass, before k_flux: Lz = -(H_{k+1/2} - H_{k-1/2}) / dz at every
// interior cell, from the split z fluxes reconstructed as in x and y, written to A.lz; the
// x-y tiles then add it to L and complete the outputs (ghost images in all three directions,
// recovery), so no output is read back and written again.  Blocks of 64 (x) x 16 (z) threads:
// one x row of one y row per wavefront, the z stencil through LDS with two halo planes on each
// side (12 interior planes per block, no x halo).  Every thread of the block reaches every
// barrier.
template <int M>
__global__ __launch_bounds__(1024) void k_flux_z(FluxArgs A)
{
    constexpr int NC = Model<M>::NC, NP = Model<M>::NP;
    constexpr int BX = 64, BZ = 16, TZ = BZ - 4, G = 2;
    __shared__ double sfp[G][BZ][BX], sfm[G][BZ][BX], shp[G][BZ][BX], shm[G][BZ][BX];
    const Geo &g = A.g;
    int bx, by, bz;
    xcd_tile3(bx, by, bz);
    const int tx = threadIdx.x, tz = threadIdx.y;
    const int ii = bx * BX + tx;        // interior column
    const int kk = bz * TZ + tz - 2;    // interior plane (two halo planes each side)
    const int i = min(ii + 2, g.nxg - 1);
    const int k = min(max(kk + 2, 0), g.nzg - 1);
    const long idx = (long)k * g.slab + (long)(by + 2) * g.pitch + i;

    double q[NC], w[NP], fz[NC];
#pragma unroll
    for (int v = 0; v < NC; ++v) q[v] = A.q.p[v][idx];
#pragma unroll
    for (int v = 0; v < NP; ++v) w[v] = plane_at(A.w, v, g)[idx];
    flux_z_m<M>(q, w, cell_sigma(A.P, idx), A.P, fz);

    const bool interior = ii < g.nx && tz >= 2 && tz < BZ - 2 && kk < g.nz;
    const bool do_z = tz >= 1 && tz <= BZ - 2;
#pragma unroll
    for (int v0 = 0; v0 < NC; v0 += G) {
#pragma unroll
        for (int c = 0; c < G; ++c) {
            const int v = v0 + c;
            if (v >= NC) break;
            sfp[c][tz][tx] = 0.5 * (fz[v] + q[v]);
            sfm[c][tz][tx] = 0.5 * (fz[v] - q[v]);
        }
        __syncthreads();
        if (do_z) {
#pragma unroll
            for (int c = 0; c < G; ++c) {
                if (v0 + c >= NC) break;
                double vp, vm;
                weno3_pair(sfp[c][tz - 1][tx], sfp[c][tz][tx], sfp[c][tz + 1][tx], sfm[c][tz + 1][tx], sfm[c][tz][tx],
                           sfm[c][tz - 1][tx], vp, vm);
                shp[c][tz][tx] = vp;
                shm[c][tz][tx] = vm;
            }
        }
        __syncthreads();
        if (interior) {
#pragma unroll
            for (int c = 0; c < G; ++c) {
                const int v = v0 + c;
                if (v >= NC) break;
                plane_at(A.lz, v, g)[idx] =
                    -((shp[c][tz][tx] + shm[c][tz + 1][tx]) - (shp[c][tz - 1][tx] + shm[c][tz][tx])) * g.idz;
            }
        }
        // sfp/sfm are rewritten only after every thread has passed the second barrier above,
        // shp/shm only after the next round's first barrier
    }
}

// ---------------------------------------------------------------------------------------
// host-side set-up shared by the single-grid and batched paths
// ---------------------------------------------------------------------------------------
// Sum the statistics slots into the public record.
static inline void stats_fold(const unsigned long long *raw, rmhd_stats *out)
{
    unsigned long long h[STATS_HIST + STATS_NHIST] = {};
    for (int sl = 0; sl < STATS_SLOTS; ++sl)
        for (int k = 0; k < STATS_HIST + STATS_NHIST; ++k) {
            const unsigned long long x = raw[sl * STATS_STRIDE + k];
            h[k] = k == 4 ? (x > h[k] ? x : h[k]) : h[k] + x;
        }
    out->stage_cells = (int64_t)h[0];
    out->newton_iters = (int64_t)h[1];
    out->c2p_iters = (int64_t)h[2];
    out->failures = (int32_t)h[3];
    out->newton_max = (int32_t)h[4];
    out->residual_evals = (int64_t)h[5];
    unsigned long long jac = 0;
    for (int sl = 0; sl < STATS_SLOTS; ++sl) jac += raw[sl * STATS_STRIDE + STATS_JAC];
    out->jacobian_evals = (int64_t)jac;
    for (int b = 0; b < STATS_NHIST; ++b) out->newton_hist[b] = (int64_t)h[STATS_HIST + b];
    unsigned long long g = 0;
    for (int sl = 0; sl < STATS_SLOTS; ++sl) g = raw[sl * STATS_STRIDE + STATS_RES] > g ? raw[sl * STATS_STRIDE + STATS_RES] : g;
    memcpy(&out->residual_max, &g, sizeof(double));
}
static inline void layout_from(const rmhd_params *p, rmhd_layout *out)
{
    out->nxg = p->nx + 4;
    out->nyg = p->ndim >= 2 ? p->ny + 4 : 1;
    out->nzg = p->ndim == 3 ? p->nz + 4 : 1;
    out->pitch = (out->nxg + 7) / 8 * 8;
    out->slab = out->pitch * out->nyg;
    out->plane = out->slab * out->nzg;
    out->ncons = p->model == RMHD_SINGLE_FLUID ? 14 : p->model == RMHD_TWO_FLUID ? 18 : 9;
    out->nprim = p->model == RMHD_TWO_FLUID ? 10 : 5;
}

static inline Geo geo_from(const rmhd_params *p, const rmhd_layout &L)
{
    Geo g{};
    g.nx = p->nx;
    g.ny = p->ndim >= 2 ? p->ny : 1;
    g.nz = p->ndim == 3 ? p->nz : 1;
    g.nxg = (int)L.nxg;
    g.nyg = (int)L.nyg;
    g.nzg = (int)L.nzg;
    g.rows = (int)(L.nyg * L.nzg);
    g.pitch = (int)L.pitch;
    g.slab = L.slab;
    g.ndim = p->ndim;
    g.bc = p->bc;
    g.plane = L.plane;
    g.idx = p->nx / (p->x1 - p->x0);
    g.idy = p->ndim >= 2 ? p->ny / (p->y1 - p->y0) : 0.0;
    g.idz = p->ndim == 3 ? p->nz / (p->z1 - p->z0) : 0.0;
    return g;
}

static inline Phys phys_from(const rmhd_params *p)
{
    Phys P{};
    P.gamma = p->gamma_eos;
    P.gk = (p->gamma_eos - 1.0) / p->gamma_eos;
    P.hk = p->gamma_eos / (p->gamma_eos - 1.0);
    P.sigma = p->sigma;
    P.sigma_cell = p->sigma_cell;
    P.mu1 = p->mu1;
    P.mu2 = p->mu2;
    P.kappa = p->kappa;
    P.c2p_tol = p->c2p_tol;
    P.newton_tol = p->newton_tol;
    P.max_c2p = p->max_c2p_iter;
    P.max_newton = p->max_newton_iter;
    P.friction_covariant = p->friction_covariant;
    P.c2p_fallback = p->c2p_primary_only ? 0 : 1;
    // Jacobian reuse after a step that cut the residual tenfold (measured on the two-fluid
    // 1024^2 sheet: Jacobians per cell and stage 1.39 -> 1.00 at the same Newton step count,
    // step 1.43 -> 1.24 ms; every first step there cuts it by more than tenfold)
    P.jac_keep = 0.1;
    return P;
}

static inline double cfl_dt(const rmhd_params *p)
{
    const double dx = (p->x1 - p->x0) / p->nx;
    if (p->ndim == 1) return p->cfl * dx;
    const double dy = (p->y1 - p->y0) / p->ny;
    if (p->ndim == 2) return p->cfl / (1.0 / dx + 1.0 / dy);
    const double dz = (p->z1 - p->z0) / p->nz;
    return p->cfl / (1.0 / dx + 1.0 / dy + 1.0 / dz);
}

}  // namespace rmhd
