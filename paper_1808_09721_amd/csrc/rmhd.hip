// rmhd.hip -- gfx950 kernels and the C ABI (include/rmhd.h) of the resistive single-fluid and
// two-fluid SRMHD SSP2(222) IMEX hot path (Wright & Hawke, arXiv:1808.09721).
//
// Kernels
//   k_init    prim -> cons on the interior, rho_e = div E (Sec. 2.1.1 Eq. 2; Sec. 2.1.2 Eq. 6)
//   k_bc      ghost fill (outflow copy / periodic wrap) of any set of planes
//   k_c2p     primitive recovery on every cell (Sec. 2.1.3)
//   k_stage   implicit-stage Newton solve per cell, ghosts included (Sec. 2.2.1 Eq. 10)
//   k_flux    FVS + WENO3 flux divergence L (Sec. 2.2.2 Eq. 12), fused with the SSP2 stage
//             combiners (Eqs. 10-11, Table 2) and with the ghost fill of its first output
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <new>
#include <string>

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

struct Geo {
    int nx, ny, nxg, nyg;
    int pitch, ndim, bc, pad_;
    long plane;
    double idx, idy;  // 1/dx, 1/dy
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

// components that carry a source term
__host__ __device__ constexpr bool has_source(int M, int v)
{
    return M == 0 ? (v == sf::EX || v == sf::EY || v == sf::EZ || v == sf::PSI || v == sf::PHI)
                  : (v == tf::SBX || v == tf::SBY || v == tf::SBZ || v == tf::TAUB || v == tf::EX ||
                     v == tf::EY || v == tf::EZ || v == tf::PSI || v == tf::PHI);
}

__device__ __forceinline__ bool is_interior(const Geo &g, int i, int j)
{
    return i >= 2 && i < g.nx + 2 && (g.ndim == 1 || (j >= 2 && j < g.ny + 2));
}

// padded index of the interior cell that a ghost (or interior) index copies
__device__ __forceinline__ int bc_src(int i, int n, int bc)
{
    if (i >= 2 && i < n + 2) return i;
    if (bc == RMHD_BC_PERIODIC) return i < 2 ? i + n : i - n;
    return i < 2 ? 2 : n + 1;
}

// ---------------------------------------------------------------------------------------
// ghost fill
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bc(Planes a, int nvar, Geo g)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t % g.pitch), j = (int)(t / g.pitch);
    if (i >= g.nxg || j >= g.nyg || is_interior(g, i, j)) return;
    const int si = bc_src(i, g.nx, g.bc);
    const int sj = g.ndim == 2 ? bc_src(j, g.ny, g.bc) : 0;
    const long d = (long)j * g.pitch + i, s = (long)sj * g.pitch + si;
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
    const int i = (int)(t % g.pitch), j = (int)(t / g.pitch);
    if (i >= g.nxg || j >= g.nyg || !is_interior(g, i, j)) return;
    const long idx = (long)j * g.pitch + i;
    double w[NP], eb[6], q[NC];
#pragma unroll
    for (int v = 0; v < NP; ++v) w[v] = prims.p[v][idx];
#pragma unroll
    for (int v = 0; v < 6; ++v) eb[v] = EB.p[v][idx];
    if constexpr (M == 0) {
        // Gauss's law rho_e = div E, central differences; neighbours through the boundary map
        const long xm = (long)j * g.pitch + bc_src(i - 1, g.nx, g.bc);
        const long xp = (long)j * g.pitch + bc_src(i + 1, g.nx, g.bc);
        double div = (EB.p[3][xp] - EB.p[3][xm]) * (0.5 * g.idx);
        if (g.ndim == 2) {
            const long ym = (long)bc_src(j - 1, g.ny, g.bc) * g.pitch + i;
            const long yp = (long)bc_src(j + 1, g.ny, g.bc) * g.pitch + i;
            div += (EB.p[4][yp] - EB.p[4][ym]) * (0.5 * g.idy);
        }
        sf_prim2cons(w, eb, div, P, q);
    } else {
        tf_prim2cons(w, eb, P, q);
    }
#pragma unroll
    for (int v = 0; v < NC; ++v) cons.p[v][idx] = q[v];
}

// ---------------------------------------------------------------------------------------
// primitive recovery
// ---------------------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(256) void k_c2p(CPlanes cons, Planes prims, int8_t *status, int32_t *iters, Geo g,
                                             Phys P)
{
    constexpr int NC = Model<M>::NC, NP = Model<M>::NP;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t % g.pitch), j = (int)(t / g.pitch);
    if (i >= g.nxg || j >= g.nyg) return;
    const long idx = (long)j * g.pitch + i;
    double q[NC], w[NP];
#pragma unroll
    for (int v = 0; v < NC; ++v) q[v] = cons.p[v][idx];
#pragma unroll
    for (int v = 0; v < NP; ++v) w[v] = prims.p[v][idx];
    int it = 0;
    const int st = M == 0 ? sf_cons2prim(q, w, P, it) : tf_cons2prim(q, w, P, it);
#pragma unroll
    for (int v = 0; v < NP; ++v) prims.p[v][idx] = w[v];
    if (status) status[idx] = (int8_t)st;
    if (iters) iters[idx] = it;
}

// ---------------------------------------------------------------------------------------
// implicit stage
// ---------------------------------------------------------------------------------------
// statistics counters: STATS_SLOTS slots of STATS_STRIDE (128 bytes) each, summed on read
constexpr int STATS_SLOTS = 64;
constexpr int STATS_STRIDE = 16;

struct StageArgs {
    CPlanes R, guess, win;
    Planes Q, wout;
    int8_t *status;
    int32_t *iters;
    unsigned long long *stats;  // [0] cells [1] newton [2] c2p [3] failures [4] newton max [5] residuals
    double a;
    Geo g;
    Phys P;
    int write_all;
    int use_guess;
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

template <int M>
__global__ __launch_bounds__(256) void k_stage(StageArgs A)
{
    constexpr int NC = Model<M>::NC, NP = Model<M>::NP, NX = Model<M>::NX;
    const Geo &g = A.g;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t % g.pitch), j = (int)(t / g.pitch);
    const bool live = i < g.nxg && j < g.nyg;
    int nit = 0, cit = 0, rit = 0, st = CELL_OK;
    if (live) {
        const long idx = (long)j * g.pitch + i;
        const double sig = cell_sigma(A.P, idx);
        double R[NC], w[NP], x[NX];
#pragma unroll
        for (int v = 0; v < NC; ++v) R[v] = A.R.p[v][idx];
#pragma unroll
        for (int v = 0; v < NP; ++v) w[v] = A.win.p[v][idx];
        const double aK = 1.0 / (1.0 + A.a * A.P.kappa);
        if constexpr (M == 0) {
            const CPlanes &X0 = A.use_guess ? A.guess : A.R;
            x[0] = X0.p[sf::EX][idx]; x[1] = X0.p[sf::EY][idx]; x[2] = X0.p[sf::EZ][idx];
            st = sf_stage(R, A.a, sig, A.P, x, w, nit, cit, rit);
            A.Q.p[sf::EX][idx] = x[0]; A.Q.p[sf::EY][idx] = x[1]; A.Q.p[sf::EZ][idx] = x[2];
            A.Q.p[sf::PHI][idx] = R[sf::PHI] * aK;
            A.Q.p[sf::PSI][idx] = (R[sf::PSI] + A.a * R[sf::RHOE]) * aK;
        } else {
            const CPlanes &X0 = A.use_guess ? A.guess : A.R;
            const double isc = 1.0 / fabs(A.P.mu1);
            x[0] = X0.p[tf::SBX][idx] * isc; x[1] = X0.p[tf::SBY][idx] * isc; x[2] = X0.p[tf::SBZ][idx] * isc;
            x[3] = X0.p[tf::TAUB][idx] * isc;
            x[4] = X0.p[tf::EX][idx]; x[5] = X0.p[tf::EY][idx]; x[6] = X0.p[tf::EZ][idx];
            st = tf_stage(R, A.a, sig, A.P, x, w, nit, cit, rit);
            const double sc = fabs(A.P.mu1);
            A.Q.p[tf::SBX][idx] = x[0] * sc; A.Q.p[tf::SBY][idx] = x[1] * sc; A.Q.p[tf::SBZ][idx] = x[2] * sc;
            A.Q.p[tf::TAUB][idx] = x[3] * sc;
            A.Q.p[tf::EX][idx] = x[4]; A.Q.p[tf::EY][idx] = x[5]; A.Q.p[tf::EZ][idx] = x[6];
            A.Q.p[tf::PHI][idx] = R[tf::PHI] * aK;
            A.Q.p[tf::PSI][idx] = (R[tf::PSI] + A.a * R[tf::DB]) * aK;
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
    if (A.stats) {
        // block reduction (wave shuffles, then LDS), one atomic per counter per block, spread
        // over STATS_SLOTS padded slots so blocks rarely contend on one address
        __shared__ unsigned long long red[4][6];
        const bool counted = live && is_interior(g, i, j);
        unsigned long long v[6] = {counted ? 1ull : 0ull, counted ? (unsigned long long)nit : 0ull,
                                   counted ? (unsigned long long)cit : 0ull,
                                   counted && st != CELL_OK ? 1ull : 0ull, 0ull,
                                   counted ? (unsigned long long)rit : 0ull};
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] = k == 4 ? (unsigned long long)wave_max(counted ? nit : 0) : wave_sum(v[k]);
        const int wave = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0)
#pragma unroll
            for (int k = 0; k < 6; ++k) red[wave][k] = v[k];
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t[6] = {0, 0, 0, 0, 0, 0};
            for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv)
#pragma unroll
                for (int k = 0; k < 6; ++k) t[k] = k == 4 ? max(t[k], red[wv][k]) : t[k] + red[wv][k];
            if (t[0]) {
                unsigned long long *slot = A.stats + (blockIdx.x % STATS_SLOTS) * STATS_STRIDE;
                atomicAdd(&slot[0], t[0]);
                atomicAdd(&slot[1], t[1]);
                atomicAdd(&slot[2], t[2]);
                if (t[3]) atomicAdd(&slot[3], t[3]);
                atomicMax(&slot[4], t[4]);
                atomicAdd(&slot[5], t[5]);
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// flux pass: FVS + WENO3 and the fused stage combiners
// ---------------------------------------------------------------------------------------
struct FluxArgs {
    CPlanes q, w, base;   // base.p[0] == nullptr: no base term
    Planes out0, out1;    // out1.p[0] == nullptr: one output
    double c0L, c0S, c1L, c1S;  // out_k = base + ckL L + ckS Psi
    Geo g;
    Phys P;
    int fuse_bc;          // also write the ghost images of out0
};

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

template <int M, int NDIM, int BX, int BY>
__global__ __launch_bounds__(BX *BY) void k_flux(FluxArgs A)
{
    constexpr int NC = Model<M>::NC, NP = Model<M>::NP;
    constexpr int TX = BX - 4, TY = NDIM == 2 ? BY - 4 : 1;
    // split fluxes f+ / f- per direction, then the half reconstructions: cell i holds
    // f+ at its right face (i+1/2) and f- at its left face (i-1/2)
    __shared__ double sfp[NDIM][BY][BX], sfm[NDIM][BY][BX];
    __shared__ double shp[NDIM][BY][BX], shm[NDIM][BY][BX];
    const Geo &g = A.g;
    const int tx = threadIdx.x, ty = NDIM == 2 ? threadIdx.y : 0;
    const int ii = blockIdx.x * TX + tx - 2;
    const int jj = NDIM == 2 ? (int)blockIdx.y * TY + ty - 2 : 0;
    const int i = min(max(ii + 2, 0), g.nxg - 1);
    const int j = NDIM == 2 ? min(max(jj + 2, 0), g.nyg - 1) : 0;
    const long idx = (long)j * g.pitch + i;

    double q[NC], w[NP], fx[NC], fy[NC], src[NC];
#pragma unroll
    for (int v = 0; v < NC; ++v) q[v] = A.q.p[v][idx];
#pragma unroll
    for (int v = 0; v < NP; ++v) w[v] = A.w.p[v][idx];
    const double sig = cell_sigma(A.P, idx);
    if constexpr (M == 0) sf_flux_source(q, w, sig, A.P, fx, fy, src);
    else tf_flux_source(q, w, sig, A.P, fx, fy, src);

    const bool interior = tx >= 2 && tx < BX - 2 && ii < g.nx &&
                          (NDIM == 1 || (ty >= 2 && ty < BY - 2 && jj < g.ny));
    const bool do_x = tx >= 1 && tx <= BX - 2 && (NDIM == 1 || (ty >= 2 && ty <= BY - 3));
    const bool do_y = NDIM == 2 && ty >= 1 && ty <= BY - 2 && tx >= 2 && tx <= BX - 3;

    // ghost images of this interior cell (fused boundary fill of out0)
    int xi[3] = {i, -1, -1}, yj[3] = {j, -1, -1};
    if (A.fuse_bc && interior) {
        if (g.bc == RMHD_BC_PERIODIC) {
            if (ii < 2) xi[1] = i + g.nx;
            if (ii >= g.nx - 2) xi[2] = i - g.nx;
            if (NDIM == 2) {
                if (jj < 2) yj[1] = j + g.ny;
                if (jj >= g.ny - 2) yj[2] = j - g.ny;
            }
        } else {
            if (ii == 0) { xi[1] = 0; xi[2] = 1; }
            if (ii == g.nx - 1) { xi[1] = g.nx + 2; xi[2] = g.nx + 3; }
            if (NDIM == 2) {
                if (jj == 0) { yj[1] = 0; yj[2] = 1; }
                if (jj == g.ny - 1) { yj[1] = g.ny + 2; yj[2] = g.ny + 3; }
            }
        }
    }
    const bool has_base = A.base.p[0] != nullptr, two_out = A.out1.p[0] != nullptr;

#pragma unroll
    for (int v = 0; v < NC; ++v) {
        sfp[0][ty][tx] = 0.5 * (fx[v] + q[v]);
        sfm[0][ty][tx] = 0.5 * (fx[v] - q[v]);
        if constexpr (NDIM == 2) {
            sfp[NDIM - 1][ty][tx] = 0.5 * (fy[v] + q[v]);
            sfm[NDIM - 1][ty][tx] = 0.5 * (fy[v] - q[v]);
        }
        __syncthreads();
        if (do_x) {
            double vp, vm;
            weno3_pair(sfp[0][ty][tx - 1], sfp[0][ty][tx], sfp[0][ty][tx + 1], sfm[0][ty][tx + 1], sfm[0][ty][tx],
                       sfm[0][ty][tx - 1], vp, vm);
            shp[0][ty][tx] = vp;
            shm[0][ty][tx] = vm;
        }
        if constexpr (NDIM == 2) {
            if (do_y) {
                double vp, vm;
                weno3_pair(sfp[NDIM - 1][ty - 1][tx], sfp[NDIM - 1][ty][tx], sfp[NDIM - 1][ty + 1][tx],
                           sfm[NDIM - 1][ty + 1][tx], sfm[NDIM - 1][ty][tx], sfm[NDIM - 1][ty - 1][tx], vp, vm);
                shp[NDIM - 1][ty][tx] = vp;
                shm[NDIM - 1][ty][tx] = vm;
            }
        }
        __syncthreads();
        if (interior) {
            double L = -((shp[0][ty][tx] + shm[0][ty][tx + 1]) - (shp[0][ty][tx - 1] + shm[0][ty][tx])) * g.idx;
            if constexpr (NDIM == 2)
                L -= ((shp[NDIM - 1][ty][tx] + shm[NDIM - 1][ty + 1][tx]) -
                      (shp[NDIM - 1][ty - 1][tx] + shm[NDIM - 1][ty][tx])) * g.idy;
            const double S = has_source(M, v) ? src[v] : 0.0;
            const double b = has_base ? A.base.p[v][idx] : 0.0;
            const double o0 = b + A.c0L * L + A.c0S * S;
#pragma unroll
            for (int aa = 0; aa < 3; ++aa)
#pragma unroll
                for (int bb = 0; bb < (NDIM == 2 ? 3 : 1); ++bb)
                    if (xi[aa] >= 0 && yj[bb] >= 0) A.out0.p[v][(long)yj[bb] * g.pitch + xi[aa]] = o0;
            if (two_out) A.out1.p[v][idx] = b + A.c1L * L + A.c1S * S;
        }
    }
}

}  // namespace rmhd

// =======================================================================================
// host side
// =======================================================================================
using namespace rmhd;

struct rmhd_ctx {
    rmhd_params prm;
    rmhd_layout lay;
    hipStream_t stream;
    Geo geo;
    Phys phys;
    int device;
    // scratch owned by the library
    double *q1src;    // stage-1 source-carrying components (NX + 2 planes)
    double *w1;       // stage-1 primitives (nprim planes)
    double *r2;       // stage-2 right-hand side, solved in place (ncons planes)
    double *acc;      // q^n + dt/2 [L(Q1) + Psi(Q1)] (ncons planes)
    int8_t *status;   // one plane
    int32_t *iters;   // one plane
    unsigned long long *stats;  // STATS_SLOTS x STATS_STRIDE counters
    // per-kernel event timing of rmhd_imex_step
    int timing;
    hipEvent_t ev[10];
    rmhd_timing times;
    std::string err;
};

static std::string g_err;  // errors before a context exists

static int fail(rmhd_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    else g_err = msg;
    return code;
}

static int hip_check(rmhd_ctx *c, hipError_t e, const char *what)
{
    if (e == hipSuccess) return RMHD_OK;
    return fail(c, RMHD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

static int check_params(const rmhd_params *p, rmhd_ctx *c)
{
    if (!p) return fail(c, RMHD_EINVAL, "params is NULL");
    if (p->model != RMHD_SINGLE_FLUID && p->model != RMHD_TWO_FLUID) return fail(c, RMHD_EINVAL, "model must be 0 or 1");
    if (p->ndim != 1 && p->ndim != 2) return fail(c, RMHD_EINVAL, "ndim must be 1 or 2");
    if (p->nx < 4 || (p->ndim == 2 && p->ny < 4) || (p->ndim == 1 && p->ny != 1))
        return fail(c, RMHD_EINVAL, "need nx >= 4 (and ny >= 4 in 2-D, ny == 1 in 1-D)");
    if ((long)p->nx * (p->ndim == 2 ? p->ny : 1) > (1l << 30)) return fail(c, RMHD_EINVAL, "grid too large");
    if (p->bc != RMHD_BC_OUTFLOW && p->bc != RMHD_BC_PERIODIC) return fail(c, RMHD_EINVAL, "bc must be 0 or 1");
    if (!(p->x1 > p->x0) || (p->ndim == 2 && !(p->y1 > p->y0))) return fail(c, RMHD_EINVAL, "empty domain");
    if (!(p->gamma_eos > 1.0 && p->gamma_eos <= 2.0)) return fail(c, RMHD_EINVAL, "gamma_eos must lie in (1, 2]");
    if (p->model == RMHD_TWO_FLUID && !(p->mu1 != p->mu2 && p->mu1 != 0.0))
        return fail(c, RMHD_EINVAL, "two-fluid model needs mu1 != mu2 and mu1 != 0");
    if (p->model == RMHD_TWO_FLUID && !p->sigma_cell && !(p->sigma > 0.0))
        return fail(c, RMHD_EINVAL, "two-fluid model needs sigma > 0 (eta = 1/sigma)");
    if (p->max_c2p_iter < 1 || p->max_newton_iter < 1) return fail(c, RMHD_EINVAL, "iteration caps must be >= 1");
    if (!(p->c2p_tol > 0.0) || !(p->newton_tol > 0.0)) return fail(c, RMHD_EINVAL, "tolerances must be > 0");
    return RMHD_OK;
}

extern "C" int rmhd_layout_of(const rmhd_params *p, rmhd_layout *out)
{
    int rc = check_params(p, nullptr);
    if (rc) return rc;
    if (!out) return fail(nullptr, RMHD_EINVAL, "out is NULL");
    out->nxg = p->nx + 4;
    out->nyg = p->ndim == 2 ? p->ny + 4 : 1;
    out->pitch = (out->nxg + 7) / 8 * 8;
    out->plane = out->pitch * out->nyg;
    out->ncons = p->model == RMHD_SINGLE_FLUID ? 14 : 18;
    out->nprim = p->model == RMHD_SINGLE_FLUID ? 5 : 10;
    return RMHD_OK;
}

static Planes planes_of(double *base, const rmhd_layout &L, int n)
{
    Planes P{};
    for (int v = 0; v < n; ++v) P.p[v] = base + v * L.plane;
    return P;
}
static CPlanes cplanes_of(const double *base, const rmhd_layout &L, int n)
{
    CPlanes P{};
    for (int v = 0; v < n; ++v) P.p[v] = base + v * L.plane;
    return P;
}
static CPlanes as_const(const Planes &a)
{
    CPlanes c{};
    for (int v = 0; v < 18; ++v) c.p[v] = a.p[v];
    return c;
}

extern "C" int rmhd_create(const rmhd_params *p, void *stream, rmhd_ctx **out)
{
    if (!out) return fail(nullptr, RMHD_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_params(p, nullptr);
    if (rc) return rc;
    rmhd_ctx *c = new (std::nothrow) rmhd_ctx();
    if (!c) return fail(nullptr, RMHD_ENOMEM, "host allocation failed");
    c->prm = *p;
    rmhd_layout_of(p, &c->lay);
    c->stream = (hipStream_t)stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(nullptr, RMHD_EHIP, "no HIP device");
    }
    const rmhd_layout &L = c->lay;
    c->geo.nx = p->nx;
    c->geo.ny = p->ndim == 2 ? p->ny : 1;
    c->geo.nxg = (int)L.nxg;
    c->geo.nyg = (int)L.nyg;
    c->geo.pitch = (int)L.pitch;
    c->geo.ndim = p->ndim;
    c->geo.bc = p->bc;
    c->geo.plane = L.plane;
    c->geo.idx = p->nx / (p->x1 - p->x0);
    c->geo.idy = p->ndim == 2 ? p->ny / (p->y1 - p->y0) : 0.0;
    Phys &P = c->phys;
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
    const size_t pl = (size_t)L.plane * sizeof(double);
    const int nsrc = p->model == RMHD_SINGLE_FLUID ? 5 : 9;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc((void **)&c->q1src, pl * nsrc);
    if (e == hipSuccess) e = hipMalloc((void **)&c->w1, pl * L.nprim);
    if (e == hipSuccess) e = hipMalloc((void **)&c->r2, pl * L.ncons);
    if (e == hipSuccess) e = hipMalloc((void **)&c->acc, pl * L.ncons);
    if (e == hipSuccess) e = hipMalloc((void **)&c->status, (size_t)L.plane);
    if (e == hipSuccess) e = hipMalloc((void **)&c->iters, (size_t)L.plane * sizeof(int32_t));
    const size_t stats_bytes = (size_t)STATS_SLOTS * STATS_STRIDE * sizeof(unsigned long long);
    if (e == hipSuccess) e = hipMalloc((void **)&c->stats, stats_bytes);
    if (e == hipSuccess) e = hipMemsetAsync(c->stats, 0, stats_bytes, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        std::string m = std::string("scratch allocation: ") + hipGetErrorString(e);
        rmhd_destroy(c);
        return fail(nullptr, e == hipErrorOutOfMemory ? RMHD_ENOMEM : RMHD_EHIP, m);
    }
    *out = c;
    return RMHD_OK;
}

extern "C" void rmhd_destroy(rmhd_ctx *c)
{
    if (!c) return;
    if (c->timing)
        for (int k = 0; k < 10; ++k) hipEventDestroy(c->ev[k]);
    hipFree(c->q1src);
    hipFree(c->w1);
    hipFree(c->r2);
    hipFree(c->acc);
    hipFree(c->status);
    hipFree(c->iters);
    hipFree(c->stats);
    delete c;
}

static dim3 cells_grid(const rmhd_ctx *c) { return dim3((unsigned)((c->lay.plane + 255) / 256)); }

static int launch_bc(rmhd_ctx *c, double *arr, int nvar)
{
    hipLaunchKernelGGL(k_bc, cells_grid(c), dim3(256), 0, c->stream, planes_of(arr, c->lay, nvar), nvar, c->geo);
    return hip_check(c, hipGetLastError(), "k_bc launch");
}

static int launch_stage(rmhd_ctx *c, const StageArgs &A)
{
    if (c->prm.model == RMHD_SINGLE_FLUID)
        hipLaunchKernelGGL(k_stage<0>, cells_grid(c), dim3(256), 0, c->stream, A);
    else
        hipLaunchKernelGGL(k_stage<1>, cells_grid(c), dim3(256), 0, c->stream, A);
    return hip_check(c, hipGetLastError(), "k_stage launch");
}

template <int M>
static void launch_flux_m(rmhd_ctx *c, const FluxArgs &A)
{
    if (c->prm.ndim == 1) {
        constexpr int BX = 256;
        dim3 grid((c->prm.nx + (BX - 4) - 1) / (BX - 4));
        hipLaunchKernelGGL((k_flux<M, 1, BX, 1>), grid, dim3(BX, 1), 0, c->stream, A);
    } else {
        constexpr int BX = 64, BY = 16;
        dim3 grid((c->prm.nx + (BX - 4) - 1) / (BX - 4), (c->prm.ny + (BY - 4) - 1) / (BY - 4));
        hipLaunchKernelGGL((k_flux<M, 2, BX, BY>), grid, dim3(BX, BY), 0, c->stream, A);
    }
}

static int launch_flux(rmhd_ctx *c, const FluxArgs &A)
{
    if (c->prm.model == RMHD_SINGLE_FLUID) launch_flux_m<0>(c, A);
    else launch_flux_m<1>(c, A);
    return hip_check(c, hipGetLastError(), "k_flux launch");
}

extern "C" int rmhd_init_state(rmhd_ctx *c, const double *prims, const double *EB, double *cons)
{
    if (!c || !prims || !EB || !cons) return fail(c, RMHD_EINVAL, "rmhd_init_state: NULL argument");
    const rmhd_layout &L = c->lay;
    if (c->prm.model == RMHD_SINGLE_FLUID)
        hipLaunchKernelGGL(k_init<0>, cells_grid(c), dim3(256), 0, c->stream, cplanes_of(prims, L, L.nprim),
                           cplanes_of(EB, L, 6), planes_of(cons, L, L.ncons), c->geo, c->phys);
    else
        hipLaunchKernelGGL(k_init<1>, cells_grid(c), dim3(256), 0, c->stream, cplanes_of(prims, L, L.nprim),
                           cplanes_of(EB, L, 6), planes_of(cons, L, L.ncons), c->geo, c->phys);
    int rc = hip_check(c, hipGetLastError(), "k_init launch");
    if (rc) return rc;
    return launch_bc(c, cons, L.ncons);
}

extern "C" int rmhd_cons2prim(rmhd_ctx *c, const double *cons, double *prims, int8_t *status, int32_t *iters)
{
    if (!c || !cons || !prims) return fail(c, RMHD_EINVAL, "rmhd_cons2prim: NULL argument");
    const rmhd_layout &L = c->lay;
    if (c->prm.model == RMHD_SINGLE_FLUID)
        hipLaunchKernelGGL(k_c2p<0>, cells_grid(c), dim3(256), 0, c->stream, cplanes_of(cons, L, L.ncons),
                           planes_of(prims, L, L.nprim), status, iters, c->geo, c->phys);
    else
        hipLaunchKernelGGL(k_c2p<1>, cells_grid(c), dim3(256), 0, c->stream, cplanes_of(cons, L, L.ncons),
                           planes_of(prims, L, L.nprim), status, iters, c->geo, c->phys);
    return hip_check(c, hipGetLastError(), "k_c2p launch");
}

extern "C" int rmhd_F(rmhd_ctx *c, double *cons, double *prims, double *Lout)
{
    if (!c || !cons || !prims || !Lout) return fail(c, RMHD_EINVAL, "rmhd_F: NULL argument");
    const rmhd_layout &L = c->lay;
    int rc = launch_bc(c, cons, L.ncons);
    if (!rc) rc = launch_bc(c, prims, L.nprim);
    if (rc) return rc;
    FluxArgs A{};
    A.q = cplanes_of(cons, L, L.ncons);
    A.w = cplanes_of(prims, L, L.nprim);
    A.out0 = planes_of(Lout, L, L.ncons);
    A.c0L = 1.0;
    A.g = c->geo;
    A.P = c->phys;
    return launch_flux(c, A);
}

extern "C" int rmhd_implicit_stage(rmhd_ctx *c, double a, const double *R, const double *guess, double *Q,
                                   double *prims, int8_t *status, int32_t *iters)
{
    if (!c || !R || !Q || !prims) return fail(c, RMHD_EINVAL, "rmhd_implicit_stage: NULL argument");
    if (!(a >= 0.0)) return fail(c, RMHD_EINVAL, "rmhd_implicit_stage: a must be >= 0");
    const rmhd_layout &L = c->lay;
    StageArgs A{};
    A.R = cplanes_of(R, L, L.ncons);
    if (guess) A.guess = cplanes_of(guess, L, L.ncons);
    A.use_guess = guess != nullptr;
    A.win = cplanes_of(prims, L, L.nprim);
    A.wout = planes_of(prims, L, L.nprim);
    A.Q = planes_of(Q, L, L.ncons);
    A.status = status;
    A.iters = iters;
    A.stats = c->stats;
    A.a = a;
    A.g = c->geo;
    A.P = c->phys;
    A.write_all = Q != R;
    return launch_stage(c, A);
}

extern "C" int rmhd_imex_step(rmhd_ctx *c, double dt, double *cons, double *prims)
{
    if (!c || !cons || !prims) return fail(c, RMHD_EINVAL, "rmhd_imex_step: NULL argument");
    if (!(dt > 0.0)) return fail(c, RMHD_EINVAL, "rmhd_imex_step: dt must be > 0");
    const rmhd_layout &L = c->lay;
    const double gm = 1.0 - 1.0 / sqrt(2.0);
    const int M = c->prm.model;
    // Q1: the source-free components are those of q^n; the others live in scratch
    Planes Q1 = planes_of(cons, L, L.ncons);
    {
        int k = 0;
        for (int v = 0; v < L.ncons; ++v)
            if (has_source(M, v)) Q1.p[v] = c->q1src + (k++) * L.plane;
    }
    // stage 1: Q1 = q^n + gamma dt Psi(Q1)
    StageArgs S{};
    S.R = cplanes_of(cons, L, L.ncons);
    S.win = cplanes_of(prims, L, L.nprim);
    S.wout = planes_of(c->w1, L, L.nprim);
    S.Q = Q1;
    S.status = c->status;
    S.iters = c->iters;
    S.stats = c->stats;
    S.a = gm * dt;
    S.g = c->geo;
    S.P = c->phys;
    S.write_all = 0;
    auto mark = [&](int k) {
        if (c->timing) hipEventRecord(c->ev[k], c->stream);
    };
    mark(0);
    int rc = launch_stage(c, S);
    mark(1);
    if (rc) return rc;
    // R2 = q^n + dt L(Q1) + (1 - 2 gamma) dt Psi(Q1);  ACC = q^n + dt/2 L(Q1) + dt/2 Psi(Q1)
    FluxArgs F{};
    F.q = as_const(Q1);
    F.w = cplanes_of(c->w1, L, L.nprim);
    F.base = cplanes_of(cons, L, L.ncons);
    F.out0 = planes_of(c->r2, L, L.ncons);
    F.out1 = planes_of(c->acc, L, L.ncons);
    F.c0L = dt;
    F.c0S = (1.0 - 2.0 * gm) * dt;
    F.c1L = 0.5 * dt;
    F.c1S = 0.5 * dt;
    F.g = c->geo;
    F.P = c->phys;
    F.fuse_bc = 1;
    mark(2);
    rc = launch_flux(c, F);
    mark(3);
    if (rc) return rc;
    // stage 2: Q2 = R2 + gamma dt Psi(Q2), in place; primitives into the caller's array
    S.R = cplanes_of(c->r2, L, L.ncons);
    S.win = cplanes_of(c->w1, L, L.nprim);
    S.wout = planes_of(prims, L, L.nprim);
    S.Q = planes_of(c->r2, L, L.ncons);
    mark(4);
    rc = launch_stage(c, S);
    mark(5);
    if (rc) return rc;
    // q^{n+1} = ACC + dt/2 L(Q2) + dt/2 Psi(Q2), ghosts included
    F.q = cplanes_of(c->r2, L, L.ncons);
    F.w = cplanes_of(prims, L, L.nprim);
    F.base = cplanes_of(c->acc, L, L.ncons);
    F.out0 = planes_of(cons, L, L.ncons);
    F.out1 = Planes{};
    F.c0L = 0.5 * dt;
    F.c0S = 0.5 * dt;
    mark(6);
    rc = launch_flux(c, F);
    mark(7);
    if (rc) return rc;
    // primitives of q^{n+1} (starting from those of Q2)
    mark(8);
    rc = rmhd_cons2prim(c, cons, prims, nullptr, nullptr);
    mark(9);
    if (rc || !c->timing) return rc;
    rc = hip_check(c, hipEventSynchronize(c->ev[9]), "timing sync");
    if (rc) return rc;
    float ms[5];
    for (int k = 0; k < 5; ++k) hipEventElapsedTime(&ms[k], c->ev[2 * k], c->ev[2 * k + 1]);
    c->times.stage_ms += ms[0] + ms[2];
    c->times.flux_ms += ms[1] + ms[3];
    c->times.c2p_ms += ms[4];
    c->times.stage_launches += 2;
    c->times.flux_launches += 2;
    c->times.c2p_launches += 1;
    c->times.steps += 1;
    return RMHD_OK;
}

extern "C" int rmhd_set_timing(rmhd_ctx *c, int enable)
{
    if (!c) return fail(c, RMHD_EINVAL, "rmhd_set_timing: NULL context");
    if (enable && !c->timing) {
        for (int k = 0; k < 10; ++k) {
            int rc = hip_check(c, hipEventCreate(&c->ev[k]), "hipEventCreate");
            if (rc) {
                for (int m = 0; m < k; ++m) hipEventDestroy(c->ev[m]);
                return rc;
            }
        }
        c->timing = 1;
    } else if (!enable && c->timing) {
        hipStreamSynchronize(c->stream);
        for (int k = 0; k < 10; ++k) hipEventDestroy(c->ev[k]);
        c->timing = 0;
    }
    return RMHD_OK;
}

extern "C" int rmhd_get_timing(rmhd_ctx *c, rmhd_timing *out, int reset)
{
    if (!c || !out) return fail(c, RMHD_EINVAL, "rmhd_get_timing: NULL argument");
    int rc = hip_check(c, hipStreamSynchronize(c->stream), "timing sync");
    if (rc) return rc;
    *out = c->times;
    if (reset) c->times = rmhd_timing{};
    return RMHD_OK;
}

extern "C" double rmhd_dt(const rmhd_ctx *c)
{
    if (!c) return 0.0;
    const double dx = (c->prm.x1 - c->prm.x0) / c->prm.nx;
    if (c->prm.ndim == 1) return c->prm.cfl * dx;
    const double dy = (c->prm.y1 - c->prm.y0) / c->prm.ny;
    return c->prm.cfl / (1.0 / dx + 1.0 / dy);
}

extern "C" int rmhd_get_stats(rmhd_ctx *c, rmhd_stats *out, int reset)
{
    if (!c || !out) return fail(c, RMHD_EINVAL, "rmhd_get_stats: NULL argument");
    unsigned long long raw[STATS_SLOTS * STATS_STRIDE], h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int rc = hip_check(c, hipMemcpyAsync(raw, c->stats, sizeof(raw), hipMemcpyDeviceToHost, c->stream), "stats copy");
    if (!rc && reset) rc = hip_check(c, hipMemsetAsync(c->stats, 0, sizeof(raw), c->stream), "stats reset");
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "stats sync");
    if (rc) return rc;
    for (int sl = 0; sl < STATS_SLOTS; ++sl)
        for (int k = 0; k < 6; ++k) {
            const unsigned long long x = raw[sl * STATS_STRIDE + k];
            h[k] = k == 4 ? (x > h[k] ? x : h[k]) : h[k] + x;
        }
    out->stage_cells = (int64_t)h[0];
    out->newton_iters = (int64_t)h[1];
    out->c2p_iters = (int64_t)h[2];
    out->failures = (int32_t)h[3];
    out->newton_max = (int32_t)h[4];
    out->residual_evals = (int64_t)h[5];
    return RMHD_OK;
}

extern "C" const char *rmhd_last_error(const rmhd_ctx *c) { return c ? c->err.c_str() : g_err.c_str(); }
