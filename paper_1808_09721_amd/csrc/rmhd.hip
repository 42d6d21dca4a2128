// rmhd.hip -- C ABI (include/rmhd.h) of the single-grid resistive single-fluid and two-fluid
// SRMHD SSP2(222) IMEX hot path (Wright & Hawke, arXiv:1808.09721); kernels in kernels.hpp.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "kernels.hpp"
#include "mlp.hpp"

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
    int cus;          // compute units of the device
    // scratch owned by the library
    double *q1src;    // stage-1 source-carrying components (NX + 2 planes)
    double *w1;       // stage-1 primitives (nprim planes)
    double *r2;       // stage-2 right-hand side, solved in place (ncons planes)
    double *acc;      // q^n + sum_j w_j dt [L(Q_j) + Psi(Q_j)], accumulated (ncons planes)
    double *r3, *w2;  // SSP3(332): third-stage right-hand side, solved in place (ncons planes);
                      // second-stage primitives (nprim planes)
    double *lz;       // 3-D: the z term of a flux pass (ncons planes)
    int8_t *status;   // one plane
    int32_t *iters;   // one plane
    unsigned long long *stats;  // STATS_SLOTS x STATS_STRIDE counters
    unsigned long long *wstats; // nwslots x STATS_WAVE per-wavefront counters (folded on read)
    long nwslots;
    // per-cell conductivity: the library's own copy of the caller's plane, ghosts filled
    double *sigma_own;
    // learned starting guess (two fluid): network, and the seven planes it writes
    const rmhd_mlp *mlp;
    double *guess;
    // harvest of (features, target) rows
    float *hx, *ht;
    long hcap, hcount;
    // flux tile rows (0 = default); detailed statistics (histogram, largest residual)
    int flux_rows, stats_detail;
    // convergence-compacted queue of the implicit stage (one entry per cell at most)
    int cap;
    int *qidx, *qit;
    double *qx, *qp;
    unsigned *qcount;
    // the step captured in a HIP graph (rmhd_set_graph), keyed by its arguments
    int use_graph;
    hipStream_t gstream;
    hipGraph_t graph;
    hipGraphExec_t exec;
    double g_dt;
    double *g_cons, *g_prims;
    // per-kernel event timing of rmhd_imex_step
    int timing;
    hipEvent_t ev[14];
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

static int check_params_impl(const rmhd_params *p, rmhd_ctx *c)
{
    if (!p) return fail(c, RMHD_EINVAL, "params is NULL");
    if (p->model != RMHD_SINGLE_FLUID && p->model != RMHD_TWO_FLUID && p->model != RMHD_IDEAL)
        return fail(c, RMHD_EINVAL, "model must be 0, 1 or 2");
    if (p->ndim < 1 || p->ndim > 3) return fail(c, RMHD_EINVAL, "ndim must be 1, 2 or 3");
    if (p->nx < 4 || (p->ndim >= 2 && p->ny < 4) || (p->ndim == 1 && p->ny != 1))
        return fail(c, RMHD_EINVAL, "need nx >= 4 (and ny >= 4 in 2-D and 3-D, ny == 1 in 1-D)");
    if ((p->ndim == 3 && p->nz < 4) || (p->ndim < 3 && p->nz != 0 && p->nz != 1))
        return fail(c, RMHD_EINVAL, "need nz >= 4 in 3-D (nz 0 or 1 below 3-D)");
    if (p->ndim == 3 && (p->ny > 65535 || p->nz > 65535)) return fail(c, RMHD_EINVAL, "3-D: ny, nz <= 65535");
    if (p->reserved_ != 0) return fail(c, RMHD_EINVAL, "reserved_ must be 0");
    if ((long)p->nx * (p->ndim >= 2 ? p->ny : 1) * (p->ndim == 3 ? p->nz : 1) > (1l << 30) ||
        (long)(p->nx + 4) * (p->ndim >= 2 ? p->ny + 4 : 1) * (p->ndim == 3 ? p->nz + 4 : 1) >= (1l << 31))
        return fail(c, RMHD_EINVAL, "grid too large");
    if (p->bc != RMHD_BC_OUTFLOW && p->bc != RMHD_BC_PERIODIC) return fail(c, RMHD_EINVAL, "bc must be 0 or 1");
    if (!(p->x1 > p->x0) || (p->ndim >= 2 && !(p->y1 > p->y0)) || (p->ndim == 3 && !(p->z1 > p->z0)))
        return fail(c, RMHD_EINVAL, "empty domain");
    if (!(p->gamma_eos > 1.0 && p->gamma_eos <= 2.0)) return fail(c, RMHD_EINVAL, "gamma_eos must lie in (1, 2]");
    if (p->model == RMHD_TWO_FLUID && !(p->mu1 != p->mu2 && p->mu1 != 0.0))
        return fail(c, RMHD_EINVAL, "two-fluid model needs mu1 != mu2 and mu1 != 0");
    if (p->model == RMHD_TWO_FLUID && !p->sigma_cell && !(p->sigma > 0.0))
        return fail(c, RMHD_EINVAL, "two-fluid model needs sigma > 0 (eta = 1/sigma)");
    if (p->max_c2p_iter < 1 || p->max_newton_iter < 1) return fail(c, RMHD_EINVAL, "iteration caps must be >= 1");
    if (p->integrator != RMHD_SSP2_222 && p->integrator != RMHD_SSP3_332)
        return fail(c, RMHD_EINVAL, "integrator must be RMHD_SSP2_222 or RMHD_SSP3_332");
    if (p->c2p_primary_only != 0 && p->c2p_primary_only != 1)
        return fail(c, RMHD_EINVAL, "c2p_primary_only must be 0 or 1");
    if (!(p->c2p_tol > 0.0) || !(p->newton_tol > 0.0)) return fail(c, RMHD_EINVAL, "tolerances must be > 0");
    return RMHD_OK;
}

// parameter validation shared with the batched path (message into *msg)
int rmhd_validate_params(const rmhd_params *p, std::string *msg)
{
    const int rc = check_params_impl(p, nullptr);
    if (rc && msg) *msg = g_err;
    return rc;
}

extern "C" int rmhd_layout_of(const rmhd_params *p, rmhd_layout *out)
{
    int rc = check_params_impl(p, nullptr);
    if (rc) return rc;
    if (!out) return fail(nullptr, RMHD_EINVAL, "out is NULL");
    layout_from(p, out);
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
    int rc = check_params_impl(p, nullptr);
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
    c->geo = geo_from(p, L);
    c->phys = phys_from(p);
    if (hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || c->cus < 1)
        c->cus = 256;
    const size_t pl = (size_t)L.plane * sizeof(double);
    const int nsrc = p->model == RMHD_SINGLE_FLUID ? 5 : p->model == RMHD_TWO_FLUID ? 9 : 1;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc((void **)&c->q1src, pl * nsrc);
    if (e == hipSuccess) e = hipMalloc((void **)&c->w1, pl * L.nprim);
    if (e == hipSuccess) e = hipMalloc((void **)&c->r2, pl * L.ncons);
    if (e == hipSuccess) e = hipMalloc((void **)&c->acc, pl * L.ncons);
    if (e == hipSuccess && p->integrator == RMHD_SSP3_332) e = hipMalloc((void **)&c->r3, pl * L.ncons);
    if (e == hipSuccess && p->integrator == RMHD_SSP3_332) e = hipMalloc((void **)&c->w2, pl * L.nprim);
    if (e == hipSuccess && p->ndim == 3) e = hipMalloc((void **)&c->lz, pl * L.ncons);
    if (e == hipSuccess) e = hipMalloc((void **)&c->status, (size_t)L.plane);
    if (e == hipSuccess) e = hipMalloc((void **)&c->iters, (size_t)L.plane * sizeof(int32_t));
    const int nx_unk = p->model == RMHD_TWO_FLUID ? 7 : 3;
    // 0: the default cap, chosen per stage launch (launch_stage_m)
    c->cap = 0;
    if (e == hipSuccess) e = hipMalloc((void **)&c->qidx, (size_t)L.plane * 2 * sizeof(int));
    if (e == hipSuccess) e = hipMalloc((void **)&c->qx, pl * (nx_unk + 2));
    if (e == hipSuccess) e = hipMalloc((void **)&c->qcount, 256);
    if (e == hipSuccess) {
        c->qit = c->qidx + L.plane;
        c->qp = c->qx + (size_t)nx_unk * L.plane;
    }
    const size_t stats_bytes = (size_t)STATS_SLOTS * STATS_STRIDE * sizeof(unsigned long long);
    if (e == hipSuccess) e = hipMalloc((void **)&c->stats, stats_bytes);
    if (e == hipSuccess) e = hipMemsetAsync(c->stats, 0, stats_bytes, c->stream);
    // one slot per wavefront of a stage launch (k_stage and k_drain use the same grid)
    c->nwslots = (long)((L.plane + 255) / 256) * 4;
    const size_t wstats_bytes = (size_t)c->nwslots * STATS_WAVE * sizeof(unsigned long long);
    if (e == hipSuccess) e = hipMalloc((void **)&c->wstats, wstats_bytes);
    if (e == hipSuccess) e = hipMemsetAsync(c->wstats, 0, wstats_bytes, c->stream);
    // per-cell conductivity: copy the caller's plane (only its interior cells matter) and
    // fill the copy's ghost cells by the boundary condition, as the state's are
    if (e == hipSuccess && p->sigma_cell) {
        e = hipMalloc((void **)&c->sigma_own, pl);
        if (e == hipSuccess) e = hipMemcpyAsync(c->sigma_own, p->sigma_cell, pl, hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_bc, dim3((unsigned)((L.plane + 255) / 256)), dim3(256), 0, c->stream,
                               planes_of(c->sigma_own, L, 1), 1, c->geo);
            e = hipGetLastError();
        }
        c->phys.sigma_cell = c->sigma_own;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        std::string m = std::string("scratch allocation: ") + hipGetErrorString(e);
        rmhd_destroy(c);
        return fail(nullptr, e == hipErrorOutOfMemory ? RMHD_ENOMEM : RMHD_EHIP, m);
    }
    *out = c;
    return RMHD_OK;
}

static void free_graph(rmhd_ctx *c)
{
    if (c->exec) hipGraphExecDestroy(c->exec);
    if (c->graph) hipGraphDestroy(c->graph);
    c->exec = nullptr;
    c->graph = nullptr;
}

extern "C" void rmhd_destroy(rmhd_ctx *c)
{
    if (!c) return;
    free_graph(c);
    if (c->gstream) hipStreamDestroy(c->gstream);
    if (c->timing)
        for (int k = 0; k < 14; ++k) hipEventDestroy(c->ev[k]);
    hipFree(c->q1src);
    hipFree(c->w1);
    hipFree(c->r2);
    hipFree(c->acc);
    hipFree(c->r3);
    hipFree(c->lz);
    hipFree(c->w2);
    hipFree(c->status);
    hipFree(c->iters);
    hipFree(c->stats);
    hipFree(c->wstats);
    hipFree(c->qidx);
    hipFree(c->qx);
    hipFree(c->qcount);
    hipFree(c->sigma_own);
    hipFree(c->guess);
    delete c;
}

static dim3 cells_grid(const rmhd_ctx *c) { return dim3((unsigned)((c->lay.plane + 255) / 256)); }

static int launch_bc(rmhd_ctx *c, double *arr, int nvar)
{
    hipLaunchKernelGGL(k_bc, cells_grid(c), dim3(256), 0, c->stream, planes_of(arr, c->lay, nvar), nvar, c->geo);
    return hip_check(c, hipGetLastError(), "k_bc launch");
}

// Default cap (none set): no queue.  Measured on the two-fluid 1024^2 sheet with Jacobian
// reuse on: a queue after one Newton step makes the learned-guess step slower (1.48 against
// 1.42 ms); without reuse it was faster there (1.48 against 1.61 ms), since a queued cell's
// second step took a fresh Jacobian either way.  From the plain guess the queue is 12-14 %
// slower on the 512^2 and 128^3 sheets, and slower on every single-fluid grid measured.
template <int M>
static int launch_stage_m(rmhd_ctx *c, StageArgs B)
{
    B.cap = c->cap ? c->cap : 1 << 30;
    B.stats_detail = c->stats_detail;
    B.qcap = (int)c->lay.plane;
    B.qidx = c->qidx;
    B.qit = c->qit;
    B.qx = c->qx;
    B.qp = c->qp;
    B.qcount = c->qcount;
    const bool queue = B.cap < c->prm.max_newton_iter;
    if (queue) hipLaunchKernelGGL(k_qreset, dim3(1), dim3(64), 0, c->stream, c->qcount);
    // one wavefront per block: a stage block ends when its slowest cell converges, and a
    // SIMD that holds a one-wavefront block takes the next block as soon as its own wavefront
    // is done instead of waiting for three others (two-fluid 1024^2 sheet: 309 -> 287 us
    // against 256-thread blocks, 293 us with 128)
    constexpr int STAGE_BLOCK = 64;
    hipLaunchKernelGGL(k_stage<M>, dim3((unsigned)((c->lay.plane + STAGE_BLOCK - 1) / STAGE_BLOCK)), dim3(STAGE_BLOCK), 0,
                       c->stream, B);
    if (queue) hipLaunchKernelGGL(k_drain<M>, cells_grid(c), dim3(256), 0, c->stream, B);
    return hip_check(c, hipGetLastError(), "k_stage launch");
}

static int launch_stage(rmhd_ctx *c, const StageArgs &A)
{
    if (c->prm.model == RMHD_SINGLE_FLUID) return launch_stage_m<0>(c, A);
    StageArgs B = A;
    // learned starting point, unless the caller gave one.  The network runs in a kernel of its
    // own: evaluated inside the stage kernel (one wavefront per SIMD there) the stage took
    // 0.61 ms instead of 0.44 + 0.06 ms on the two-fluid 1024^2 sheet, its matrix products,
    // LDS hand-offs and transcendentals exposed with no other wavefront to hide them
    if (c->mlp && !A.use_guess) {
        Planes G{};
        int k = 0;
        for (int v : {tf::SBX, tf::SBY, tf::SBZ, tf::TAUB, tf::EX, tf::EY, tf::EZ}) G.p[v] = c->guess + (k++) * c->lay.plane;
        if (mlp_launch_guess(c->mlp, c->stream, A.R, G, c->geo, c->phys, A.a))
            return fail(c, RMHD_EHIP, "k_guess launch failed");
        B.guess = as_const(G);
        B.use_guess = 1;
        // no comparison with the plain start: measured on the two-fluid 1024^2 sheet, it
        // leaves the Newton steps per cell unchanged (2.06) and costs one residual per cell
        B.compare_start = 0;
    }
    const long cells = (long)c->prm.nx * c->geo.ny * c->geo.nz;
    if (c->hx && c->hcount + cells <= c->hcap) {
        B.hx = c->hx;
        B.ht = c->ht;
        B.hbase = c->hcount;
        c->hcount += cells;
    }
    return launch_stage_m<1>(c, B);
}

// Flux tiles: a CU holds one tile block at a time (register and LDS bound), so a pass takes
// (rounds of tiles over the CUs) x (time per tile).  Cost of a pass, in units of a reference
// tile's time (x100), with tiles of tx x ty interior cells over `planes` z planes.
static long tile_cost(const rmhd_ctx *c, int tx, int ty, long planes, long rel)
{
    const long tiles = (long)((c->prm.nx + tx - 1) / tx) * ((c->prm.ny + ty - 1) / ty) * planes;
    return rel * ((tiles + c->cus - 1) / c->cus);
}

// Single-fluid and ideal tiles: 64 x 16 (the x stencil across the lanes of a row) or 32 x 32
// (both stencils through LDS, 28 x 28 interior cells), whose tile takes 1.18 times as long
// but wastes less of a narrow grid's last column of tiles: Kelvin-Helmholtz 128 x 256 x 128,
// x-y kernel 33 rounds of 64 x 16 tiles 870 us per pass, 25 rounds of 32 x 32 777 us; on
// 256 x 512 (one round either way) 27 against 29 us.
static int sf_rows(const rmhd_ctx *c, long planes)
{
    return tile_cost(c, 28, 28, planes, 118) < tile_cost(c, 60, 12, planes, 100) ? 32 : 16;
}

// Thread rows of a 2-D flux tile block (24: the 32-column two-fluid tile, 32: the 32 x 32
// single-fluid and ideal tile).  Two-fluid grids take the cheapest of 64 x 12, 32 x 24 and
// 64 x 16 with per-tile times relative to 64 x 12 (60 x 8 interior cells) of 1.19 for 32 x 24
// (28 x 20) and 1.45 for 64 x 16 (60 x 12; spills, and the step then needs a separate
// recovery kernel); measured: 1024^2 sheet 64 x 12 (9 rounds) 223 us per pass, 32 x 24 (7.5
// rounds) 235 us; 512^2 sheet 64 x 12 (2.25 rounds) 70 us, 32 x 24 (1.9 rounds) 59 us;
// 1024 x 128, 64 x 16 (one round) 36 us, 64 x 12 (1.1 rounds) 50 us.
static int flux_rows_2d(const rmhd_ctx *c)
{
    if (c->flux_rows) return c->flux_rows;
    if (c->prm.model != RMHD_TWO_FLUID) return sf_rows(c, 1);
    const long c12 = tile_cost(c, 60, 8, 1, 100), c24 = tile_cost(c, 28, 20, 1, 119),
               c16 = tile_cost(c, 60, 12, 1, 145);
    if (c16 < c12 && c16 < c24) return 16;
    return c24 < c12 ? 24 : 12;
}

// The same choices for the x-y tiles of a 3-D grid: two fluid 64 x 12 or 32 x 24, the other
// models 64 x 16 or 32 x 32 (a requested shape among those is kept).
static int flux_rows_3d(const rmhd_ctx *c)
{
    if (c->prm.model == RMHD_TWO_FLUID) {
        if (c->flux_rows == 12 || c->flux_rows == 24) return c->flux_rows;
        return tile_cost(c, 28, 20, c->prm.nz, 119) < tile_cost(c, 60, 8, c->prm.nz, 100) ? 24 : 12;
    }
    if (c->flux_rows == 16 || c->flux_rows == 32) return c->flux_rows;
    return sf_rows(c, c->prm.nz);
}

template <int M, int NO, bool BQ>
static void launch_flux_shape(rmhd_ctx *c, const FluxArgs &A)
{
    if (c->prm.ndim == 3) {
        // the z term of every interior cell first, then the x and y terms per interior z plane
        // (64 x 16 or 32 x 32 tiles, two fluid 64 x 12 or 32 x 24), which add it, complete the outputs, write their
        // ghost images in all three directions and recover the primitives
        constexpr int BX = 64;
        FluxArgs Az = A;
        Az.lz = planes_of(c->lz, c->lay, c->lay.ncons);
        const dim3 gz((unsigned)((c->prm.nx + BX - 1) / BX), (unsigned)c->prm.ny, (unsigned)((c->prm.nz + 11) / 12));
        hipLaunchKernelGGL((k_flux_z<M>), gz, dim3(BX, 16), 0, c->stream, Az);
        const unsigned gx = (unsigned)((c->prm.nx + (BX - 4) - 1) / (BX - 4));
        if constexpr (M == RMHD_TWO_FLUID) {   // 64 x 12 or 32 x 24: the two-fluid tile's registers without spills
            if (flux_rows_3d(c) == 24)
                hipLaunchKernelGGL((k_flux<M, 3, 32, 24, NO, BQ>),
                                   dim3((unsigned)((c->prm.nx + 27) / 28), (unsigned)((c->prm.ny + 19) / 20),
                                        (unsigned)c->prm.nz),
                                   dim3(32, 24), 0, c->stream, Az);
            else
                hipLaunchKernelGGL((k_flux<M, 3, BX, 12, NO, BQ>),
                                   dim3(gx, (unsigned)((c->prm.ny + 7) / 8), (unsigned)c->prm.nz), dim3(BX, 12), 0,
                                   c->stream, Az);
        } else if (flux_rows_3d(c) == 32)
            hipLaunchKernelGGL((k_flux<M == RMHD_TWO_FLUID ? RMHD_SINGLE_FLUID : M, 3, 32, 32, NO, BQ>),
                               dim3((unsigned)((c->prm.nx + 27) / 28), (unsigned)((c->prm.ny + 27) / 28),
                                    (unsigned)c->prm.nz),
                               dim3(32, 32), 0, c->stream, Az);
        else
            hipLaunchKernelGGL((k_flux<M, 3, BX, 16, NO, BQ>), dim3(gx, (unsigned)((c->prm.ny + 11) / 12), (unsigned)c->prm.nz),
                               dim3(BX, 16), 0, c->stream, Az);
    } else if (c->prm.ndim == 1) {
        constexpr int BX = 256;
        dim3 grid((c->prm.nx + (BX - 4) - 1) / (BX - 4));
        hipLaunchKernelGGL((k_flux<M, 1, BX, 1, NO, BQ>), grid, dim3(BX, 1), 0, c->stream, A);
    } else {
        // 64 x 16 or 32 x 32 tiles for the single-fluid and ideal models; two-fluid grids
        // choose between 64 x 12, 32 x 24 and 64 x 16 (flux_rows_2d): the 768-thread blocks fit
        // the two-fluid tile's registers without spills and let the last pass recover the
        // primitives (1024^2 sheet: 221 against 239 us per pass for 64 x 16); 64 x 8 (4 rows)
        // on request.
        // Measured on the 256 x 512 single-fluid grid, whose 16-row tiles leave some CUs idle,
        // 16 rows are still faster (30 us against 41 us at 8 rows, 40 us at 12).
        constexpr int BX = 64;
        const unsigned gx = (unsigned)((c->prm.nx + (BX - 4) - 1) / (BX - 4));
        const int rows = flux_rows_2d(c);
        if (rows == 8)
            hipLaunchKernelGGL((k_flux<M, 2, BX, 8, NO, BQ>), dim3(gx, (c->prm.ny + 3) / 4), dim3(BX, 8), 0, c->stream, A);
        else if (rows == 12)
            hipLaunchKernelGGL((k_flux<M, 2, BX, 12, NO, BQ>), dim3(gx, (c->prm.ny + 7) / 8), dim3(BX, 12), 0, c->stream, A);
        else if (M == RMHD_TWO_FLUID && rows == 24)
            hipLaunchKernelGGL((k_flux<RMHD_TWO_FLUID, 2, 32, 24, NO, BQ>),
                               dim3((c->prm.nx + 27) / 28, (c->prm.ny + 19) / 20), dim3(32, 24), 0, c->stream, A);
        else if (M != RMHD_TWO_FLUID && rows == 32)
            hipLaunchKernelGGL((k_flux<M == RMHD_TWO_FLUID ? RMHD_SINGLE_FLUID : M, 2, 32, 32, NO, BQ>),
                               dim3((c->prm.nx + 27) / 28, (c->prm.ny + 27) / 28), dim3(32, 32), 0, c->stream, A);
        else
            hipLaunchKernelGGL((k_flux<M, 2, BX, 16, NO, BQ>), dim3(gx, (c->prm.ny + 11) / 12), dim3(BX, 16), 0,
                               c->stream, A);
    }
}

// Outputs that all share one base whose source-free planes are q's (the first pass of a step)
// take those base values from the state the tile already holds (base_terms, BQ).
template <int M, int NO>
static void launch_flux_mo(rmhd_ctx *c, const FluxArgs &A)
{
    bool bq = NO >= 2 && A.o[0].base.p[0] != nullptr;
    for (int k = 1; k < NO && bq; ++k) bq = A.o[k].base.p[0] == A.o[0].base.p[0];
    for (int v = 0; v < c->lay.ncons && bq; ++v)
        if (!has_source(M, v)) bq = A.o[0].base.p[0] + (long)v * c->geo.plane == A.q.p[v];
    if constexpr (NO >= 2) {
        if (bq) {
            launch_flux_shape<M, NO, true>(c, A);
            return;
        }
    }
    launch_flux_shape<M, NO, false>(c, A);
}

template <int M>
static void launch_flux_m(rmhd_ctx *c, const FluxArgs &A)
{
    const int n = A.o[2].out.p[0] ? 3 : A.o[1].out.p[0] ? 2 : 1;
    if (n == 3) launch_flux_mo<M, 3>(c, A);
    else if (n == 2) launch_flux_mo<M, 2>(c, A);
    else launch_flux_mo<M, 1>(c, A);
}

static int launch_flux(rmhd_ctx *c, const FluxArgs &A)
{
    if (c->prm.model == RMHD_SINGLE_FLUID) launch_flux_m<0>(c, A);
    else if (c->prm.model == RMHD_TWO_FLUID) launch_flux_m<1>(c, A);
    else launch_flux_m<2>(c, A);
    return hip_check(c, hipGetLastError(), "k_flux launch");
}

extern "C" int rmhd_init_state(rmhd_ctx *c, const double *prims, const double *EB, double *cons)
{
    if (!c || !prims || !EB || !cons) return fail(c, RMHD_EINVAL, "rmhd_init_state: NULL argument");
    const rmhd_layout &L = c->lay;
    const CPlanes P = cplanes_of(prims, L, L.nprim), F = cplanes_of(EB, L, 6);
    const Planes Q = planes_of(cons, L, L.ncons);
    if (c->prm.model == RMHD_SINGLE_FLUID)
        hipLaunchKernelGGL(k_init<0>, cells_grid(c), dim3(256), 0, c->stream, P, F, Q, c->geo, c->phys);
    else if (c->prm.model == RMHD_TWO_FLUID)
        hipLaunchKernelGGL(k_init<1>, cells_grid(c), dim3(256), 0, c->stream, P, F, Q, c->geo, c->phys);
    else
        hipLaunchKernelGGL(k_init<2>, cells_grid(c), dim3(256), 0, c->stream, P, F, Q, c->geo, c->phys);
    int rc = hip_check(c, hipGetLastError(), "k_init launch");
    if (rc) return rc;
    return launch_bc(c, cons, L.ncons);
}

// Recovery on every cell, starting from prims' own values.
static int launch_c2p(rmhd_ctx *c, const double *cons, double *prims, int8_t *status, int32_t *iters)
{
    const rmhd_layout &L = c->lay;
    const CPlanes Q = cplanes_of(cons, L, L.ncons);
    const Planes W = planes_of(prims, L, L.nprim);
    if (c->prm.model == RMHD_SINGLE_FLUID)
        hipLaunchKernelGGL(k_c2p<0>, cells_grid(c), dim3(256), 0, c->stream, Q, W, status, iters, c->geo, c->phys);
    else if (c->prm.model == RMHD_TWO_FLUID)
        hipLaunchKernelGGL(k_c2p<1>, cells_grid(c), dim3(256), 0, c->stream, Q, W, status, iters, c->geo, c->phys);
    else
        hipLaunchKernelGGL(k_c2p<2>, cells_grid(c), dim3(256), 0, c->stream, Q, W, status, iters, c->geo, c->phys);
    return hip_check(c, hipGetLastError(), "k_c2p launch");
}

extern "C" int rmhd_cons2prim(rmhd_ctx *c, const double *cons, double *prims, int8_t *status, int32_t *iters)
{
    if (!c || !cons || !prims) return fail(c, RMHD_EINVAL, "rmhd_cons2prim: NULL argument");
    return launch_c2p(c, cons, prims, status, iters);
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
    A.o[0].out = planes_of(Lout, L, L.ncons);
    A.o[0].cL = 1.0;
    A.g = c->geo;
    A.P = c->phys;
    return launch_flux(c, A);
}

extern "C" int rmhd_implicit_stage(rmhd_ctx *c, double a, const double *R, const double *guess, double *Q,
                                   double *prims, int8_t *status, int32_t *iters)
{
    if (!c || !R || !Q || !prims) return fail(c, RMHD_EINVAL, "rmhd_implicit_stage: NULL argument");
    if (c->prm.model == RMHD_IDEAL) return fail(c, RMHD_EINVAL, "rmhd_implicit_stage: the ideal model has no implicit stage");
    if (!(a >= 0.0)) return fail(c, RMHD_EINVAL, "rmhd_implicit_stage: a must be >= 0");
    const rmhd_layout &L = c->lay;
    StageArgs A{};
    A.R = cplanes_of(R, L, L.ncons);
    if (guess) A.guess = cplanes_of(guess, L, L.ncons);
    A.use_guess = guess != nullptr;
    A.compare_start = 1;
    A.win = cplanes_of(prims, L, L.nprim);
    A.wout = planes_of(prims, L, L.nprim);
    A.Q = planes_of(Q, L, L.ncons);
    A.status = status;
    A.iters = iters;
    A.stats = c->stats;
    A.wstats = c->wstats;
    A.a = a;
    A.g = c->geo;
    A.P = c->phys;
    A.write_all = Q != R;
    return launch_stage(c, A);
}

static int enqueue_imex(rmhd_ctx *c, double dt, double *cons, double *prims);

extern "C" int rmhd_imex_step(rmhd_ctx *c, double dt, double *cons, double *prims)
{
    if (!c || !cons || !prims) return fail(c, RMHD_EINVAL, "rmhd_imex_step: NULL argument");
    if (!(dt > 0.0)) return fail(c, RMHD_EINVAL, "rmhd_imex_step: dt must be > 0");
    // the graph holds fixed kernel arguments: not while timing or harvesting (both change
    // per call)
    if (!c->use_graph || c->timing || c->hx) return enqueue_imex(c, dt, cons, prims);
    if (!c->exec || dt != c->g_dt || cons != c->g_cons || prims != c->g_prims) {
        free_graph(c);
        int rc = RMHD_OK;
        if (!c->gstream)
            rc = hip_check(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking), "capture stream");
        if (rc) return rc;
        rc = hip_check(c, hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal), "begin capture");
        if (rc) return rc;
        const hipStream_t own = c->stream;
        c->stream = c->gstream;
        rc = enqueue_imex(c, dt, cons, prims);
        c->stream = own;
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(c->gstream, &g);
        if (rc) {
            if (g) hipGraphDestroy(g);
            return rc;
        }
        rc = hip_check(c, e, "end capture");
        if (rc) return rc;
        c->graph = g;
        rc = hip_check(c, hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0), "graph instantiate");
        if (rc) {
            free_graph(c);
            return rc;
        }
        c->g_dt = dt;
        c->g_cons = cons;
        c->g_prims = prims;
    }
    return hip_check(c, hipGraphLaunch(c->exec, c->stream), "graph launch");
}

static FluxOut flux_out(const double *base, double *out, const rmhd_layout &L, double cL, double cS)
{
    FluxOut o{};
    if (base) o.base = cplanes_of(base, L, L.ncons);
    o.out = planes_of(out, L, L.ncons);
    o.cL = cL;
    o.cS = cS;
    return o;
}

// The step as a sequence of launches (Pareschi-Russo stage sums, Table 2 or Table 3):
//   SSP2(222)  stage 1: Q1 = q^n + g dt Psi(Q1)
//              flux 1:  R2 = q^n + dt L1 + (1-2g) dt Psi1,   ACC = q^n + dt/2 (L1 + Psi1)
//              stage 2: Q2 = R2 + g dt Psi(Q2)
//              flux 2:  q^{n+1} = ACC + dt/2 (L2 + Psi2)
//   SSP3(332)  stage 1 as above
//              flux 1:  R2 as above,  R3 = q^n + dt/4 L1 + (1/2-g) dt Psi1,  ACC = q^n + dt/6 (L1 + Psi1)
//              stage 2: Q2 = R2 + g dt Psi(Q2)
//              flux 2:  R3 += dt/4 L2,  ACC += dt/6 (L2 + Psi2)
//              stage 3: Q3 = R3 + g dt Psi(Q3)
//              flux 3:  q^{n+1} = ACC + 2 dt/3 (L3 + Psi3)
// Every flux pass writes the ghost images of its first output; the last one also recovers the
// primitives (single fluid; two fluid: a separate recovery kernel), from the last stage's.
static int enqueue_explicit(rmhd_ctx *c, double dt, double *cons, double *prims);

// Wait for a timed step's last event and add its event pairs to the per-kind totals
// (0 stage, 1 flux pass, 2 recovery).
static int record_timing(rmhd_ctx *c, int nev, const int *kinds)
{
    int rc = hip_check(c, hipEventSynchronize(c->ev[nev - 1]), "timing sync");
    if (rc) return rc;
    for (int k = 0; 2 * k < nev; ++k) {
        float ms = 0.0f;
        hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]);
        if (kinds[k] == 0) { c->times.stage_ms += ms; c->times.stage_launches += 1; }
        if (kinds[k] == 1) { c->times.flux_ms += ms; c->times.flux_launches += 1; }
        if (kinds[k] == 2) { c->times.c2p_ms += ms; c->times.c2p_launches += 1; }
    }
    c->times.steps += 1;
    return RMHD_OK;
}

// The ideal model's step: the explicit halves of the tableaux, with the cleaning source
// (the model's only one) explicit as well, K = L + Psi:
//   SSP2(222)  flux 1: R2 = q^n + dt K1,  ACC = q^n + dt/2 K1
//              flux 2: q^{n+1} = ACC + dt/2 K(R2)
//   SSP3(332)  flux 1: R2 = q^n + dt K1,  R3 = q^n + dt/4 K1,  ACC = q^n + dt/6 K1
//              flux 2: R3 += dt/4 K(R2),  ACC += dt/6 K(R2)
//              flux 3: q^{n+1} = ACC + 2 dt/3 K(R3)
// Each pass writes the ghost images of its first output and recovers its primitives in the
// kernel that completes that output, each recovery starting from the primitives of the
// state the pass read.
static int enqueue_explicit(rmhd_ctx *c, double dt, double *cons, double *prims)
{
    const rmhd_layout &L = c->lay;
    const bool ssp3 = c->prm.integrator == RMHD_SSP3_332;
    int nev = 0, kinds[7];
    auto begin = [&]() {
        if (c->timing) hipEventRecord(c->ev[nev], c->stream);
    };
    auto end = [&](int kind) {
        if (c->timing) hipEventRecord(c->ev[nev + 1], c->stream);
        kinds[nev / 2] = kind;
        nev += 2;
    };
    // one pass reading (q, w), writing outputs with the recovered primitives of output 0 in wout
    auto pass = [&](const double *q, const double *w, double *wout, const FluxOut *o, int n) {
        FluxArgs F{};
        F.q = cplanes_of(q, L, L.ncons);
        F.w = cplanes_of(w, L, L.nprim);
        F.g = c->geo;
        F.P = c->phys;
        F.fuse_bc = 1;
        for (int k = 0; k < n; ++k) F.o[k] = o[k];
        F.wnew = planes_of(wout, L, L.nprim);
        begin();
        int rc = launch_flux(c, F);
        end(1);
        return rc;
    };
    int rc;
    if (!ssp3) {
        const FluxOut o1[2] = {flux_out(cons, c->r2, L, dt, dt), flux_out(cons, c->acc, L, 0.5 * dt, 0.5 * dt)};
        rc = pass(cons, prims, c->w1, o1, 2);
        if (rc) return rc;
        const FluxOut o2[1] = {flux_out(c->acc, cons, L, 0.5 * dt, 0.5 * dt)};
        rc = pass(c->r2, c->w1, prims, o2, 1);
    } else {
        const FluxOut o1[3] = {flux_out(cons, c->r2, L, dt, dt), flux_out(cons, c->r3, L, 0.25 * dt, 0.25 * dt),
                               flux_out(cons, c->acc, L, dt / 6.0, dt / 6.0)};
        rc = pass(cons, prims, c->w1, o1, 3);
        if (rc) return rc;
        const FluxOut o2[2] = {flux_out(c->r3, c->r3, L, 0.25 * dt, 0.25 * dt),
                               flux_out(c->acc, c->acc, L, dt / 6.0, dt / 6.0)};
        rc = pass(c->r2, c->w1, c->w2, o2, 2);
        if (rc) return rc;
        const FluxOut o3[1] = {flux_out(c->acc, cons, L, 2.0 * dt / 3.0, 2.0 * dt / 3.0)};
        rc = pass(c->r3, c->w2, prims, o3, 1);
    }
    if (rc || !c->timing) return rc;
    return record_timing(c, nev, kinds);
}

static int enqueue_imex(rmhd_ctx *c, double dt, double *cons, double *prims)
{
    if (c->prm.model == RMHD_IDEAL) return enqueue_explicit(c, dt, cons, prims);
    const rmhd_layout &L = c->lay;
    const double gm = SSP2_GAMMA;
    const int M = c->prm.model;
    const bool ssp3 = c->prm.integrator == RMHD_SSP3_332;
    // the last flux pass also recovers the primitives, except in two-fluid steps on 3-D grids
    // and with 16-row 2-D tiles, which run a separate recovery kernel: the recovery's
    // registers make those tiles spill.  Measured: 1024^2 sheet (12-row tiles) 1.118 ->
    // 1.099 ms per step fused; 512^2 sheet (16-row tiles) 0.321 -> 0.328 ms fused
    const bool fused = M == RMHD_SINGLE_FLUID || c->prm.ndim != 2 || flux_rows_2d(c) == 12 || flux_rows_2d(c) == 24;
    // event pairs: stages, flux passes, recovery (kinds 0, 1, 2)
    int nev = 0, kinds[7];
    auto begin = [&]() {
        if (c->timing) hipEventRecord(c->ev[nev], c->stream);
    };
    auto end = [&](int kind) {
        if (c->timing) hipEventRecord(c->ev[nev + 1], c->stream);
        kinds[nev / 2] = kind;
        nev += 2;
    };
    // Q1: the source-free components are those of q^n; the others live in scratch
    Planes Q1 = planes_of(cons, L, L.ncons);
    {
        int k = 0;
        for (int v = 0; v < L.ncons; ++v)
            if (has_source(M, v)) Q1.p[v] = c->q1src + (k++) * L.plane;
    }
    StageArgs S{};
    S.R = cplanes_of(cons, L, L.ncons);
    S.win = cplanes_of(prims, L, L.nprim);
    S.wout = planes_of(c->w1, L, L.nprim);
    S.Q = Q1;
    S.status = c->status;
    S.iters = c->iters;
    S.stats = c->stats;
    S.wstats = c->wstats;
    S.a = gm * dt;
    S.g = c->geo;
    S.P = c->phys;
    S.write_all = 0;
    begin();
    int rc = launch_stage(c, S);
    end(0);
    if (rc) return rc;

    FluxArgs F{};
    F.q = as_const(Q1);
    F.w = cplanes_of(c->w1, L, L.nprim);
    F.g = c->geo;
    F.P = c->phys;
    F.fuse_bc = 1;
    F.o[0] = flux_out(cons, c->r2, L, dt, (1.0 - 2.0 * gm) * dt);
    if (ssp3) {
        F.o[1] = flux_out(cons, c->r3, L, 0.25 * dt, (0.5 - gm) * dt);
        F.o[2] = flux_out(cons, c->acc, L, dt / 6.0, dt / 6.0);
    } else {
        F.o[1] = flux_out(cons, c->acc, L, 0.5 * dt, 0.5 * dt);
    }
    begin();
    rc = launch_flux(c, F);
    end(1);
    if (rc) return rc;

    // stage 2, in place in R2
    double *w_last = ssp3 ? c->w2 : (fused ? c->w1 : prims);   // primitives of the last stage
    S.R = cplanes_of(c->r2, L, L.ncons);
    S.win = cplanes_of(c->w1, L, L.nprim);
    S.wout = planes_of(ssp3 ? c->w2 : w_last, L, L.nprim);
    S.Q = planes_of(c->r2, L, L.ncons);
    begin();
    rc = launch_stage(c, S);
    end(0);
    if (rc) return rc;

    double *Qlast = c->r2;
    if (ssp3) {
        F = FluxArgs{};
        F.q = cplanes_of(c->r2, L, L.ncons);
        F.w = cplanes_of(c->w2, L, L.nprim);
        F.g = c->geo;
        F.P = c->phys;
        F.fuse_bc = 1;
        F.o[0] = flux_out(c->r3, c->r3, L, 0.25 * dt, 0.0);
        F.o[1] = flux_out(c->acc, c->acc, L, dt / 6.0, dt / 6.0);
        begin();
        rc = launch_flux(c, F);
        end(1);
        if (rc) return rc;
        // stage 3, in place in R3
        w_last = fused ? c->w1 : prims;
        S.R = cplanes_of(c->r3, L, L.ncons);
        S.win = cplanes_of(c->w2, L, L.nprim);
        S.wout = planes_of(w_last, L, L.nprim);
        S.Q = planes_of(c->r3, L, L.ncons);
        begin();
        rc = launch_stage(c, S);
        end(0);
        if (rc) return rc;
        Qlast = c->r3;
    }

    // q^{n+1} = ACC + w_last dt (L + Psi) of the last stage, ghosts included, and its
    // primitives (recovered by the thread that forms each cell, from the last stage's)
    const double wl = ssp3 ? 2.0 * dt / 3.0 : 0.5 * dt;
    F = FluxArgs{};
    F.q = cplanes_of(Qlast, L, L.ncons);
    F.w = cplanes_of(w_last, L, L.nprim);
    F.g = c->geo;
    F.P = c->phys;
    F.fuse_bc = 1;
    F.o[0] = flux_out(c->acc, cons, L, wl, wl);
    F.wnew = fused ? planes_of(prims, L, L.nprim) : Planes{};
    begin();
    rc = launch_flux(c, F);
    end(1);
    if (rc) return rc;
    if (!fused) {
        begin();
        rc = rmhd_cons2prim(c, cons, prims, nullptr, nullptr);
        end(2);
        if (rc) return rc;
    }
    if (!c->timing) return RMHD_OK;
    return record_timing(c, nev, kinds);
}

extern "C" int rmhd_set_timing(rmhd_ctx *c, int enable)
{
    if (!c) return fail(c, RMHD_EINVAL, "rmhd_set_timing: NULL context");
    if (enable && !c->timing) {
        for (int k = 0; k < 14; ++k) {
            int rc = hip_check(c, hipEventCreate(&c->ev[k]), "hipEventCreate");
            if (rc) {
                for (int m = 0; m < k; ++m) hipEventDestroy(c->ev[m]);
                return rc;
            }
        }
        c->timing = 1;
    } else if (!enable && c->timing) {
        hipStreamSynchronize(c->stream);
        for (int k = 0; k < 14; ++k) hipEventDestroy(c->ev[k]);
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

extern "C" double rmhd_dt(const rmhd_ctx *c) { return c ? cfl_dt(&c->prm) : 0.0; }

extern "C" int rmhd_get_stats(rmhd_ctx *c, rmhd_stats *out, int reset)
{
    if (!c || !out) return fail(c, RMHD_EINVAL, "rmhd_get_stats: NULL argument");
    unsigned long long raw[STATS_SLOTS * STATS_STRIDE];
    hipLaunchKernelGGL(k_wave_stats_fold, dim3(wave_stats_fold_blocks(c->nwslots)), dim3(256), 0, c->stream, c->wstats,
                       c->nwslots, c->stats);
    int rc = hip_check(c, hipGetLastError(), "k_wave_stats_fold launch");
    if (!rc) rc = hip_check(c, hipMemcpyAsync(raw, c->stats, sizeof(raw), hipMemcpyDeviceToHost, c->stream), "stats copy");
    if (!rc && reset) rc = hip_check(c, hipMemsetAsync(c->stats, 0, sizeof(raw), c->stream), "stats reset");
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "stats sync");
    if (rc) return rc;
    stats_fold(raw, out);
    return RMHD_OK;
}

extern "C" const char *rmhd_last_error(const rmhd_ctx *c) { return c ? c->err.c_str() : g_err.c_str(); }

// ---- learned starting guess and harvest (include/rmhd_mlp.h) ---------------------------
extern "C" int rmhd_set_harvest(rmhd_ctx *c, float *X, float *T, long capacity)
{
    if (!c) return fail(c, RMHD_EINVAL, "rmhd_set_harvest: NULL context");
    if (c->prm.model != RMHD_TWO_FLUID) return fail(c, RMHD_EINVAL, "rmhd_set_harvest: two-fluid contexts only");
    if ((X == nullptr) != (T == nullptr)) return fail(c, RMHD_EINVAL, "rmhd_set_harvest: give both arrays or neither");
    if (X && capacity < 0) return fail(c, RMHD_EINVAL, "rmhd_set_harvest: capacity must be >= 0");
    c->hx = X;
    c->ht = T;
    c->hcap = X ? capacity : 0;
    c->hcount = 0;
    return RMHD_OK;
}

extern "C" long rmhd_harvest_count(const rmhd_ctx *c) { return c ? c->hcount : 0; }

extern "C" int rmhd_set_guess_model(rmhd_ctx *c, const rmhd_mlp *m)
{
    if (!c) return fail(c, RMHD_EINVAL, "rmhd_set_guess_model: NULL context");
    if (c->prm.model != RMHD_TWO_FLUID) return fail(c, RMHD_EINVAL, "rmhd_set_guess_model: two-fluid contexts only");
    if (m && !c->guess) {
        const hipError_t e = hipMalloc(&c->guess, sizeof(double) * 7 * c->lay.plane);
        if (e != hipSuccess) {
            c->guess = nullptr;
            return fail(c, e == hipErrorOutOfMemory ? RMHD_ENOMEM : RMHD_EHIP, "rmhd_set_guess_model: guess planes");
        }
    }
    c->mlp = m;
    free_graph(c);   // kernel sequence changed: capture again
    return RMHD_OK;
}

extern "C" int rmhd_learned_guess(rmhd_ctx *c, const rmhd_mlp *m, double a, const double *R, double *guess)
{
    if (!c || !m || !R || !guess) return fail(c, RMHD_EINVAL, "rmhd_learned_guess: NULL argument");
    if (c->prm.model != RMHD_TWO_FLUID) return fail(c, RMHD_EINVAL, "rmhd_learned_guess: two-fluid contexts only");
    if (!(a > 0.0)) return fail(c, RMHD_EINVAL, "rmhd_learned_guess: a must be > 0");
    const rmhd_layout &L = c->lay;
    if (mlp_launch_guess(m, c->stream, cplanes_of(R, L, L.ncons), planes_of(guess, L, L.ncons), c->geo, c->phys, a))
        return fail(c, RMHD_EHIP, "k_guess launch failed");
    return RMHD_OK;
}

extern "C" int rmhd_set_newton_cap(rmhd_ctx *c, int cap)
{
    if (!c) return fail(c, RMHD_EINVAL, "rmhd_set_newton_cap: NULL context");
    if (cap < 1) return fail(c, RMHD_EINVAL, "rmhd_set_newton_cap: cap must be >= 1");
    c->cap = cap;
    free_graph(c);   // kernel arguments changed: capture again
    return RMHD_OK;
}

extern "C" int rmhd_set_jacobian_reuse(rmhd_ctx *c, double keep)
{
    if (!c) return fail(c, RMHD_EINVAL, "rmhd_set_jacobian_reuse: NULL context");
    if (!(keep >= 0.0 && keep < 1.0)) return fail(c, RMHD_EINVAL, "rmhd_set_jacobian_reuse: keep must lie in [0, 1)");
    c->phys.jac_keep = keep;
    free_graph(c);   // kernel arguments changed: capture again
    return RMHD_OK;
}

extern "C" int rmhd_set_flux_rows(rmhd_ctx *c, int rows)
{
    if (!c) return fail(c, RMHD_EINVAL, "rmhd_set_flux_rows: NULL context");
    if (rows != 0 && rows != 8 && rows != 12 && rows != 16 && rows != 24 && rows != 32)
        return fail(c, RMHD_EINVAL, "rmhd_set_flux_rows: rows must be 0, 8, 12, 16, 24 or 32");
    if (rows == 24 && c->prm.model != RMHD_TWO_FLUID)
        return fail(c, RMHD_EINVAL, "rmhd_set_flux_rows: 32 x 24 tiles are for the two-fluid model only");
    if (rows == 32 && c->prm.model == RMHD_TWO_FLUID)
        return fail(c, RMHD_EINVAL, "rmhd_set_flux_rows: 32 x 32 tiles are for the single-fluid and ideal models");
    c->flux_rows = rows;
    free_graph(c);   // kernel arguments changed: capture again
    return RMHD_OK;
}

extern "C" int rmhd_set_stats_detail(rmhd_ctx *c, int detail)
{
    if (!c) return fail(c, RMHD_EINVAL, "rmhd_set_stats_detail: NULL context");
    c->stats_detail = detail != 0;
    free_graph(c);   // kernel arguments changed: capture again
    return RMHD_OK;
}

extern "C" int rmhd_set_graph(rmhd_ctx *c, int enable)
{
    if (!c) return fail(c, RMHD_EINVAL, "rmhd_set_graph: NULL context");
    c->use_graph = enable != 0;
    free_graph(c);
    return RMHD_OK;
}

// ---- the step without allocation (include/rmhd.h: rmhd_imex_step_noalloc) ---------------
// The stage scratch of one step (stage-1 source parts and primitives, R2, ACC, and for
// SSP3(332) R3 and the second stage's primitives) lives in this file-scope array instead
// of memory allocated by rmhd_create.  Every GPU the library runs on holds its own copy from
// the time the code object is loaded until the process ends.  In host code the name only
// stands in for the symbol: the device address of each GPU's copy comes from
// hipGetSymbolAddress with that GPU current, and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[RMHD_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];   // device address of scratch per device, once looked up
}  // namespace

// Address of the current device's copy of scratch (looked up once per device).
static int noalloc_scratch(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, RMHD_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, RMHD_EINVAL, "rmhd_imex_step_noalloc: device index too large");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(nullptr, RMHD_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return RMHD_OK;
}

// Bytes of scratch one step of this parameter set needs (each part rounded up to 256 bytes).
static size_t noalloc_bytes(const rmhd_params *p, const rmhd_layout &L)
{
    const size_t pl = ((size_t)L.plane * sizeof(double) + 255) & ~(size_t)255;
    const int nsrc = p->model == RMHD_SINGLE_FLUID ? 5 : p->model == RMHD_TWO_FLUID ? 9 : 1;
    size_t n = (size_t)nsrc + L.nprim + 2 * (size_t)L.ncons;
    if (p->integrator == RMHD_SSP3_332) n += (size_t)L.ncons + L.nprim;
    if (p->ndim == 3) n += L.ncons;
    return n * pl;
}

extern "C" size_t rmhd_noalloc_scratch_bytes(const rmhd_params *p)
{
    if (check_params_impl(p, nullptr)) return 0;
    rmhd_layout L;
    layout_from(p, &L);
    return noalloc_bytes(p, L);
}

extern "C" int rmhd_imex_step_noalloc(const rmhd_params *p, void *hip_stream, double dt, double *cons, double *prims)
{
    int rc = check_params_impl(p, nullptr);
    if (rc) return rc;
    if (!cons || !prims) return fail(nullptr, RMHD_EINVAL, "rmhd_imex_step_noalloc: NULL argument");
    if (!(dt > 0.0)) return fail(nullptr, RMHD_EINVAL, "rmhd_imex_step_noalloc: dt must be > 0");
    if (p->sigma_cell)
        return fail(nullptr, RMHD_EINVAL,
                    "rmhd_imex_step_noalloc: per-cell conductivity needs a context (rmhd_create keeps a ghost-filled copy)");
    rmhd_ctx c{};
    c.prm = *p;
    layout_from(p, &c.lay);
    const size_t need = noalloc_bytes(p, c.lay);
    if (need > (size_t)RMHD_NOALLOC_SCRATCH_BYTES)
        return fail(nullptr, RMHD_EINVAL,
                    "rmhd_imex_step_noalloc: grid needs " + std::to_string(need) + " bytes of scratch, more than the " +
                        std::to_string((size_t)RMHD_NOALLOC_SCRATCH_BYTES) + " the library holds; use rmhd_create");
    void *base = nullptr;
    rc = noalloc_scratch(&base);
    if (rc) return rc;
    c.stream = (hipStream_t)hip_stream;
    c.geo = geo_from(p, c.lay);
    c.phys = phys_from(p);
    hipGetDevice(&c.device);
    if (hipDeviceGetAttribute(&c.cus, hipDeviceAttributeMultiprocessorCount, c.device) != hipSuccess || c.cus < 1)
        c.cus = 256;
    const size_t pl = ((size_t)c.lay.plane * sizeof(double) + 255) & ~(size_t)255;
    unsigned char *s = (unsigned char *)base;
    auto take = [&](int nplanes) {
        double *q = (double *)s;
        s += (size_t)nplanes * pl;
        return q;
    };
    const int nsrc = p->model == RMHD_SINGLE_FLUID ? 5 : p->model == RMHD_TWO_FLUID ? 9 : 1;
    // every plane below is written before it is read within the step, so nothing is cleared;
    // no statistics, status or iteration planes and no stage queue (cap left at the plain
    // default, which is none)
    c.q1src = take(nsrc);
    c.w1 = take(c.lay.nprim);
    c.r2 = take(c.lay.ncons);
    c.acc = take(c.lay.ncons);
    if (p->integrator == RMHD_SSP3_332) {
        c.r3 = take(c.lay.ncons);
        c.w2 = take(c.lay.nprim);
    }
    if (p->ndim == 3) c.lz = take(c.lay.ncons);
    rc = enqueue_imex(&c, dt, cons, prims);
    if (rc) g_err = c.err;
    return rc;
}
