// batch.hip -- batched form of the SSP2(222) IMEX hot path: many independent single-fluid
// domains of uneven size and stiffness advanced together, one launch per kernel of the step
// for all domains, with a convergence-compacted queue for the implicit stage, the whole
// step captured in a HIP graph, and launch shapes chosen by a built-in autotuner.
//
// Per step (each domain with its own dt, sigma, grid and boundary):
//   reset counters | stage 1 (all cells of all domains, Newton capped at K iterations;
//   unconverged cells are appended to a compacted queue) | queue drain (full wavefronts of
//   hard cells continue Newton) | flux pass 1 over all (domain, tile) pairs | reset |
//   stage 2 | drain | flux pass 2 | primitive recovery of all cells.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace rmhd {

// Everything a kernel needs about one domain (device-resident table, read with scalar loads).
struct DomainDev {
    Geo g;
    Phys P;
    double dt;
    double *cons, *prims;            // caller arrays
    double *q1src, *w1, *r2, *acc;   // pooled stage scratch
};

struct BatchArgs {
    const DomainDev *dom;
    const int2 *items;          // (domain, first linear index) of each 256-cell chunk
    int nitems;
    int chunks_per_item;        // persistent mode: chunks taken per atomic grab
    int persistent;             // 1: loop over grabbed items; 0: one chunk per block
    unsigned *counters;         // [0] item head  [1] queue tail
    int phase;                  // 1 or 2 (selects the stage buffers)
    int K;                      // Newton steps from unconverged iterates before a cell is queued
    int stats_detail;           // also the Newton-step histogram and the largest final residual
    int *qdom, *qidx, *qit;     // compacted queue of unconverged cells
    double *qx, *qp;            // their current unknowns (3 per entry) and pressure
    int qcap;
    unsigned long long *stats;
    unsigned long long *wstats;  // per-wavefront slots of the basic counters (detail off), or nullptr
};

// source-carrying single-fluid components in the order of the scratch planes
__device__ __forceinline__ int sf_src_slot(int v)
{
    return v == sf::EX ? 0 : v == sf::EY ? 1 : v == sf::EZ ? 2 : v == sf::PSI ? 3 : 4;
}

// Solve (or continue) the stage of one cell of domain D.  First pass (resume false): at
// most cap Newton steps from unconverged iterates; CELL_QUEUED tells the caller to queue
// the cell.  Resumed pass: up to budget more steps, no cap.
__device__ __forceinline__ int batch_cell(const DomainDev &D, int phase, long idx, double (&x)[3], double *w,
                                          int cap, int budget, bool resume, int &nit, int &cit, int &rit,
                                          double &gres, int &jit)
{
    const Geo &g = D.g;
    (void)g;
    const double gm = SSP2_GAMMA;
    const double a = gm * D.dt;
    const double *Rb = phase == 1 ? D.cons : D.r2;
    double R[sf::NC];
#pragma unroll
    for (int v = 0; v < sf::NC; ++v) R[v] = Rb[v * g.plane + idx];
    if (!resume) {
        const double *wb = phase == 1 ? D.prims : D.w1;
        w[4] = wb[4 * g.plane + idx];
        x[0] = R[sf::EX];
        x[1] = R[sf::EY];
        x[2] = R[sf::EZ];
    }
    Phys P = D.P;
    if (resume) P.max_newton = budget;
    int n = 0, c = 0, r = 0;
    const int st = sf_stage(R, a, cell_sigma(D.P, idx), P, x, w, n, c, r, resume ? 1 << 30 : cap, &gres, &jit);
    nit += n;
    cit += c;
    rit += r;
    return st;
}

__device__ __forceinline__ void batch_write(const DomainDev &D, int phase, long idx, const double (&x)[3],
                                            const double *w)
{
    const Geo &g = D.g;
    const double gm = SSP2_GAMMA;
    const double a = gm * D.dt;
    const double aK = 1.0 / (1.0 + a * D.P.kappa);
    const double *Rb = phase == 1 ? D.cons : D.r2;
    double *Qs = phase == 1 ? D.q1src : D.r2;
    // phase 1: source parts into the scratch planes (slot order E, psi, phi);
    // phase 2: in place into R2's own planes
    auto qplane = [&](int v) -> double * {
        return phase == 1 ? Qs + sf_src_slot(v) * g.plane : Qs + v * g.plane;
    };
    qplane(sf::EX)[idx] = x[0];
    qplane(sf::EY)[idx] = x[1];
    qplane(sf::EZ)[idx] = x[2];
    qplane(sf::PHI)[idx] = Rb[sf::PHI * g.plane + idx] * aK;
    qplane(sf::PSI)[idx] = (Rb[sf::PSI * g.plane + idx] + a * Rb[sf::RHOE * g.plane + idx]) * aK;
    // both stages' primitives go to w1 (the second stage's in place): the second flux pass
    // reads them as its guess and recovers the new primitives into prims itself
    double *wo = D.w1;
#pragma unroll
    for (int v = 0; v < sf::NP; ++v) wo[v * g.plane + idx] = w[v];
}

// Stage over all cells of all domains.  Cells still unconverged after K Newton iterations
// are appended to the queue (one atomic per block and chunk, prefix sums in LDS).
__global__ __launch_bounds__(256) void kb_stage(BatchArgs A)
{
    __shared__ int s_item;
    __shared__ int s_wcount[4];
    __shared__ int s_base;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int grabbed = 0, pos_in_item = 0;
    int item = A.persistent ? -1 : (int)blockIdx.x;
    // basic counters: per-lane sums over this block's chunks, one wavefront slot write at the end
    const bool wave_stats = A.stats && A.wstats && !A.stats_detail;
    WaveStats ws{};
    if (wave_stats) wave_stats_begin(A.wstats, ws);
    unsigned a_cells = 0, a_nit = 0, a_nmax = 0, a_cit = 0, a_fail = 0, a_rit = 0, a_jit = 0;
    for (;;) {
        if (A.persistent) {
            if (pos_in_item == 0 || pos_in_item >= A.chunks_per_item) {
                if (threadIdx.x == 0) s_item = (int)atomicAdd(&A.counters[0], 1u);
                __syncthreads();
                grabbed = s_item;
                __syncthreads();
                pos_in_item = 0;
            }
            item = grabbed * A.chunks_per_item + pos_in_item;
            ++pos_in_item;
            if (grabbed * A.chunks_per_item >= A.nitems) break;
            if (item >= A.nitems) { pos_in_item = A.chunks_per_item; continue; }
        } else if (item >= A.nitems) {
            break;
        }
        const int2 it = A.items[item];
        const DomainDev &D = A.dom[it.x];
        const Geo &g = D.g;
        const long idx = (long)it.y + threadIdx.x;
        const int i = (int)(idx % g.pitch), j = (int)(idx / g.pitch);
        const bool live = idx < g.plane && i < g.nxg && j < g.nyg;
        int nit = 0, cit = 0, rit = 0, jit = 0, st = CELL_OK;
        double x[3] = {0, 0, 0}, w[sf::NP] = {0, 0, 0, 0, 0}, gres = 0.0;
        if (live) st = batch_cell(D, A.phase, idx, x, w, A.K, 0, false, nit, cit, rit, gres, jit);
        const bool push = live && st == CELL_QUEUED;
        if (live && !push) batch_write(D, A.phase, idx, x, w);
        // block-aggregated queue append
        const unsigned long long mask = __ballot(push);
        if (lane == 0) s_wcount[wave] = __popcll(mask);
        __syncthreads();
        if (threadIdx.x == 0) {
            const int tot = s_wcount[0] + s_wcount[1] + s_wcount[2] + s_wcount[3];
            s_base = tot ? (int)atomicAdd(&A.counters[1], (unsigned)tot) : 0;
        }
        __syncthreads();
        if (push) {
            int off = s_base;
            for (int wv = 0; wv < wave; ++wv) off += s_wcount[wv];
            off += __popcll(mask & ((1ull << lane) - 1ull));
            if (off < A.qcap) {
                A.qdom[off] = it.x;
                A.qidx[off] = (int)idx;
                A.qit[off] = nit;
                A.qx[3 * off + 0] = x[0];
                A.qx[3 * off + 1] = x[1];
                A.qx[3 * off + 2] = x[2];
                A.qp[off] = w[4];
            }
        }
        if (A.stats) {
            const bool c = live && is_interior(g, i, j);
            if (wave_stats) {
                a_cells += c;
                a_nit += c ? nit : 0;
                a_nmax = max(a_nmax, c ? (unsigned)nit : 0u);
                a_cit += c ? cit : 0;
                a_fail += c && !push && st != CELL_OK;
                a_rit += c ? rit : 0;
                a_jit += c ? jit : 0;
            } else {
                stats_block_add(A.stats, c, c ? nit : 0, c ? nit : 0, c ? cit : 0, c && !push && st != CELL_OK,
                                c ? rit : 0, c && !push ? nit : -1, gres, A.stats_detail != 0, c ? jit : 0);
            }
        }
        if (!A.persistent) break;
        __syncthreads();  // s_wcount / s_base are rewritten by the next chunk
    }
    if (wave_stats) wave_stats_end(ws, a_cells, a_nit, a_nmax, a_cit, a_fail, a_rit, a_jit);
}

// Drain the queue: each lane continues one queued cell from its saved unknowns.  The grid is
// sized for the largest possible queue; blocks past the queue's tail exit at once.
__global__ __launch_bounds__(256) void kb_drain(BatchArgs A)
{
    const int tail = min((int)A.counters[1], A.qcap);
    const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if ((int)(blockIdx.x * blockDim.x) >= tail) return;   // whole block past the tail
    const bool live = e < tail;
    int nit = 0, cit = 0, rit = 0, jit = 0, st = CELL_OK, done_it = 0;
    double gres = 0.0;
    bool interior = false;
    const bool wave_stats = A.stats && A.wstats && !A.stats_detail;
    WaveStats ws{};
    if (wave_stats) wave_stats_begin(A.wstats, ws);
    if (live) {
        const DomainDev &D = A.dom[A.qdom[e]];
        const long idx = A.qidx[e];
        interior = is_interior(D.g, (int)(idx % D.g.pitch), (int)(idx / D.g.pitch));
        double x[3] = {A.qx[3 * e], A.qx[3 * e + 1], A.qx[3 * e + 2]}, w[sf::NP] = {0, 0, 0, 0, A.qp[e]};
        done_it = A.qit[e];
        st = batch_cell(D, A.phase, idx, x, w, 0, max(1, D.P.max_newton - done_it), true, nit, cit, rit, gres, jit);
        batch_write(D, A.phase, idx, x, w);
    }
    // the cell was counted by kb_stage; only iterations and failures are added here
    if (A.stats) {
        const bool c = live && interior;
        if (wave_stats)
            wave_stats_end(ws, 0u, c ? nit : 0, c ? nit + done_it : 0, c ? cit : 0, c && st != CELL_OK, c ? rit : 0,
                           c ? jit : 0);
        else
            stats_block_add(A.stats, 0u, c ? nit : 0, c ? nit + done_it : 0, c ? cit : 0, c && st != CELL_OK,
                            c ? rit : 0, c ? nit + done_it : -1, gres, A.stats_detail != 0, c ? jit : 0);
    }
}

__global__ void kb_reset(unsigned *counters)
{
    if (threadIdx.x < 4) counters[threadIdx.x] = 0u;
}

// Flux pass over a list of (domain, tile x, tile y) for domains of one dimensionality.
struct BatchFluxArgs {
    const DomainDev *dom;
    const int4 *tiles;
};

// PASS 1: L(Q1) -> R2, ACC;  PASS 2: L(Q2) -> q^{n+1} and its primitives (recovered by the
// thread that forms each cell, from the second stage's, with their ghost images).  One
// kernel per pass, so that each is allocated registers of its own (the 64 x 16 tile with
// both passes in one kernel spilled 44 bytes per lane).
template <int NDIM, int BX, int BY, int PASS>
__global__ __launch_bounds__(BX *BY) void kb_flux(BatchFluxArgs B)
{
    // tiles are listed domain by domain in row-major order: the XCD-aware renumbering keeps
    // neighbouring tiles of a domain on one XCD
    const int4 t = B.tiles[xcd_order(blockIdx.x, gridDim.x)];
    const DomainDev &D = B.dom[t.x];
    const Geo &g = D.g;
    const double gm = SSP2_GAMMA;
    FluxArgs A{};
    A.g = g;
    A.P = D.P;
    A.fuse_bc = 1;
    const double dt = D.dt;
    if constexpr (PASS == 1) {
        int k = 0;
        for (int v = 0; v < sf::NC; ++v) {
            A.q.p[v] = has_source(0, v) ? D.q1src + (k++) * g.plane : D.cons + v * g.plane;
            A.o[0].base.p[v] = D.cons + v * g.plane;
            A.o[0].out.p[v] = D.r2 + v * g.plane;
            A.o[1].base.p[v] = D.cons + v * g.plane;
            A.o[1].out.p[v] = D.acc + v * g.plane;
        }
        for (int v = 0; v < sf::NP; ++v) A.w.p[v] = D.w1 + v * g.plane;
        A.o[0].cL = dt;
        A.o[0].cS = (1.0 - 2.0 * gm) * dt;
        A.o[1].cL = 0.5 * dt;
        A.o[1].cS = 0.5 * dt;
    } else {
        for (int v = 0; v < sf::NC; ++v) {
            A.q.p[v] = D.r2 + v * g.plane;
            A.o[0].base.p[v] = D.acc + v * g.plane;
            A.o[0].out.p[v] = D.cons + v * g.plane;
        }
        for (int v = 0; v < sf::NP; ++v) {
            A.w.p[v] = D.w1 + v * g.plane;
            A.wnew.p[v] = D.prims + v * g.plane;
        }
        A.o[0].cL = 0.5 * dt;
        A.o[0].cS = 0.5 * dt;
    }
    // pass 1: both outputs have q^n as base, whose source-free planes q shares
    if constexpr (PASS == 1) flux_tile<0, NDIM, BX, BY, 2, false, false, true>(A, t.y, t.z);
    else flux_tile<0, NDIM, BX, BY, 1>(A, t.y, t.z);
}

}  // namespace rmhd

// =======================================================================================
// host side
// =======================================================================================
using namespace rmhd;

int rmhd_validate_params(const rmhd_params *p, std::string *msg);

struct rmhd_batch {
    int n = 0;
    std::vector<rmhd_params> prm;
    std::vector<rmhd_layout> lay;
    std::vector<DomainDev> hdom;
    hipStream_t stream = nullptr;    // caller's stream (work is ordered on it)
    hipStream_t cap = nullptr;       // private stream used only to capture the step graph
    DomainDev *ddom = nullptr;
    double *pool = nullptr;
    int2 *items = nullptr;
    int nitems = 0;
    int4 *tiles1 = nullptr, *tiles2_16 = nullptr, *tiles2_8 = nullptr;
    int ntiles1 = 0, ntiles2_16 = 0, ntiles2_8 = 0;
    unsigned *counters = nullptr;    // [0..3] stage 1, [4..7] stage 2
    int *qdom = nullptr, *qidx = nullptr, *qit = nullptr;
    double *qx = nullptr, *qp = nullptr;
    int qcap = 0;
    int max_newton = 50;
    unsigned long long *stats = nullptr;
    unsigned long long *wstats = nullptr;   // per-wavefront counter slots (folded on read)
    long nwslots = 0;
    rmhd_batch_tuning tune{};
    int stats_detail = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool table_dirty = true;
    std::string err;
};

static int bfail(rmhd_batch *b, int code, const std::string &m)
{
    if (b) b->err = m;
    return code;
}
static int bcheck(rmhd_batch *b, hipError_t e, const char *what)
{
    return e == hipSuccess ? RMHD_OK : bfail(b, RMHD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

static void free_graph(rmhd_batch *b)
{
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

extern "C" void rmhd_batch_destroy(rmhd_batch *b)
{
    if (!b) return;
    free_graph(b);
    if (b->cap) hipStreamDestroy(b->cap);
    hipFree(b->ddom);
    hipFree(b->pool);
    hipFree(b->items);
    hipFree(b->tiles1);
    hipFree(b->tiles2_16);
    hipFree(b->tiles2_8);
    hipFree(b->counters);
    hipFree(b->qdom);
    hipFree(b->qidx);
    hipFree(b->qit);
    hipFree(b->qx);
    hipFree(b->qp);
    hipFree(b->stats);
    hipFree(b->wstats);
    delete b;
}

template <class T>
static hipError_t upload(T **dst, const std::vector<T> &src)
{
    if (src.empty()) return hipSuccess;
    hipError_t e = hipMalloc((void **)dst, sizeof(T) * src.size());
    if (e == hipSuccess) e = hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
    return e;
}

static std::vector<int4> tile_list(const rmhd_batch *b, int ndim, int TX, int TY)
{
    std::vector<int4> t;
    for (int d = 0; d < b->n; ++d) {
        const rmhd_params &p = b->prm[d];
        if (p.ndim != ndim) continue;
        const int nbx = (p.nx + TX - 1) / TX, nby = ndim == 2 ? (p.ny + TY - 1) / TY : 1;
        for (int by = 0; by < nby; ++by)
            for (int bx = 0; bx < nbx; ++bx) t.push_back(make_int4(d, bx, by, 0));
    }
    return t;
}

extern "C" int rmhd_batch_create(const rmhd_params *domains, int n, void *stream, rmhd_batch **out)
{
    if (!out) return RMHD_EINVAL;
    *out = nullptr;
    rmhd_batch *b = new (std::nothrow) rmhd_batch();
    if (!b) return RMHD_ENOMEM;
    *out = b;   // returned even on failure so rmhd_batch_last_error() can explain; destroy it
    if (!domains || n < 1) return bfail(b, RMHD_EINVAL, "rmhd_batch_create: need at least one domain");
    b->n = n;
    b->stream = (hipStream_t)stream;
    size_t total_planes_doubles = 0;
    long total_cells = 0;
    for (int d = 0; d < n; ++d) {
        std::string msg;
        if (rmhd_validate_params(&domains[d], &msg))
            return bfail(b, RMHD_EINVAL, "domain " + std::to_string(d) + ": " + msg);
        if (domains[d].model != RMHD_SINGLE_FLUID)
            return bfail(b, RMHD_EINVAL, "rmhd_batch_create: batched domains must be single-fluid");
        if (domains[d].integrator != RMHD_SSP2_222)
            return bfail(b, RMHD_EINVAL, "rmhd_batch_create: batched domains use the SSP2(222) integrator");
        if (domains[d].ndim == 3)
            return bfail(b, RMHD_EINVAL, "rmhd_batch_create: batched domains are 1-D or 2-D");
        if (domains[d].sigma_cell)
            return bfail(b, RMHD_EINVAL, "rmhd_batch_create: per-cell conductivity is not batched");
        rmhd_layout L;
        layout_from(&domains[d], &L);
        b->prm.push_back(domains[d]);
        b->lay.push_back(L);
        total_planes_doubles += (size_t)L.plane * (5 + 5 + 14 + 14);
        total_cells += L.plane;
        b->max_newton = std::max(b->max_newton, domains[d].max_newton_iter);
    }
    if (total_cells > (1l << 30)) return bfail(b, RMHD_EINVAL, "rmhd_batch_create: batch too large");
    hipError_t e = hipMalloc((void **)&b->pool, total_planes_doubles * sizeof(double));
    // domain table, 256-cell chunks, tile lists
    std::vector<int2> items;
    size_t off = 0;
    for (int d = 0; d < n && e == hipSuccess; ++d) {
        const rmhd_layout &L = b->lay[d];
        DomainDev D{};
        D.g = geo_from(&b->prm[d], L);
        D.P = phys_from(&b->prm[d]);
        D.dt = cfl_dt(&b->prm[d]);
        D.q1src = b->pool + off; off += 5 * L.plane;
        D.w1 = b->pool + off;    off += 5 * L.plane;
        D.r2 = b->pool + off;    off += 14 * L.plane;
        D.acc = b->pool + off;   off += 14 * L.plane;
        b->hdom.push_back(D);
        for (long s = 0; s < L.plane; s += 256) items.push_back(make_int2(d, (int)s));
    }
    b->nitems = (int)items.size();
    b->qcap = (int)total_cells;
    const auto t1 = tile_list(b, 1, 252, 1), t16 = tile_list(b, 2, 60, 12), t8 = tile_list(b, 2, 60, 4);
    b->ntiles1 = (int)t1.size();
    b->ntiles2_16 = (int)t16.size();
    b->ntiles2_8 = (int)t8.size();
    if (e == hipSuccess) e = hipMalloc((void **)&b->ddom, sizeof(DomainDev) * n);
    if (e == hipSuccess) e = upload(&b->items, items);
    if (e == hipSuccess) e = upload(&b->tiles1, t1);
    if (e == hipSuccess) e = upload(&b->tiles2_16, t16);
    if (e == hipSuccess) e = upload(&b->tiles2_8, t8);
    if (e == hipSuccess) e = hipMalloc((void **)&b->counters, 8 * sizeof(unsigned));
    if (e == hipSuccess) e = hipMalloc((void **)&b->qdom, sizeof(int) * b->qcap);
    if (e == hipSuccess) e = hipMalloc((void **)&b->qidx, sizeof(int) * b->qcap);
    if (e == hipSuccess) e = hipMalloc((void **)&b->qit, sizeof(int) * b->qcap);
    if (e == hipSuccess) e = hipMalloc((void **)&b->qx, sizeof(double) * 3 * b->qcap);
    if (e == hipSuccess) e = hipMalloc((void **)&b->qp, sizeof(double) * b->qcap);
    const size_t sb = (size_t)STATS_SLOTS * STATS_STRIDE * sizeof(unsigned long long);
    if (e == hipSuccess) e = hipMalloc((void **)&b->stats, sb);
    if (e == hipSuccess) e = hipMemset(b->stats, 0, sb);
    {
        // slots for the default launch shapes (a larger persistent grid set by the caller
        // falls back to the block-level counters)
        int dev = 0, ncu = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        const long blocks = std::max({(long)b->nitems, 8L * std::max(1, ncu), (long)((b->qcap + 255) / 256)});
        b->nwslots = blocks * 4;
        const size_t wb = (size_t)b->nwslots * STATS_WAVE * sizeof(unsigned long long);
        if (e == hipSuccess) e = hipMalloc((void **)&b->wstats, wb);
        if (e == hipSuccess) e = hipMemset(b->wstats, 0, wb);
    }
    if (e == hipSuccess) e = hipMemset(b->counters, 0, 8 * sizeof(unsigned));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return bfail(b, e == hipErrorOutOfMemory ? RMHD_ENOMEM : RMHD_EHIP,
                                      std::string("rmhd_batch_create: ") + hipGetErrorString(e));
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    b->tune.persistent = 0;
    b->tune.chunks_per_item = 16;
    b->tune.persistent_blocks = std::max(1, cus) * 4;
    b->tune.newton_cap = 2;
    b->tune.flux_rows = 16;
    b->tune.use_graph = 1;
    b->tune.step_ms = 0.0;
    return RMHD_OK;
}

// enqueue one step's kernels on stream s (also used while capturing the graph)
// One flux pass over every domain: the 1-D tile list, then the 2-D list of the tuned height.
template <int PASS>
static void launch_batch_flux(rmhd_batch *b, BatchFluxArgs F, int rows, hipStream_t s)
{
    if (b->ntiles1) {
        F.tiles = b->tiles1;
        hipLaunchKernelGGL((kb_flux<1, 256, 1, PASS>), dim3(b->ntiles1), dim3(256, 1), 0, s, F);
    }
    if (rows == 8 && b->ntiles2_8) {
        F.tiles = b->tiles2_8;
        hipLaunchKernelGGL((kb_flux<2, 64, 8, PASS>), dim3(b->ntiles2_8), dim3(64, 8), 0, s, F);
    } else if (b->ntiles2_16) {
        F.tiles = b->tiles2_16;
        hipLaunchKernelGGL((kb_flux<2, 64, 16, PASS>), dim3(b->ntiles2_16), dim3(64, 16), 0, s, F);
    }
}

static int enqueue_step(rmhd_batch *b, hipStream_t s)
{
    const rmhd_batch_tuning &T = b->tune;
    BatchArgs A{};
    A.dom = b->ddom;
    A.items = b->items;
    A.nitems = b->nitems;
    A.chunks_per_item = std::max(1, T.chunks_per_item);
    A.persistent = T.persistent;
    A.K = std::max(1, std::min(T.newton_cap, b->max_newton));
    A.stats_detail = b->stats_detail;
    A.qdom = b->qdom;
    A.qidx = b->qidx;
    A.qit = b->qit;
    A.qx = b->qx;
    A.qp = b->qp;
    A.qcap = b->qcap;
    A.stats = b->stats;
    const dim3 sgrid(T.persistent ? (unsigned)std::max(1, T.persistent_blocks) : (unsigned)b->nitems);
    const dim3 dgrid((unsigned)((b->qcap + 255) / 256));
    A.wstats = (long)std::max(sgrid.x, dgrid.x) * 4 <= b->nwslots ? b->wstats : nullptr;
    BatchFluxArgs F{};
    F.dom = b->ddom;
    for (int phase = 1; phase <= 2; ++phase) {
        A.phase = phase;
        A.counters = b->counters + 4 * (phase - 1);
        hipLaunchKernelGGL(kb_reset, dim3(1), dim3(64), 0, s, A.counters);
        hipLaunchKernelGGL(kb_stage, sgrid, dim3(256), 0, s, A);
        if (A.K < b->max_newton) hipLaunchKernelGGL(kb_drain, dgrid, dim3(256), 0, s, A);
        if (phase == 1) launch_batch_flux<1>(b, F, T.flux_rows, s);
        else launch_batch_flux<2>(b, F, T.flux_rows, s);
    }
    return bcheck(b, hipGetLastError(), "batch step launch");
}

static int set_arrays(rmhd_batch *b, const double *dt, double *const *cons, double *const *prims)
{
    bool changed = b->table_dirty;
    for (int d = 0; d < b->n; ++d) {
        if (!cons[d] || !prims[d]) return bfail(b, RMHD_EINVAL, "rmhd_batch_step: NULL state array");
        const double h = dt ? dt[d] : cfl_dt(&b->prm[d]);
        if (!(h > 0.0)) return bfail(b, RMHD_EINVAL, "rmhd_batch_step: dt must be > 0");
        DomainDev &D = b->hdom[d];
        if (D.cons != cons[d] || D.prims != prims[d] || D.dt != h) changed = true;
        D.cons = cons[d];
        D.prims = prims[d];
        D.dt = h;
    }
    if (changed) {
        // ordered before the step on the caller's stream; the graph reads the table at run time
        int rc = bcheck(b, hipMemcpyAsync(b->ddom, b->hdom.data(), sizeof(DomainDev) * b->n, hipMemcpyHostToDevice,
                                          b->stream), "domain table upload");
        if (rc) return rc;
        rc = bcheck(b, hipStreamSynchronize(b->stream), "domain table sync");
        if (rc) return rc;
        b->table_dirty = false;
    }
    return RMHD_OK;
}

extern "C" int rmhd_batch_step(rmhd_batch *b, const double *dt, double *const *cons, double *const *prims)
{
    if (!b || !cons || !prims) return bfail(b, RMHD_EINVAL, "rmhd_batch_step: NULL argument");
    int rc = set_arrays(b, dt, cons, prims);
    if (rc) return rc;
    if (!b->tune.use_graph) return enqueue_step(b, b->stream);
    if (!b->exec) {
        rc = bcheck(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "begin capture");
        if (rc) return rc;
        rc = enqueue_step(b, b->cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->cap, &g);
        if (rc) {
            if (g) hipGraphDestroy(g);
            return rc;
        }
        rc = bcheck(b, e, "end capture");
        if (rc) return rc;
        b->graph = g;
        rc = bcheck(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "graph instantiate");
        if (rc) {
            free_graph(b);
            return rc;
        }
    }
    return bcheck(b, hipGraphLaunch(b->exec, b->stream), "graph launch");
}

extern "C" int rmhd_batch_set_tuning(rmhd_batch *b, const rmhd_batch_tuning *t)
{
    if (!b || !t) return bfail(b, RMHD_EINVAL, "rmhd_batch_set_tuning: NULL argument");
    if (t->flux_rows != 8 && t->flux_rows != 16) return bfail(b, RMHD_EINVAL, "flux_rows must be 8 or 16");
    if (t->newton_cap < 1 || t->chunks_per_item < 1 || t->persistent_blocks < 1)
        return bfail(b, RMHD_EINVAL, "newton_cap, chunks_per_item and persistent_blocks must be >= 1");
    b->tune = *t;
    free_graph(b);   // launch shapes changed: capture again on the next step
    return RMHD_OK;
}

extern "C" int rmhd_batch_set_stats_detail(rmhd_batch *b, int detail)
{
    if (!b) return RMHD_EINVAL;
    b->stats_detail = detail != 0;
    free_graph(b);   // the kernels' arguments changed: capture again on the next step
    return RMHD_OK;
}

extern "C" int rmhd_batch_get_tuning(const rmhd_batch *b, rmhd_batch_tuning *t)
{
    if (!b || !t) return RMHD_EINVAL;
    *t = b->tune;
    return RMHD_OK;
}

// Time one candidate: stage 1 (+ drain) and flux pass 1, which read the state and write only
// the library's scratch, so the caller's state is left untouched.
static int time_candidate(rmhd_batch *b, const rmhd_batch_tuning &t, int reps, float *ms)
{
    const rmhd_batch_tuning keep = b->tune;
    b->tune = t;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    BatchArgs A{};
    A.dom = b->ddom;
    A.items = b->items;
    A.nitems = b->nitems;
    A.chunks_per_item = t.chunks_per_item;
    A.persistent = t.persistent;
    A.K = std::max(1, std::min(t.newton_cap, b->max_newton));
    A.qdom = b->qdom; A.qidx = b->qidx; A.qit = b->qit; A.qx = b->qx; A.qp = b->qp;
    A.qcap = b->qcap;
    A.stats = nullptr;
    A.phase = 1;
    A.counters = b->counters;
    BatchFluxArgs F{};
    F.dom = b->ddom;
    float best = 1e30f;
    for (int r = 0; r < reps + 1; ++r) {
        hipEventRecord(e0, b->stream);
        hipLaunchKernelGGL(kb_reset, dim3(1), dim3(64), 0, b->stream, A.counters);
        hipLaunchKernelGGL(kb_stage, dim3(t.persistent ? (unsigned)t.persistent_blocks : (unsigned)b->nitems),
                           dim3(256), 0, b->stream, A);
        if (A.K < b->max_newton)
            hipLaunchKernelGGL(kb_drain, dim3((unsigned)((b->qcap + 255) / 256)), dim3(256), 0, b->stream, A);
        launch_batch_flux<1>(b, F, t.flux_rows, b->stream);
        hipEventRecord(e1, b->stream);
        hipEventSynchronize(e1);
        float m = 0.f;
        hipEventElapsedTime(&m, e0, e1);
        if (r > 0) best = std::min(best, m);   // first run warms up
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    b->tune = keep;
    *ms = best;
    return bcheck(b, hipGetLastError(), "autotune launch");
}

extern "C" int rmhd_batch_autotune(rmhd_batch *b, double *const *cons, double *const *prims, rmhd_batch_tuning *out)
{
    if (!b || !cons || !prims) return bfail(b, RMHD_EINVAL, "rmhd_batch_autotune: NULL argument");
    int rc = set_arrays(b, nullptr, cons, prims);
    if (rc) return rc;
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    rmhd_batch_tuning best = b->tune;
    float best_ms = 1e30f;
    const int caps[] = {1, 2, 1 << 20};
    for (int persistent = 0; persistent <= 1; ++persistent)
        for (int rows : {8, 16})
            for (int cap : caps)
                for (int blocks_per_cu : {2, 4, 8}) {
                    if (!persistent && blocks_per_cu != 2) continue;
                    rmhd_batch_tuning t = b->tune;
                    t.persistent = persistent;
                    t.flux_rows = rows;
                    t.newton_cap = std::min(cap, b->max_newton);
                    t.persistent_blocks = std::max(1, cus) * blocks_per_cu;
                    t.chunks_per_item = 16;
                    float ms = 0.f;
                    rc = time_candidate(b, t, 3, &ms);
                    if (rc) return rc;
                    if (ms < best_ms) {
                        best_ms = ms;
                        best = t;
                    }
                }
    best.step_ms = best_ms;
    best.use_graph = b->tune.use_graph;
    rc = rmhd_batch_set_tuning(b, &best);
    if (rc) return rc;
    b->tune.step_ms = best_ms;
    if (out) *out = b->tune;
    return RMHD_OK;
}

extern "C" int rmhd_batch_get_stats(rmhd_batch *b, rmhd_stats *out, int reset)
{
    if (!b || !out) return bfail(b, RMHD_EINVAL, "rmhd_batch_get_stats: NULL argument");
    unsigned long long raw[STATS_SLOTS * STATS_STRIDE];
    hipLaunchKernelGGL(k_wave_stats_fold, dim3(wave_stats_fold_blocks(b->nwslots)), dim3(256), 0, b->stream, b->wstats,
                       b->nwslots, b->stats);
    int rc = bcheck(b, hipGetLastError(), "k_wave_stats_fold launch");
    if (!rc) rc = bcheck(b, hipMemcpyAsync(raw, b->stats, sizeof(raw), hipMemcpyDeviceToHost, b->stream), "stats copy");
    if (!rc && reset) rc = bcheck(b, hipMemsetAsync(b->stats, 0, sizeof(raw), b->stream), "stats reset");
    if (!rc) rc = bcheck(b, hipStreamSynchronize(b->stream), "stats sync");
    if (rc) return rc;
    stats_fold(raw, out);
    return RMHD_OK;
}

extern "C" const char *rmhd_batch_last_error(const rmhd_batch *b) { return b ? b->err.c_str() : ""; }
