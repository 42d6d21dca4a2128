/*
 * rmhd.h -- C ABI of librmhd.so: the MI355X (gfx950) hot path of the finite-volume IMEX
 * scheme for resistive single-fluid and two-fluid special-relativistic MHD of Wright &
 * Hawke, "Resistive and multi-fluid RMHD on graphics processing units" (arXiv:1808.09721).
 *
 * The problem is the balance law  d_t q = L(q) + Psi(q)  (Sec. 2.2.1, Eq. 9) with
 * L(q) = -d_k f^k(q) (one flux difference per dimension, in 1-D, 2-D or 3-D) from
 * Lax-Friedrichs flux-vector splitting and WENO3 (Sec. 2.2.2, Eq. 12) and the stiff source Psi (Sec. 2.1.1 Eq. 1; Appendix A Eq. A2), advanced by the
 * SSP2(222) IMEX Runge-Kutta scheme (Sec. 2.2.1, Eqs. 10-11, Table 2).
 *
 * Memory.  Every array argument is a DEVICE pointer owned by the caller; the library never
 * frees or reallocates it.  Arrays are FP64 structure-of-arrays: variable v of cell (i, j, k)
 * lives at  base[v * plane + k * slab + j * pitch + i],  i = 0 .. nx+3 (two ghost cells each
 * side), j = 0 .. ny+3 in 2-D and 3-D (j = 0 in 1-D), k = 0 .. nz+3 in 3-D (k = 0 below);
 * interior cells are i = 2 .. nx+1 (and j = 2 .. ny+1, k = 2 .. nz+1 where present).
 * pitch, slab and plane come from rmhd_layout_of(); pitch is nx+4 rounded up to a multiple
 * of 8 doubles (columns beyond nx+3 are padding that is never read); slab = pitch * nyg.
 * Status arrays (int8) and iteration arrays (int32) use one plane of the same indexing.
 *
 * Variable orders:
 *   single fluid  conserved (14): D, Sx, Sy, Sz, tau, Bx, By, Bz, Ex, Ey, Ez, rho_e, psi, phi
 *                 primitive  (5): rho, vx, vy, vz, p
 *   two fluid     conserved (18): D, Sx, Sy, Sz, tau, Dbar, Sbx, Sby, Sbz, taubar,
 *                                 Bx, By, Bz, Ex, Ey, Ez, psi, phi
 *                 primitive (10): rho1, v1x, v1y, v1z, p1, rho2, v2x, v2y, v2z, p2
 *   ideal         conserved  (9): D, Sx, Sy, Sz, tau, Bx, By, Bz, phi   (E = -v x B)
 *                 primitive  (5): rho, vx, vy, vz, p
 *   fields EB (6, init only):     Bx, By, Bz, Ex, Ey, Ez (the ideal model reads B only)
 *
 * Streams.  All work is enqueued on the HIP stream given to rmhd_create() and is ordered
 * with the caller's other work on that stream; calls return before the GPU finishes,
 * except rmhd_get_stats(), which synchronises the stream.
 *
 * Errors.  Functions return RMHD_OK (0) or a negative code; the message is available from
 * rmhd_last_error(ctx) (or rmhd_last_error(NULL) for failures before a context exists).
 * A cell whose root-finds do not converge is NOT an error return: it is reported in the
 * per-cell status array and in the counters of rmhd_get_stats().  No C++ exception crosses
 * this interface.  A context is not thread-safe; distinct contexts are independent.
 */
#ifndef RMHD_H
#define RMHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RMHD_SINGLE_FLUID 0
#define RMHD_TWO_FLUID 1
#define RMHD_IDEAL 2       /* ideal RMHD, advanced by explicit steps (see rmhd_imex_step) */
#define RMHD_BC_OUTFLOW 0  /* zero-gradient copy of the nearest interior cell */
#define RMHD_BC_PERIODIC 1

#define RMHD_OK 0
#define RMHD_EINVAL (-1)
#define RMHD_EHIP (-2)
#define RMHD_ENOMEM (-3)

/* per-cell status codes */
#define RMHD_CELL_OK 0
#define RMHD_CELL_C2P_NOCONV 1
#define RMHD_CELL_C2P_UNPHYSICAL 2
#define RMHD_CELL_NEWTON_NOCONV 3
#define RMHD_CELL_LINESEARCH 4

/* IMEX integrators (Sec. 2.2.1, Eqs. 10-11) */
#define RMHD_SSP2_222 0
#define RMHD_SSP3_332 1

typedef struct rmhd_params {
    int32_t model;            /* RMHD_SINGLE_FLUID, RMHD_TWO_FLUID or RMHD_IDEAL */
    int32_t ndim;             /* 1, 2 or 3 */
    int32_t nx, ny;           /* interior cells (ny = 1 in 1-D); nz below */
    int32_t bc;               /* RMHD_BC_OUTFLOW or RMHD_BC_PERIODIC, all sides */
    int32_t max_c2p_iter;     /* primitive-recovery iteration cap (e.g. 100) */
    int32_t max_newton_iter;  /* implicit-stage iteration cap (e.g. 50) */
    int32_t friction_covariant; /* two-fluid friction: 0 = eta (J - rho_e u) as printed in
                                   Eq. A2, 1 = eta (J - rho_0 u) with the rest-frame charge */
    double x0, x1, y0, y1;    /* domain; dx = (x1-x0)/nx, dy = (y1-y0)/ny */
    double gamma_eos;         /* Gamma-law index (both species) */
    double sigma;             /* conductivity; two-fluid resistivity eta = 1/sigma */
    const double *sigma_cell; /* optional device plane of per-cell conductivities (same
                                 indexing as a state plane), or NULL.  Only its interior cells
                                 are read, once, by rmhd_create: the context keeps its own
                                 copy and fills that copy's ghost cells by the boundary
                                 condition, so the caller's ghost values are ignored and the
                                 plane may be released after rmhd_create returns */
    double mu1, mu2;          /* two-fluid charge-to-mass ratios */
    double kappa;             /* divergence-cleaning damping rate (1 in the paper) */
    double cfl;               /* CFL number for rmhd_dt() */
    double c2p_tol;           /* primitive-recovery residual tolerance (1e-13, Sec. 2.1.3) */
    double newton_tol;        /* implicit-stage residual tolerance (e.g. 1e-12) */
    int32_t integrator;       /* RMHD_SSP2_222 (0, Table 2) or RMHD_SSP3_332 (1, Table 3) */
    int32_t c2p_primary_only; /* 0: where the recovery's z = rho h W^2 iteration does not
                                 converge, a Newton iteration on the pressure takes over (the
                                 paper keeps two residuals, Sec. 2.1.3); 1: z iteration only */
    int32_t nz;               /* 3-D: interior cells along z (>= 4); 0 or 1 below 3-D */
    int32_t reserved_;        /* must be 0 */
    double z0, z1;            /* 3-D: domain along z; dz = (z1-z0)/nz */
} rmhd_params;

typedef struct rmhd_layout {
    int64_t nxg, nyg;         /* cells per row / rows per z plane, ghosts included */
    int64_t pitch;            /* doubles between rows */
    int64_t plane;            /* doubles between variables */
    int32_t ncons, nprim;
    int64_t nzg;              /* z planes, ghosts included (1 below 3-D) */
    int64_t slab;             /* doubles between z planes (pitch * nyg) */
} rmhd_layout;

typedef struct rmhd_stats {
    int64_t stage_cells;      /* cell solves counted (interior cells x implicit stages) */
    int64_t newton_iters;     /* their Newton iterations, summed */
    int64_t residual_evals;   /* their residual evaluations (Newton trials included), summed */
    int64_t c2p_iters;        /* primitive-recovery iterations inside them, summed */
    int32_t newton_max;       /* largest Newton iteration count of one cell */
    int32_t failures;         /* cell solves that ended with a nonzero status */
    /* collected only while detailed statistics are on (rmhd_set_stats_detail): */
    int64_t newton_hist[16];  /* cell solves by Newton iteration count (last bin: 15 or more) */
    double residual_max;      /* largest final |G|_inf / max(1, |R_x|_inf) of a converged cell */
    int64_t jacobian_evals;   /* Jacobian evaluations of the counted cell solves, summed (the
                                 polishing step after convergence reuses the last one) */
} rmhd_stats;

/* Per-kernel GPU time of rmhd_imex_step, from HIP events recorded on the context's stream
 * around every launch while timing is enabled (rmhd_set_timing). */
typedef struct rmhd_timing {
    double stage_ms;          /* implicit-stage kernels (learned guess, solve, queue), summed */
    double flux_ms;           /* flux-divergence + combiner kernel, summed */
    double c2p_ms;            /* separate primitive-recovery kernel, summed (0: the step
                                 recovers the primitives inside its second flux pass) */
    int64_t stage_launches, flux_launches, c2p_launches;
    int64_t steps;
} rmhd_timing;

typedef struct rmhd_ctx rmhd_ctx;

/* Array geometry for a parameter set (no GPU work).  Returns RMHD_EINVAL on bad sizes. */
int rmhd_layout_of(const rmhd_params *params, rmhd_layout *out);

/* Create a context on the current HIP device: validates params, allocates the library's
 * own scratch (stage buffers, counters, the copy of sigma_cell) and binds the stream
 * (hipStream_t, NULL = default).  The params are copied; sigma_cell is read before return. */
int rmhd_create(const rmhd_params *params, void *hip_stream, rmhd_ctx **out);
void rmhd_destroy(rmhd_ctx *ctx);

/* Initial data (Sec. 2.1.1, Eq. 2; Sec. 2.1.2, Eq. 6): cons on every cell from the interior
 * primitives and fields; rho_e = div E by second-order central differences (Gauss's law,
 * Sec. 2.1.1); psi = phi = 0; ghost cells of cons are filled by the boundary condition.
 * prims/EB: interior read only.  cons: written everywhere. */
int rmhd_init_state(rmhd_ctx *ctx, const double *prims, const double *EB, double *cons);

/* Primitive recovery (Sec. 2.1.3) on every cell, ghosts included.  prims holds the pressure
 * guesses on entry (non-physical values are replaced by a bracket midpoint) and the
 * primitives on exit.  status/iters (int8 / int32 planes) may be NULL. */
int rmhd_cons2prim(rmhd_ctx *ctx, const double *cons, double *prims, int8_t *status, int32_t *iters);

/* L(q) = -d_k f^k(q) (Eq. 9; FVS + WENO3, Sec. 2.2.2) on the interior cells.  First fills the
 * ghost cells of cons and prims in place from their interior by the boundary condition.
 * L: written on the interior only. */
int rmhd_F(rmhd_ctx *ctx, double *cons, double *prims, double *L);

/* Implicit stage (Sec. 2.2.1, Eq. 10; resistive models only): solve Q = R + a Psi(Q) per cell, a = a_ii dt, on every
 * cell including ghosts (so Q's ghosts follow R's).  guess: optional array of conserved
 * variables whose source-carrying components start Newton (NULL = the plain guess R; two
 * fluid: Newton starts from whichever of guess and R has the smaller residual); a cell whose
 * Newton fails from guess is solved again from R.
 * prims: pressure guesses on entry, primitives of Q on exit.  Q may alias R.  status and
 * iters (Newton iterations) may be NULL. */
int rmhd_implicit_stage(rmhd_ctx *ctx, double a, const double *R, const double *guess, double *Q,
                        double *prims, int8_t *status, int32_t *iters);

/* One IMEX step of size dt (Sec. 2.2.1, Eqs. 10-11) with the context's integrator: SSP2(222)
 * (Table 2, two implicit stages, gamma = 1 - 1/sqrt 2) or SSP3(332) (Table 3, three).
 * RMHD_IDEAL contexts, which have no stiff source, take the explicit half of the same
 * tableau (Heun's method, or the three-stage SSP Runge-Kutta method) with the divergence
 * cleaning's damping explicit too; their recovery is the two-dimensional root-find of
 * Sec. 2.1.3 (with a one-dimensional bracketed fallback unless c2p_primary_only).
 * cons (ghosts valid) is advanced in place; prims holds the primitives of cons on entry
 * (used as root-find starting points) and those of the new cons on exit, ghosts included.
 * Counters of the stage solves are accumulated into the context's statistics. */
int rmhd_imex_step(rmhd_ctx *ctx, double dt, double *cons, double *prims);

/* With enable = 1, rmhd_imex_step captures its kernels once into a HIP graph (on a private
 * stream) and replays it on the context's stream while (dt, cons, prims) and the context's
 * settings stay the same; any change captures again.  Steps with timing or harvesting on
 * are launched directly.  Results are identical either way.  Default 0. */
int rmhd_set_graph(rmhd_ctx *ctx, int enable);

/* Time step CFL / sum_d (1/dx_d) over the grid's dimensions (maximum signal speed c = 1). */
double rmhd_dt(const rmhd_ctx *ctx);

/* Copy the accumulated statistics (synchronises the stream); reset != 0 zeroes them. */
int rmhd_get_stats(rmhd_ctx *ctx, rmhd_stats *out, int reset);

/* Detailed statistics (1) or the six basic counters only (0, default): the histogram and the
 * residual maximum cost a few microseconds per stage launch. */
int rmhd_set_stats_detail(rmhd_ctx *ctx, int detail);

/* Newton steps a cell may take from unconverged iterates in the first pass of an implicit
 * stage (rmhd_implicit_stage, rmhd_imex_step) before it moves to a compacted queue that a
 * second kernel finishes in full wavefronts: the first pass then costs what its fastest
 * cells need instead of what the slowest cell of each wavefront needs.  cap >=
 * max_newton_iter disables the queue and gives the uninterrupted solve bit for bit; a queued
 * cell resumes from its saved unknowns and pressures with a fresh Jacobian, which agrees with
 * the uninterrupted solve to the Newton tolerance.  Default (until a cap is set): no queue.
 * cap must be >= 1. */
int rmhd_set_newton_cap(rmhd_ctx *ctx, int cap);

/* Jacobian reuse in the implicit stage's Newton iteration (resistive models): after a step
 * that cut ||G||_inf to at most keep times its previous value, the next step reuses the same
 * factorised Jacobian (a chord step) instead of forming it at the new iterate; a chord step
 * is accepted only at full length and only if it cuts ||G||_inf by the same factor, else the
 * Jacobian is formed afresh there.  The stopping rule and the polishing step are unchanged,
 * so results agree with the iteration without reuse to the Newton tolerance.  Default 0.1
 * (also in the batched form); keep = 0: a fresh Jacobian at every unconverged iterate.  keep
 * must lie in [0, 1). */
int rmhd_set_jacobian_reuse(rmhd_ctx *ctx, double keep);

/* Shape of the 2-D flux-pass thread block: 16 (64 x 16 threads, 60 x 12 interior cells), 12
 * (64 x 12, 60 x 8), 8 (64 x 8, 60 x 4: more blocks and more halo work); for the two-fluid
 * model only 24 (32 x 24 threads, 28 x 20 interior cells), for the single-fluid and ideal
 * models only 32 (32 x 32 threads, 28 x 28 interior cells); RMHD_EINVAL otherwise.
 * 0 (default): whichever of the model's shapes (single fluid and ideal 16 and 32; two fluid
 * 12, 24 and 16) needs the fewest tile rounds over the compute units, weighted by each tile's
 * measured time.  Results do not depend on it beyond rounding (the two-fluid shapes, and 8,
 * 12 and 16 among themselves, give identical results; 32 forms the x stencil through LDS
 * instead of across lanes, which changes the last bits).  The x-y tiles of 3-D grids: two
 * fluid 12 or 24, the other models 16 or 32 (a requested one of those is kept, otherwise
 * chosen as in 2-D). */
int rmhd_set_flux_rows(rmhd_ctx *ctx, int rows);

/* Enable (1) or disable (0) per-kernel event timing of rmhd_imex_step.  While enabled each
 * step waits for its own kernels to finish (to read the events), so it is meant for a
 * measurement pass, not for production stepping. */
int rmhd_set_timing(rmhd_ctx *ctx, int enable);

/* Copy the accumulated per-kernel times; reset != 0 zeroes them. */
int rmhd_get_timing(rmhd_ctx *ctx, rmhd_timing *out, int reset);

/* Message of the last failing call on ctx (or of the last failing rmhd_create/layout call
 * when ctx is NULL).  Owned by the library; valid until the next call on the same ctx. */
const char *rmhd_last_error(const rmhd_ctx *ctx);

/* ------------------------------------------------------------------------------------
 * The step without allocation, for callers that cannot allocate device memory: code being
 * captured into a HIP graph, tight serving loops, harnesses that forbid hipMalloc.
 * rmhd_imex_step_noalloc() does what rmhd_imex_step() does on a context made from *params
 * (same kernels, results equal bit for bit), but needs no context: its stage scratch lives
 * in one array of RMHD_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends, and the call itself allocates nothing (no hipMalloc, hipFree or
 * allocating library routine) and launches kernels only (no memset, no copy), on hip_stream.
 * Limits: the grid's scratch (rmhd_noalloc_scratch_bytes) must fit the array -- e.g. the
 * single-fluid 256 x 512 grid needs 41 MB with SSP2(222), 62 MB with SSP3(332) -- else
 * RMHD_EINVAL; sigma_cell must be NULL (scalar conductivity); no statistics, timing, stage
 * queue or learned guess.  Every call on one GPU shares that GPU's array: calls that overlap
 * in time on one GPU (two streams, two threads) race and give wrong results; calls ordered
 * on one stream are safe.  Nothing in the array has to start at zero.  Errors are reported
 * by rmhd_last_error(NULL).
 * ------------------------------------------------------------------------------------ */
#define RMHD_NOALLOC_SCRATCH_BYTES (64u << 20)

/* Scratch bytes rmhd_imex_step_noalloc() needs for *params (0 if params are invalid). */
size_t rmhd_noalloc_scratch_bytes(const rmhd_params *params);

/* One IMEX step of size dt of cons/prims (device arrays laid out as rmhd_layout_of(params)
 * gives, exactly as for rmhd_imex_step()), enqueued on hip_stream (hipStream_t, NULL =
 * default), with no context and no allocation. */
int rmhd_imex_step_noalloc(const rmhd_params *params, void *hip_stream, double dt, double *cons, double *prims);

/* ------------------------------------------------------------------------------------
 * Batched form: many independent single-fluid domains of uneven size and stiffness advanced
 * by one launch per kernel of the SSP2(222) step for all of them (each domain with its own
 * grid, boundary, sigma and dt), with a convergence-compacted queue for the implicit stage
 * (cells still unconverged after newton_cap Newton steps continue in full wavefronts),
 * the step captured once in a HIP graph, and launch shapes chosen by rmhd_batch_autotune().
 * The method per cell is exactly the one of rmhd_imex_step (Sec. 2.2.1, Eqs. 10-11): with
 * newton_cap >= max_newton_iter the results equal rmhd_imex_step's bit for bit; a queued cell
 * resumes from its saved unknowns and pressure with a fresh Jacobian, which agrees with the
 * uninterrupted solve to the Newton tolerance.
 * ------------------------------------------------------------------------------------ */
typedef struct rmhd_batch rmhd_batch;

typedef struct rmhd_batch_tuning {
    int32_t persistent;         /* stage launch: 1 = persistent grid pulling work items from an
                                   atomic counter, 0 = one block per 256-cell chunk */
    int32_t chunks_per_item;    /* persistent mode: 256-cell chunks per counter grab */
    int32_t persistent_blocks;  /* persistent mode: blocks in the grid */
    int32_t newton_cap;         /* Newton steps from unconverged iterates before a cell moves to
                                   the compacted queue (a cell converged by then still takes its
                                   polishing step)
                                   (>= max_newton_iter: no queue) */
    int32_t flux_rows;          /* rows of a 2-D flux tile block: 8 or 16 */
    int32_t use_graph;          /* 1: capture the step in a HIP graph and replay it */
    double step_ms;             /* set by rmhd_batch_autotune: time of the chosen shape for one
                                   implicit stage plus one flux pass (half an SSP2 step; the
                                   best of three timed repetitions) */
} rmhd_batch_tuning;

/* Create a batch of n domains (each validated as for rmhd_create; single fluid, 1-D or 2-D,
 * scalar sigma).  Allocates pooled stage scratch for all domains.  *out is set even on failure so
 * that rmhd_batch_last_error() can explain it; always release with rmhd_batch_destroy(). */
int rmhd_batch_create(const rmhd_params *domains, int n, void *hip_stream, rmhd_batch **out);
void rmhd_batch_destroy(rmhd_batch *batch);

/* One SSP2(222) step of every domain.  dt: host array of n time steps, or NULL for each
 * domain's CFL time step.  cons, prims: host arrays of n device pointers, laid out per domain
 * as in rmhd_layout_of(); advanced in place exactly as rmhd_imex_step() does. */
int rmhd_batch_step(rmhd_batch *batch, const double *dt, double *const *cons, double *const *prims);

/* Time the candidate launch shapes on the given state (only library scratch is written) and
 * keep the fastest; the choice is returned in *out (may be NULL). */
int rmhd_batch_autotune(rmhd_batch *batch, double *const *cons, double *const *prims, rmhd_batch_tuning *out);
int rmhd_batch_set_tuning(rmhd_batch *batch, const rmhd_batch_tuning *tuning);
int rmhd_batch_get_tuning(const rmhd_batch *batch, rmhd_batch_tuning *tuning);

/* Statistics of the stage solves of all domains (synchronises the stream). */
int rmhd_batch_get_stats(rmhd_batch *batch, rmhd_stats *out, int reset);
int rmhd_batch_set_stats_detail(rmhd_batch *batch, int detail);   /* as rmhd_set_stats_detail */
const char *rmhd_batch_last_error(const rmhd_batch *batch);

#ifdef __cplusplus
}
#endif
#endif
