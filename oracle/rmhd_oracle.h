/*
 * rmhd_oracle.h -- plain FP64 CPU reference ("the oracle") for the finite-volume
 * IMEX scheme for resistive single-fluid and two-fluid special-relativistic MHD of
 * Wright & Hawke, "Resistive and multi-fluid RMHD on graphics processing units"
 * (arXiv:1808.09721).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load, link or call
 * this library: only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * implementation; the two meet only through the seeded input generators (which
 * hold none of the method's arithmetic) and through numpy arrays in the tests.
 *
 * Layout used by every grid-level routine here (independent of the GPU layout):
 *   array[v][k][j][i], v = variable, k = 0..NZ-1, j = 0..NY-1, i = 0..NX-1, x fastest,
 *   where NX = nx + 4, NY = ny + 4 in 2-D and 3-D (1 in 1-D), NZ = nz + 4 in 3-D (1
 *   below): two ghost cells per side in every simulated direction.  Interior cell
 *   (ix, iy, iz) sits at i = ix + 2, j = iy + 2, k = iz + 2 (or 0 where absent).
 *
 * Variable orders:
 *   single fluid, conserved (14): D, Sx, Sy, Sz, tau, Bx, By, Bz, Ex, Ey, Ez, rho_e, psi, phi
 *   single fluid, primitive (5):  rho, vx, vy, vz, p
 *   two fluid, conserved (18):    D, Sx, Sy, Sz, tau, Dbar, Sbx, Sby, Sbz, taubar,
 *                                 Bx, By, Bz, Ex, Ey, Ez, psi, phi
 *   two fluid, primitive (10):    rho1, v1x, v1y, v1z, p1, rho2, v2x, v2y, v2z, p2
 *                                 (species 1 has charge-to-mass ratio mu1, species 2 mu2)
 *   ideal, conserved (9):         D, Sx, Sy, Sz, tau, Bx, By, Bz, phi
 *   ideal, primitive (5):         rho, vx, vy, vz, p
 * The ideal model has no stiff source: orc_ssp2_step / orc_ssp3_step advance it with the
 * explicit halves of the same tableaux (no implicit stage).
 */
#ifndef RMHD_ORACLE_H
#define RMHD_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_params {
    int model;              /* 0 = resistive single fluid, 1 = resistive two fluid, 2 = ideal */
    int ndim;               /* 1, 2 or 3 */
    int nx, ny;             /* interior cells (ny = 1 in 1-D) */
    int bc;                 /* 0 = outflow (zero-gradient copy), 1 = periodic */
    int max_c2p_iter;
    int max_newton_iter;
    int friction_covariant; /* two-fluid friction term: 0 = as printed (rho_e u), 1 = rest-frame charge (rho_0 u) */
    double dx, dy;
    double gamma;           /* Gamma-law index, both species */
    double sigma;           /* conductivity; two-fluid resistivity eta = 1/sigma */
    double mu1, mu2;        /* two-fluid charge-to-mass ratios */
    double kappa;           /* divergence-cleaning damping rate */
    double c2p_tol;         /* primitive-recovery residual tolerance */
    double newton_tol;      /* implicit-stage residual tolerance */
    const double *sigma_cell; /* optional per-cell conductivity [NZ][NY][NX], or NULL */
    int nz;                 /* interior cells along z in 3-D (unused below 3-D) */
    double dz;
} orc_params;

/* Status codes written per cell. */
#define ORC_OK            0
#define ORC_C2P_NOCONV    1
#define ORC_C2P_UNPHYS    2
#define ORC_NEWTON_NOCONV 3
#define ORC_LINESEARCH    4

int orc_ncons(int model);
int orc_nprim(int model);

/* ---- per-cell routines (arrays of length ncons / nprim) ---- */
void orc_prim2cons_cell(const orc_params *p, const double *w, const double *EB,
                        double rho_e, double *q);
int  orc_cons2prim_cell(const orc_params *p, const double *q, double *w, int *iters);
void orc_flux_cell(const orc_params *p, const double *q, const double *w, double sigma,
                   int dir, double *f);
void orc_source_cell(const orc_params *p, const double *q, const double *w, double sigma,
                     double *s);
int  orc_implicit_cell(const orc_params *p, double a, double sigma, const double *R,
                       double *Q, double *w, int *iters);
int  orc_implicit_cell_from(const orc_params *p, double a, double sigma, const double *R,
                            const double *Qstart, double *Q, double *w, int *iters);
int  orc_implicit_residual_cell(const orc_params *p, double a, double sigma,
                                const double *R, const double *Q, double *G, int *nG);
void orc_weno3_face(const double *fm1, const double *f0, const double *fp1,
                    double *out, int n);

/* ---- grid routines (layout described above) ---- */
void   orc_bc_fill(const orc_params *p, double *arr, int nvar);
void   orc_init_state(const orc_params *p, const double *prims, const double *EB, double *cons);
void   orc_cons2prim(const orc_params *p, const double *cons, double *prims,
                     signed char *status, int *iters);
void   orc_rhs(const orc_params *p, const double *cons, const double *prims, double *L);
void   orc_implicit(const orc_params *p, double a, const double *R, double *Q, double *prims,
                    signed char *status, int *iters);
int    orc_ssp2_step(const orc_params *p, double dt, double *cons, double *prims,
                     long long *newton_iters, int *max_newton, int *nfail);
/* One SSP3(332) IMEX step (Table 3 tableau), same conventions as orc_ssp2_step. */
int    orc_ssp3_step(const orc_params *p, double dt, double *cons, double *prims,
                     long long *newton_iters, int *max_newton, int *nfail);
double orc_dt(const orc_params *p, double cfl);

/* OpenMP threads of the grid loops (n <= 0: unchanged); returns the number in effect. */
int orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
