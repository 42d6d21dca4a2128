/*
 * rmhd_oracle.c -- plain FP64 CPU reference ("the oracle") for the IMEX finite-volume
 * scheme for resistive single-fluid and two-fluid special-relativistic MHD of
 * Wright & Hawke (arXiv:1808.09721).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It shares no code
 * with the HIP implementation.
 *
 * Every routine writes out the definition the paper gives, in the paper's order,
 * with no blocking, fusion or reordering.  Where the paper is silent the reading
 * taken is stated at the routine.  Build: gcc -O2 -ffp-contract=off -fopenmp.
 */
#include "rmhd_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* Conserved / primitive indices (variable orders in rmhd_oracle.h). */
enum { SF_D, SF_SX, SF_SY, SF_SZ, SF_TAU, SF_BX, SF_BY, SF_BZ, SF_EX, SF_EY, SF_EZ,
       SF_RHOE, SF_PSI, SF_PHI, SF_NC };
enum { TF_D, TF_SX, TF_SY, TF_SZ, TF_TAU, TF_DB, TF_SBX, TF_SBY, TF_SBZ, TF_TAUB,
       TF_BX, TF_BY, TF_BZ, TF_EX, TF_EY, TF_EZ, TF_PSI, TF_PHI, TF_NC };
enum { ID_D, ID_SX, ID_SY, ID_SZ, ID_TAU, ID_BX, ID_BY, ID_BZ, ID_PHI, ID_NC };
enum { P_RHO, P_VX, P_VY, P_VZ, P_P, FLUID_NP };
#define MAXC 18
#define MAXP 10

int orc_ncons(int model) { return model == 0 ? SF_NC : model == 1 ? TF_NC : ID_NC; }
int orc_nprim(int model) { return model == 1 ? 2 * FLUID_NP : FLUID_NP; }

static void ideal_prim2cons(const orc_params *p, const double *w, const double *B, double *q);
static int ideal_c2p(const orc_params *p, const double *q, double *w, int *iters);
static void ideal_flux(const orc_params *p, const double *q, const double *w, int k, double *f);

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Lorentz factor W = 1/sqrt(1 - v_i v^i) and Gamma-law specific enthalpy
 * h = 1 + Gamma p / (rho (Gamma - 1))  (Sec. 2.1.1, Eqs. 3-4; EOS p = rho e (Gamma-1), Sec. 2.1). */
static double lorentz(const double *v) { return 1.0 / sqrt(1.0 - dot3(v, v)); }
static double enthalpy(double gam, double rho, double p) { return 1.0 + gam * p / (rho * (gam - 1.0)); }

/* ------------------------------------------------------------------------------------------
 * prim -> cons
 * ---------------------------------------------------------------------------------------- */

/* Single fluid, Sec. 2.1.1 Eq. 2:  D = rho W,  S = rho h W^2 v + E x B,
 * tau = rho h W^2 - p + (E^2 + B^2)/2 - rho W;  B, E copied;  rho_e given; psi = phi = 0
 * at t = 0 (divergence cleaning, end of Sec. 2.1.1).
 * Two fluid, Sec. 2.1.2 Eq. 6, summed over the species s = 1, 2. */
void orc_prim2cons_cell(const orc_params *p, const double *w, const double *EB, double rho_e, double *q)
{
    if (p->model == 2) {
        ideal_prim2cons(p, w, EB, q);
        return;
    }
    const double *B = EB, *E = EB + 3;
    double ExB[3];
    cross3(E, B, ExB);
    const double em = 0.5 * (dot3(E, E) + dot3(B, B));
    if (p->model == 0) {
        const double rho = w[P_RHO], *v = w + P_VX, pr = w[P_P];
        const double W = lorentz(v), h = enthalpy(p->gamma, rho, pr);
        q[SF_D] = rho * W;
        for (int i = 0; i < 3; ++i) q[SF_SX + i] = rho * h * W * W * v[i] + ExB[i];
        q[SF_TAU] = rho * h * W * W - pr + em - rho * W;
        for (int i = 0; i < 3; ++i) { q[SF_BX + i] = B[i]; q[SF_EX + i] = E[i]; }
        q[SF_RHOE] = rho_e;
        q[SF_PSI] = 0.0;
        q[SF_PHI] = 0.0;
    } else {
        const double mu[2] = { p->mu1, p->mu2 };
        for (int k = 0; k < TF_NC; ++k) q[k] = 0.0;
        for (int s = 0; s < 2; ++s) {
            const double *ws = w + FLUID_NP * s;
            const double rho = ws[P_RHO], *v = ws + P_VX, pr = ws[P_P];
            const double W = lorentz(v), h = enthalpy(p->gamma, rho, pr);
            q[TF_D] += rho * W;
            for (int i = 0; i < 3; ++i) q[TF_SX + i] += rho * h * W * W * v[i];
            q[TF_TAU] += rho * h * W * W - pr - rho * W;
            q[TF_DB] += mu[s] * rho * W;
            for (int i = 0; i < 3; ++i) q[TF_SBX + i] += mu[s] * rho * h * W * W * v[i];
            q[TF_TAUB] += mu[s] * (rho * h * W * W - pr - rho * W);
        }
        for (int i = 0; i < 3; ++i) q[TF_SX + i] += ExB[i];
        q[TF_TAU] += em;
        for (int i = 0; i < 3; ++i) { q[TF_BX + i] = B[i]; q[TF_EX + i] = E[i]; }
        q[TF_PSI] = 0.0;
        q[TF_PHI] = 0.0;
    }
}

/* ------------------------------------------------------------------------------------------
 * cons -> prim (Sec. 2.1.3)
 * ---------------------------------------------------------------------------------------- */

/* Pressure residual of one ideal-gas fluid with hydrodynamic conserved part
 * (D, St, taut):  with Q = taut + D + p (= rho h W^2),  v = St/Q,  W = (1 - v^2)^(-1/2),
 * rho = D/W,  rho eps = Q/W^2 - rho - p, the residual is f(p) = (Gamma - 1) rho eps - p and
 * f'(p) = (Gamma - 1) v^2 (1 - D W / Q) - 1  (< 0 for Gamma <= 2, so the root is unique). */
static void fluid_residual(double gam, double D, double s2, double Eh, double pr, double *f, double *df)
{
    const double Q = Eh + pr;
    const double v2 = s2 / (Q * Q);
    const double W = 1.0 / sqrt(1.0 - v2);
    const double rho = D / W;
    const double rhoeps = Q / (W * W) - rho - pr;
    *f = (gam - 1.0) * rhoeps - pr;
    *df = (gam - 1.0) * v2 * (1.0 - D * W / Q) - 1.0;
}

/* Recover (rho, v, p) of one fluid.  The paper minimises a single residual by Newton-
 * Raphson to an absolute tolerance of 1e-13 (Sec. 2.1.3) without printing the residual;
 * the reading taken is the pressure residual above, stopped at |f| <= tol * max(1, p),
 * after which one more Newton step is taken, so the answer sits at round-off.  Newton is
 * safeguarded by bisection on the bracket (p_lo, p_hi): p_lo = max(|St| - taut - D, 0)
 * keeps v < 1 and f(p_hi) <= 0 at p_hi = (Gamma - 1)(taut + D). */
static int fluid_c2p(double gam, double D, const double *St, double taut, double pguess, double tol,
                     int maxit, double *w, int *iters)
{
    const double Eh = taut + D;
    const double s2 = dot3(St, St);
    const double s = sqrt(s2);
    *iters = 0;
    if (!(D > 0.0) || !(Eh > 0.0) || !isfinite(s2)) return ORC_C2P_UNPHYS;
    double lo = s - Eh > 0.0 ? s - Eh : 0.0;
    double hi = (gam - 1.0) * Eh;
    if (!(hi > lo)) return ORC_C2P_UNPHYS;
    double pr = pguess;
    if (!(pr > lo && pr < hi)) pr = 0.5 * (lo + hi);
    int conv = 0, it;
    for (it = 1; it <= maxit; ++it) {
        double f, df;
        fluid_residual(gam, D, s2, Eh, pr, &f, &df);
        if (f > 0.0) lo = pr; else hi = pr;
        double pn = pr - f / df;
        if (fabs(f) <= tol * (pr > 1.0 ? pr : 1.0)) {
            if (pn >= 0.0 && Eh + pn > s) pr = pn; /* the extra (polishing) Newton step */
            conv = 1;
            break;
        }
        if (!(pn > lo && pn < hi)) pn = 0.5 * (lo + hi);
        pr = pn;
    }
    *iters = conv ? it : maxit;
    const double Q = Eh + pr;
    for (int i = 0; i < 3; ++i) w[P_VX + i] = St[i] / Q;
    const double W = lorentz(w + P_VX);
    w[P_RHO] = D / W;
    w[P_P] = pr;
    if (!conv) return ORC_C2P_NOCONV;
    if (!(w[P_RHO] > 0.0) || !isfinite(W)) return ORC_C2P_UNPHYS;
    return ORC_OK;
}

/* Full cons2prim.  First the electromagnetic parts are removed:  St = S - E x B and
 * taut = tau - (E^2 + B^2)/2 (Eq. 2; Sec. 2.1.3).  Two fluid: the totals and the
 * charge-to-mass weighted sums are split into species (Sec. 2.1.3, Eqs. 7-8):
 *   X_1 = (Xbar - mu2 X)/(mu1 - mu2),   X_2 = (Xbar - mu1 X)/(mu2 - mu1)
 * for X = D, St_i, taut (the printed Eq. 8 subtracts the EM part from the barred momentum;
 * the reading taken subtracts it from the total momentum S, the only one that carries it).
 * w holds the pressure guess(es) on entry and the primitives on exit. */
int orc_cons2prim_cell(const orc_params *p, const double *q, double *w, int *iters)
{
    if (p->model == 2) return ideal_c2p(p, q, w, iters);
    const int model = p->model;
    const double *B = q + (model == 0 ? SF_BX : TF_BX), *E = q + (model == 0 ? SF_EX : TF_EX);
    double ExB[3], St[3];
    cross3(E, B, ExB);
    const double em = 0.5 * (dot3(E, E) + dot3(B, B));
    if (model == 0) {
        for (int i = 0; i < 3; ++i) St[i] = q[SF_SX + i] - ExB[i];
        const double taut = q[SF_TAU] - em;
        return fluid_c2p(p->gamma, q[SF_D], St, taut, w[P_P], p->c2p_tol, p->max_c2p_iter, w, iters);
    }
    const double m1 = p->mu1, m2 = p->mu2;
    for (int i = 0; i < 3; ++i) St[i] = q[TF_SX + i] - ExB[i];
    const double taut = q[TF_TAU] - em;
    const double D1 = (q[TF_DB] - m2 * q[TF_D]) / (m1 - m2);
    const double D2 = (q[TF_DB] - m1 * q[TF_D]) / (m2 - m1);
    double S1[3], S2[3];
    for (int i = 0; i < 3; ++i) {
        S1[i] = (q[TF_SBX + i] - m2 * St[i]) / (m1 - m2);
        S2[i] = (q[TF_SBX + i] - m1 * St[i]) / (m2 - m1);
    }
    const double t1 = (q[TF_TAUB] - m2 * taut) / (m1 - m2);
    const double t2 = (q[TF_TAUB] - m1 * taut) / (m2 - m1);
    int it1 = 0, it2 = 0;
    int st1 = fluid_c2p(p->gamma, D1, S1, t1, w[P_P], p->c2p_tol, p->max_c2p_iter, w, &it1);
    int st2 = fluid_c2p(p->gamma, D2, S2, t2, w[FLUID_NP + P_P], p->c2p_tol, p->max_c2p_iter,
                        w + FLUID_NP, &it2);
    *iters = it1 + it2;
    if (st1 == ORC_C2P_UNPHYS || st2 == ORC_C2P_UNPHYS) return ORC_C2P_UNPHYS;
    if (st1 != ORC_OK) return st1;
    return st2;
}

/* ------------------------------------------------------------------------------------------
 * fluxes and sources
 * ---------------------------------------------------------------------------------------- */

/* Ohm's law current of the single-fluid model (Sec. 2.1.1, Eq. 2):
 * J = rho_e v + W sigma [E + v x B - (v.E) v]. */
static void sf_current(const double *q, const double *w, double sigma, double *J)
{
    const double *v = w + P_VX, *B = q + SF_BX, *E = q + SF_EX;
    const double W = lorentz(v);
    double vxB[3];
    cross3(v, B, vxB);
    const double vE = dot3(v, E);
    for (int i = 0; i < 3; ++i) J[i] = q[SF_RHOE] * v[i] + W * sigma * (E[i] + vxB[i] - vE * v[i]);
}

/* Flux of B_i and E_i in direction k (Eq. 1; Appendix A, Eq. A1): F(B_i) = -eps_ijk E_j +
 * delta_ik phi and F(E_i) = eps_ijk B_j + delta_ik psi;  F(psi) = E_k, F(phi) = B_k. */
static void em_flux(const double *B, const double *E, double psi, double phi, int k, double *fB,
                    double *fE, double *fpsi, double *fphi)
{
    static const int eps[3][3][3] = { { { 0, 0, 0 }, { 0, 0, 1 }, { 0, -1, 0 } },
                                      { { 0, 0, -1 }, { 0, 0, 0 }, { 1, 0, 0 } },
                                      { { 0, 1, 0 }, { -1, 0, 0 }, { 0, 0, 0 } } };
    for (int i = 0; i < 3; ++i) {
        fB[i] = (i == k) ? phi : 0.0;
        fE[i] = (i == k) ? psi : 0.0;
        for (int j = 0; j < 3; ++j) {
            fB[i] -= eps[i][j][k] * E[j];
            fE[i] += eps[i][j][k] * B[j];
        }
    }
    *fpsi = E[k];
    *fphi = B[k];
}

/* Flux vector f^k(q) in direction k (0 = x, 1 = y).
 * Single fluid (Eq. 1 with Eq. 2): F(D) = D v^k, F(S_i) = S_ik = rho h W^2 v_i v_k +
 * [p + (E^2+B^2)/2] delta_ik - E_i E_k - B_i B_k, F(tau) = S^k - D v^k, F(rho_e) = J^k.
 * Two fluid (Appendix A, Eqs. A1 and A3; the stress uses each species' own velocity v_s^k):
 * F(D) = sum rho_s W_s v_s^k, F(S_i) = sum (rho_s h_s W_s^2 v_si v_s^k + p_s delta_ik)
 * - E_i E_k - B_i B_k + (E^2 + B^2)/2 delta_ik, F(tau) = S^k - sum D_s v_s^k,
 * F(Dbar) = sum mu_s rho_s W_s v_s^k, F(Sbar_i) = sum mu_s (rho_s h_s W_s^2 v_si v_s^k +
 * p_s delta_ik), F(taubar) = sum (taubar_s + mu_s p_s) v_s^k with
 * taubar_s = mu_s (rho_s h_s W_s^2 - p_s - rho_s W_s). */
void orc_flux_cell(const orc_params *p, const double *q, const double *w, double sigma, int k,
                   double *f)
{
    if (p->model == 2) {
        ideal_flux(p, q, w, k, f);
        return;
    }
    if (p->model == 0) {
        const double *B = q + SF_BX, *E = q + SF_EX, *v = w + P_VX;
        const double rho = w[P_RHO], pr = w[P_P];
        const double W = lorentz(v), h = enthalpy(p->gamma, rho, pr);
        const double em = 0.5 * (dot3(E, E) + dot3(B, B));
        f[SF_D] = q[SF_D] * v[k];
        for (int i = 0; i < 3; ++i)
            f[SF_SX + i] = rho * h * W * W * v[i] * v[k] + ((i == k) ? pr + em : 0.0) - E[i] * E[k]
                           - B[i] * B[k];
        f[SF_TAU] = q[SF_SX + k] - q[SF_D] * v[k];
        em_flux(B, E, q[SF_PSI], q[SF_PHI], k, f + SF_BX, f + SF_EX, f + SF_PSI, f + SF_PHI);
        double J[3];
        sf_current(q, w, sigma, J);
        f[SF_RHOE] = J[k];
        return;
    }
    const double *B = q + TF_BX, *E = q + TF_EX;
    const double mu[2] = { p->mu1, p->mu2 };
    const double em = 0.5 * (dot3(E, E) + dot3(B, B));
    for (int c = 0; c < TF_NC; ++c) f[c] = 0.0;
    double Dv = 0.0;
    for (int s = 0; s < 2; ++s) {
        const double *ws = w + FLUID_NP * s;
        const double rho = ws[P_RHO], *v = ws + P_VX, pr = ws[P_P];
        const double W = lorentz(v), h = enthalpy(p->gamma, rho, pr);
        f[TF_D] += rho * W * v[k];
        Dv += rho * W * v[k];
        for (int i = 0; i < 3; ++i) {
            const double Sik = rho * h * W * W * v[i] * v[k] + ((i == k) ? pr : 0.0);
            f[TF_SX + i] += Sik;
            f[TF_SBX + i] += mu[s] * Sik;
        }
        f[TF_DB] += mu[s] * rho * W * v[k];
        const double taubar_s = mu[s] * (rho * h * W * W - pr - rho * W);
        f[TF_TAUB] += (taubar_s + mu[s] * pr) * v[k];
    }
    for (int i = 0; i < 3; ++i) f[TF_SX + i] += -E[i] * E[k] - B[i] * B[k] + ((i == k) ? em : 0.0);
    f[TF_TAU] = q[TF_SX + k] - Dv;
    em_flux(B, E, q[TF_PSI], q[TF_PHI], k, f + TF_BX, f + TF_EX, f + TF_PSI, f + TF_PHI);
}

/* Source vector Psi(q).
 * Single fluid (Eq. 1): Psi(E) = -J, Psi(psi) = rho_e - kappa psi, Psi(phi) = -kappa phi,
 * zero otherwise.
 * Two fluid (Appendix A, Eqs. A2-A3), with eta = 1/sigma (the paper never defines eta
 * beyond calling the two-fluid coefficient a conductivity; the reading is eta = 1/sigma):
 *   omega_p^2 = sum mu_s^2 rho_s,  W = sum mu_s^2 rho_s W_s / omega_p^2,
 *   u = sum mu_s^2 rho_s W_s v_s / omega_p^2,  rho_e = sum mu_s rho_s W_s,
 *   J = sum mu_s rho_s W_s v_s,  rho_0 = W rho_e - J.u,
 *   Psi(Sbar) = omega_p^2 [W E + u x B - eta (J - rho_e u)]   (as printed; the rest-frame
 *               reading rho_0 u is selected by friction_covariant),
 *   Psi(taubar) = omega_p^2 [u.E - eta (rho_e - rho_0 W)],
 *   Psi(E) = -J,  Psi(psi) = rho_e - kappa psi,  Psi(phi) = -kappa phi.
 * rho_e in Psi(psi) is the conserved Dbar, which equals sum mu_s rho_s W_s by Eq. 6. */
void orc_source_cell(const orc_params *p, const double *q, const double *w, double sigma, double *s)
{
    if (p->model == 2) {   /* ideal: only the divergence cleaning damps */
        for (int c = 0; c < ID_NC; ++c) s[c] = 0.0;
        s[ID_PHI] = -p->kappa * q[ID_PHI];
        return;
    }
    if (p->model == 0) {
        for (int c = 0; c < SF_NC; ++c) s[c] = 0.0;
        double J[3];
        sf_current(q, w, sigma, J);
        for (int i = 0; i < 3; ++i) s[SF_EX + i] = -J[i];
        s[SF_PSI] = q[SF_RHOE] - p->kappa * q[SF_PSI];
        s[SF_PHI] = -p->kappa * q[SF_PHI];
        return;
    }
    const double mu[2] = { p->mu1, p->mu2 };
    const double *B = q + TF_BX, *E = q + TF_EX;
    double wp2 = 0.0, Wsum = 0.0, usum[3] = { 0, 0, 0 }, rhoe = 0.0, J[3] = { 0, 0, 0 };
    for (int sp = 0; sp < 2; ++sp) {
        const double *ws = w + FLUID_NP * sp;
        const double rho = ws[P_RHO], *v = ws + P_VX;
        const double W = lorentz(v);
        wp2 += mu[sp] * mu[sp] * rho;
        Wsum += mu[sp] * mu[sp] * rho * W;
        for (int i = 0; i < 3; ++i) usum[i] += mu[sp] * mu[sp] * rho * W * v[i];
        rhoe += mu[sp] * rho * W;
        for (int i = 0; i < 3; ++i) J[i] += mu[sp] * rho * W * v[i];
    }
    const double Wb = Wsum / wp2;
    double u[3];
    for (int i = 0; i < 3; ++i) u[i] = usum[i] / wp2;
    const double rho0 = Wb * rhoe - dot3(J, u);
    const double eta = 1.0 / sigma;
    double uxB[3];
    cross3(u, B, uxB);
    const double fric = p->friction_covariant ? rho0 : rhoe;
    for (int c = 0; c < TF_NC; ++c) s[c] = 0.0;
    for (int i = 0; i < 3; ++i) s[TF_SBX + i] = wp2 * (Wb * E[i] + uxB[i] - eta * (J[i] - fric * u[i]));
    s[TF_TAUB] = wp2 * (dot3(u, E) - eta * (rhoe - rho0 * Wb));
    for (int i = 0; i < 3; ++i) s[TF_EX + i] = -J[i];
    s[TF_PSI] = q[TF_DB] - p->kappa * q[TF_PSI];
    s[TF_PHI] = -p->kappa * q[TF_PHI];
}

/* ------------------------------------------------------------------------------------------
 * Implicit stage (Sec. 2.2.1, Eq. 10): find Q with G(Q) = Q - R - a Psi(Q) = 0, a = a_ii dt.
 * Components with zero source equal R.  phi and psi enter Psi linearly and only through
 * themselves and the (fixed) charge density, so they have the closed forms
 *   phi = R_phi / (1 + a kappa),   psi = (R_psi + a rho_e) / (1 + a kappa).
 * The remaining unknowns x solve a small nonlinear system whose every evaluation runs the
 * nested primitive recovery (Sec. 2.2.1):  single fluid x = E (3);  two fluid
 * x = (Sbar/|mu1|, taubar/|mu1|, E) (7; the barred unknowns are scaled to order one).
 * The paper solves the full system with a Powell hybrid method (CMINPACK, Sec. 3.3.2); the
 * root is the definition, and this oracle reaches it by plain Newton with a central-
 * difference Jacobian, Gaussian elimination with partial pivoting and step halving.  It
 * stops at ||G||_inf <= tol * max(1, ||R_x||_inf) and then takes one more Newton step.
 * ---------------------------------------------------------------------------------------- */
typedef struct {
    const orc_params *p;
    double a, sigma;
    const double *R;
    double q[MAXC]; /* state with closed-form components set */
    int n;          /* number of nonlinear unknowns */
    double xs;      /* scale of the two-fluid barred unknowns */
} stage_t;

static void stage_state(const stage_t *c, const double *x, double *q)
{
    memcpy(q, c->q, sizeof(double) * MAXC);
    if (c->p->model == 0) {
        for (int i = 0; i < 3; ++i) q[SF_EX + i] = x[i];
    } else {
        for (int i = 0; i < 3; ++i) q[TF_SBX + i] = x[i] * c->xs;
        q[TF_TAUB] = x[3] * c->xs;
        for (int i = 0; i < 3; ++i) q[TF_EX + i] = x[4 + i];
    }
}

static void stage_unknowns(const stage_t *c, const double *q, double *x)
{
    if (c->p->model == 0) {
        for (int i = 0; i < 3; ++i) x[i] = q[SF_EX + i];
    } else {
        for (int i = 0; i < 3; ++i) x[i] = q[TF_SBX + i] / c->xs;
        x[3] = q[TF_TAUB] / c->xs;
        for (int i = 0; i < 3; ++i) x[4 + i] = q[TF_EX + i];
    }
}

/* G(x) in the scaled unknowns; w holds the c2p guess on entry and the primitives on exit. */
static int stage_residual(const stage_t *c, const double *x, double *w, double *G)
{
    double q[MAXC], s[MAXC];
    stage_state(c, x, q);
    int it;
    int st = orc_cons2prim_cell(c->p, q, w, &it);
    if (st != ORC_OK) return st;
    orc_source_cell(c->p, q, w, c->sigma, s);
    for (int k = 0; k < orc_ncons(c->p->model); ++k)
        if (!isfinite(s[k])) return ORC_C2P_UNPHYS;
    const double *R = c->R, a = c->a;
    if (c->p->model == 0) {
        for (int i = 0; i < 3; ++i) G[i] = q[SF_EX + i] - R[SF_EX + i] - a * s[SF_EX + i];
    } else {
        for (int i = 0; i < 3; ++i) G[i] = (q[TF_SBX + i] - R[TF_SBX + i] - a * s[TF_SBX + i]) / c->xs;
        G[3] = (q[TF_TAUB] - R[TF_TAUB] - a * s[TF_TAUB]) / c->xs;
        for (int i = 0; i < 3; ++i) G[4 + i] = q[TF_EX + i] - R[TF_EX + i] - a * s[TF_EX + i];
    }
    return ORC_OK;
}

static double norm_inf(const double *x, int n)
{
    double m = 0.0;
    for (int i = 0; i < n; ++i) m = fabs(x[i]) > m ? fabs(x[i]) : m;
    return m;
}

/* Solve A x = b (n x n, row-major, overwritten) by Gaussian elimination with partial pivoting. */
static int gauss_solve(double *A, double *b, int n)
{
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(A[r * n + col]) > fabs(A[piv * n + col])) piv = r;
        if (A[piv * n + col] == 0.0 || !isfinite(A[piv * n + col])) return -1;
        if (piv != col) {
            for (int k = 0; k < n; ++k) {
                double t = A[col * n + k];
                A[col * n + k] = A[piv * n + k];
                A[piv * n + k] = t;
            }
            double t = b[col];
            b[col] = b[piv];
            b[piv] = t;
        }
        for (int r = col + 1; r < n; ++r) {
            const double m = A[r * n + col] / A[col * n + col];
            for (int k = col; k < n; ++k) A[r * n + k] -= m * A[col * n + k];
            b[r] -= m * b[col];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double acc = b[r];
        for (int k = r + 1; k < n; ++k) acc -= A[r * n + k] * b[k];
        b[r] = acc / A[r * n + r];
    }
    return 0;
}

static void stage_setup(stage_t *c, const orc_params *p, double a, double sigma, const double *R)
{
    c->p = p;
    c->a = a;
    c->sigma = sigma;
    c->R = R;
    const int nc = orc_ncons(p->model);
    memset(c->q, 0, sizeof(c->q));
    memcpy(c->q, R, sizeof(double) * nc);
    if (p->model == 0) {
        c->n = 3;
        c->xs = 1.0;
        c->q[SF_PHI] = R[SF_PHI] / (1.0 + a * p->kappa);
        c->q[SF_PSI] = (R[SF_PSI] + a * R[SF_RHOE]) / (1.0 + a * p->kappa);
    } else {
        c->n = 7;
        c->xs = fabs(p->mu1);
        c->q[TF_PHI] = R[TF_PHI] / (1.0 + a * p->kappa);
        c->q[TF_PSI] = (R[TF_PSI] + a * R[TF_DB]) / (1.0 + a * p->kappa);
    }
}

int orc_implicit_cell(const orc_params *p, double a, double sigma, const double *R, double *Q, double *w,
                      int *iters)
{
    return orc_implicit_cell_from(p, a, sigma, R, NULL, Q, w, iters);
}

/* As orc_implicit_cell, starting Newton from the unknowns of Qstart (NULL: the plain guess
 * x0 = R_x). */
int orc_implicit_cell_from(const orc_params *p, double a, double sigma, const double *R, const double *Qstart,
                           double *Q, double *w, int *iters)
{
    stage_t c;
    stage_setup(&c, p, a, sigma, R);
    const int n = c.n, np = orc_nprim(p->model);
    double x[7], Rx[7], G[7], wcur[MAXP];
    stage_unknowns(&c, R, Rx);
    if (Qstart) stage_unknowns(&c, Qstart, x);
    else memcpy(x, Rx, sizeof(double) * n); /* plain initial guess x0 = R_x */
    memcpy(wcur, w, sizeof(double) * np);
    *iters = 0;
    int st = stage_residual(&c, x, wcur, G);
    if (st != ORC_OK) {
        double qf[MAXC];
        stage_state(&c, x, qf);
        memcpy(Q, qf, sizeof(double) * orc_ncons(p->model));
        memcpy(w, wcur, sizeof(double) * np);
        return st;
    }
    const double target = p->newton_tol * (norm_inf(Rx, n) > 1.0 ? norm_inf(Rx, n) : 1.0);
    int status = ORC_NEWTON_NOCONV;
    for (int it = 0; it < p->max_newton_iter; ++it) {
        const double nrm = norm_inf(G, n);
        const int conv = nrm <= target;
        /* central-difference Jacobian dG/dx */
        double Jm[49], dx[7];
        int jst = ORC_OK;
        for (int j = 0; j < n && jst == ORC_OK; ++j) {
            const double scale = fabs(x[j]) > 0.1 ? fabs(x[j]) : 0.1;
            double xp[7], xm[7], Gp[7], Gm[7], wp[MAXP], wm[MAXP];
            memcpy(xp, x, sizeof(double) * n);
            memcpy(xm, x, sizeof(double) * n);
            xp[j] = x[j] + 6e-6 * scale;
            xm[j] = x[j] - 6e-6 * scale;
            const double h2 = xp[j] - xm[j];
            memcpy(wp, wcur, sizeof(double) * np);
            memcpy(wm, wcur, sizeof(double) * np);
            jst = stage_residual(&c, xp, wp, Gp);
            if (jst == ORC_OK) jst = stage_residual(&c, xm, wm, Gm);
            for (int i = 0; i < n; ++i) Jm[i * n + j] = (Gp[i] - Gm[i]) / h2;
        }
        if (jst != ORC_OK) { status = ORC_LINESEARCH; break; }
        for (int i = 0; i < n; ++i) dx[i] = -G[i];
        if (gauss_solve(Jm, dx, n) != 0) { status = ORC_LINESEARCH; break; }
        /* step halving: accept the first step that keeps the primitives physical and
         * lowers ||G|| (the final, polishing step only has to stay physical) */
        double lam = 1.0, xt[7], Gt[7], wt[MAXP];
        int ok = 0;
        for (int h = 0; h <= 30; ++h) {
            for (int i = 0; i < n; ++i) xt[i] = x[i] + lam * dx[i];
            memcpy(wt, wcur, sizeof(double) * np);
            if (stage_residual(&c, xt, wt, Gt) == ORC_OK && (conv || norm_inf(Gt, n) < nrm)) {
                ok = 1;
                break;
            }
            lam *= 0.5;
        }
        if (!ok) { status = conv ? ORC_OK : ORC_LINESEARCH; break; }
        memcpy(x, xt, sizeof(double) * n);
        memcpy(G, Gt, sizeof(double) * n);
        memcpy(wcur, wt, sizeof(double) * np);
        *iters = it + 1;
        if (conv) { status = ORC_OK; break; }
    }
    double qf[MAXC];
    stage_state(&c, x, qf);
    memcpy(Q, qf, sizeof(double) * orc_ncons(p->model));
    memcpy(w, wcur, sizeof(double) * np);
    return status;
}

/* Residual of the implicit stage at a given Q: runs this oracle's own primitive recovery on
 * Q and returns G in the scaled unknowns (length written to *nG), so that a candidate
 * solution can be judged independently of how it was found. */
int orc_implicit_residual_cell(const orc_params *p, double a, double sigma, const double *R,
                               const double *Q, double *G, int *nG)
{
    stage_t c;
    stage_setup(&c, p, a, sigma, R);
    double x[7], w[MAXP];
    stage_unknowns(&c, Q, x);
    for (int k = 0; k < MAXP; ++k) w[k] = -1.0; /* no guess: bracket midpoint */
    *nG = c.n;
    return stage_residual(&c, x, w, G);
}

/* ------------------------------------------------------------------------------------------
 * Flux-vector splitting + WENO3 (Sec. 2.2.2).
 * Lax-Friedrichs splitting f^(+-) = (f +- alpha q)/2 with alpha = c = 1 (Eq. 12).  Each
 * split flux is reconstructed component-wise at the faces with the third-order WENO scheme
 * of Shu (1997); its constants are not printed, the reading is the Jiang-Shu r = 2 form:
 * candidates p0 = -a/2 + 3b/2, p1 = b/2 + c/2 on the upwind stencil (a, b, c), smoothness
 * beta0 = (b - a)^2, beta1 = (c - b)^2, linear weights d = (1/3, 2/3), eps = 1e-6,
 * alpha_k = d_k / (eps + beta_k)^2, value = (alpha0 p0 + alpha1 p1) / (alpha0 + alpha1).
 * f+ at face i+1/2 uses (a, b, c) = (f_{i-1}, f_i, f_{i+1}); f- at face i+1/2 is the mirror
 * image, (a, b, c) = (f_{i+2}, f_{i+1}, f_i).  The face flux is F_{i+1/2} = f+ + f-.
 * ---------------------------------------------------------------------------------------- */
void orc_weno3_face(const double *fa, const double *fb, const double *fc, double *out, int n)
{
    for (int v = 0; v < n; ++v) {
        const double a = fa[v], b = fb[v], c = fc[v];
        const double p0 = -0.5 * a + 1.5 * b;
        const double p1 = 0.5 * b + 0.5 * c;
        const double beta0 = (b - a) * (b - a);
        const double beta1 = (c - b) * (c - b);
        const double eps = 1e-6;
        const double al0 = (1.0 / 3.0) / ((eps + beta0) * (eps + beta0));
        const double al1 = (2.0 / 3.0) / ((eps + beta1) * (eps + beta1));
        out[v] = (al0 * p0 + al1 * p1) / (al0 + al1);
    }
}

/* ------------------------------------------------------------------------------------------
 * Ideal RMHD, the comparison model advanced with explicit integrators (Sec. 2.1 lists it
 * among the models; its recovery is a two-dimensional root-find in the formulation of the
 * cited Anton et al. 2010, Sec. 2.1.3).  Conserved (9): D, Sx, Sy, Sz, tau, Bx, By, Bz, phi;
 * primitive (5): rho, vx, vy, vz, p.  The electric field is E = -v x B, and the magnetic
 * field is cleaned as in the resistive models: d_t phi + d_k B^k = -kappa phi, the flux of
 * B^i gaining phi along i.
 * ---------------------------------------------------------------------------------------- */

/* D = rho W, S = (rho h W^2 + B^2) v - (v.B) B,
 * tau = rho h W^2 - p + (B^2 + v^2 B^2 - (v.B)^2)/2 - D  (the resistive expressions with
 * E = -v x B: E x B = v B^2 - (v.B) B and E^2 = v^2 B^2 - (v.B)^2); phi = 0 at t = 0. */
static void ideal_prim2cons(const orc_params *p, const double *w, const double *B, double *q)
{
    const double rho = w[P_RHO], *v = w + P_VX, pr = w[P_P];
    const double W = lorentz(v), h = enthalpy(p->gamma, rho, pr);
    const double vB = dot3(v, B), B2 = dot3(B, B), v2 = dot3(v, v);
    q[ID_D] = rho * W;
    for (int i = 0; i < 3; ++i) q[ID_SX + i] = (rho * h * W * W + B2) * v[i] - vB * B[i];
    q[ID_TAU] = rho * h * W * W - pr + 0.5 * (B2 + v2 * B2 - vB * vB) - rho * W;
    for (int i = 0; i < 3; ++i) q[ID_BX + i] = B[i];
    q[ID_PHI] = 0.0;
}

/* Energy residual of the recovery reduced to one unknown, Z = rho h W^2.  From
 * S^2 = (Z + B^2)^2 v^2 - (2Z + B^2) (S.B)^2 / Z^2 the velocity follows from Z,
 *   v^2(Z) = (S^2 Z^2 + (S.B)^2 (2Z + B^2)) / (Z^2 (Z + B^2)^2),
 * and with u = 1 - v^2, rho = D sqrt(u), p = (Gamma-1)/Gamma (Z u - rho) (Gamma law), the
 * energy equation tau + D = Z + B^2 - p - B^2 u / 2 - (S.B)^2 / (2 Z^2) leaves
 *   f(Z) = Z + B^2 - p - B^2 u/2 - (S.B)^2/(2 Z^2) - (tau + D).
 * Returns 0 where v^2(Z) >= 1 (Z too small); f and f' otherwise. */
static int ideal_residual(double gam, double D, double S2, double SB2, double B2, double Et, double Z,
                          double *f, double *df)
{
    const double N = S2 * Z * Z + SB2 * (2.0 * Z + B2);
    const double M = Z * Z * (Z + B2) * (Z + B2);
    const double v2 = N / M;
    if (!(v2 < 1.0)) return 0;
    const double u = 1.0 - v2, su = sqrt(u);
    const double g = (gam - 1.0) / gam;
    const double pr = g * (Z * u - D * su);
    *f = Z + B2 - pr - 0.5 * B2 * u - 0.5 * SB2 / (Z * Z) - Et;
    const double dN = 2.0 * S2 * Z + 2.0 * SB2;
    const double dM = 2.0 * Z * (Z + B2) * (2.0 * Z + B2);
    const double du = -(dN * M - N * dM) / (M * M);
    const double dp = g * (u + Z * du - D * du / (2.0 * su));
    *df = 1.0 - dp - 0.5 * B2 * du + SB2 / (Z * Z * Z);
    return 1;
}

/* Recovery: the unique Z > 0 with v^2 < 1 and f(Z) = 0, bracketed (a Z with v^2 >= 1 or
 * f < 0 lies below the root, f > 0 above) and found by Newton steps kept inside the bracket
 * (bisection otherwise), until the step is at rounding level; then v = (S + (S.B) B / Z) /
 * (Z + B^2), rho = D sqrt(1 - v^2) and p as above.  The guess in w is not needed. */
static int ideal_c2p(const orc_params *p, const double *q, double *w, int *iters)
{
    const double D = q[ID_D], *S = q + ID_SX, *B = q + ID_BX;
    const double Et = q[ID_TAU] + D, S2 = dot3(S, S), SB = dot3(S, B), B2 = dot3(B, B), SB2 = SB * SB;
    *iters = 0;
    if (!(D > 0.0) || !(Et > 0.0) || !isfinite(S2 + B2)) return ORC_C2P_UNPHYS;
    double lo = 0.0, hi = 2.0 * Et + 1.0, f, df;
    int k;
    for (k = 0; k < 200; ++k) {   /* an upper end where f > 0 */
        if (ideal_residual(p->gamma, D, S2, SB2, B2, Et, hi, &f, &df) && f > 0.0) break;
        lo = hi;
        hi *= 2.0;
    }
    if (k == 200) return ORC_C2P_UNPHYS;
    double Z = 0.5 * (lo + hi);
    int conv = 0, it;
    for (it = 1; it <= 400; ++it) {
        double Zn;
        if (!ideal_residual(p->gamma, D, S2, SB2, B2, Et, Z, &f, &df)) {
            lo = Z;
            Zn = 0.5 * (lo + hi);
        } else {
            if (f > 0.0) hi = Z; else lo = Z;
            Zn = (df > 0.0 && it <= 60) ? Z - f / df : 0.5 * (lo + hi);   /* bisection after 60 */
            if (!(Zn > lo && Zn < hi)) Zn = 0.5 * (lo + hi);
        }
        const double step = fabs(Zn - Z);
        Z = Zn;
        if (step <= 4.0 * 2.220446049250313e-16 * Z || hi - lo <= 4.0 * 2.220446049250313e-16 * hi) {
            conv = 1;
            break;
        }
    }
    *iters = it;
    if (!conv) return ORC_C2P_NOCONV;
    /* a bracket that closed on the edge v^2 = 1 rather than on a sign change of f holds no
     * root: the state has no physical primitives */
    if (!ideal_residual(p->gamma, D, S2, SB2, B2, Et, Z, &f, &df) || fabs(f) > 1e-8 * (Et > 1.0 ? Et : 1.0))
        return ORC_C2P_UNPHYS;
    for (int i = 0; i < 3; ++i) w[P_VX + i] = (S[i] + SB * B[i] / Z) / (Z + B2);
    const double u = 1.0 - dot3(w + P_VX, w + P_VX);
    w[P_RHO] = D * sqrt(u);
    w[P_P] = (p->gamma - 1.0) / p->gamma * (Z * u - w[P_RHO]);
    if (!(w[P_RHO] > 0.0) || !(w[P_P] > 0.0) || !(u > 0.0)) return ORC_C2P_UNPHYS;
    return ORC_OK;
}

/* Fluxes along k (Anton et al. 2010 form): with b^0 = W (v.B), b^i = B^i / W + b^0 v^i,
 * b^2 = B^2 / W^2 + (v.B)^2,
 *   f(D) = D v^k,  f(S_i) = S_i v^k + (p + b^2/2) delta_ik - b_i B^k / W,
 *   f(tau) = S_k - D v^k,  f(B^i) = v^k B^i - v^i B^k + phi delta_ik,  f(phi) = B^k. */
static void ideal_flux(const orc_params *p, const double *q, const double *w, int k, double *f)
{
    const double *v = w + P_VX, pr = w[P_P], *B = q + ID_BX;
    const double W = lorentz(v), vB = dot3(v, B), B2 = dot3(B, B);
    const double b0 = W * vB, b2 = B2 / (W * W) + vB * vB;
    (void)p;
    f[ID_D] = q[ID_D] * v[k];
    for (int i = 0; i < 3; ++i) {
        const double bi = B[i] / W + b0 * v[i];
        f[ID_SX + i] = q[ID_SX + i] * v[k] + ((i == k) ? pr + 0.5 * b2 : 0.0) - bi * B[k] / W;
    }
    f[ID_TAU] = q[ID_SX + k] - q[ID_D] * v[k];
    for (int i = 0; i < 3; ++i) f[ID_BX + i] = v[k] * B[i] - v[i] * B[k] + ((i == k) ? q[ID_PHI] : 0.0);
    f[ID_PHI] = B[k];
}

/* ------------------------------------------------------------------------------------------
 * Grid helpers
 * ---------------------------------------------------------------------------------------- */
/* Cell (i, j, k) of a [var][NZ][NY][NX] array lives at v * plane + (k * NY + j) * NX + i;
 * NY = 1 in 1-D, NZ = 1 below 3-D.  The interior rows (j, k) are numbered r = 0, 1, ... with
 * j fastest. */
static int NXg(const orc_params *p) { return p->nx + 4; }
static int NYg(const orc_params *p) { return p->ndim >= 2 ? p->ny + 4 : 1; }
static int NZg(const orc_params *p) { return p->ndim == 3 ? p->nz + 4 : 1; }
static long plane(const orc_params *p) { return (long)NXg(p) * NYg(p) * NZg(p); }
static long nrows(const orc_params *p)
{
    return (long)(p->ndim >= 2 ? p->ny : 1) * (p->ndim == 3 ? p->nz : 1);
}
static long row_base(const orc_params *p, long r)
{
    const int ny = p->ndim >= 2 ? p->ny : 1;
    const long j = r % ny + (p->ndim >= 2 ? 2 : 0);
    const long k = r / ny + (p->ndim == 3 ? 2 : 0);
    return (k * NYg(p) + j) * NXg(p);
}
static double cell_sigma(const orc_params *p, long idx) { return p->sigma_cell ? p->sigma_cell[idx] : p->sigma; }

static void gather(const double *arr, long pl, long idx, int n, double *out)
{
    for (int v = 0; v < n; ++v) out[v] = arr[v * pl + idx];
}
static void scatter(double *arr, long pl, long idx, int n, const double *in)
{
    for (int v = 0; v < n; ++v) arr[v * pl + idx] = in[v];
}

/* Boundary conditions on two ghost layers: outflow copies the nearest interior cell (zero
 * gradient), periodic wraps.  x ghosts are filled on the interior rows first, then y ghosts
 * on every column of the interior z planes, then z ghosts on every (x, y) column, which
 * fills edges and corners consistently. */
void orc_bc_fill(const orc_params *p, double *arr, int nvar)
{
    const int NX = NXg(p), NY = NYg(p), nx = p->nx, ny = p->ny, nz = p->nz;
    const long pl = plane(p), slab = (long)NX * NY;
    for (int v = 0; v < nvar; ++v) {
        double *a = arr + v * pl;
        for (long r = 0; r < nrows(p); ++r) {
            double *row = a + row_base(p, r);
            for (int g = 0; g < 2; ++g) {
                const int il = g, ir = nx + 2 + g; /* ghost columns 0,1 and nx+2,nx+3 */
                if (p->bc == 1) {
                    row[il] = row[il + nx];
                    row[ir] = row[ir - nx];
                } else {
                    row[il] = row[2];
                    row[ir] = row[nx + 1];
                }
            }
        }
        if (p->ndim >= 2)
            for (int k = (p->ndim == 3 ? 2 : 0); k < (p->ndim == 3 ? nz + 2 : 1); ++k) {
                double *b = a + k * slab;
                for (int i = 0; i < NX; ++i)
                    for (int g = 0; g < 2; ++g) {
                        const int jl = g, jr = ny + 2 + g;
                        if (p->bc == 1) {
                            b[(long)jl * NX + i] = b[(long)(jl + ny) * NX + i];
                            b[(long)jr * NX + i] = b[(long)(jr - ny) * NX + i];
                        } else {
                            b[(long)jl * NX + i] = b[(long)2 * NX + i];
                            b[(long)jr * NX + i] = b[(long)(ny + 1) * NX + i];
                        }
                    }
            }
        if (p->ndim == 3)
            for (long c = 0; c < slab; ++c)
                for (int g = 0; g < 2; ++g) {
                    const int kl = g, kr = nz + 2 + g;
                    if (p->bc == 1) {
                        a[kl * slab + c] = a[(kl + nz) * slab + c];
                        a[kr * slab + c] = a[(kr - nz) * slab + c];
                    } else {
                        a[kl * slab + c] = a[2 * slab + c];
                        a[kr * slab + c] = a[(nz + 1) * slab + c];
                    }
                }
    }
}

/* Initial data: conserved variables from primitives and fields.  rho_e is initialised by
 * Gauss's law, rho_e = div E (Sec. 2.1.1), discretised by second-order central differences
 * (the discretisation is not printed); psi = phi = 0. */
void orc_init_state(const orc_params *p, const double *prims, const double *EB, double *cons)
{
    const int NX = NXg(p);
    const long pl = plane(p), slab = (long)NX * NYg(p);
    const int np = orc_nprim(p->model), nc = orc_ncons(p->model);
    double *E = (double *)malloc(sizeof(double) * 6 * pl);
    memcpy(E, EB, sizeof(double) * 6 * pl);
    orc_bc_fill(p, E, 6);
    for (long r = 0; r < nrows(p); ++r)
        for (int i = 2; i < p->nx + 2; ++i) {
            const long idx = row_base(p, r) + i;
            double w[MAXP], eb[6], q[MAXC];
            gather(prims, pl, idx, np, w);
            gather(E, pl, idx, 6, eb);
            double div = (E[3 * pl + idx + 1] - E[3 * pl + idx - 1]) / (2.0 * p->dx);
            if (p->ndim >= 2) div += (E[4 * pl + idx + NX] - E[4 * pl + idx - NX]) / (2.0 * p->dy);
            if (p->ndim == 3) div += (E[5 * pl + idx + slab] - E[5 * pl + idx - slab]) / (2.0 * p->dz);
            orc_prim2cons_cell(p, w, eb, div, q);
            scatter(cons, pl, idx, nc, q);
        }
    orc_bc_fill(p, cons, nc);
    free(E);
}

/* Primitive recovery on every cell, ghosts included; prims holds the guesses on entry. */
void orc_cons2prim(const orc_params *p, const double *cons, double *prims, signed char *status, int *iters)
{
    const long pl = plane(p);
    const int np = orc_nprim(p->model), nc = orc_ncons(p->model);
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < pl; ++idx) {
        double q[MAXC], w[MAXP];
        int it = 0;
        gather(cons, pl, idx, nc, q);
        gather(prims, pl, idx, np, w);
        int st = orc_cons2prim_cell(p, q, w, &it);
        scatter(prims, pl, idx, np, w);
        if (status) status[idx] = (signed char)st;
        if (iters) iters[idx] = it;
    }
}

/* Numerical flux function L(q) = -d_k f^k(q) (Sec. 2.2.1, Eq. 9) on the interior cells:
 * L_i = -(F_{i+1/2} - F_{i-1/2})/dx - (G_{j+1/2} - G_{j-1/2})/dy - (H_{k+1/2} - H_{k-1/2})/dz,
 * one term per dimension, with the face fluxes from the split-and-reconstruct procedure
 * above.  Ghost cells of cons and prims must be valid. */
void orc_rhs(const orc_params *p, const double *cons, const double *prims, double *L)
{
    const int NX = NXg(p), nc = orc_ncons(p->model), np = orc_nprim(p->model);
    const long pl = plane(p);
    for (long k = 0; k < nc * pl; ++k) L[k] = 0.0;
#pragma omp parallel for schedule(static)
    for (long r = 0; r < nrows(p); ++r)
        for (int i = 2; i < p->nx + 2; ++i) {
            const long c = row_base(p, r) + i;
            double Lc[MAXC];
            for (int v = 0; v < nc; ++v) Lc[v] = 0.0;
            for (int dir = 0; dir < p->ndim; ++dir) {
                const long stride = dir == 0 ? 1 : dir == 1 ? NX : (long)NX * NYg(p);
                const double h = dir == 0 ? p->dx : dir == 1 ? p->dy : p->dz;
                /* split fluxes at the five cells i-2..i+2 along dir */
                double fp[5][MAXC], fm[5][MAXC];
                for (int o = -2; o <= 2; ++o) {
                    const long idx = c + o * stride;
                    double q[MAXC], w[MAXP], f[MAXC];
                    gather(cons, pl, idx, nc, q);
                    gather(prims, pl, idx, np, w);
                    orc_flux_cell(p, q, w, cell_sigma(p, idx), dir, f);
                    for (int v = 0; v < nc; ++v) {
                        fp[o + 2][v] = 0.5 * (f[v] + q[v]);
                        fm[o + 2][v] = 0.5 * (f[v] - q[v]);
                    }
                }
                /* face i+1/2: f+ from (i-1, i, i+1), f- from (i+2, i+1, i)
                 * face i-1/2: f+ from (i-2, i-1, i), f- from (i+1, i, i-1) */
                double Fr_p[MAXC], Fr_m[MAXC], Fl_p[MAXC], Fl_m[MAXC];
                orc_weno3_face(fp[1], fp[2], fp[3], Fr_p, nc);
                orc_weno3_face(fm[4], fm[3], fm[2], Fr_m, nc);
                orc_weno3_face(fp[0], fp[1], fp[2], Fl_p, nc);
                orc_weno3_face(fm[3], fm[2], fm[1], Fl_m, nc);
                for (int v = 0; v < nc; ++v)
                    Lc[v] -= ((Fr_p[v] + Fr_m[v]) - (Fl_p[v] + Fl_m[v])) / h;
            }
            scatter(L, pl, c, nc, Lc);
        }
}

/* Source Psi on the interior cells (zero elsewhere). */
static void source_grid(const orc_params *p, const double *cons, const double *prims, double *S)
{
    const int nc = orc_ncons(p->model), np = orc_nprim(p->model);
    const long pl = plane(p);
    for (long k = 0; k < nc * pl; ++k) S[k] = 0.0;
#pragma omp parallel for schedule(static)
    for (long r = 0; r < nrows(p); ++r)
        for (int i = 2; i < p->nx + 2; ++i) {
            const long idx = row_base(p, r) + i;
            double q[MAXC], w[MAXP], s[MAXC];
            gather(cons, pl, idx, nc, q);
            gather(prims, pl, idx, np, w);
            orc_source_cell(p, q, w, cell_sigma(p, idx), s);
            scatter(S, pl, idx, nc, s);
        }
}

/* Implicit stage on the interior cells, then the boundary fill of Q and prims.
 * prims holds the c2p guesses on entry. */
void orc_implicit(const orc_params *p, double a, const double *R, double *Q, double *prims, signed char *status,
                  int *iters)
{
    const int nc = orc_ncons(p->model), np = orc_nprim(p->model);
    const long pl = plane(p);
    memcpy(Q, R, sizeof(double) * nc * pl);
#pragma omp parallel for schedule(dynamic, 16)
    for (long r = 0; r < nrows(p); ++r)
        for (int i = 2; i < p->nx + 2; ++i) {
            const long idx = row_base(p, r) + i;
            double r[MAXC], q[MAXC], w[MAXP];
            int it = 0;
            gather(R, pl, idx, nc, r);
            gather(prims, pl, idx, np, w);
            int st = orc_implicit_cell(p, a, cell_sigma(p, idx), r, q, w, &it);
            scatter(Q, pl, idx, nc, q);
            scatter(prims, pl, idx, np, w);
            if (status) status[idx] = (signed char)st;
            if (iters) iters[idx] = it;
        }
    orc_bc_fill(p, Q, nc);
    orc_bc_fill(p, prims, np);
}

/* One SSP2(222) IMEX step (Sec. 2.2.1, Eqs. 10-11 with the Table 2 tableau,
 * gamma = 1 - 1/sqrt(2)).  The stage sums are read in the standard form
 * q(i) = q^n + dt sum_{j<i} at_ij L(q(j)) + dt sum_{j<=i} a_ij Psi(q(j)):
 *   Q1 = q^n + gamma dt Psi(Q1)
 *   Q2 = q^n + dt L(Q1) + (1 - 2 gamma) dt Psi(Q1) + gamma dt Psi(Q2)
 *   q^{n+1} = q^n + dt/2 [L(Q1) + L(Q2)] + dt/2 [Psi(Q1) + Psi(Q2)]
 * Psi(Q_i) is evaluated from the converged primitives.  The primitives of q^{n+1} are then
 * recovered (guess: those of Q2).  Returns the number of cells with a nonzero status. */
static int explicit_step(const orc_params *p, double dt, int stages, double *cons, double *prims, int *nfail);

int orc_ssp2_step(const orc_params *p, double dt, double *cons, double *prims, long long *newton_iters,
                  int *max_newton, int *nfail)
{
    if (p->model == 2) return explicit_step(p, dt, 2, cons, prims, nfail);
    const double g = 1.0 - 1.0 / sqrt(2.0);
    const int nc = orc_ncons(p->model), np = orc_nprim(p->model);
    const long pl = plane(p);
    double *Q1 = malloc(sizeof(double) * nc * pl), *Q2 = malloc(sizeof(double) * nc * pl);
    double *R2 = malloc(sizeof(double) * nc * pl);
    double *L1 = malloc(sizeof(double) * nc * pl), *L2 = malloc(sizeof(double) * nc * pl);
    double *S1 = malloc(sizeof(double) * nc * pl), *S2 = malloc(sizeof(double) * nc * pl);
    double *w1 = malloc(sizeof(double) * np * pl), *w2 = malloc(sizeof(double) * np * pl);
    signed char *st = malloc(pl);
    int *it = malloc(sizeof(int) * pl);
    long long nit = 0;
    int mx = 0, bad = 0;

    memcpy(w1, prims, sizeof(double) * np * pl);
    orc_implicit(p, g * dt, cons, Q1, w1, st, it);
    for (long r = 0; r < nrows(p); ++r)
        for (int i = 2; i < p->nx + 2; ++i) {
            const long idx = row_base(p, r) + i;
            nit += it[idx];
            mx = it[idx] > mx ? it[idx] : mx;
            bad += st[idx] != ORC_OK;
        }
    orc_rhs(p, Q1, w1, L1);
    source_grid(p, Q1, w1, S1);
    for (long k = 0; k < nc * pl; ++k) R2[k] = cons[k] + dt * L1[k] + (1.0 - 2.0 * g) * dt * S1[k];

    memcpy(w2, w1, sizeof(double) * np * pl);
    orc_implicit(p, g * dt, R2, Q2, w2, st, it);
    for (long r = 0; r < nrows(p); ++r)
        for (int i = 2; i < p->nx + 2; ++i) {
            const long idx = row_base(p, r) + i;
            nit += it[idx];
            mx = it[idx] > mx ? it[idx] : mx;
            bad += st[idx] != ORC_OK;
        }
    orc_rhs(p, Q2, w2, L2);
    source_grid(p, Q2, w2, S2);
    for (int v = 0; v < nc; ++v)
        for (long r = 0; r < nrows(p); ++r)
            for (int i = 2; i < p->nx + 2; ++i) {
                const long k = v * pl + row_base(p, r) + i;
                cons[k] = cons[k] + 0.5 * dt * (L1[k] + L2[k]) + 0.5 * dt * (S1[k] + S2[k]);
            }
    orc_bc_fill(p, cons, nc);
    memcpy(prims, w2, sizeof(double) * np * pl);
    orc_cons2prim(p, cons, prims, st, it);
    for (long idx = 0; idx < pl; ++idx) bad += st[idx] != ORC_OK;

    if (newton_iters) *newton_iters += nit;
    if (max_newton && mx > *max_newton) *max_newton = mx;
    if (nfail) *nfail += bad;
    free(Q1); free(Q2); free(R2); free(L1); free(L2); free(S1); free(S2); free(w1); free(w2);
    free(st); free(it);
    return bad;
}

/* Add the iteration counts and failures of one implicit stage over the interior cells. */
static void stage_tally(const orc_params *p, const signed char *st, const int *it, long long *nit, int *mx,
                        int *bad)
{
    for (long r = 0; r < nrows(p); ++r)
        for (int i = 2; i < p->nx + 2; ++i) {
            const long idx = row_base(p, r) + i;
            *nit += it[idx];
            *mx = it[idx] > *mx ? it[idx] : *mx;
            *bad += st[idx] != ORC_OK;
        }
}

/* One SSP3(332) IMEX step (Sec. 2.2.1, Eqs. 10-11 with the Table 3 tableau, gamma as for
 * SSP2(222)), in the same standard reading of the stage sums:
 *   Q1 = q^n + gamma dt Psi(Q1)
 *   Q2 = q^n + dt L(Q1) + (1 - 2 gamma) dt Psi(Q1) + gamma dt Psi(Q2)
 *   Q3 = q^n + dt/4 [L(Q1) + L(Q2)] + (1/2 - gamma) dt Psi(Q1) + gamma dt Psi(Q3)
 *   q^{n+1} = q^n + dt [L(Q1)/6 + L(Q2)/6 + 2 L(Q3)/3] + dt [Psi(Q1)/6 + Psi(Q2)/6 + 2 Psi(Q3)/3]
 * Each stage starts its recovery from the previous stage's primitives; the primitives of
 * q^{n+1} are recovered from those of Q3.  Returns the number of cells with a nonzero status. */
int orc_ssp3_step(const orc_params *p, double dt, double *cons, double *prims, long long *newton_iters,
                  int *max_newton, int *nfail)
{
    if (p->model == 2) return explicit_step(p, dt, 3, cons, prims, nfail);
    const double g = 1.0 - 1.0 / sqrt(2.0);
    const int nc = orc_ncons(p->model), np = orc_nprim(p->model);
    const long pl = plane(p);
    const size_t bc = sizeof(double) * nc * pl, bp = sizeof(double) * np * pl;
    double *Q1 = malloc(bc), *Q2 = malloc(bc), *Q3 = malloc(bc), *R = malloc(bc);
    double *L1 = malloc(bc), *L2 = malloc(bc), *L3 = malloc(bc);
    double *S1 = malloc(bc), *S2 = malloc(bc), *S3 = malloc(bc);
    double *w = malloc(bp);
    signed char *st = malloc(pl);
    int *it = malloc(sizeof(int) * pl);
    long long nit = 0;
    int mx = 0, bad = 0;

    memcpy(w, prims, bp);
    orc_implicit(p, g * dt, cons, Q1, w, st, it);
    stage_tally(p, st, it, &nit, &mx, &bad);
    orc_rhs(p, Q1, w, L1);
    source_grid(p, Q1, w, S1);

    for (long k = 0; k < nc * pl; ++k) R[k] = cons[k] + dt * L1[k] + (1.0 - 2.0 * g) * dt * S1[k];
    orc_implicit(p, g * dt, R, Q2, w, st, it);
    stage_tally(p, st, it, &nit, &mx, &bad);
    orc_rhs(p, Q2, w, L2);
    source_grid(p, Q2, w, S2);

    for (long k = 0; k < nc * pl; ++k) R[k] = cons[k] + 0.25 * dt * (L1[k] + L2[k]) + (0.5 - g) * dt * S1[k];
    orc_implicit(p, g * dt, R, Q3, w, st, it);
    stage_tally(p, st, it, &nit, &mx, &bad);
    orc_rhs(p, Q3, w, L3);
    source_grid(p, Q3, w, S3);

    for (int v = 0; v < nc; ++v)
        for (long r = 0; r < nrows(p); ++r)
            for (int i = 2; i < p->nx + 2; ++i) {
                const long k = v * pl + row_base(p, r) + i;
                cons[k] = cons[k] + dt * (L1[k] / 6.0 + L2[k] / 6.0 + 2.0 * L3[k] / 3.0) +
                          dt * (S1[k] / 6.0 + S2[k] / 6.0 + 2.0 * S3[k] / 3.0);
            }
    orc_bc_fill(p, cons, nc);
    memcpy(prims, w, bp);
    orc_cons2prim(p, cons, prims, st, it);
    for (long idx = 0; idx < pl; ++idx) bad += st[idx] != ORC_OK;

    if (newton_iters) *newton_iters += nit;
    if (max_newton && mx > *max_newton) *max_newton = mx;
    if (nfail) *nfail += bad;
    free(Q1); free(Q2); free(Q3); free(R); free(L1); free(L2); free(L3); free(S1); free(S2); free(S3);
    free(w); free(st); free(it);
    return bad;
}

/* The ideal model's explicit step: the explicit halves of the IMEX tableaux (Eq. 11),
 * Table 2 (stages = 2: at_21 = 1, weights 1/2, 1/2) or Table 3 (stages = 3: at_21 = 1,
 * at_31 = at_32 = 1/4, weights 1/6, 1/6, 2/3), with the cleaning source explicit too:
 *   q(i) = q^n + dt sum_{j<i} at_ij K_j,   q^{n+1} = q^n + dt sum_i w_i K_i,
 *   K_j = L(q(j)) + Psi(q(j)).
 * Each stage's primitives are recovered from the previous ones; returns the number of cells
 * whose recovery failed. */
static int explicit_step(const orc_params *p, double dt, int stages, double *cons, double *prims, int *nfail)
{
    const double at[3][3] = { { 0.0, 0.0, 0.0 }, { 1.0, 0.0, 0.0 }, { 0.25, 0.25, 0.0 } };
    const double w2[3] = { 0.5, 0.5, 0.0 }, w3[3] = { 1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0 };
    const double *wt = stages == 2 ? w2 : w3;
    const int nc = orc_ncons(p->model), np = orc_nprim(p->model);
    const long pl = plane(p);
    const size_t bc = sizeof(double) * nc * pl, bp = sizeof(double) * np * pl;
    double *K[3], *q = malloc(bc), *w = malloc(bp), *S = malloc(bc);
    signed char *st = malloc(pl);
    int *it = malloc(sizeof(int) * pl);
    int bad = 0;
    for (int i = 0; i < stages; ++i) K[i] = malloc(bc);
    memcpy(q, cons, bc);
    memcpy(w, prims, bp);
    for (int i = 0; i < stages; ++i) {
        if (i > 0) {
            for (long k = 0; k < nc * pl; ++k) {
                double sum = 0.0;
                for (int j = 0; j < i; ++j) sum += at[i][j] * K[j][k];
                q[k] = cons[k] + dt * sum;
            }
            orc_bc_fill(p, q, nc);
            orc_cons2prim(p, q, w, st, it);
            for (long idx = 0; idx < pl; ++idx) bad += st[idx] != ORC_OK;
        }
        orc_rhs(p, q, w, K[i]);
        source_grid(p, q, w, S);
        for (long k = 0; k < nc * pl; ++k) K[i][k] += S[k];
    }
    for (int v = 0; v < nc; ++v)
        for (long r = 0; r < nrows(p); ++r)
            for (int i = 2; i < p->nx + 2; ++i) {
                const long k = v * pl + row_base(p, r) + i;
                double sum = 0.0;
                for (int j = 0; j < stages; ++j) sum += wt[j] * K[j][k];
                cons[k] = cons[k] + dt * sum;
            }
    orc_bc_fill(p, cons, nc);
    memcpy(prims, w, bp);
    orc_cons2prim(p, cons, prims, st, it);
    for (long idx = 0; idx < pl; ++idx) bad += st[idx] != ORC_OK;
    if (nfail) *nfail += bad;
    for (int i = 0; i < stages; ++i) free(K[i]);
    free(q); free(w); free(S); free(st); free(it);
    return bad;
}

/* Time step dt = CFL / sum_d (1/dx_d) with the maximum signal speed c = 1 (the CFL number is
 * given per workload; the 2-D combination is the reading taken). */
double orc_dt(const orc_params *p, double cfl)
{
    if (p->ndim == 1) return cfl * p->dx;
    if (p->ndim == 2) return cfl / (1.0 / p->dx + 1.0 / p->dy);
    return cfl / (1.0 / p->dx + 1.0 / p->dy + 1.0 / p->dz);
}

/* Harness control, no arithmetic of the method: OpenMP threads used by the grid loops
 * (n <= 0 leaves the setting); returns the number now in effect. */
int orc_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}
