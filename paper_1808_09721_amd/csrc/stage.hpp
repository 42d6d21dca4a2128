// stage.hpp -- per-cell implicit-stage solve of the SSP2(222) IMEX scheme (Sec. 2.2.1, Eq. 10):
// Q = R + a Psi(Q).  Components with zero source equal R; phi and psi are linear:
//   phi = R_phi / (1 + a kappa),  psi = (R_psi + a rho_e) / (1 + a kappa);
// the remaining unknowns solve a small nonlinear system whose every residual evaluation
// runs the nested primitive recovery:
//   single fluid  x = E                              (3 unknowns)
//   two fluid     x = (Sbar/|mu1|, taubar/|mu1|, E)   (7 unknowns, barred parts scaled to O(1))
// Newton with the exact Jacobian (single fluid: one forward pass of three-tangent dual numbers;
// two fluid: the chain rule written out through the residual's structure), in which the
// recovery root z = rho h W^2 is differentiated by the implicit-function theorem at the
// converged root instead of iterating in tangent arithmetic.  Steps are halved (up to 30
// times) until the primitives stay physical and ||G||_inf drops; at ||G||_inf <= tol max(1,
// ||R_x||_inf) one further Newton step is taken with the last Jacobian (it changed by the
// order of the last step only), so the answer sits at round-off whatever the starting point.
// With P.jac_keep > 0 a step that cut ||G||_inf to at most jac_keep times its previous value
// lets the next step reuse the same factorised Jacobian (a chord step, about a tenth of the
// cost of a Jacobian evaluation in the two-fluid stage); a reused Jacobian's step is taken
// whole or not at all, and where it does not cut ||G|| by that factor the Jacobian is formed
// afresh at the current iterate.
#pragma once

#include "lu.hpp"
#include "physics.hpp"

namespace rmhd {

template <int N>
__device__ __forceinline__ double maxabs(const double (&g)[N])
{
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) m = fmax(m, fabs(g[i]));
    return m;
}

// ---------------------------------------------------------------------------------------
// single fluid
// ---------------------------------------------------------------------------------------
struct SFCell {
    double D, tau, rhoe, B2, a, sig;
    vec3<double> S, B, RE;
};

// The cell's constants from its right-hand side R (14 conserved values), stage coefficient a
// and conductivity sig.
__device__ __forceinline__ SFCell sf_cell(const double *R, double a, double sig)
{
    SFCell c;
    c.D = R[sf::D];
    c.tau = R[sf::TAU];
    c.rhoe = R[sf::RHOE];
    c.S = v3(R[sf::SX], R[sf::SY], R[sf::SZ]);
    c.B = v3(R[sf::BX], R[sf::BY], R[sf::BZ]);
    c.B2 = dot(c.B, c.B);
    c.RE = v3(R[sf::EX], R[sf::EY], R[sf::EZ]);
    c.a = a;
    c.sig = sig;
    return c;
}

// Hydrodynamic inputs of the recovery at field E: St = S - E x B, Eh = tau - (E^2 + B^2)/2 + D.
template <class T>
__device__ __forceinline__ void sf_split(const SFCell &c, const vec3<T> &E, vec3<T> &St, T &s2, T &Eh)
{
    const auto ExB = cross(E, c.B);
    St = v3<T>(c.S.x - ExB.x, c.S.y - ExB.y, c.S.z - ExB.z);
    s2 = dot(St, St);
    Eh = c.tau + c.D - 0.5 * (dot(E, E) + c.B2);
}

template <class T>
__device__ __forceinline__ void sf_finish(const SFCell &c, const vec3<T> &E, const vec3<T> &St, T z, T (&G)[3])
{
    const T iz = recip(z);
    const vec3<T> v = v3<T>(St.x * iz, St.y * iz, St.z * iz);
    const T W = rsqrt_t(1.0 - dot(v, v));
    const vec3<T> J = sf_current(v, W, E, c.B, c.rhoe, c.sig);
    G[0] = E.x - c.RE.x + c.a * J.x;
    G[1] = E.y - c.RE.y + c.a * J.y;
    G[2] = E.z - c.RE.z + c.a * J.z;
}

// Primal residual; solves the recovery from the pressure guess pg. Returns a cell status.
__device__ __forceinline__ int sf_residual(const SFCell &c, const double (&x)[3], double pg, const Phys &P,
                                           double (&G)[3], Root &r, double &Eh, int &c2p_it)
{
    const vec3<double> E = v3(x[0], x[1], x[2]);
    vec3<double> St;
    double s2;
    sf_split(c, E, St, s2, Eh);
    r = fluid_root(c.D, s2, Eh, Eh + pg, P);
    c2p_it += r.iters;
    if (r.status != CELL_OK) return r.status;
    sf_finish(c, E, St, r.z, G);
    if (!isfinite(G[0]) || !isfinite(G[1]) || !isfinite(G[2])) return CELL_C2P_UNPHYS;
    return CELL_OK;
}

// Exact 3x3 Jacobian dG/dE in one forward pass with three tangents.
__device__ __forceinline__ void sf_jacobian(const SFCell &c, const double (&x)[3], const Root &r, const Phys &P,
                                            double (&A)[3][3])
{
    const vec3<dual3> E = v3(dual3{x[0], 1.0, 0.0, 0.0}, dual3{x[1], 0.0, 1.0, 0.0}, dual3{x[2], 0.0, 0.0, 1.0});
    vec3<dual3> St;
    dual3 s2, Eh;
    sf_split(c, E, St, s2, Eh);
    const dual3 z = root_tangent(r, c.D, s2, Eh, P);
    dual3 G[3];
    sf_finish(c, E, St, z, G);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        A[i][0] = G[i].d0;
        A[i][1] = G[i].d1;
        A[i][2] = G[i].d2;
    }
}

// Inverse of a 3x3 matrix by its adjugate; false if singular or not finite.
__device__ __forceinline__ bool inverse3(const double (&A)[3][3], double (&Ai)[3][3])
{
    const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
    const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
    const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
    if (!(det != 0.0) || !isfinite(det)) return false;
    const double id = frcp(det);
    Ai[0][0] = c00 * id;
    Ai[1][0] = c01 * id;
    Ai[2][0] = c02 * id;
    Ai[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id;
    Ai[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id;
    Ai[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id;
    Ai[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id;
    Ai[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id;
    Ai[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id;
    return true;
}

// Solve one single-fluid cell.  R: the 14 conserved right-hand-side values; x: start of E on
// entry, solution on exit; w: pressure guess in w[4] on entry, primitives on exit.
// The polishing step after convergence reuses the last Jacobian (its change over the last
// step is of the order of that step, so the polished iterate still sits at round-off).
// cap: Newton steps allowed from unconverged iterates in this call; a cell still unconverged
// after them returns CELL_QUEUED with x and w (pressure) ready for a later call to resume.
__device__ inline int sf_stage(const double *R, double a, double sig, const Phys &P, double (&x)[3], double *w,
                               int &newton_it, int &c2p_it, int &res_it, int cap = 1 << 30, double *gres = nullptr,
                               int *jac_it = nullptr)
{
    const SFCell c = sf_cell(R, a, sig);
    newton_it = 0;
    double G[3], Eh;
    Root r;
    double pg = w[4];
    res_it = 1;
    int st = sf_residual(c, x, pg, P, G, r, Eh, c2p_it);
    const double gscale = fmax(1.0, fmax(fabs(c.RE.x), fmax(fabs(c.RE.y), fabs(c.RE.z))));
    if (st == CELL_OK) {
        const double target = P.newton_tol * gscale;
        st = CELL_NEWTON_NOCONV;
        double Ji[3][3];
        bool have_J = false, fresh = false;
        double ratio = 1.0;   // ||G|| after the last accepted step over ||G|| before it
        for (int it = 0; it < P.max_newton; ++it) {
            const double nrm = maxabs(G);
            const bool conv = nrm <= target;
            if (!conv && it >= cap) { st = CELL_QUEUED; break; }
            fresh = !have_J || (!conv && !(ratio <= P.jac_keep));
            if (fresh) {
                double A[3][3];
                sf_jacobian(c, x, r, P, A);
                if (jac_it) ++*jac_it;
                if (!inverse3(A, Ji)) { st = CELL_LINESEARCH; break; }
                have_J = true;
            }
            double dx[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) dx[i] = -(Ji[i][0] * G[0] + Ji[i][1] * G[1] + Ji[i][2] * G[2]);
            double lam = 1.0, xt[3], Gt[3], Eht;
            Root rt;
            bool ok = false;
            const double pcur = r.z - Eh;
            // a reused Jacobian's step must cut ||G|| by the reuse factor at full length
            const double accept = fresh ? nrm : P.jac_keep * nrm;
            for (int h = 0; h <= (fresh || conv ? 30 : 0); ++h) {
#pragma unroll
                for (int i = 0; i < 3; ++i) xt[i] = x[i] + lam * dx[i];
                ++res_it;
                if (sf_residual(c, xt, pcur, P, Gt, rt, Eht, c2p_it) == CELL_OK && (conv || maxabs(Gt) < accept)) {
                    ok = true;
                    break;
                }
                lam *= 0.5;
            }
            if (!ok && !fresh && !conv) { ratio = 1.0; continue; }   // form the Jacobian afresh
            if (!ok) { st = conv ? CELL_OK : CELL_LINESEARCH; break; }
            ratio = nrm > 0.0 ? maxabs(Gt) * frcp(nrm) : 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) { x[i] = xt[i]; G[i] = Gt[i]; }
            r = rt;
            Eh = Eht;
            newton_it = it + 1;
            if (conv) { st = CELL_OK; break; }
        }
    }
    if (gres) *gres = st == CELL_OK ? maxabs(G) * frcp(gscale) : 0.0;
    // primitives at the final point
    const vec3<double> E = v3(x[0], x[1], x[2]);
    vec3<double> St;
    double s2;
    sf_split(c, E, St, s2, Eh);
    const double iz = frcp(r.z);
    w[0] = c.D * r.iW;
    w[1] = St.x * iz; w[2] = St.y * iz; w[3] = St.z * iz;
    w[4] = r.z - Eh;
    return st;
}

// ---------------------------------------------------------------------------------------
// two fluid
// ---------------------------------------------------------------------------------------
struct TFCell {
    double D, tau, B2, a, eta, sc, isc, i12, Ds[2], rhoe;
    vec3<double> S, B, RSb, RE;
    double Rtb;
};

// The cell's constants from its right-hand side R (18 conserved values), stage coefficient a
// and conductivity sig; D_s = rho_s W_s of each species from D and Dbar (Sec. 2.1.3).
__device__ __forceinline__ TFCell tf_cell(const double *R, double a, double sig, const Phys &P)
{
    TFCell c;
    c.D = R[tf::D];
    c.tau = R[tf::TAU];
    c.S = v3(R[tf::SX], R[tf::SY], R[tf::SZ]);
    c.B = v3(R[tf::BX], R[tf::BY], R[tf::BZ]);
    c.B2 = dot(c.B, c.B);
    c.RSb = v3(R[tf::SBX], R[tf::SBY], R[tf::SBZ]);
    c.Rtb = R[tf::TAUB];
    c.RE = v3(R[tf::EX], R[tf::EY], R[tf::EZ]);
    c.a = a;
    c.eta = frcp(sig);
    c.sc = fabs(P.mu1);
    c.isc = frcp(c.sc);
    c.i12 = frcp(P.mu1 - P.mu2);
    c.Ds[0] = (R[tf::DB] - P.mu2 * c.D) * c.i12;
    c.Ds[1] = -(R[tf::DB] - P.mu1 * c.D) * c.i12;
    c.rhoe = R[tf::DB];
    return c;
}

// Species recovery inputs at unknowns x (Sec. 2.1.3, Eqs. 7-8).
template <class T>
__device__ __forceinline__ void tf_split(const TFCell &c, const T (&x)[7], const Phys &P, vec3<T> (&Ss)[2],
                                         T (&s2)[2], T (&Eh)[2])
{
    const vec3<T> E = v3<T>(x[4], x[5], x[6]);
    const vec3<T> Sb = v3<T>(x[0] * c.sc, x[1] * c.sc, x[2] * c.sc);
    const T tb = x[3] * c.sc;
    const auto ExB = cross(E, c.B);
    const vec3<T> St = v3<T>(c.S.x - ExB.x, c.S.y - ExB.y, c.S.z - ExB.z);
    const T tt = c.tau - 0.5 * (dot(E, E) + c.B2);
    const double i12 = c.i12;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const double m = s == 0 ? P.mu2 : P.mu1, sg = s == 0 ? i12 : -i12;
        Ss[s] = v3<T>((Sb.x - m * St.x) * sg, (Sb.y - m * St.y) * sg, (Sb.z - m * St.z) * sg);
        s2[s] = dot(Ss[s], Ss[s]);
        Eh[s] = (tb - m * tt) * sg + c.Ds[s];
    }
}

template <class T>
__device__ __forceinline__ void tf_finish(const TFCell &c, const T (&x)[7], const vec3<T> (&Ss)[2], const T (&z)[2],
                                          const Phys &P, T (&G)[7])
{
    T Dw[2], rho[2];
    vec3<T> v[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const T iz = recip(z[s]);
        v[s] = v3<T>(Ss[s].x * iz, Ss[s].y * iz, Ss[s].z * iz);
        rho[s] = c.Ds[s] * dsqrt(1.0 - dot(v[s], v[s]));
        Dw[s] = lift<T>(c.Ds[s]);  // rho_s W_s = D_s, fixed during the stage
    }
    const vec3<T> E = v3<T>(x[4], x[5], x[6]);
    const TFSource<T> src = tf_source_terms<T>(Dw, rho, v, E, c.B, c.eta, P);
    const double isc = c.isc;
    G[0] = x[0] - (c.RSb.x + c.a * src.Sb.x) * isc;
    G[1] = x[1] - (c.RSb.y + c.a * src.Sb.y) * isc;
    G[2] = x[2] - (c.RSb.z + c.a * src.Sb.z) * isc;
    G[3] = x[3] - (c.Rtb + c.a * src.taub) * isc;
    G[4] = x[4] - c.RE.x + c.a * src.J.x;
    G[5] = x[5] - c.RE.y + c.a * src.J.y;
    G[6] = x[6] - c.RE.z + c.a * src.J.z;
}

__device__ __forceinline__ int tf_residual(const TFCell &c, const double (&x)[7], const double (&pg)[2],
                                           const Phys &P, double (&G)[7], Root (&r)[2], double (&Eh)[2],
                                           int &c2p_it)
{
    vec3<double> Ss[2];
    double s2[2];
    tf_split(c, x, P, Ss, s2, Eh);
    double z[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        r[s] = fluid_root(c.Ds[s], s2[s], Eh[s], Eh[s] + pg[s], P);
        c2p_it += r[s].iters;
        if (r[s].status != CELL_OK) return r[s].status;
        z[s] = r[s].z;
    }
    tf_finish(c, x, Ss, z, P, G);
#pragma unroll
    for (int i = 0; i < 7; ++i)
        if (!isfinite(G[i])) return CELL_C2P_UNPHYS;
    return CELL_OK;
}

// Exact Jacobian dG/dx by the chain rule through the residual's structure, the primal values
// formed once and the seven directions propagated as plain tangents (no dual arithmetic, no
// products with structurally zero tangents).  Per species s (mass-to-charge weight m, sign
// sg = +-1/(mu1 - mu2) as in tf_split):
//   dSs   = sg (sc dx_{0..2} - m B x dE)         ds2 = 2 Ss.dSs
//   dEh   = sg (sc dx_3 + m E.dE)                dz  = (dEh - dg/ds2 ds2) / (dg/dz)
//   dv    = (dSs - v dz) / z                     drho = -D_s (v.dv) / sqrt(1 - v^2)
// and through the source terms (D_s W-weights fixed): d(omega_p^2), dU, dJ, d rho_0, then
//   dPsi(Sbar) = M2 dE + dU x B - eta (d(omega_p^2) J + omega_p^2 dJ - dfr U - fr dU)
//   dPsi(taubar) = dU.E + U.dE - eta (d(omega_p^2) rho_e - d rho_0 M2)
// r: the recovery roots at x (from the residual evaluation at x).
__device__ __forceinline__ void tf_jacobian(const TFCell &c, const double (&x)[7], const Root (&r)[2], const Phys &P,
                                            double (&A)[7][7])
{
    const vec3<double> E = v3(x[4], x[5], x[6]);
    const vec3<double> &B = c.B;
    vec3<double> Ss[2];
    double s2[2], Eh[2];
    tf_split(c, x, P, Ss, s2, Eh);
    const double mu[2] = {P.mu1, P.mu2};
    vec3<double> v[2], SxB[2];
    double rho[2], kr[2], sgsc[2], sgm[2];
    RootPartials q[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const double m = s == 0 ? P.mu2 : P.mu1, sg = s == 0 ? c.i12 : -c.i12;
        q[s] = root_partials(r[s], c.Ds[s], s2[s], P);
        v[s] = v3(Ss[s].x * q[s].iz, Ss[s].y * q[s].iz, Ss[s].z * q[s].iz);
        const double u = 1.0 - dot(v[s], v[s]), rs = frsqrt(u);
        rho[s] = c.Ds[s] * (u * rs);
        kr[s] = -c.Ds[s] * rs;
        sgsc[s] = sg * c.sc;
        sgm[s] = sg * m;
        SxB[s] = cross(Ss[s], B);
    }
    const double cU[2] = {mu[0] * mu[0] * c.Ds[0], mu[1] * mu[1] * c.Ds[1]};
    const double cJ[2] = {mu[0] * c.Ds[0], mu[1] * c.Ds[1]};
    const double wp2 = mu[0] * mu[0] * rho[0] + mu[1] * mu[1] * rho[1];
    const double iwp2 = frcp(wp2);
    const double M2 = cU[0] + cU[1];
    const double rhoe = cJ[0] + cJ[1];
    const vec3<double> U = v3(cU[0] * v[0].x + cU[1] * v[1].x, cU[0] * v[0].y + cU[1] * v[1].y,
                              cU[0] * v[0].z + cU[1] * v[1].z);
    const vec3<double> J = v3(cJ[0] * v[0].x + cJ[1] * v[1].x, cJ[0] * v[0].y + cJ[1] * v[1].y,
                              cJ[0] * v[0].z + cJ[1] * v[1].z);
    const double rho0 = (M2 * rhoe - dot(J, U)) * iwp2;
    const bool cov = P.friction_covariant;
    const double fr = cov ? rho0 : rhoe;
    const double eta = c.eta, ka = c.a * c.isc;
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        // tangents of v_s and rho_s along x_k
        vec3<double> dv[2];
        double drho[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const double vs[3] = {v[s].x, v[s].y, v[s].z};
            double dS[3];      // dSs, entries flagged false are structurally zero
            bool nz[3];
            double ds2, dz;
            if (k < 3) {
#pragma unroll
                for (int i = 0; i < 3; ++i) { nz[i] = i == k; dS[i] = sgsc[s]; }
                const double Sk = k == 0 ? Ss[s].x : k == 1 ? Ss[s].y : Ss[s].z;
                ds2 = 2.0 * sgsc[s] * Sk;
                dz = -(q[s].dgds2 * ds2) * q[s].idgdz;
            } else if (k == 3) {
#pragma unroll
                for (int i = 0; i < 3; ++i) { nz[i] = false; dS[i] = 0.0; }
                dz = sgsc[s] * q[s].idgdz;
            } else {
                // -sg m (B x e_l), l = k - 4
                const int l = k - 4;
                const double bx[3][3] = {{0.0, B.z, -B.y}, {-B.z, 0.0, B.x}, {B.y, -B.x, 0.0}};
#pragma unroll
                for (int i = 0; i < 3; ++i) { nz[i] = i != l; dS[i] = -sgm[s] * bx[l][i]; }
                const double SxBl = l == 0 ? SxB[s].x : l == 1 ? SxB[s].y : SxB[s].z;
                const double El = l == 0 ? E.x : l == 1 ? E.y : E.z;
                ds2 = -2.0 * sgm[s] * SxBl;
                dz = (sgm[s] * El - q[s].dgds2 * ds2) * q[s].idgdz;
            }
            double d[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) d[i] = (nz[i] ? dS[i] - vs[i] * dz : -(vs[i] * dz)) * q[s].iz;
            dv[s] = v3(d[0], d[1], d[2]);
            drho[s] = kr[s] * dot(v[s], dv[s]);
        }
        const double dwp2 = mu[0] * mu[0] * drho[0] + mu[1] * mu[1] * drho[1];
        const vec3<double> dU = v3(cU[0] * dv[0].x + cU[1] * dv[1].x, cU[0] * dv[0].y + cU[1] * dv[1].y,
                                   cU[0] * dv[0].z + cU[1] * dv[1].z);
        const vec3<double> dJ = v3(cJ[0] * dv[0].x + cJ[1] * dv[1].x, cJ[0] * dv[0].y + cJ[1] * dv[1].y,
                                   cJ[0] * dv[0].z + cJ[1] * dv[1].z);
        const double drho0 = -(dot(dJ, U) + dot(J, dU) + rho0 * dwp2) * iwp2;
        const double dfr = cov ? drho0 : 0.0;
        const vec3<double> dUxB = cross(dU, B);
        const double Jc[3] = {J.x, J.y, J.z}, Uc[3] = {U.x, U.y, U.z};
        const double dJc[3] = {dJ.x, dJ.y, dJ.z}, dUc[3] = {dU.x, dU.y, dU.z}, dUxBc[3] = {dUxB.x, dUxB.y, dUxB.z};
        double dtaub = dot(dU, E) - eta * (dwp2 * rhoe - drho0 * M2);
        if (k >= 4) dtaub += Uc[k - 4];
        double col[7];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double dSb = dUxBc[i] - eta * (dwp2 * Jc[i] + wp2 * dJc[i] - dfr * Uc[i] - fr * dUc[i]);
            if (k == 4 + i) dSb += M2;
            col[i] = -ka * dSb;
            col[4 + i] = c.a * dJc[i];
        }
        col[3] = -ka * dtaub;
        col[k] += 1.0;
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            // column k, selected without dynamic register indexing
#pragma unroll
            for (int kk = 0; kk < 7; ++kk)
                if (kk == k) A[i][kk] = col[i];
        }
    }
}

// Solve one two-fluid cell.  x: start (scaled unknowns) on entry, solution on exit;
// w: pressure guesses w[4], w[9] on entry, primitives on exit.  alt: optional second start;
// Newton begins at whichever of x and alt has the smaller residual.  cap: as for sf_stage.
__device__ inline int tf_stage(const double *R, double a, double sig, const Phys &P, double (&x)[7], double *w,
                               int &newton_it, int &c2p_it, int &res_it, const double *alt = nullptr,
                               int cap = 1 << 30, double *gres = nullptr, int *jac_it = nullptr)
{
    const TFCell c = tf_cell(R, a, sig, P);
    newton_it = 0;
    double G[7], Eh[2];
    Root r[2];
    double pg[2] = {w[4], w[9]};
    res_it = 1;
    int st = tf_residual(c, x, pg, P, G, r, Eh, c2p_it);
    if (alt) {
        double xa[7], Ga[7], Eha[2];
        Root ra[2];
#pragma unroll
        for (int i = 0; i < 7; ++i) xa[i] = alt[i];
        ++res_it;
        if (tf_residual(c, xa, pg, P, Ga, ra, Eha, c2p_it) == CELL_OK && (st != CELL_OK || maxabs(Ga) < maxabs(G))) {
#pragma unroll
            for (int i = 0; i < 7; ++i) { x[i] = xa[i]; G[i] = Ga[i]; }
            r[0] = ra[0];
            r[1] = ra[1];
            Eh[0] = Eha[0];
            Eh[1] = Eha[1];
            st = CELL_OK;
        }
    }
    double rx = 0.0;
    rx = fmax(rx, fabs(c.RSb.x * c.isc)); rx = fmax(rx, fabs(c.RSb.y * c.isc)); rx = fmax(rx, fabs(c.RSb.z * c.isc));
    rx = fmax(rx, fabs(c.Rtb * c.isc));
    rx = fmax(rx, fabs(c.RE.x)); rx = fmax(rx, fabs(c.RE.y)); rx = fmax(rx, fabs(c.RE.z));
    const double gscale = fmax(1.0, rx);
    if (st == CELL_OK) {
        const double target = P.newton_tol * gscale;
        st = CELL_NEWTON_NOCONV;
        double A[7][7];
        unsigned long long swaps = 0ull;
        bool have_J = false, fresh = false;
        double ratio = 1.0;   // ||G|| after the last accepted step over ||G|| before it
        for (int it = 0; it < P.max_newton; ++it) {
            const double nrm = maxabs(G);
            const bool conv = nrm <= target;
            if (!conv && it >= cap) { st = CELL_QUEUED; break; }
            fresh = !have_J || (!conv && !(ratio <= P.jac_keep));
            if (fresh) {
                tf_jacobian(c, x, r, P, A);
                if (jac_it) ++*jac_it;
                if (!lu_factor<7>(A, swaps)) { st = CELL_LINESEARCH; break; }
                have_J = true;
            }
            double dx[7];
#pragma unroll
            for (int i = 0; i < 7; ++i) dx[i] = -G[i];
            lu_solve<7>(A, swaps, dx);
            double lam = 1.0, xt[7], Gt[7], Eht[2];
            Root rt[2];
            bool ok = false;
            const double pcur[2] = {r[0].z - Eh[0], r[1].z - Eh[1]};
            // a reused Jacobian's step must cut ||G|| by the reuse factor at full length
            const double accept = fresh ? nrm : P.jac_keep * nrm;
            for (int h = 0; h <= (fresh || conv ? 30 : 0); ++h) {
#pragma unroll
                for (int i = 0; i < 7; ++i) xt[i] = x[i] + lam * dx[i];
                ++res_it;
                if (tf_residual(c, xt, pcur, P, Gt, rt, Eht, c2p_it) == CELL_OK && (conv || maxabs(Gt) < accept)) {
                    ok = true;
                    break;
                }
                lam *= 0.5;
            }
            if (!ok && !fresh && !conv) { ratio = 1.0; continue; }   // form the Jacobian afresh
            if (!ok) { st = conv ? CELL_OK : CELL_LINESEARCH; break; }
            ratio = nrm > 0.0 ? maxabs(Gt) * frcp(nrm) : 0.0;
#pragma unroll
            for (int i = 0; i < 7; ++i) { x[i] = xt[i]; G[i] = Gt[i]; }
            r[0] = rt[0]; r[1] = rt[1];
            Eh[0] = Eht[0]; Eh[1] = Eht[1];
            newton_it = it + 1;
            if (conv) { st = CELL_OK; break; }
        }
    }
    if (gres) *gres = st == CELL_OK ? maxabs(G) * frcp(gscale) : 0.0;
    vec3<double> Ss[2];
    double s2[2];
    tf_split(c, x, P, Ss, s2, Eh);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const double iz = frcp(r[s].z);
        double *ws = w + 5 * s;
        ws[0] = c.Ds[s] * r[s].iW;
        ws[1] = Ss[s].x * iz; ws[2] = Ss[s].y * iz; ws[3] = Ss[s].z * iz;
        ws[4] = r[s].z - Eh[s];
    }
    return st;
}

}  // namespace rmhd
