// physics.hpp -- device-side physics of the resistive single-fluid and two-fluid SRMHD
// model of Wright & Hawke (arXiv:1808.09721) for the gfx950 kernels: conserved <-> primitive
// maps, flux vectors, sources, and the per-cell implicit-stage Newton solve.
//
// Everything here is FP64 (Sec. 3: the 1e-13 recovery tolerance needs double precision).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace rmhd {

// ---------------------------------------------------------------------------------------
// variable orders (as documented in include/rmhd.h)
// ---------------------------------------------------------------------------------------
namespace sf {
enum { D, SX, SY, SZ, TAU, BX, BY, BZ, EX, EY, EZ, RHOE, PSI, PHI, NC };
constexpr int NP = 5;
}  // namespace sf
namespace tf {
enum { D, SX, SY, SZ, TAU, DB, SBX, SBY, SBZ, TAUB, BX, BY, BZ, EX, EY, EZ, PSI, PHI, NC };
constexpr int NP = 10;
}  // namespace tf
namespace id {   // ideal RMHD (E = -v x B), the explicit comparison model
enum { D, SX, SY, SZ, TAU, BX, BY, BZ, PHI, NC };
constexpr int NP = 5;
}  // namespace id

enum CellStatus { CELL_OK = 0, CELL_C2P_NOCONV = 1, CELL_C2P_UNPHYS = 2, CELL_NEWTON_NOCONV = 3,
                  CELL_LINESEARCH = 4,
                  CELL_QUEUED = 5 };  // internal: stopped unconverged at the step cap, to be resumed

// Per-launch physics constants (by value in every kernel).
struct Phys {
    double gamma;      // Gamma-law index
    double gk;         // (Gamma - 1) / Gamma
    double hk;         // Gamma / (Gamma - 1):  rho h = rho + hk p
    double sigma;      // scalar conductivity (two fluid: eta = 1/sigma)
    const double *sigma_cell;  // per-cell conductivity plane or nullptr
    double mu1, mu2, kappa;
    double c2p_tol, newton_tol;
    int max_c2p, max_newton;
    int friction_covariant;
    int c2p_fallback;  // 1: the pressure residual takes over where the z residual fails
    double jac_keep;   // implicit stage: a Newton step that cut ||G|| to at most this fraction
                       // of its previous value lets the next step reuse the same Jacobian
                       // (0: a fresh Jacobian at every unconverged iterate)
};

__device__ __forceinline__ double cell_sigma(const Phys &P, long idx)
{
    return P.sigma_cell ? P.sigma_cell[idx] : P.sigma;
}

// ---------------------------------------------------------------------------------------
// reciprocal and reciprocal square root: the hardware estimate (v_rcp_f64 / v_rsq_f64)
// refined by two Newton-Raphson steps in FMA form, accurate to about one ulp for the normal,
// finite, positive arguments used here (instead of the IEEE-exact division and square-root
// sequences with their scaling and fix-up instructions)
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double frcp(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ double frsqrt(double x)
{
    double r = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    double e = fma(-h * r, r, 0.5);
    r = fma(r, e, r);
    e = fma(-h * r, r, 0.5);
    return fma(r, e, r);
}
// square root as x / sqrt(x) from the refined reciprocal square root (about two ulp): 0 at 0,
// NaN below 0, where the state is unphysical anyway
__device__ __forceinline__ double fsqrt(double x)
{
    const double r = x * frsqrt(x);
    return x > 0.0 ? r : (x == 0.0 ? 0.0 : __builtin_nan(""));
}

// ---------------------------------------------------------------------------------------
// forward-mode dual number with three tangents for the exact single-fluid stage Jacobian: one
// forward pass yields the whole 3x3 Jacobian
// ---------------------------------------------------------------------------------------
struct dual3 {
    double v, d0, d1, d2;
};
__device__ __forceinline__ dual3 operator+(dual3 a, dual3 b) { return {a.v + b.v, a.d0 + b.d0, a.d1 + b.d1, a.d2 + b.d2}; }
__device__ __forceinline__ dual3 operator-(dual3 a, dual3 b) { return {a.v - b.v, a.d0 - b.d0, a.d1 - b.d1, a.d2 - b.d2}; }
__device__ __forceinline__ dual3 operator-(dual3 a) { return {-a.v, -a.d0, -a.d1, -a.d2}; }
__device__ __forceinline__ dual3 operator*(dual3 a, dual3 b)
{
    return {a.v * b.v, a.v * b.d0 + a.d0 * b.v, a.v * b.d1 + a.d1 * b.v, a.v * b.d2 + a.d2 * b.v};
}
__device__ __forceinline__ dual3 operator+(dual3 a, double b) { return {a.v + b, a.d0, a.d1, a.d2}; }
__device__ __forceinline__ dual3 operator+(double b, dual3 a) { return {a.v + b, a.d0, a.d1, a.d2}; }
__device__ __forceinline__ dual3 operator-(dual3 a, double b) { return {a.v - b, a.d0, a.d1, a.d2}; }
__device__ __forceinline__ dual3 operator-(double b, dual3 a) { return {b - a.v, -a.d0, -a.d1, -a.d2}; }
__device__ __forceinline__ dual3 operator*(dual3 a, double b) { return {a.v * b, a.d0 * b, a.d1 * b, a.d2 * b}; }
__device__ __forceinline__ dual3 operator*(double b, dual3 a) { return {a.v * b, a.d0 * b, a.d1 * b, a.d2 * b}; }
__device__ __forceinline__ dual3 recip(dual3 a)
{
    const double r = frcp(a.v), m = -r * r;
    return {r, a.d0 * m, a.d1 * m, a.d2 * m};
}
__device__ __forceinline__ dual3 dsqrt(dual3 a)
{
    const double s = fsqrt(a.v), h = 0.5 * frcp(s);
    return {s, a.d0 * h, a.d1 * h, a.d2 * h};
}

// 1/sqrt for scalars and duals
__device__ __forceinline__ double rsqrt_t(double a) { return frsqrt(a); }
__device__ __forceinline__ dual3 rsqrt_t(dual3 a)
{
    const double r = frsqrt(a.v), m = -0.5 * r * r * r;
    return {r, a.d0 * m, a.d1 * m, a.d2 * m};
}

template <class T>
__device__ __forceinline__ T lift(double v);
template <>
__device__ __forceinline__ double lift<double>(double v) { return v; }
template <>
__device__ __forceinline__ dual3 lift<dual3>(double v) { return dual3{v, 0.0, 0.0, 0.0}; }
__device__ __forceinline__ double recip(double a) { return frcp(a); }
__device__ __forceinline__ double dsqrt(double a) { return fsqrt(a); }

template <class T>
struct vec3 {
    T x, y, z;
};
template <class T>
__device__ __forceinline__ vec3<T> v3(T a, T b, T c) { return vec3<T>{a, b, c}; }
template <class T, class U>
__device__ __forceinline__ auto dot(const vec3<T> &a, const vec3<U> &b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T, class U>
__device__ __forceinline__ auto cross(const vec3<T> &a, const vec3<U> &b)
{
    using R = decltype(a.x * b.x);
    return vec3<R>{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// ---------------------------------------------------------------------------------------
// Primitive recovery of one fluid (Sec. 2.1.3).
// Unknown z = rho h W^2 (= taut + D + p).  With v^2 = s^2/z^2, 1/W = sqrt(1 - v^2),
// rho = D/W, the Gamma law gives p(z) = (Gamma-1)/Gamma (z (1 - v^2) - D/W), and the root of
// g(z) = z - Eh - p(z), Eh = taut + D, is sought.  g is increasing for Gamma <= 2 on the
// physical bracket z in (max(s, Eh), Gamma Eh].  Newton, safeguarded by bisection, stops at
// |g| <= tol max(1, p) and then takes one more Newton step.
// ---------------------------------------------------------------------------------------
struct Root {
    double z;    // rho h W^2 at the root
    double iW;   // 1/W
    int status;  // CELL_OK / CELL_C2P_NOCONV / CELL_C2P_UNPHYS
    int iters;
};

__device__ __forceinline__ Root fluid_root_z(double D, double s2, double Eh, double zguess, const Phys &P)
{
    Root r;
    r.iters = 0;
    r.z = zguess;
    r.iW = 1.0;
    const double s = fsqrt(s2);
    double lo = fmax(s, Eh);
    double hi = P.gamma * Eh;
    if (!(D > 0.0) || !(Eh > 0.0) || !(hi > lo)) {
        r.status = CELL_C2P_UNPHYS;
        return r;
    }
    double z = (zguess > lo && zguess < hi) ? zguess : 0.5 * (lo + hi);
    r.status = CELL_C2P_NOCONV;
    for (int it = 1; it <= P.max_c2p; ++it) {
        const double iz = frcp(z);
        const double v2 = s2 * iz * iz;
        const double u = 1.0 - v2;
        const double W = frsqrt(u);
        const double iW = u * W;
        const double p = P.gk * (z * u - D * iW);
        const double g = z - Eh - p;
        const double dg = 1.0 - P.gk * (1.0 + v2 - D * v2 * iz * W);
        if (g < 0.0) lo = z; else hi = z;
        double zn = z - g * frcp(dg);
        if (fabs(g) <= P.c2p_tol * fmax(1.0, p)) {
            if (zn > s && zn >= Eh) z = zn;
            r.status = CELL_OK;
            r.iters = it;
            break;
        }
        if (!(zn > lo && zn < hi)) zn = 0.5 * (lo + hi);
        z = zn;
        r.iters = it;
    }
    r.z = z;
    const double iz = frcp(z);
    const double u = 1.0 - s2 * iz * iz;
    r.iW = u * frsqrt(u);
    if (r.status == CELL_OK && !(r.iW > 0.0)) r.status = CELL_C2P_UNPHYS;
    return r;
}

// The second recovery residual (Sec. 2.1.3 keeps two, so that one can take over where the
// other fails): Newton on the pressure, f(p) = (Gamma - 1) rho eps - p with Q = E_h + p,
// v^2 = s^2/Q^2, rho = D sqrt(1 - v^2), rho eps = Q (1 - v^2) - rho - p, and
// f'(p) = (Gamma - 1) v^2 (1 - D W / Q) - 1, bracketed on (max(s - E_h, 0), (Gamma - 1) E_h]
// with bisection where a Newton step leaves the bracket.  Same root as fluid_root_z
// (z = Q = E_h + p), returned in the same form.
__device__ __forceinline__ Root fluid_root_p(double D, double s2, double Eh, double pguess, const Phys &P)
{
    Root r;
    r.iters = 0;
    r.iW = 1.0;
    const double s = fsqrt(s2);
    double lo = fmax(s - Eh, 0.0), hi = (P.gamma - 1.0) * Eh;
    r.z = Eh + pguess;
    if (!(D > 0.0) || !(Eh > 0.0) || !(hi > lo)) {
        r.status = CELL_C2P_UNPHYS;
        return r;
    }
    double p = (pguess > lo && pguess < hi) ? pguess : 0.5 * (lo + hi);
    r.status = CELL_C2P_NOCONV;
    for (int it = 1; it <= P.max_c2p; ++it) {
        const double Q = Eh + p, iQ = frcp(Q);
        const double v2 = s2 * iQ * iQ, u = 1.0 - v2;
        const double W = frsqrt(u);
        const double f = (P.gamma - 1.0) * (Q * u - D * u * W - p) - p;
        const double df = (P.gamma - 1.0) * v2 * (1.0 - D * W * iQ) - 1.0;
        if (f > 0.0) lo = p; else hi = p;
        double pn = p - f * frcp(df);
        if (fabs(f) <= P.c2p_tol * fmax(1.0, p)) {
            if (pn >= 0.0 && Eh + pn > s) p = pn;
            r.status = CELL_OK;
            r.iters = it;
            break;
        }
        if (!(pn > lo && pn < hi)) pn = 0.5 * (lo + hi);
        p = pn;
        r.iters = it;
    }
    r.z = Eh + p;
    const double iz = frcp(r.z);
    const double u = 1.0 - s2 * iz * iz;
    r.iW = u * frsqrt(u);
    if (r.status == CELL_OK && !(r.iW > 0.0)) r.status = CELL_C2P_UNPHYS;
    return r;
}

// Recovery of one fluid: the z residual, and where it does not converge (unless
// P.c2p_fallback is 0) the pressure residual, started from the last z iterate.  The z
// residual stalls above its tolerance where rounding in z - Eh exceeds it (large rho h W^2
// against max(1, p)); the pressure residual then usually still converges.  The iterations
// of both count.
__device__ __forceinline__ Root fluid_root(double D, double s2, double Eh, double zguess, const Phys &P)
{
    Root r = fluid_root_z(D, s2, Eh, zguess, P);
    if (r.status == CELL_C2P_NOCONV && P.c2p_fallback) {
        const int used = r.iters;
        r = fluid_root_p(D, s2, Eh, r.z - Eh, P);
        r.iters += used;
    }
    return r;
}

// Tangent of the root z through the implicit-function theorem: with z fixed at the root,
// dg = dg/ds2 ds2 + dg/dEh dEh, and dz = -(dg/ds2 ds2 + dg/dEh dEh) / (dg/dz).  Since
// dg/dEh = -1, dz = (dEh - dg/ds2 ds2) / (dg/dz); root_partials gives dg/ds2 and 1/(dg/dz)
// at the root (iz = 1/z).
struct RootPartials {
    double iz, dgds2, idgdz;
};
__device__ __forceinline__ RootPartials root_partials(const Root &r, double D, double s2, const Phys &P)
{
    RootPartials q;
    const double iz = frcp(r.z), W = frcp(r.iW);
    const double v2 = s2 * iz * iz;
    q.iz = iz;
    q.idgdz = frcp(1.0 - P.gk * (1.0 + v2 - D * v2 * iz * W));
    q.dgds2 = P.gk * (iz - 0.5 * D * iz * iz * W);
    return q;
}
__device__ __forceinline__ dual3 root_tangent(const Root &r, double D, dual3 s2, dual3 Eh, const Phys &P)
{
    const RootPartials q = root_partials(r, D, s2.v, P);
    return dual3{r.z, (Eh.d0 - q.dgds2 * s2.d0) * q.idgdz, (Eh.d1 - q.dgds2 * s2.d1) * q.idgdz,
                 (Eh.d2 - q.dgds2 * s2.d2) * q.idgdz};
}
__device__ __forceinline__ double root_tangent(const Root &r, double, double, double, const Phys &) { return r.z; }

// ---------------------------------------------------------------------------------------
// Single fluid (Sec. 2.1.1, Eqs. 1-2)
// ---------------------------------------------------------------------------------------
// Ohm's law J = rho_e v + W sigma [E + v x B - (v.E) v]
template <class T>
__device__ __forceinline__ vec3<T> sf_current(const vec3<T> &v, T W, const vec3<T> &E, const vec3<double> &B,
                                               double rhoe, double sig)
{
    const vec3<T> vxB = cross(v, B);
    const T vE = dot(v, E);
    const T sW = sig * W;
    return v3<T>(rhoe * v.x + sW * (E.x + vxB.x - vE * v.x), rhoe * v.y + sW * (E.y + vxB.y - vE * v.y),
                 rhoe * v.z + sW * (E.z + vxB.z - vE * v.z));
}

// prim (rho, v, p), B, E, rho_e -> 14 conserved
__device__ inline void sf_prim2cons(const double *w, const double *EB, double rhoe, const Phys &P, double *q)
{
    const vec3<double> v = v3(w[1], w[2], w[3]), B = v3(EB[0], EB[1], EB[2]), E = v3(EB[3], EB[4], EB[5]);
    const double W2 = 1.0 / (1.0 - dot(v, v));
    const double W = sqrt(W2);
    const double A = (w[0] + P.hk * w[4]) * W2;  // rho h W^2
    const vec3<double> ExB = cross(E, B);
    q[sf::D] = w[0] * W;
    q[sf::SX] = A * v.x + ExB.x;
    q[sf::SY] = A * v.y + ExB.y;
    q[sf::SZ] = A * v.z + ExB.z;
    q[sf::TAU] = A - w[4] - w[0] * W + 0.5 * (dot(E, E) + dot(B, B));
    q[sf::BX] = B.x; q[sf::BY] = B.y; q[sf::BZ] = B.z;
    q[sf::EX] = E.x; q[sf::EY] = E.y; q[sf::EZ] = E.z;
    q[sf::RHOE] = rhoe;
    q[sf::PSI] = 0.0;
    q[sf::PHI] = 0.0;
}

// 14 conserved -> (rho, v, p); w[4] holds the pressure guess on entry
__device__ inline int sf_cons2prim(const double *q, double *w, const Phys &P, int &iters)
{
    const vec3<double> B = v3(q[sf::BX], q[sf::BY], q[sf::BZ]), E = v3(q[sf::EX], q[sf::EY], q[sf::EZ]);
    const vec3<double> ExB = cross(E, B);
    const vec3<double> St = v3(q[sf::SX] - ExB.x, q[sf::SY] - ExB.y, q[sf::SZ] - ExB.z);
    const double Eh = q[sf::TAU] - 0.5 * (dot(E, E) + dot(B, B)) + q[sf::D];
    const Root r = fluid_root(q[sf::D], dot(St, St), Eh, Eh + w[4], P);
    iters = r.iters;
    const double iz = frcp(r.z);
    w[0] = q[sf::D] * r.iW;
    w[1] = St.x * iz; w[2] = St.y * iz; w[3] = St.z * iz;
    w[4] = r.z - Eh;
    return r.status;
}

// Flux vectors f^x and f^y and source Psi of one cell from (q, w).
__device__ inline void sf_flux_source(const double *q, const double *w, double sig, const Phys &P, double *fx,
                                      double *fy, double *src)
{
    const vec3<double> v = v3(w[1], w[2], w[3]);
    const vec3<double> B = v3(q[sf::BX], q[sf::BY], q[sf::BZ]), E = v3(q[sf::EX], q[sf::EY], q[sf::EZ]);
    const double W = frsqrt(1.0 - dot(v, v));
    const double W2 = W * W;
    const double A = (w[0] + P.hk * w[4]) * W2;
    const double pt = w[4] + 0.5 * (dot(E, E) + dot(B, B));
    const vec3<double> J = sf_current(v, W, E, B, q[sf::RHOE], sig);
    // x
    fx[sf::D] = q[sf::D] * v.x;
    fx[sf::SX] = A * v.x * v.x + pt - E.x * E.x - B.x * B.x;
    fx[sf::SY] = A * v.y * v.x - E.y * E.x - B.y * B.x;
    fx[sf::SZ] = A * v.z * v.x - E.z * E.x - B.z * B.x;
    fx[sf::TAU] = q[sf::SX] - q[sf::D] * v.x;
    fx[sf::BX] = q[sf::PHI]; fx[sf::BY] = -E.z; fx[sf::BZ] = E.y;
    fx[sf::EX] = q[sf::PSI]; fx[sf::EY] = B.z; fx[sf::EZ] = -B.y;
    fx[sf::RHOE] = J.x;
    fx[sf::PSI] = E.x;
    fx[sf::PHI] = B.x;
    // y
    fy[sf::D] = q[sf::D] * v.y;
    fy[sf::SX] = A * v.x * v.y - E.x * E.y - B.x * B.y;
    fy[sf::SY] = A * v.y * v.y + pt - E.y * E.y - B.y * B.y;
    fy[sf::SZ] = A * v.z * v.y - E.z * E.y - B.z * B.y;
    fy[sf::TAU] = q[sf::SY] - q[sf::D] * v.y;
    fy[sf::BX] = E.z; fy[sf::BY] = q[sf::PHI]; fy[sf::BZ] = -E.x;
    fy[sf::EX] = -B.z; fy[sf::EY] = q[sf::PSI]; fy[sf::EZ] = B.x;
    fy[sf::RHOE] = J.y;
    fy[sf::PSI] = E.y;
    fy[sf::PHI] = B.y;
    // source: only E, psi, phi carry one
    for (int k = 0; k < sf::NC; ++k) src[k] = 0.0;
    src[sf::EX] = -J.x; src[sf::EY] = -J.y; src[sf::EZ] = -J.z;
    src[sf::PSI] = q[sf::RHOE] - P.kappa * q[sf::PSI];
    src[sf::PHI] = -P.kappa * q[sf::PHI];
}

// Flux vector f^z of one cell from (q, w), for 3-D grids: the z column of the fluxes of
// Eq. 1 (induction -E x, Ampere +B x, cleaning psi, phi along z).
__device__ inline void sf_flux_z(const double *q, const double *w, double sig, const Phys &P, double *fz)
{
    const vec3<double> v = v3(w[1], w[2], w[3]);
    const vec3<double> B = v3(q[sf::BX], q[sf::BY], q[sf::BZ]), E = v3(q[sf::EX], q[sf::EY], q[sf::EZ]);
    const double W = frsqrt(1.0 - dot(v, v));
    const double A = (w[0] + P.hk * w[4]) * (W * W);
    const double pt = w[4] + 0.5 * (dot(E, E) + dot(B, B));
    const vec3<double> J = sf_current(v, W, E, B, q[sf::RHOE], sig);
    fz[sf::D] = q[sf::D] * v.z;
    fz[sf::SX] = A * v.x * v.z - E.x * E.z - B.x * B.z;
    fz[sf::SY] = A * v.y * v.z - E.y * E.z - B.y * B.z;
    fz[sf::SZ] = A * v.z * v.z + pt - E.z * E.z - B.z * B.z;
    fz[sf::TAU] = q[sf::SZ] - q[sf::D] * v.z;
    fz[sf::BX] = -E.y; fz[sf::BY] = E.x; fz[sf::BZ] = q[sf::PHI];
    fz[sf::EX] = B.y; fz[sf::EY] = -B.x; fz[sf::EZ] = q[sf::PSI];
    fz[sf::RHOE] = J.z;
    fz[sf::PSI] = E.z;
    fz[sf::PHI] = B.z;
}

// ---------------------------------------------------------------------------------------
// Two fluid (Sec. 2.1.2 Eq. 6; Appendix A Eqs. A1-A3)
// ---------------------------------------------------------------------------------------
__device__ inline void tf_prim2cons(const double *w, const double *EB, const Phys &P, double *q)
{
    const vec3<double> B = v3(EB[0], EB[1], EB[2]), E = v3(EB[3], EB[4], EB[5]);
    const double mu[2] = {P.mu1, P.mu2};
    double Dn = 0, Db = 0, tn = 0, tb = 0;
    vec3<double> Sn = v3(0.0, 0.0, 0.0), Sb = v3(0.0, 0.0, 0.0);
    for (int s = 0; s < 2; ++s) {
        const double *ws = w + 5 * s;
        const vec3<double> v = v3(ws[1], ws[2], ws[3]);
        const double W2 = 1.0 / (1.0 - dot(v, v));
        const double Ds = ws[0] * sqrt(W2);
        const double A = (ws[0] + P.hk * ws[4]) * W2;
        const double ts = A - ws[4] - Ds;
        Dn += Ds; Db += mu[s] * Ds;
        tn += ts; tb += mu[s] * ts;
        Sn.x += A * v.x; Sn.y += A * v.y; Sn.z += A * v.z;
        Sb.x += mu[s] * A * v.x; Sb.y += mu[s] * A * v.y; Sb.z += mu[s] * A * v.z;
    }
    const vec3<double> ExB = cross(E, B);
    q[tf::D] = Dn;
    q[tf::SX] = Sn.x + ExB.x; q[tf::SY] = Sn.y + ExB.y; q[tf::SZ] = Sn.z + ExB.z;
    q[tf::TAU] = tn + 0.5 * (dot(E, E) + dot(B, B));
    q[tf::DB] = Db;
    q[tf::SBX] = Sb.x; q[tf::SBY] = Sb.y; q[tf::SBZ] = Sb.z;
    q[tf::TAUB] = tb;
    q[tf::BX] = B.x; q[tf::BY] = B.y; q[tf::BZ] = B.z;
    q[tf::EX] = E.x; q[tf::EY] = E.y; q[tf::EZ] = E.z;
    q[tf::PSI] = 0.0;
    q[tf::PHI] = 0.0;
}

// Species split of the hydrodynamic parts (Sec. 2.1.3, Eqs. 7-8): X_1 = (Xbar - mu2 X)/(mu1 - mu2),
// X_2 = (Xbar - mu1 X)/(mu2 - mu1), X = D, St (= S - E x B), taut (= tau - (E^2+B^2)/2).
__device__ inline int tf_cons2prim(const double *q, double *w, const Phys &P, int &iters)
{
    const vec3<double> B = v3(q[tf::BX], q[tf::BY], q[tf::BZ]), E = v3(q[tf::EX], q[tf::EY], q[tf::EZ]);
    const vec3<double> ExB = cross(E, B);
    const vec3<double> St = v3(q[tf::SX] - ExB.x, q[tf::SY] - ExB.y, q[tf::SZ] - ExB.z);
    const double tt = q[tf::TAU] - 0.5 * (dot(E, E) + dot(B, B));
    const double i12 = 1.0 / (P.mu1 - P.mu2);
    int status = CELL_OK;
    iters = 0;
    for (int s = 0; s < 2; ++s) {
        // species 1: (Xbar - mu2 X)/(mu1 - mu2); species 2: -(Xbar - mu1 X)/(mu1 - mu2)
        const double m = s == 0 ? P.mu2 : P.mu1, sg = s == 0 ? i12 : -i12;
        const double Ds = (q[tf::DB] - m * q[tf::D]) * sg;
        const vec3<double> Ss = v3((q[tf::SBX] - m * St.x) * sg, (q[tf::SBY] - m * St.y) * sg,
                                   (q[tf::SBZ] - m * St.z) * sg);
        const double Eh = (q[tf::TAUB] - m * tt) * sg + Ds;
        double *ws = w + 5 * s;
        const Root r = fluid_root(Ds, dot(Ss, Ss), Eh, Eh + ws[4], P);
        iters += r.iters;
        const double iz = frcp(r.z);
        ws[0] = Ds * r.iW;
        ws[1] = Ss.x * iz; ws[2] = Ss.y * iz; ws[3] = Ss.z * iz;
        ws[4] = r.z - Eh;
        if (r.status != CELL_OK && status != CELL_C2P_UNPHYS) status = r.status;
    }
    return status;
}

// Two-fluid source from the primitives, arranged around omega_p^2 W = sum mu_s^2 D_s and
// omega_p^2 u = sum mu_s^2 D_s v_s (D_s = rho_s W_s), so no division by omega_p^2 is needed
// except in rho_0 = W rho_e - J.u.
template <class T>
struct TFSource {
    vec3<T> Sb;  // Psi(Sbar)
    T taub;      // Psi(taubar)
    vec3<T> J;   // current; Psi(E) = -J
};

template <class T>
__device__ __forceinline__ TFSource<T> tf_source_terms(const T Dw[2], const T rho[2], const vec3<T> v[2],
                                                      const vec3<T> &E, const vec3<double> &B, double eta,
                                                      const Phys &P)
{
    const double mu[2] = {P.mu1, P.mu2};
    const T wp2 = mu[0] * mu[0] * rho[0] + mu[1] * mu[1] * rho[1];
    const T M2 = mu[0] * mu[0] * Dw[0] + mu[1] * mu[1] * Dw[1];   // omega_p^2 W
    const T rhoe = mu[0] * Dw[0] + mu[1] * Dw[1];                 // rho_e
    const vec3<T> U = v3<T>(mu[0] * mu[0] * Dw[0] * v[0].x + mu[1] * mu[1] * Dw[1] * v[1].x,
                            mu[0] * mu[0] * Dw[0] * v[0].y + mu[1] * mu[1] * Dw[1] * v[1].y,
                            mu[0] * mu[0] * Dw[0] * v[0].z + mu[1] * mu[1] * Dw[1] * v[1].z);  // omega_p^2 u
    const vec3<T> J = v3<T>(mu[0] * Dw[0] * v[0].x + mu[1] * Dw[1] * v[1].x,
                            mu[0] * Dw[0] * v[0].y + mu[1] * Dw[1] * v[1].y,
                            mu[0] * Dw[0] * v[0].z + mu[1] * Dw[1] * v[1].z);
    const T rho0 = (M2 * rhoe - dot(J, U)) * recip(wp2);
    const T fr = P.friction_covariant ? rho0 : rhoe;
    const vec3<T> UxB = cross(U, B);
    TFSource<T> s;
    s.Sb = v3<T>(M2 * E.x + UxB.x - eta * (wp2 * J.x - fr * U.x), M2 * E.y + UxB.y - eta * (wp2 * J.y - fr * U.y),
                 M2 * E.z + UxB.z - eta * (wp2 * J.z - fr * U.z));
    s.taub = dot(U, E) - eta * (wp2 * rhoe - rho0 * M2);
    s.J = J;
    return s;
}

// need_src false: the source terms are not wanted (left zero), e.g. for the halo rows of a flux
// tile, whose cells only contribute face fluxes.
__device__ inline void tf_flux_source(const double *q, const double *w, double sig, const Phys &P, double *fx,
                                      double *fy, double *src, bool need_src = true)
{
    const vec3<double> B = v3(q[tf::BX], q[tf::BY], q[tf::BZ]), E = v3(q[tf::EX], q[tf::EY], q[tf::EZ]);
    const double mu[2] = {P.mu1, P.mu2};
    const double em = 0.5 * (dot(E, E) + dot(B, B));
    double Dw[2], rho[2], A[2], p[2];
    vec3<double> v[2];
    for (int s = 0; s < 2; ++s) {
        const double *ws = w + 5 * s;
        v[s] = v3(ws[1], ws[2], ws[3]);
        const double Wl = frsqrt(1.0 - dot(v[s], v[s]));
        const double W2 = Wl * Wl;
        rho[s] = ws[0];
        p[s] = ws[4];
        Dw[s] = ws[0] * Wl;
        A[s] = (ws[0] + P.hk * ws[4]) * W2;
    }
    for (int k = 0; k < tf::NC; ++k) { fx[k] = 0.0; fy[k] = 0.0; }
    for (int s = 0; s < 2; ++s) {
        const vec3<double> vs = v[s];
        const double Sxx = A[s] * vs.x * vs.x + p[s], Syx = A[s] * vs.y * vs.x, Szx = A[s] * vs.z * vs.x;
        const double Syy = A[s] * vs.y * vs.y + p[s], Szy = A[s] * vs.z * vs.y;
        fx[tf::D] += Dw[s] * vs.x;               fy[tf::D] += Dw[s] * vs.y;
        fx[tf::SX] += Sxx; fx[tf::SY] += Syx; fx[tf::SZ] += Szx;
        fy[tf::SX] += Syx; fy[tf::SY] += Syy; fy[tf::SZ] += Szy;
        fx[tf::DB] += mu[s] * Dw[s] * vs.x;      fy[tf::DB] += mu[s] * Dw[s] * vs.y;
        fx[tf::SBX] += mu[s] * Sxx; fx[tf::SBY] += mu[s] * Syx; fx[tf::SBZ] += mu[s] * Szx;
        fy[tf::SBX] += mu[s] * Syx; fy[tf::SBY] += mu[s] * Syy; fy[tf::SBZ] += mu[s] * Szy;
        fx[tf::TAUB] += mu[s] * (A[s] - Dw[s]) * vs.x;
        fy[tf::TAUB] += mu[s] * (A[s] - Dw[s]) * vs.y;
    }
    fx[tf::SX] += em - E.x * E.x - B.x * B.x; fx[tf::SY] += -E.y * E.x - B.y * B.x; fx[tf::SZ] += -E.z * E.x - B.z * B.x;
    fy[tf::SX] += -E.x * E.y - B.x * B.y; fy[tf::SY] += em - E.y * E.y - B.y * B.y; fy[tf::SZ] += -E.z * E.y - B.z * B.y;
    fx[tf::TAU] = q[tf::SX] - fx[tf::D];
    fy[tf::TAU] = q[tf::SY] - fy[tf::D];
    fx[tf::BX] = q[tf::PHI]; fx[tf::BY] = -E.z; fx[tf::BZ] = E.y;
    fx[tf::EX] = q[tf::PSI]; fx[tf::EY] = B.z; fx[tf::EZ] = -B.y;
    fy[tf::BX] = E.z; fy[tf::BY] = q[tf::PHI]; fy[tf::BZ] = -E.x;
    fy[tf::EX] = -B.z; fy[tf::EY] = q[tf::PSI]; fy[tf::EZ] = B.x;
    fx[tf::PSI] = E.x; fx[tf::PHI] = B.x;
    fy[tf::PSI] = E.y; fy[tf::PHI] = B.y;
    for (int k = 0; k < tf::NC; ++k) src[k] = 0.0;
    if (need_src) {
        const TFSource<double> S = tf_source_terms<double>(Dw, rho, v, E, B, frcp(sig), P);
        src[tf::SBX] = S.Sb.x; src[tf::SBY] = S.Sb.y; src[tf::SBZ] = S.Sb.z;
        src[tf::TAUB] = S.taub;
        src[tf::EX] = -S.J.x; src[tf::EY] = -S.J.y; src[tf::EZ] = -S.J.z;
    }
    src[tf::PSI] = q[tf::DB] - P.kappa * q[tf::PSI];
    src[tf::PHI] = -P.kappa * q[tf::PHI];
}

// Flux vector f^z of one cell from (q, w), for 3-D grids (Appendix A Eq. A3, z column).
__device__ inline void tf_flux_z(const double *q, const double *w, const Phys &P, double *fz)
{
    const vec3<double> B = v3(q[tf::BX], q[tf::BY], q[tf::BZ]), E = v3(q[tf::EX], q[tf::EY], q[tf::EZ]);
    const double mu[2] = {P.mu1, P.mu2};
    const double em = 0.5 * (dot(E, E) + dot(B, B));
    for (int k = 0; k < tf::NC; ++k) fz[k] = 0.0;
    for (int s = 0; s < 2; ++s) {
        const double *ws = w + 5 * s;
        const vec3<double> vs = v3(ws[1], ws[2], ws[3]);
        const double Wl = frsqrt(1.0 - dot(vs, vs));
        const double Dw = ws[0] * Wl, A = (ws[0] + P.hk * ws[4]) * (Wl * Wl);
        const double Sxz = A * vs.x * vs.z, Syz = A * vs.y * vs.z, Szz = A * vs.z * vs.z + ws[4];
        fz[tf::D] += Dw * vs.z;
        fz[tf::SX] += Sxz; fz[tf::SY] += Syz; fz[tf::SZ] += Szz;
        fz[tf::DB] += mu[s] * Dw * vs.z;
        fz[tf::SBX] += mu[s] * Sxz; fz[tf::SBY] += mu[s] * Syz; fz[tf::SBZ] += mu[s] * Szz;
        fz[tf::TAUB] += mu[s] * (A - Dw) * vs.z;
    }
    fz[tf::SX] += -E.x * E.z - B.x * B.z; fz[tf::SY] += -E.y * E.z - B.y * B.z; fz[tf::SZ] += em - E.z * E.z - B.z * B.z;
    fz[tf::TAU] = q[tf::SZ] - fz[tf::D];
    fz[tf::BX] = -E.y; fz[tf::BY] = E.x; fz[tf::BZ] = q[tf::PHI];
    fz[tf::EX] = B.y; fz[tf::EY] = -B.x; fz[tf::EZ] = q[tf::PSI];
    fz[tf::PSI] = E.z; fz[tf::PHI] = B.z;
}

// ---------------------------------------------------------------------------------------
// Ideal RMHD (Sec. 2.1 lists it; recovery by a two-dimensional root-find, Sec. 2.1.3): the
// conserved state (D, S, tau, B, phi) of a perfectly conducting fluid, E = -v x B, with the
// resistive models' cleaning of B (flux of B^i gains phi along i; d_t phi + div B = -kappa phi).
// ---------------------------------------------------------------------------------------
__device__ inline void id_prim2cons(const double *w, const double *EB, const Phys &P, double *q)
{
    const vec3<double> v = v3(w[1], w[2], w[3]), B = v3(EB[0], EB[1], EB[2]);
    const double W = frsqrt(1.0 - dot(v, v));
    const double Z = (w[0] + P.hk * w[4]) * (W * W);   // rho h W^2
    const double vB = dot(v, B), B2 = dot(B, B);
    q[id::D] = w[0] * W;
    q[id::SX] = (Z + B2) * v.x - vB * B.x;
    q[id::SY] = (Z + B2) * v.y - vB * B.y;
    q[id::SZ] = (Z + B2) * v.z - vB * B.z;
    // E^2 = v^2 B^2 - (v.B)^2 for E = -v x B
    q[id::TAU] = Z - w[4] + 0.5 * (B2 + dot(v, v) * B2 - vB * vB) - q[id::D];
    q[id::BX] = B.x; q[id::BY] = B.y; q[id::BZ] = B.z;
    q[id::PHI] = 0.0;
}

// The two equations of the recovery in the unknowns (Z = rho h W^2, y = v^2):
//   F1 = y (Z + B^2)^2 - (S.B)^2 (B^2 + 2 Z) / Z^2 - S^2                 (momentum)
//   F2 = Z + B^2 - p - B^2 (1 - y) / 2 - (S.B)^2 / (2 Z^2) - (tau + D)    (energy)
// with p = (Gamma-1)/Gamma (Z (1 - y) - D sqrt(1 - y)) for the Gamma law.
struct IdealSys {
    double D, S2, SB2, B2, Et, gk;
};
__device__ __forceinline__ void id_residual(const IdealSys &s, double Z, double y, double &F1, double &F2,
                                            double J[4])
{
    const double iZ = frcp(Z), u = 1.0 - y, su = fsqrt(u);
    const double ZB = Z + s.B2;
    const double p = s.gk * (Z * u - s.D * su);
    F1 = y * ZB * ZB - s.SB2 * (s.B2 + 2.0 * Z) * iZ * iZ - s.S2;
    F2 = ZB - p - 0.5 * s.B2 * u - 0.5 * s.SB2 * iZ * iZ - s.Et;
    J[0] = 2.0 * y * ZB + 2.0 * s.SB2 * ZB * iZ * iZ * iZ;   // dF1/dZ
    J[1] = ZB * ZB;                                          // dF1/dy
    J[2] = 1.0 - s.gk * u + s.SB2 * iZ * iZ * iZ;            // dF2/dZ
    J[3] = s.gk * (Z - 0.5 * s.D * frcp(su)) + 0.5 * s.B2;   // dF2/dy
}

// Second route, where the two-dimensional iteration does not converge: y from F1 = 0 in
// closed form, y(Z) = (S^2 Z^2 + (S.B)^2 (2 Z + B^2)) / (Z^2 (Z + B^2)^2), and F2(Z, y(Z))
// bracketed on Z (y >= 1 or F2 < 0 below the root, F2 > 0 above) and bisected to rounding.
// A bracket that closes on the edge y = 1 instead of a sign change of F2 holds no root: the
// state has no physical primitives (status CELL_C2P_UNPHYS).
__device__ inline int id_root_1d(const IdealSys &s, double &Z, double &y, int &iters)
{
    auto eval = [&](double z, double &yy, double &f) -> bool {
        const double iz = frcp(z), zb = z + s.B2;
        yy = (s.S2 * z * z + s.SB2 * (2.0 * z + s.B2)) * iz * iz * frcp(zb * zb);
        if (!(yy < 1.0)) return false;
        const double u = 1.0 - yy;
        f = zb - s.gk * (z * u - s.D * fsqrt(u)) - 0.5 * s.B2 * u - 0.5 * s.SB2 * iz * iz - s.Et;
        return true;
    };
    double lo = 0.0, hi = 2.0 * s.Et + 1.0, yy = 0.0, f = 0.0;
    int k = 0;
    while (k < 64 && !(eval(hi, yy, f) && f > 0.0)) {
        lo = hi;
        hi *= 2.0;
        ++k;
    }
    if (k == 64) return CELL_C2P_UNPHYS;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        if (eval(mid, yy, f) && f > 0.0) hi = mid; else lo = mid;
        ++iters;
    }
    Z = hi;
    if (!eval(Z, y, f) || fabs(f) > 1e-8 * fmax(1.0, s.Et)) return CELL_C2P_UNPHYS;
    return CELL_OK;
}

// 9 conserved -> (rho, v, p).  Newton on (Z, y) from the guess w (rho h W^2 and v^2 of w;
// a start outside Z > 0, 0 <= y < 1 is replaced by Z = tau + D, y = 0), steps halved until
// they stay inside; stop at |F1| <= tol max(1, S^2 + B^4) and |F2| <= tol max(1, tau + D) and
// take one more step.  Where it does not converge (unless P.c2p_fallback is 0) the
// one-dimensional route takes over.
__device__ inline int id_cons2prim(const double *q, double *w, const Phys &P, int &iters)
{
    const vec3<double> S = v3(q[id::SX], q[id::SY], q[id::SZ]), B = v3(q[id::BX], q[id::BY], q[id::BZ]);
    IdealSys s;
    s.D = q[id::D];
    s.S2 = dot(S, S);
    const double SB = dot(S, B);
    s.SB2 = SB * SB;
    s.B2 = dot(B, B);
    s.Et = q[id::TAU] + q[id::D];
    s.gk = P.gk;
    iters = 0;
    if (!(s.D > 0.0) || !(s.Et > 0.0) || !isfinite(s.S2 + s.B2)) return CELL_C2P_UNPHYS;
    double y = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
    double Z = (w[0] + P.hk * w[4]) * frcp(1.0 - y);
    if (!(Z > 0.0) || !(y >= 0.0 && y < 1.0) || !(w[0] > 0.0) || !(w[4] > 0.0)) {
        Z = s.Et;
        y = 0.0;
    }
    const double t1 = P.c2p_tol * fmax(1.0, s.S2 + s.B2 * s.B2), t2 = P.c2p_tol * fmax(1.0, s.Et);
    int st = CELL_C2P_NOCONV;
    for (int it = 1; it <= P.max_c2p; ++it) {
        double F1, F2, J[4];
        id_residual(s, Z, y, F1, F2, J);
        const double idet = frcp(J[0] * J[3] - J[1] * J[2]);
        const double dZ = -(J[3] * F1 - J[1] * F2) * idet, dy = -(J[0] * F2 - J[2] * F1) * idet;
        const bool done = fabs(F1) <= t1 && fabs(F2) <= t2;
        double lam = 1.0;
        for (int h = 0; h < 30 && !(Z + lam * dZ > 0.0 && y + lam * dy >= 0.0 && y + lam * dy < 1.0); ++h)
            lam *= 0.5;
        iters = it;
        if (!(Z + lam * dZ > 0.0 && y + lam * dy >= 0.0 && y + lam * dy < 1.0)) break;
        Z += lam * dZ;
        y += lam * dy;
        if (done) {
            st = CELL_OK;
            break;
        }
    }
    if (st != CELL_OK && P.c2p_fallback) st = id_root_1d(s, Z, y, iters);
    if (st != CELL_OK) return st;
    const double iZB = frcp(Z + s.B2), sZ = SB * frcp(Z);
    w[1] = (S.x + sZ * B.x) * iZB;
    w[2] = (S.y + sZ * B.y) * iZB;
    w[3] = (S.z + sZ * B.z) * iZB;
    // rho and p from the velocity actually returned, so that (rho, v, p) are consistent
    const double uw = 1.0 - (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
    w[0] = s.D * fsqrt(uw);
    w[4] = P.gk * (Z * uw - w[0]);
    if (!(w[0] > 0.0) || !(w[4] > 0.0) || !(uw > 0.0)) return CELL_C2P_UNPHYS;
    return CELL_OK;
}

// Flux of one cell along direction K (0, 1, 2) from (q, w), and the cleaning source.
template <int K>
__device__ __forceinline__ void id_flux_dir(const double *q, const vec3<double> &v, double W, double pstar,
                                           const double *b, const vec3<double> &B, double *f)
{
    const double vk = K == 0 ? v.x : K == 1 ? v.y : v.z;
    const double Bk = K == 0 ? B.x : K == 1 ? B.y : B.z;
    const double iW = frcp(W);
    f[id::D] = q[id::D] * vk;
    f[id::SX] = q[id::SX] * vk + (K == 0 ? pstar : 0.0) - b[0] * Bk * iW;
    f[id::SY] = q[id::SY] * vk + (K == 1 ? pstar : 0.0) - b[1] * Bk * iW;
    f[id::SZ] = q[id::SZ] * vk + (K == 2 ? pstar : 0.0) - b[2] * Bk * iW;
    f[id::TAU] = q[id::SX + K] - q[id::D] * vk;
    f[id::BX] = vk * B.x - v.x * Bk + (K == 0 ? q[id::PHI] : 0.0);
    f[id::BY] = vk * B.y - v.y * Bk + (K == 1 ? q[id::PHI] : 0.0);
    f[id::BZ] = vk * B.z - v.z * Bk + (K == 2 ? q[id::PHI] : 0.0);
    f[id::PHI] = Bk;
}

// Comoving-field quantities of the fluxes: b^i = B^i / W + b^0 v^i, b^0 = W (v.B),
// p* = p + b^2 / 2, b^2 = B^2 / W^2 + (v.B)^2.
__device__ __forceinline__ void id_fields(const double *q, const double *w, vec3<double> &v, vec3<double> &B,
                                         double &W, double &pstar, double b[3])
{
    v = v3(w[1], w[2], w[3]);
    B = v3(q[id::BX], q[id::BY], q[id::BZ]);
    W = frsqrt(1.0 - dot(v, v));
    const double vB = dot(v, B), iW = frcp(W), b0 = W * vB;
    b[0] = B.x * iW + b0 * v.x;
    b[1] = B.y * iW + b0 * v.y;
    b[2] = B.z * iW + b0 * v.z;
    pstar = w[4] + 0.5 * (dot(B, B) * (iW * iW) + vB * vB);
}

__device__ inline void id_flux_source(const double *q, const double *w, const Phys &P, double *fx, double *fy,
                                      double *src)
{
    vec3<double> v, B;
    double W, pstar, b[3];
    id_fields(q, w, v, B, W, pstar, b);
    id_flux_dir<0>(q, v, W, pstar, b, B, fx);
    id_flux_dir<1>(q, v, W, pstar, b, B, fy);
    for (int k = 0; k < id::NC; ++k) src[k] = 0.0;
    src[id::PHI] = -P.kappa * q[id::PHI];
}

__device__ inline void id_flux_z(const double *q, const double *w, const Phys &P, double *fz)
{
    vec3<double> v, B;
    double W, pstar, b[3];
    id_fields(q, w, v, B, W, pstar, b);
    id_flux_dir<2>(q, v, W, pstar, b, B, fz);
    (void)P;   // the ideal fluxes need no physics constants beyond the state
}

// ---------------------------------------------------------------------------------------
// Flux components one at a time (for the row-form flux tile, which works through the
// conserved variables in rounds): the per-cell quantities shared by the components are
// formed once, and each component of f^x (K = 0) or f^y (K = 1) and of the source is an
// expression in them and in q, so only the current round's values are live.  Same values as
// sf_flux_source / id_flux_source.
// ---------------------------------------------------------------------------------------
struct SFRow {
    double vx, vy, vz, A, pt, Jx, Jy, Jz;
};
__device__ __forceinline__ SFRow sf_row(const double *q, const double *w, double sig, const Phys &P)
{
    const vec3<double> v = v3(w[1], w[2], w[3]);
    const vec3<double> B = v3(q[sf::BX], q[sf::BY], q[sf::BZ]), E = v3(q[sf::EX], q[sf::EY], q[sf::EZ]);
    const double W = frsqrt(1.0 - dot(v, v));
    const vec3<double> J = sf_current(v, W, E, B, q[sf::RHOE], sig);
    return SFRow{v.x, v.y, v.z, (w[0] + P.hk * w[4]) * (W * W), w[4] + 0.5 * (dot(E, E) + dot(B, B)), J.x, J.y, J.z};
}
template <int K>
__device__ __forceinline__ double sf_row_flux(int c, const double *q, const SFRow &I)
{
    const double vk = K == 0 ? I.vx : I.vy, Ek = q[sf::EX + K], Bk = q[sf::BX + K];
    switch (c) {
    case sf::D: return q[sf::D] * vk;
    case sf::SX: return I.A * I.vx * vk + (K == 0 ? I.pt : 0.0) - q[sf::EX] * Ek - q[sf::BX] * Bk;
    case sf::SY: return I.A * I.vy * vk + (K == 1 ? I.pt : 0.0) - q[sf::EY] * Ek - q[sf::BY] * Bk;
    case sf::SZ: return I.A * I.vz * vk - q[sf::EZ] * Ek - q[sf::BZ] * Bk;
    case sf::TAU: return q[sf::SX + K] - q[sf::D] * vk;
    case sf::BX: return K == 0 ? q[sf::PHI] : q[sf::EZ];
    case sf::BY: return K == 0 ? -q[sf::EZ] : q[sf::PHI];
    case sf::BZ: return K == 0 ? q[sf::EY] : -q[sf::EX];
    case sf::EX: return K == 0 ? q[sf::PSI] : -q[sf::BZ];
    case sf::EY: return K == 0 ? q[sf::BZ] : q[sf::PSI];
    case sf::EZ: return K == 0 ? -q[sf::BY] : q[sf::BX];
    case sf::RHOE: return K == 0 ? I.Jx : I.Jy;
    case sf::PSI: return Ek;
    default: return Bk;   // PHI
    }
}
__device__ __forceinline__ double sf_row_src(int c, const double *q, const SFRow &I, const Phys &P)
{
    switch (c) {
    case sf::EX: return -I.Jx;
    case sf::EY: return -I.Jy;
    case sf::EZ: return -I.Jz;
    case sf::PSI: return q[sf::RHOE] - P.kappa * q[sf::PSI];
    case sf::PHI: return -P.kappa * q[sf::PHI];
    default: return 0.0;
    }
}

struct IdRow {
    double vx, vy, vz, iW, pstar, bx, by, bz;
};
__device__ __forceinline__ IdRow id_row(const double *q, const double *w)
{
    vec3<double> v, B;
    double W, pstar, b[3];
    id_fields(q, w, v, B, W, pstar, b);
    return IdRow{v.x, v.y, v.z, frcp(W), pstar, b[0], b[1], b[2]};
}
template <int K>
__device__ __forceinline__ double id_row_flux(int c, const double *q, const IdRow &I)
{
    const double vk = K == 0 ? I.vx : I.vy, Bk = q[id::BX + K];
    switch (c) {
    case id::D: return q[id::D] * vk;
    case id::SX: return q[id::SX] * vk + (K == 0 ? I.pstar : 0.0) - I.bx * Bk * I.iW;
    case id::SY: return q[id::SY] * vk + (K == 1 ? I.pstar : 0.0) - I.by * Bk * I.iW;
    case id::SZ: return q[id::SZ] * vk - I.bz * Bk * I.iW;
    case id::TAU: return q[id::SX + K] - q[id::D] * vk;
    case id::BX: return vk * q[id::BX] - I.vx * Bk + (K == 0 ? q[id::PHI] : 0.0);
    case id::BY: return vk * q[id::BY] - I.vy * Bk + (K == 1 ? q[id::PHI] : 0.0);
    case id::BZ: return vk * q[id::BZ] - I.vz * Bk;
    default: return Bk;   // PHI
    }
}

}  // namespace rmhd
