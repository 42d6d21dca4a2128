"""The implicit stage's exact Jacobians (csrc/stage.hpp) checked against central finite
differences of the stage residual they differentiate, with the stage code compiled for the
host: the two-fluid Jacobian written out by the chain rule through the residual's structure
(species split, recovery root by the implicit-function theorem, source terms), and the
single-fluid one by three-tangent dual numbers.  Random physical states of both species
(speeds up to 0.9), both friction forms, two charge-to-mass pairs and stage coefficients
a sigma from 1e-2 to 1e2, so that the resistive terms carry weight in every column.

A stand-in for the HIP runtime header maps the device qualifiers away and the hardware
reciprocal and reciprocal square root onto exact host arithmetic; everything else is the
device source as it is compiled for the GPU.  Newton converges at the same rate whatever
the Jacobian's rounding, so the kernels' results do not depend on these last bits; a wrong
term, however, slows or stalls the iteration, and no parity test would name it."""
import ctypes
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1808_09721_amd", "csrc")

SHIM = r"""
#pragma once
#include <cmath>
#define __host__
#define __device__
#define __forceinline__ inline
#define __global__
using std::fma; using std::sqrt; using std::fabs; using std::isfinite; using std::fmax; using std::fmin;
inline double __builtin_amdgcn_rcp(double x) { return 1.0 / x; }
inline double __builtin_amdgcn_rsq(double x) { return 1.0 / std::sqrt(x); }
"""

HARNESS = r"""
#include <hip/hip_runtime.h>
#include "stage.hpp"
using namespace rmhd;

static Phys phys(const double *pp)
{
    Phys P{};
    P.gamma = pp[0];
    P.gk = (P.gamma - 1.0) / P.gamma;
    P.hk = P.gamma / (P.gamma - 1.0);
    P.mu1 = pp[1];
    P.mu2 = pp[2];
    P.friction_covariant = (int)pp[3];
    P.c2p_tol = 1e-13;
    P.newton_tol = 1e-12;
    P.max_c2p = 100;
    P.max_newton = 50;
    P.c2p_fallback = 1;
    P.jac_keep = 0.1;
    return P;
}

// Jacobian of the two-fluid stage residual at the stage's plain start x = R_x: the kernel's
// (Jc) and central differences with steps h max(1, |x_k|) (Jf), row-major 7x7.
extern "C" int tf_jac(const double *pp, const double *w, const double *EB, double a, double sig, double h,
                      double *Jc, double *Jf)
{
    const Phys P = phys(pp);
    double R[tf::NC];
    tf_prim2cons(w, EB, P, R);
    const TFCell c = tf_cell(R, a, sig, P);
    double x[7] = {R[tf::SBX] * c.isc, R[tf::SBY] * c.isc, R[tf::SBZ] * c.isc, R[tf::TAUB] * c.isc,
                   R[tf::EX], R[tf::EY], R[tf::EZ]};
    const double pg[2] = {w[4], w[9]};
    double G[7], Eh[2];
    Root r[2];
    int it = 0;
    if (tf_residual(c, x, pg, P, G, r, Eh, it) != CELL_OK) return -1;
    double A[7][7];
    tf_jacobian(c, x, r, P, A);
    for (int i = 0; i < 7; ++i)
        for (int j = 0; j < 7; ++j) Jc[7 * i + j] = A[i][j];
    for (int k = 0; k < 7; ++k) {
        const double hk = h * fmax(1.0, fabs(x[k]));
        double xp[7], xm[7], Gp[7], Gm[7];
        for (int i = 0; i < 7; ++i) { xp[i] = x[i]; xm[i] = x[i]; }
        xp[k] += hk;
        xm[k] -= hk;
        if (tf_residual(c, xp, pg, P, Gp, r, Eh, it) != CELL_OK) return -2;
        if (tf_residual(c, xm, pg, P, Gm, r, Eh, it) != CELL_OK) return -2;
        for (int i = 0; i < 7; ++i) Jf[7 * i + k] = (Gp[i] - Gm[i]) / (xp[k] - xm[k]);
    }
    return 0;
}

// The same for the single-fluid stage (x = E, 3x3).
extern "C" int sf_jac(const double *pp, const double *w, const double *EB, double rhoe, double a, double sig,
                      double h, double *Jc, double *Jf)
{
    const Phys P = phys(pp);
    double R[sf::NC];
    sf_prim2cons(w, EB, rhoe, P, R);
    const SFCell c = sf_cell(R, a, sig);
    double x[3] = {R[sf::EX], R[sf::EY], R[sf::EZ]};
    double G[3], Eh;
    Root r;
    int it = 0;
    if (sf_residual(c, x, w[4], P, G, r, Eh, it) != CELL_OK) return -1;
    double A[3][3];
    sf_jacobian(c, x, r, P, A);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Jc[3 * i + j] = A[i][j];
    for (int k = 0; k < 3; ++k) {
        const double hk = h * fmax(1.0, fabs(x[k]));
        double xp[3] = {x[0], x[1], x[2]}, xm[3] = {x[0], x[1], x[2]}, Gp[3], Gm[3];
        xp[k] += hk;
        xm[k] -= hk;
        if (sf_residual(c, xp, w[4], P, Gp, r, Eh, it) != CELL_OK) return -2;
        if (sf_residual(c, xm, w[4], P, Gm, r, Eh, it) != CELL_OK) return -2;
        for (int i = 0; i < 3; ++i) Jf[3 * i + k] = (Gp[i] - Gm[i]) / (xp[k] - xm[k]);
    }
    return 0;
}
"""


def build(csrc: str = CSRC):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tempfile.mkdtemp(prefix="stage_jac_")
    os.makedirs(os.path.join(d, "hip"))
    open(os.path.join(d, "hip", "hip_runtime.h"), "w").write(SHIM)
    src, so = os.path.join(d, "h.cpp"), os.path.join(d, "libjac.so")
    open(src, "w").write(HARNESS)
    subprocess.run([cxx, "-O2", "-std=c++17", "-shared", "-fPIC", "-Wno-unknown-pragmas", "-I", d, "-I", csrc, src,
                    "-o", so], check=True)
    lib = ctypes.CDLL(so)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.tf_jac.restype = ctypes.c_int
    lib.tf_jac.argtypes = [dp, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp]
    lib.sf_jac.restype = ctypes.c_int
    lib.sf_jac.argtypes = [dp, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp]
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def random_species(rng):
    v = rng.uniform(-1, 1, 3)
    v *= 0.9 * rng.uniform() / np.linalg.norm(v)
    return [10 ** rng.uniform(-1, 1), *v, 10 ** rng.uniform(-2, 0)]


def tf_errors(lib, n=300, seed=3):
    """Largest |Jc - Jf| / max|Jf| over random two-fluid states, and the number checked."""
    rng = np.random.default_rng(seed)
    worst, checked = 0.0, 0
    for mu1, mu2 in ((1000.0, -1000.0), (-20.0, 1.0)):
        for cov in (0, 1):
            pp = np.array([4.0 / 3.0, mu1, mu2, cov, 0.0])
            for _ in range(n):
                w = np.array(random_species(rng) + random_species(rng))
                EB = rng.uniform(-1, 1, 6)
                a = 10 ** rng.uniform(-3, -1)
                sig = 10 ** rng.uniform(1, 3)
                Jc, Jf = np.zeros(49), np.zeros(49)
                rc = lib.tf_jac(_ptr(pp), _ptr(w), _ptr(EB), a, sig, 1e-6, _ptr(Jc), _ptr(Jf))
                if rc != 0:
                    continue
                checked += 1
                worst = max(worst, float(np.abs(Jc - Jf).max() / np.abs(Jf).max()))
    return worst, checked


def test_two_fluid_jacobian_matches_finite_differences():
    lib = build()
    worst, checked = tf_errors(lib)
    print(f"two-fluid: {checked} states, max |J - J_fd| / max |J_fd| = {worst:.2e}")
    assert checked >= 1000
    assert worst < 1e-6


def test_single_fluid_jacobian_matches_finite_differences():
    lib = build()
    rng = np.random.default_rng(4)
    worst, checked = 0.0, 0
    pp = np.array([4.0 / 3.0, 0.0, 0.0, 0, 0.0])
    for _ in range(600):
        w = np.array(random_species(rng))
        EB = rng.uniform(-1, 1, 6)
        rhoe = rng.uniform(-0.5, 0.5)
        a = 10 ** rng.uniform(-3, -1)
        sig = 10 ** rng.uniform(1, 3)
        Jc, Jf = np.zeros(9), np.zeros(9)
        if lib.sf_jac(_ptr(pp), _ptr(w), _ptr(EB), rhoe, a, sig, 1e-6, _ptr(Jc), _ptr(Jf)) != 0:
            continue
        checked += 1
        worst = max(worst, float(np.abs(Jc - Jf).max() / np.abs(Jf).max()))
    print(f"single fluid: {checked} states, max |J - J_fd| / max |J_fd| = {worst:.2e}")
    assert checked >= 500
    assert worst < 1e-6
