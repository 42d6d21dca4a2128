"""The implicit stage's register LU (csrc/lu.hpp) compiled for the host and checked against
numpy's solve: random 7x7 systems with pivoting at every elimination step, systems whose
pivots are forced at late steps only, and singular matrices (refused).  The stage replays
the recorded row swaps interleaved with the elimination, so the factorisation must leave
each multiplier where it was formed; moving it along with later swaps gives solutions off
by O(1) whenever a later step pivots."""
import ctypes
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1808_09721_amd", "csrc")

HARNESS = r"""
#define __host__
#define __device__
#define __forceinline__ inline
#include "lu.hpp"
extern "C" int lu_solve7(const double *a, const double *b, double *x)
{
    double A[7][7], v[7];
    for (int i = 0; i < 7; ++i) {
        v[i] = b[i];
        for (int j = 0; j < 7; ++j) A[i][j] = a[7 * i + j];
    }
    unsigned long long swaps = 0;
    if (!rmhd::lu_factor<7>(A, swaps)) return -1;
    rmhd::lu_solve<7>(A, swaps, v);
    for (int i = 0; i < 7; ++i) x[i] = v[i];
    return __builtin_popcountll(swaps);
}
"""


@pytest.fixture(scope="module")
def lu():
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tempfile.mkdtemp(prefix="lu_host_")
    src, so = os.path.join(d, "h.cpp"), os.path.join(d, "liblu.so")
    open(src, "w").write(HARNESS)
    subprocess.run([cxx, "-O2", "-std=c++17", "-shared", "-fPIC", "-Wno-unknown-pragmas", "-I", CSRC, src, "-o", so],
                   check=True)
    lib = ctypes.CDLL(so)
    lib.lu_solve7.restype = ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    lib.lu_solve7.argtypes = [dp, dp, dp]

    def solve(A, b):
        A = np.ascontiguousarray(A, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.empty(7)
        rc = lib.lu_solve7(A.ctypes.data_as(dp), b.ctypes.data_as(dp), x.ctypes.data_as(dp))
        return rc, x
    yield solve
    shutil.rmtree(d, ignore_errors=True)


def test_random_systems_match_numpy(lu):
    rng = np.random.default_rng(5)
    swaps = 0
    for _ in range(500):
        A = rng.normal(size=(7, 7)) * rng.uniform(1e-3, 1e3, size=(7, 1))
        b = rng.normal(size=7)
        rc, x = lu(A, b)
        assert rc >= 0
        swaps += rc
        # backward error of a stable factorisation: |A x - b| <= c eps (|A| |x| + |b|)
        res = np.abs(A @ x - b).max()
        assert res <= 1e-13 * (np.abs(A).max() * np.abs(x).max() + np.abs(b).max())
        ref = np.linalg.solve(A, b)
        assert np.abs(x - ref).max() <= 1e-10 * np.linalg.cond(A) * np.abs(ref).max()
    assert swaps > 500          # pivoting happened, at many steps


def test_late_pivots(lu):
    """Diagonally dominant in the first columns, so the first steps keep their rows; a small
    diagonal entry further down forces swaps at steps 3 and 5 after multipliers exist."""
    rng = np.random.default_rng(6)
    for _ in range(100):
        A = rng.normal(size=(7, 7))
        A[0, 0] += 20.0
        A[1, 1] += 20.0
        A[2, 2] += 20.0
        A[3, 3] = 1e-3
        A[5, 5] = 1e-3
        b = rng.normal(size=7)
        rc, x = lu(A, b)
        assert rc > 0
        np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)


def test_singular_is_refused(lu):
    A = np.ones((7, 7))
    rc, _ = lu(A, np.ones(7))
    assert rc == -1
