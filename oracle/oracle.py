"""Python access to the plain FP64 CPU oracle (``rmhd_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It never imports the product
package; the product never imports it.

Arrays use the oracle's own layout ``[var][NY][NX]`` (``NX = nx + 4``; ``NY = ny + 4`` in
2-D, 1 in 1-D) or, in 3-D, ``[var][NZ][NY][NX]`` (``NZ = nz + 4``), float64, C-contiguous.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rmhd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, C2P_NOCONV, C2P_UNPHYS, NEWTON_NOCONV, LINESEARCH = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, OpenMP over cells)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int), ("ndim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("bc", ctypes.c_int), ("max_c2p_iter", ctypes.c_int), ("max_newton_iter", ctypes.c_int),
        ("friction_covariant", ctypes.c_int),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("gamma", ctypes.c_double),
        ("sigma", ctypes.c_double), ("mu1", ctypes.c_double), ("mu2", ctypes.c_double),
        ("kappa", ctypes.c_double), ("c2p_tol", ctypes.c_double), ("newton_tol", ctypes.c_double),
        ("sigma_cell", ctypes.POINTER(ctypes.c_double)),
        ("nz", ctypes.c_int), ("dz", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        P = ctypes.POINTER(_Params)
        sig = {
            "orc_set_threads": (ctypes.c_int, [ctypes.c_int]),
            "orc_ncons": (ctypes.c_int, [ctypes.c_int]),
            "orc_nprim": (ctypes.c_int, [ctypes.c_int]),
            "orc_prim2cons_cell": (None, [P, dp, dp, ctypes.c_double, dp]),
            "orc_cons2prim_cell": (ctypes.c_int, [P, dp, dp, ip]),
            "orc_flux_cell": (None, [P, dp, dp, ctypes.c_double, ctypes.c_int, dp]),
            "orc_source_cell": (None, [P, dp, dp, ctypes.c_double, dp]),
            "orc_implicit_cell": (ctypes.c_int, [P, ctypes.c_double, ctypes.c_double, dp, dp, dp, ip]),
            "orc_implicit_residual_cell": (ctypes.c_int, [P, ctypes.c_double, ctypes.c_double, dp, dp, dp, ip]),
            "orc_implicit_cell_from": (ctypes.c_int, [P, ctypes.c_double, ctypes.c_double, dp, dp, dp, dp, ip]),
            "orc_weno3_face": (None, [dp, dp, dp, dp, ctypes.c_int]),
            "orc_bc_fill": (None, [P, dp, ctypes.c_int]),
            "orc_init_state": (None, [P, dp, dp, dp]),
            "orc_cons2prim": (None, [P, dp, dp, ctypes.c_void_p, ctypes.c_void_p]),
            "orc_rhs": (None, [P, dp, dp, dp]),
            "orc_implicit": (None, [P, ctypes.c_double, dp, dp, dp, ctypes.c_void_p, ctypes.c_void_p]),
            "orc_ssp2_step": (ctypes.c_int, [P, ctypes.c_double, dp, dp, ctypes.POINTER(ctypes.c_longlong), ip, ip]),
            "orc_ssp3_step": (ctypes.c_int, [P, ctypes.c_double, dp, dp, ctypes.POINTER(ctypes.c_longlong), ip, ip]),
            "orc_dt": (ctypes.c_double, [P, ctypes.c_double]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous float64"
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Grid:
    """Problem set-up handed to the oracle (mirrors the workload description)."""
    model: int
    ndim: int
    nx: int
    ny: int
    dx: float
    dy: float
    gamma: float
    sigma: float
    bc: int
    mu1: float = 0.0
    mu2: float = 0.0
    kappa: float = 1.0
    c2p_tol: float = 1e-13
    newton_tol: float = 1e-12
    max_c2p_iter: int = 100
    max_newton_iter: int = 50
    friction_covariant: int = 0
    sigma_cell: np.ndarray | None = None   # cell shape ([NY][NX], 3-D [NZ][NY][NX]) or None
    nz: int = 1
    dz: float = 1.0
    _keep: list = field(default_factory=list, repr=False)

    @property
    def NX(self) -> int:
        return self.nx + 4

    @property
    def NY(self) -> int:
        return self.ny + 4 if self.ndim >= 2 else 1

    @property
    def NZ(self) -> int:
        return self.nz + 4 if self.ndim == 3 else 1

    @property
    def cell_shape(self) -> tuple:
        """Shape of one variable's array: (NY, NX), or (NZ, NY, NX) in 3-D."""
        return (self.NZ, self.NY, self.NX) if self.ndim == 3 else (self.NY, self.NX)

    @property
    def ncons(self) -> int:
        return {0: 14, 1: 18, 2: 9}[self.model]

    @property
    def nprim(self) -> int:
        return 10 if self.model == 1 else 5

    def interior(self, a: np.ndarray) -> np.ndarray:
        """View of the interior cells of a [var][NY][NX] (3-D: [var][NZ][NY][NX]) array."""
        if self.ndim == 3:
            return a[..., 2:-2, 2:-2, 2:-2]
        if self.ndim == 2:
            return a[..., 2:-2, 2:-2]
        return a[..., :, 2:-2]

    def zeros(self, nvar: int) -> np.ndarray:
        return np.zeros((nvar,) + self.cell_shape)

    def embed(self, interior: np.ndarray) -> np.ndarray:
        """[var][ny][nx] (3-D: [var][nz][ny][nx]) interior values -> the full layout with zero
        ghosts."""
        out = self.zeros(interior.shape[0])
        self.interior(out)[...] = interior.reshape(self.interior(out).shape)
        return out

    def params(self) -> _Params:
        p = _Params()
        for name, _ in _Params._fields_:
            if name == "sigma_cell":
                continue
            setattr(p, name, getattr(self, name))
        if self.sigma_cell is not None:
            sc = np.ascontiguousarray(self.sigma_cell, dtype=np.float64)
            self._keep.append(sc)
            p.sigma_cell = _dp(sc)
        else:
            p.sigma_cell = ctypes.POINTER(ctypes.c_double)()
        return p


# ---------------------------------------------------------------------------------------------
# per-cell calls
# ---------------------------------------------------------------------------------------------
def prim2cons_cell(g: Grid, w, EB, rho_e=0.0):
    q = np.zeros(g.ncons)
    lib().orc_prim2cons_cell(ctypes.byref(g.params()), _dp(np.ascontiguousarray(w, float)),
                             _dp(np.ascontiguousarray(EB, float)), float(rho_e), _dp(q))
    return q


def cons2prim_cell(g: Grid, q, w_guess=None):
    w = np.full(g.nprim, -1.0) if w_guess is None else np.array(w_guess, dtype=float)
    it = ctypes.c_int(0)
    st = lib().orc_cons2prim_cell(ctypes.byref(g.params()), _dp(np.ascontiguousarray(q, float)), _dp(w),
                                  ctypes.byref(it))
    return w, st, it.value


def flux_cell(g: Grid, q, w, direction, sigma=None):
    f = np.zeros(g.ncons)
    lib().orc_flux_cell(ctypes.byref(g.params()), _dp(np.ascontiguousarray(q, float)),
                        _dp(np.ascontiguousarray(w, float)), float(g.sigma if sigma is None else sigma),
                        int(direction), _dp(f))
    return f


def source_cell(g: Grid, q, w, sigma=None):
    s = np.zeros(g.ncons)
    lib().orc_source_cell(ctypes.byref(g.params()), _dp(np.ascontiguousarray(q, float)),
                          _dp(np.ascontiguousarray(w, float)), float(g.sigma if sigma is None else sigma), _dp(s))
    return s


def implicit_cell(g: Grid, a, R, w_guess=None, sigma=None, Q_start=None):
    """Implicit stage of one cell; Newton starts from the unknowns of Q_start (default R)."""
    Q = np.zeros(g.ncons)
    w = np.full(g.nprim, -1.0) if w_guess is None else np.array(w_guess, dtype=float)
    it = ctypes.c_int(0)
    start = _dp(np.ascontiguousarray(Q_start, float)) if Q_start is not None else ctypes.POINTER(ctypes.c_double)()
    st = lib().orc_implicit_cell_from(ctypes.byref(g.params()), float(a), float(g.sigma if sigma is None else sigma),
                                      _dp(np.ascontiguousarray(R, float)), start, _dp(Q), _dp(w), ctypes.byref(it))
    return Q, w, st, it.value


def implicit_residual_cell(g: Grid, a, R, Q, sigma=None):
    G = np.zeros(7)
    n = ctypes.c_int(0)
    st = lib().orc_implicit_residual_cell(ctypes.byref(g.params()), float(a),
                                          float(g.sigma if sigma is None else sigma),
                                          _dp(np.ascontiguousarray(R, float)), _dp(np.ascontiguousarray(Q, float)),
                                          _dp(G), ctypes.byref(n))
    return G[:n.value], st


def weno3_face(a, b, c):
    a, b, c = (np.ascontiguousarray(np.atleast_1d(x), dtype=float) for x in (a, b, c))
    out = np.zeros_like(a)
    lib().orc_weno3_face(_dp(a), _dp(b), _dp(c), _dp(out), int(a.size))
    return out


# ---------------------------------------------------------------------------------------------
# grid calls
# ---------------------------------------------------------------------------------------------
def bc_fill(g: Grid, arr: np.ndarray) -> np.ndarray:
    lib().orc_bc_fill(ctypes.byref(g.params()), _dp(arr), int(arr.shape[0]))
    return arr


def init_state(g: Grid, prims: np.ndarray, EB: np.ndarray) -> np.ndarray:
    cons = g.zeros(g.ncons)
    lib().orc_init_state(ctypes.byref(g.params()), _dp(np.ascontiguousarray(prims)), _dp(np.ascontiguousarray(EB)),
                         _dp(cons))
    return cons


def cons2prim(g: Grid, cons: np.ndarray, prims_guess: np.ndarray):
    prims = np.array(prims_guess, dtype=np.float64, order="C")
    status = np.zeros(g.cell_shape, dtype=np.int8)
    iters = np.zeros(g.cell_shape, dtype=np.int32)
    lib().orc_cons2prim(ctypes.byref(g.params()), _dp(np.ascontiguousarray(cons)), _dp(prims),
                        status.ctypes.data, iters.ctypes.data)
    return prims, status, iters


def rhs(g: Grid, cons: np.ndarray, prims: np.ndarray) -> np.ndarray:
    L = g.zeros(g.ncons)
    lib().orc_rhs(ctypes.byref(g.params()), _dp(np.ascontiguousarray(cons)), _dp(np.ascontiguousarray(prims)),
                  _dp(L))
    return L


def implicit(g: Grid, a: float, R: np.ndarray, prims_guess: np.ndarray):
    Q = g.zeros(g.ncons)
    prims = np.array(prims_guess, dtype=np.float64, order="C")
    status = np.zeros(g.cell_shape, dtype=np.int8)
    iters = np.zeros(g.cell_shape, dtype=np.int32)
    lib().orc_implicit(ctypes.byref(g.params()), float(a), _dp(np.ascontiguousarray(R)), _dp(Q), _dp(prims),
                       status.ctypes.data, iters.ctypes.data)
    return Q, prims, status, iters


def ssp2_step(g: Grid, dt: float, cons: np.ndarray, prims: np.ndarray):
    """Advance (cons, prims) in place by one SSP2(222) step; returns (nbad, newton_iters, max_newton)."""
    nit = ctypes.c_longlong(0)
    mx = ctypes.c_int(0)
    nf = ctypes.c_int(0)
    bad = lib().orc_ssp2_step(ctypes.byref(g.params()), float(dt), _dp(cons), _dp(prims), ctypes.byref(nit),
                              ctypes.byref(mx), ctypes.byref(nf))
    return bad, nit.value, mx.value


def ssp3_step(g: Grid, dt: float, cons: np.ndarray, prims: np.ndarray):
    """Advance (cons, prims) in place by one SSP3(332) step; returns (nbad, newton_iters, max_newton)."""
    nit = ctypes.c_longlong(0)
    mx = ctypes.c_int(0)
    nf = ctypes.c_int(0)
    bad = lib().orc_ssp3_step(ctypes.byref(g.params()), float(dt), _dp(cons), _dp(prims), ctypes.byref(nit),
                              ctypes.byref(mx), ctypes.byref(nf))
    return bad, nit.value, mx.value


def dt(g: Grid, cfl: float) -> float:
    return lib().orc_dt(ctypes.byref(g.params()), float(cfl))


def set_threads(n: int) -> int:
    """OpenMP threads of the grid loops (n <= 0: unchanged); returns the number in effect."""
    return lib().orc_set_threads(int(n))
