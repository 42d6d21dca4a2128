"""Thin Python binding of librmhd.so (include/rmhd.h).

Argument marshalling only: every step of the method runs in the library's HIP kernels.
torch supplies device memory and the stream.  Functions keep the C names; arrays are
torch float64 CUDA tensors in the library's padded layout (``alloc`` builds them).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librmhd.so")

SINGLE_FLUID, TWO_FLUID = 0, 1
BC_OUTFLOW, BC_PERIODIC = 0, 1
CELL_STATUS = {0: "ok", 1: "c2p_noconv", 2: "c2p_unphysical", 3: "newton_noconv", 4: "linesearch"}


class RmhdError(RuntimeError):
    pass


class rmhd_params(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int32), ("ndim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("bc", ctypes.c_int32), ("max_c2p_iter", ctypes.c_int32), ("max_newton_iter", ctypes.c_int32),
        ("friction_covariant", ctypes.c_int32),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("gamma_eos", ctypes.c_double), ("sigma", ctypes.c_double), ("sigma_cell", ctypes.c_void_p),
        ("mu1", ctypes.c_double), ("mu2", ctypes.c_double), ("kappa", ctypes.c_double), ("cfl", ctypes.c_double),
        ("c2p_tol", ctypes.c_double), ("newton_tol", ctypes.c_double),
    ]


class rmhd_layout(ctypes.Structure):
    _fields_ = [("nxg", ctypes.c_int64), ("nyg", ctypes.c_int64), ("pitch", ctypes.c_int64),
                ("plane", ctypes.c_int64), ("ncons", ctypes.c_int32), ("nprim", ctypes.c_int32)]


class rmhd_stats(ctypes.Structure):
    _fields_ = [("stage_cells", ctypes.c_int64), ("newton_iters", ctypes.c_int64),
                ("residual_evals", ctypes.c_int64), ("c2p_iters", ctypes.c_int64),
                ("newton_max", ctypes.c_int32), ("failures", ctypes.c_int32)]


class rmhd_timing(ctypes.Structure):
    _fields_ = [("stage_ms", ctypes.c_double), ("flux_ms", ctypes.c_double), ("c2p_ms", ctypes.c_double),
                ("stage_launches", ctypes.c_int64), ("flux_launches", ctypes.c_int64),
                ("c2p_launches", ctypes.c_int64), ("steps", ctypes.c_int64)]


class rmhd_batch_tuning(ctypes.Structure):
    _fields_ = [("persistent", ctypes.c_int32), ("chunks_per_item", ctypes.c_int32),
                ("persistent_blocks", ctypes.c_int32), ("newton_cap", ctypes.c_int32),
                ("flux_rows", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("step_ms", ctypes.c_double)]


EXPORTS = ["rmhd_layout_of", "rmhd_create", "rmhd_destroy", "rmhd_init_state", "rmhd_cons2prim", "rmhd_F",
           "rmhd_implicit_stage", "rmhd_imex_step", "rmhd_dt", "rmhd_get_stats", "rmhd_set_timing",
           "rmhd_get_timing", "rmhd_last_error",
           "rmhd_batch_create", "rmhd_batch_destroy", "rmhd_batch_step", "rmhd_batch_autotune",
           "rmhd_batch_set_tuning", "rmhd_batch_get_tuning", "rmhd_batch_get_stats", "rmhd_batch_last_error"]

_lib = None


def lib() -> ctypes.CDLL:
    """Load librmhd.so; fails loudly when the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RmhdError(f"{LIB_PATH} is missing: build it first (python -m paper_1808_09721_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp = ctypes.c_void_p, ctypes.c_void_p
        P = ctypes.POINTER(rmhd_params)
        sig = {
            "rmhd_layout_of": (ctypes.c_int, [P, ctypes.POINTER(rmhd_layout)]),
            "rmhd_create": (ctypes.c_int, [P, vp, ctypes.POINTER(vp)]),
            "rmhd_destroy": (None, [vp]),
            "rmhd_init_state": (ctypes.c_int, [vp, dp, dp, dp]),
            "rmhd_cons2prim": (ctypes.c_int, [vp, dp, dp, vp, vp]),
            "rmhd_F": (ctypes.c_int, [vp, dp, dp, dp]),
            "rmhd_implicit_stage": (ctypes.c_int, [vp, ctypes.c_double, dp, dp, dp, dp, vp, vp]),
            "rmhd_imex_step": (ctypes.c_int, [vp, ctypes.c_double, dp, dp]),
            "rmhd_dt": (ctypes.c_double, [vp]),
            "rmhd_get_stats": (ctypes.c_int, [vp, ctypes.POINTER(rmhd_stats), ctypes.c_int]),
            "rmhd_set_timing": (ctypes.c_int, [vp, ctypes.c_int]),
            "rmhd_get_timing": (ctypes.c_int, [vp, ctypes.POINTER(rmhd_timing), ctypes.c_int]),
            "rmhd_last_error": (ctypes.c_char_p, [vp]),
            "rmhd_batch_create": (ctypes.c_int, [P, ctypes.c_int, vp, ctypes.POINTER(vp)]),
            "rmhd_batch_destroy": (None, [vp]),
            "rmhd_batch_step": (ctypes.c_int, [vp, vp, vp, vp]),
            "rmhd_batch_autotune": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(rmhd_batch_tuning)]),
            "rmhd_batch_set_tuning": (ctypes.c_int, [vp, ctypes.POINTER(rmhd_batch_tuning)]),
            "rmhd_batch_get_tuning": (ctypes.c_int, [vp, ctypes.POINTER(rmhd_batch_tuning)]),
            "rmhd_batch_get_stats": (ctypes.c_int, [vp, ctypes.POINTER(rmhd_stats), ctypes.c_int]),
            "rmhd_batch_last_error": (ctypes.c_char_p, [vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not (t.is_cuda and t.is_contiguous()):
        raise RmhdError("arrays must be contiguous CUDA tensors")
    return t.data_ptr()


def _check(rc: int, ctx=None):
    if rc != 0:
        msg = lib().rmhd_last_error(ctx)
        raise RmhdError(f"librmhd error {rc}: {msg.decode() if msg else ''}")


def params_from(wl, sigma_cell=None, c2p_tol=1e-13, newton_tol=1e-12, max_c2p_iter=100, max_newton_iter=50,
                friction_covariant=0) -> rmhd_params:
    """rmhd_params from a workload description (paper_1808_09721_amd.workloads.Workload)."""
    p = rmhd_params()
    p.model, p.ndim, p.nx, p.ny, p.bc = wl.model, wl.ndim, wl.nx, wl.ny if wl.ndim == 2 else 1, wl.bc
    p.max_c2p_iter, p.max_newton_iter, p.friction_covariant = max_c2p_iter, max_newton_iter, friction_covariant
    p.x0, p.x1, p.y0, p.y1 = wl.x0, wl.x1, wl.y0, wl.y1
    p.gamma_eos, p.sigma = wl.gamma, wl.sigma
    p.sigma_cell = _ptr(sigma_cell) if sigma_cell is not None else None
    p.mu1, p.mu2, p.kappa, p.cfl = wl.mu1, wl.mu2, wl.kappa, wl.cfl
    p.c2p_tol, p.newton_tol = c2p_tol, newton_tol
    return p


def rmhd_layout_of(params: rmhd_params) -> rmhd_layout:
    out = rmhd_layout()
    _check(lib().rmhd_layout_of(ctypes.byref(params), ctypes.byref(out)))
    return out


def rmhd_create(params: rmhd_params, stream=None):
    """Create a context on the current device, bound to ``stream`` (torch stream or None =
    torch's current stream)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    ctx = ctypes.c_void_p()
    _check(lib().rmhd_create(ctypes.byref(params), ctypes.c_void_p(s.cuda_stream), ctypes.byref(ctx)))
    return ctx


def rmhd_destroy(ctx):
    lib().rmhd_destroy(ctx)


def rmhd_init_state(ctx, prims, EB, cons):
    _check(lib().rmhd_init_state(ctx, _ptr(prims), _ptr(EB), _ptr(cons)), ctx)


def rmhd_cons2prim(ctx, cons, prims, status=None, iters=None):
    _check(lib().rmhd_cons2prim(ctx, _ptr(cons), _ptr(prims), _ptr(status), _ptr(iters)), ctx)


def rmhd_F(ctx, cons, prims, L):
    _check(lib().rmhd_F(ctx, _ptr(cons), _ptr(prims), _ptr(L)), ctx)


def rmhd_implicit_stage(ctx, a, R, guess, Q, prims, status=None, iters=None):
    _check(lib().rmhd_implicit_stage(ctx, float(a), _ptr(R), _ptr(guess), _ptr(Q), _ptr(prims), _ptr(status),
                                     _ptr(iters)), ctx)


def rmhd_imex_step(ctx, dt, cons, prims):
    _check(lib().rmhd_imex_step(ctx, float(dt), _ptr(cons), _ptr(prims)), ctx)


def rmhd_dt(ctx) -> float:
    return lib().rmhd_dt(ctx)


def rmhd_get_stats(ctx, reset: bool = False) -> dict:
    s = rmhd_stats()
    _check(lib().rmhd_get_stats(ctx, ctypes.byref(s), int(reset)), ctx)
    return {k: getattr(s, k) for k, _ in rmhd_stats._fields_}


def rmhd_set_timing(ctx, enable: bool):
    _check(lib().rmhd_set_timing(ctx, int(enable)), ctx)


def rmhd_get_timing(ctx, reset: bool = False) -> dict:
    t = rmhd_timing()
    _check(lib().rmhd_get_timing(ctx, ctypes.byref(t), int(reset)), ctx)
    return {k: getattr(t, k) for k, _ in rmhd_timing._fields_}


def rmhd_last_error(ctx=None) -> str:
    m = lib().rmhd_last_error(ctx)
    return m.decode() if m else ""


# ---------------------------------------------------------------------------------------------
# layout plumbing (host <-> device copies, no arithmetic of the method)
# ---------------------------------------------------------------------------------------------
class Grid:
    """Geometry of one parameter set plus helpers to move interior fields in and out."""

    def __init__(self, params: rmhd_params):
        self.params = params
        self.layout = rmhd_layout_of(params)
        self.ndim = params.ndim
        self.nx, self.ny = params.nx, params.ny

    def alloc(self, nvar: int, dtype=None, fill: float = 0.0):
        import torch
        dtype = dtype or torch.float64
        L = self.layout
        return torch.full((nvar, L.nyg, L.pitch), fill, dtype=dtype, device="cuda")

    def interior_view(self, t):
        if self.ndim == 2:
            return t[..., 2:self.ny + 2, 2:self.nx + 2]
        return t[..., :, 2:self.nx + 2]

    def all_view(self, t):
        """All cells, ghosts included, without the row padding."""
        return t[..., :, :self.layout.nxg]

    def upload_interior(self, arr: np.ndarray, nvar: int | None = None, fill: float = 0.0):
        import torch
        arr = np.asarray(arr, dtype=np.float64)
        t = self.alloc(nvar or arr.shape[0], fill=fill)
        self.interior_view(t)[...] = torch.from_numpy(arr.reshape(self.interior_view(t).shape)).cuda()
        return t

    def download_interior(self, t) -> np.ndarray:
        return self.interior_view(t).cpu().numpy().copy()

    def download_all(self, t) -> np.ndarray:
        return self.all_view(t).cpu().numpy().copy()


class Solver:
    """Convenience owner of one context and its geometry."""

    def __init__(self, params: rmhd_params, stream=None):
        self.grid = Grid(params)
        self.ctx = rmhd_create(params, stream)

    def close(self):
        if self.ctx is not None:
            rmhd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def initial_state(self, prims_interior: np.ndarray, EB_interior: np.ndarray):
        """cons and prims (ghosts filled) on the device from interior initial data."""
        g = self.grid
        L = g.layout
        prims = g.upload_interior(prims_interior, L.nprim)
        EB = g.upload_interior(EB_interior, 6)
        cons = g.alloc(L.ncons)
        rmhd_init_state(self.ctx, prims, EB, cons)
        prims_all = g.alloc(L.nprim, fill=-1.0)
        rmhd_cons2prim(self.ctx, cons, prims_all)
        return cons, prims_all

    def step(self, dt, cons, prims):
        rmhd_imex_step(self.ctx, dt, cons, prims)

    def dt(self) -> float:
        return rmhd_dt(self.ctx)

    def stats(self, reset: bool = False) -> dict:
        return rmhd_get_stats(self.ctx, reset)


# ---------------------------------------------------------------------------------------------
# batched form
# ---------------------------------------------------------------------------------------------
def _bcheck(rc: int, batch):
    if rc != 0:
        msg = lib().rmhd_batch_last_error(batch)
        raise RmhdError(f"librmhd batch error {rc}: {msg.decode() if msg else ''}")


def _ptr_array(tensors):
    arr = (ctypes.c_void_p * len(tensors))(*[_ptr(t) for t in tensors])
    return arr


def rmhd_batch_create(params_list, stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    arr = (rmhd_params * len(params_list))(*params_list)
    b = ctypes.c_void_p()
    rc = lib().rmhd_batch_create(arr, len(params_list), ctypes.c_void_p(s.cuda_stream), ctypes.byref(b))
    if rc != 0:
        msg = lib().rmhd_batch_last_error(b)
        lib().rmhd_batch_destroy(b)
        raise RmhdError(f"librmhd batch error {rc}: {msg.decode() if msg else ''}")
    return b


def rmhd_batch_destroy(b):
    lib().rmhd_batch_destroy(b)


def rmhd_batch_step(b, dt, cons_list, prims_list):
    dts = None if dt is None else (ctypes.c_double * len(dt))(*[float(x) for x in dt])
    c, p = _ptr_array(cons_list), _ptr_array(prims_list)
    _bcheck(lib().rmhd_batch_step(b, dts, c, p), b)


def rmhd_batch_autotune(b, cons_list, prims_list) -> dict:
    t = rmhd_batch_tuning()
    c, p = _ptr_array(cons_list), _ptr_array(prims_list)
    _bcheck(lib().rmhd_batch_autotune(b, c, p, ctypes.byref(t)), b)
    return {k: getattr(t, k) for k, _ in rmhd_batch_tuning._fields_}


def rmhd_batch_set_tuning(b, **kw):
    t = rmhd_batch_tuning()
    _bcheck(lib().rmhd_batch_get_tuning(b, ctypes.byref(t)), b)
    for k, v in kw.items():
        setattr(t, k, v)
    _bcheck(lib().rmhd_batch_set_tuning(b, ctypes.byref(t)), b)


def rmhd_batch_get_tuning(b) -> dict:
    t = rmhd_batch_tuning()
    _bcheck(lib().rmhd_batch_get_tuning(b, ctypes.byref(t)), b)
    return {k: getattr(t, k) for k, _ in rmhd_batch_tuning._fields_}


def rmhd_batch_get_stats(b, reset: bool = False) -> dict:
    s = rmhd_stats()
    _bcheck(lib().rmhd_batch_get_stats(b, ctypes.byref(s), int(reset)), b)
    return {k: getattr(s, k) for k, _ in rmhd_stats._fields_}


class Batch:
    """Owner of a batch and of its domains' device state (initialised per domain through the
    single-grid entry points)."""

    def __init__(self, workloads, stream=None, **param_kw):
        self.params = [params_from(wl, **param_kw) for wl in workloads]
        self.grids = [Grid(p) for p in self.params]
        self.cons, self.prims = [], []
        for wl, p in zip(workloads, self.params):
            s = Solver(p, stream)
            c, w = s.initial_state(wl.prims, wl.EB)
            s.close()
            self.cons.append(c)
            self.prims.append(w)
        self.b = rmhd_batch_create(self.params, stream)

    def step(self, dt=None):
        rmhd_batch_step(self.b, dt, self.cons, self.prims)

    def autotune(self) -> dict:
        return rmhd_batch_autotune(self.b, self.cons, self.prims)

    def tune(self, **kw):
        rmhd_batch_set_tuning(self.b, **kw)

    def tuning(self) -> dict:
        return rmhd_batch_get_tuning(self.b)

    def stats(self, reset: bool = False) -> dict:
        return rmhd_batch_get_stats(self.b, reset)

    def close(self):
        if self.b is not None:
            rmhd_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
