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

SINGLE_FLUID, TWO_FLUID, IDEAL = 0, 1, 2
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
        ("integrator", ctypes.c_int32), ("c2p_primary_only", ctypes.c_int32),
        ("nz", ctypes.c_int32), ("reserved_", ctypes.c_int32), ("z0", ctypes.c_double), ("z1", ctypes.c_double),
    ]


class rmhd_layout(ctypes.Structure):
    _fields_ = [("nxg", ctypes.c_int64), ("nyg", ctypes.c_int64), ("pitch", ctypes.c_int64),
                ("plane", ctypes.c_int64), ("ncons", ctypes.c_int32), ("nprim", ctypes.c_int32),
                ("nzg", ctypes.c_int64), ("slab", ctypes.c_int64)]


class rmhd_stats(ctypes.Structure):
    _fields_ = [("stage_cells", ctypes.c_int64), ("newton_iters", ctypes.c_int64),
                ("residual_evals", ctypes.c_int64), ("c2p_iters", ctypes.c_int64),
                ("newton_max", ctypes.c_int32), ("failures", ctypes.c_int32),
                ("newton_hist", ctypes.c_int64 * 16), ("residual_max", ctypes.c_double),
                ("jacobian_evals", ctypes.c_int64)]


class rmhd_timing(ctypes.Structure):
    _fields_ = [("stage_ms", ctypes.c_double), ("flux_ms", ctypes.c_double), ("c2p_ms", ctypes.c_double),
                ("stage_launches", ctypes.c_int64), ("flux_launches", ctypes.c_int64),
                ("c2p_launches", ctypes.c_int64), ("steps", ctypes.c_int64)]


class rmhd_batch_tuning(ctypes.Structure):
    _fields_ = [("persistent", ctypes.c_int32), ("chunks_per_item", ctypes.c_int32),
                ("persistent_blocks", ctypes.c_int32), ("newton_cap", ctypes.c_int32),
                ("flux_rows", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("step_ms", ctypes.c_double)]


EXPORTS = ["rmhd_layout_of", "rmhd_create", "rmhd_destroy", "rmhd_init_state", "rmhd_cons2prim", "rmhd_F",
           "rmhd_implicit_stage", "rmhd_imex_step", "rmhd_set_graph", "rmhd_dt", "rmhd_get_stats", "rmhd_set_newton_cap", "rmhd_set_jacobian_reuse", "rmhd_set_flux_rows", "rmhd_set_stats_detail",
           "rmhd_set_timing",
           "rmhd_get_timing", "rmhd_last_error",
           "rmhd_batch_create", "rmhd_batch_destroy", "rmhd_batch_step", "rmhd_batch_autotune",
           "rmhd_batch_set_tuning", "rmhd_batch_get_tuning", "rmhd_batch_get_stats", "rmhd_batch_set_stats_detail",
           "rmhd_batch_last_error",
           "rmhd_mlp_create", "rmhd_mlp_destroy", "rmhd_mlp_get_params", "rmhd_mlp_get_norm", "rmhd_mlp_set_norm",
           "rmhd_mlp_fit_norm", "rmhd_mlp_forward", "rmhd_mlp_loss_grad", "rmhd_mlp_train_step", "rmhd_mlp_train",
           "rmhd_mlp_steps", "rmhd_mlp_last_error", "rmhd_set_harvest", "rmhd_harvest_count", "rmhd_set_guess_model",
           "rmhd_learned_guess", "rmhd_noalloc_scratch_bytes", "rmhd_imex_step_noalloc"]

MLP_NIN, MLP_NHID, MLP_NOUT, MLP_NPARAMS, MLP_NNORM, MLP_MAX_BATCH = 19, 64, 7, 5895, 52, 65536

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
            "rmhd_set_graph": (ctypes.c_int, [vp, ctypes.c_int]),
            "rmhd_dt": (ctypes.c_double, [vp]),
            "rmhd_get_stats": (ctypes.c_int, [vp, ctypes.POINTER(rmhd_stats), ctypes.c_int]),
            "rmhd_set_newton_cap": (ctypes.c_int, [vp, ctypes.c_int]),
            "rmhd_set_flux_rows": (ctypes.c_int, [vp, ctypes.c_int]),
            "rmhd_set_jacobian_reuse": (ctypes.c_int, [vp, ctypes.c_double]),
            "rmhd_set_stats_detail": (ctypes.c_int, [vp, ctypes.c_int]),
            "rmhd_batch_set_stats_detail": (ctypes.c_int, [vp, ctypes.c_int]),
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
            "rmhd_mlp_create": (ctypes.c_int, [vp, vp, ctypes.POINTER(vp)]),
            "rmhd_mlp_destroy": (None, [vp]),
            "rmhd_mlp_get_params": (ctypes.c_int, [vp, vp]),
            "rmhd_mlp_get_norm": (ctypes.c_int, [vp, vp]),
            "rmhd_mlp_set_norm": (ctypes.c_int, [vp, vp]),
            "rmhd_mlp_fit_norm": (ctypes.c_int, [vp, vp, vp, ctypes.c_long]),
            "rmhd_mlp_forward": (ctypes.c_int, [vp, vp, ctypes.c_long, vp, ctypes.c_int]),
            "rmhd_mlp_loss_grad": (ctypes.c_int, [vp, vp, vp, ctypes.c_long, vp, vp]),
            "rmhd_mlp_train_step": (ctypes.c_int, [vp, vp, vp, ctypes.c_long, ctypes.c_long, ctypes.c_long,
                                                   ctypes.c_int, ctypes.c_float, vp]),
            "rmhd_mlp_train": (ctypes.c_int, [vp, vp, vp, ctypes.c_long, ctypes.c_int, ctypes.c_int, ctypes.c_float,
                                              ctypes.c_float, ctypes.c_ulonglong, vp]),
            "rmhd_mlp_steps": (ctypes.c_long, [vp]),
            "rmhd_mlp_last_error": (ctypes.c_char_p, [vp]),
            "rmhd_set_harvest": (ctypes.c_int, [vp, vp, vp, ctypes.c_long]),
            "rmhd_harvest_count": (ctypes.c_long, [vp]),
            "rmhd_set_guess_model": (ctypes.c_int, [vp, vp]),
            "rmhd_learned_guess": (ctypes.c_int, [vp, vp, ctypes.c_double, dp, dp]),
            "rmhd_noalloc_scratch_bytes": (ctypes.c_size_t, [P]),
            "rmhd_imex_step_noalloc": (ctypes.c_int, [P, vp, ctypes.c_double, dp, dp]),
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


SSP2_222, SSP3_332 = 0, 1


def params_from(wl, sigma_cell=None, c2p_tol=1e-13, newton_tol=1e-12, max_c2p_iter=100, max_newton_iter=50,
                friction_covariant=0, integrator=SSP2_222, c2p_primary_only=0) -> rmhd_params:
    """rmhd_params from a workload description (paper_1808_09721_amd.workloads.Workload)."""
    p = rmhd_params()
    p.model, p.ndim, p.nx, p.ny, p.bc = wl.model, wl.ndim, wl.nx, wl.ny if wl.ndim >= 2 else 1, wl.bc
    if wl.ndim == 3:
        p.nz, p.z0, p.z1 = wl.nz, wl.z0, wl.z1
    p.max_c2p_iter, p.max_newton_iter, p.friction_covariant = max_c2p_iter, max_newton_iter, friction_covariant
    p.x0, p.x1, p.y0, p.y1 = wl.x0, wl.x1, wl.y0, wl.y1
    p.gamma_eos, p.sigma = wl.gamma, wl.sigma
    p.sigma_cell = _ptr(sigma_cell) if sigma_cell is not None else None
    p.mu1, p.mu2, p.kappa, p.cfl = wl.mu1, wl.mu2, wl.kappa, wl.cfl
    p.c2p_tol, p.newton_tol = c2p_tol, newton_tol
    p.integrator = integrator
    p.c2p_primary_only = c2p_primary_only
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
    if s != torch.cuda.current_stream():
        s.wait_stream(torch.cuda.current_stream())   # sigma_cell may have been written there
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


def rmhd_noalloc_scratch_bytes(params: rmhd_params) -> int:
    return lib().rmhd_noalloc_scratch_bytes(ctypes.byref(params))


def rmhd_imex_step_noalloc(params: rmhd_params, dt, cons, prims, stream=None):
    """One step with no context and no allocation (stream: torch stream, None = current)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().rmhd_imex_step_noalloc(ctypes.byref(params), ctypes.c_void_p(s.cuda_stream), float(dt),
                                        _ptr(cons), _ptr(prims)))


def rmhd_set_graph(ctx, enable: bool):
    _check(lib().rmhd_set_graph(ctx, int(enable)), ctx)


def rmhd_dt(ctx) -> float:
    return lib().rmhd_dt(ctx)


def _stats_dict(s) -> dict:
    d = {k: getattr(s, k) for k, _ in rmhd_stats._fields_}
    d["newton_hist"] = list(s.newton_hist)
    return d


def newton_percentile(stats: dict, q: float) -> int:
    """Smallest Newton iteration count covering fraction q of the counted cell solves."""
    h = stats["newton_hist"]
    tot = sum(h)
    acc = 0
    for k, n in enumerate(h):
        acc += n
        if tot and acc >= q * tot:
            return k
    return len(h) - 1


def rmhd_get_stats(ctx, reset: bool = False) -> dict:
    s = rmhd_stats()
    _check(lib().rmhd_get_stats(ctx, ctypes.byref(s), int(reset)), ctx)
    return _stats_dict(s)


def rmhd_set_newton_cap(ctx, cap: int):
    _check(lib().rmhd_set_newton_cap(ctx, int(cap)), ctx)


def rmhd_set_jacobian_reuse(ctx, keep: float):
    _check(lib().rmhd_set_jacobian_reuse(ctx, float(keep)), ctx)


def rmhd_set_flux_rows(ctx, rows: int):
    _check(lib().rmhd_set_flux_rows(ctx, int(rows)), ctx)


def rmhd_set_stats_detail(ctx, detail: bool):
    _check(lib().rmhd_set_stats_detail(ctx, int(detail)), ctx)


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
        self.nz = params.nz if params.ndim == 3 else 1

    @property
    def cell_shape(self) -> tuple:
        """Shape of one variable's padded array: (nyg, pitch), or (nzg, nyg, pitch) in 3-D."""
        L = self.layout
        return (L.nzg, L.nyg, L.pitch) if self.ndim == 3 else (L.nyg, L.pitch)

    def alloc(self, nvar: int, dtype=None, fill: float = 0.0):
        import torch
        dtype = dtype or torch.float64
        return torch.full((nvar,) + self.cell_shape, fill, dtype=dtype, device="cuda")

    def interior_view(self, t):
        if self.ndim == 3:
            return t[..., 2:self.nz + 2, 2:self.ny + 2, 2:self.nx + 2]
        if self.ndim == 2:
            return t[..., 2:self.ny + 2, 2:self.nx + 2]
        return t[..., :, 2:self.nx + 2]

    def all_view(self, t):
        """All cells, ghosts included, without the row padding."""
        return t[..., :self.layout.nxg]

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

    def sigma_plane(self, sigma_interior: np.ndarray):
        """Per-cell conductivity as one padded device plane with its interior filled (the
        ghost cells are left NaN: rmhd_create fills its own copy's ghosts)."""
        return self.upload_interior(np.asarray(sigma_interior, dtype=np.float64)[None], nvar=1,
                                    fill=float("nan"))


class Solver:
    """Convenience owner of one context and its geometry."""

    def __init__(self, params: rmhd_params, stream=None):
        self.grid = Grid(params)
        self.ctx = rmhd_create(params, stream)

    @classmethod
    def for_workload(cls, wl, stream=None, **param_kw):
        """A solver for a workload, with its per-cell conductivity plane (if any) on the device."""
        sigma = None
        if wl.sigma_cell is not None:
            sigma = Grid(params_from(wl, **param_kw)).sigma_plane(wl.sigma_cell)
        s = cls(params_from(wl, sigma_cell=sigma, **param_kw), stream)
        del sigma                 # read by rmhd_create; the context holds its own copy
        return s

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

    def set_graph(self, enable: bool = True):
        """Replay the step from a captured HIP graph while its arguments stay the same."""
        rmhd_set_graph(self.ctx, enable)

    def set_stats_detail(self, detail: bool = True):
        """Also collect the Newton-step histogram and the largest final residual."""
        rmhd_set_stats_detail(self.ctx, detail)

    def set_newton_cap(self, cap: int):
        """Newton steps from unconverged iterates before a cell is queued (>= max: no queue)."""
        rmhd_set_newton_cap(self.ctx, cap)

    def set_flux_rows(self, rows: int):
        """Shape of the 2-D flux tile block (0: the library's choice; 8, 12 or 16 rows of 64
        threads; 24: 32 x 24 threads, two-fluid model only; 32: 32 x 32 threads, single-fluid
        and ideal models only)."""
        rmhd_set_flux_rows(self.ctx, rows)

    def set_jacobian_reuse(self, keep: float):
        """Reuse the factorised Jacobian after a step that cut the residual by at least keep."""
        rmhd_set_jacobian_reuse(self.ctx, keep)

    def set_harvest(self, X, T):
        """Harvest (features, target) rows of every following implicit stage into the float32
        CUDA tensors X[cap, 19] and T[cap, 7] (None stops)."""
        rmhd_set_harvest(self.ctx, X, T)

    def harvest_count(self) -> int:
        return rmhd_harvest_count(self.ctx)

    def set_guess_model(self, mlp):
        """Start every following implicit stage from the learned guess of ``mlp`` (None: plain)."""
        rmhd_set_guess_model(self.ctx, mlp)


# ---------------------------------------------------------------------------------------------
# learned starting guess (include/rmhd_mlp.h)
# ---------------------------------------------------------------------------------------------
def _mcheck(rc: int, m):
    if rc != 0:
        msg = lib().rmhd_mlp_last_error(m)
        raise RmhdError(f"librmhd mlp error {rc}: {msg.decode() if msg else ''}")


def _hostf(arr, n):
    a = np.ascontiguousarray(arr, dtype=np.float32)
    if a.size != n:
        raise RmhdError(f"expected {n} floats, got {a.size}")
    return a


def _f32(t, cols=None):
    if t is None:
        return None
    import torch
    if t.dtype != torch.float32:
        raise RmhdError("sample arrays must be float32")
    if cols is not None and (t.dim() != 2 or t.shape[1] != cols):
        raise RmhdError(f"sample arrays must have shape [n, {cols}]")
    return _ptr(t)


def rmhd_mlp_create(params, stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    a = _hostf(params, MLP_NPARAMS)
    m = ctypes.c_void_p()
    rc = lib().rmhd_mlp_create(a.ctypes.data, ctypes.c_void_p(s.cuda_stream), ctypes.byref(m))
    _mcheck(rc, None)
    return m


def rmhd_mlp_destroy(m):
    lib().rmhd_mlp_destroy(m)


def rmhd_mlp_get_params(m) -> np.ndarray:
    out = np.zeros(MLP_NPARAMS, dtype=np.float32)
    _mcheck(lib().rmhd_mlp_get_params(m, out.ctypes.data), m)
    return out


def rmhd_mlp_get_norm(m) -> np.ndarray:
    out = np.zeros(MLP_NNORM, dtype=np.float32)
    _mcheck(lib().rmhd_mlp_get_norm(m, out.ctypes.data), m)
    return out


def rmhd_mlp_set_norm(m, norm):
    a = _hostf(norm, MLP_NNORM)
    _mcheck(lib().rmhd_mlp_set_norm(m, a.ctypes.data), m)


def rmhd_mlp_fit_norm(m, X, T):
    _mcheck(lib().rmhd_mlp_fit_norm(m, _f32(X, MLP_NIN), _f32(T, MLP_NOUT), X.shape[0]), m)


def rmhd_mlp_forward(m, X, Y, precision: int):
    _mcheck(lib().rmhd_mlp_forward(m, _f32(X, MLP_NIN), X.shape[0], _f32(Y, MLP_NOUT), int(precision)), m)


def rmhd_mlp_loss_grad(m, X, T, grad=None, loss=None):
    _mcheck(lib().rmhd_mlp_loss_grad(m, _f32(X, MLP_NIN), _f32(T, MLP_NOUT), X.shape[0], _f32(grad), _f32(loss)), m)


def rmhd_mlp_train_step(m, X, T, first: int, stride: int, batch: int, lr: float, loss=None):
    _mcheck(lib().rmhd_mlp_train_step(m, _f32(X, MLP_NIN), _f32(T, MLP_NOUT), X.shape[0], int(first), int(stride),
                                      int(batch), float(lr), _f32(loss)), m)


def rmhd_mlp_train(m, X, T, batch: int, epochs: int, lr0: float, lr1: float, seed: int) -> np.ndarray:
    hist = np.zeros(epochs, dtype=np.float32)
    _mcheck(lib().rmhd_mlp_train(m, _f32(X, MLP_NIN), _f32(T, MLP_NOUT), X.shape[0], int(batch), int(epochs),
                                 float(lr0), float(lr1), int(seed), hist.ctypes.data), m)
    return hist


def rmhd_mlp_steps(m) -> int:
    return lib().rmhd_mlp_steps(m)


def rmhd_set_harvest(ctx, X, T):
    cap = 0 if X is None else X.shape[0]
    if X is not None and (T is None or T.shape[0] != cap):
        raise RmhdError("harvest arrays must have the same number of rows")
    _check(lib().rmhd_set_harvest(ctx, _f32(X, MLP_NIN), _f32(T, MLP_NOUT), cap), ctx)


def rmhd_harvest_count(ctx) -> int:
    return lib().rmhd_harvest_count(ctx)


def rmhd_set_guess_model(ctx, mlp):
    _check(lib().rmhd_set_guess_model(ctx, None if mlp is None else mlp.m), ctx)


def rmhd_learned_guess(ctx, mlp, a, R, guess):
    _check(lib().rmhd_learned_guess(ctx, mlp.m, float(a), _ptr(R), _ptr(guess)), ctx)


def harvest_stages(workloads, steps: int, dt_factors=(1.0,), sample_steps=None):
    """Training rows of the learned guess: every workload is run from its initial state, step
    k with dt = dt_CFL * dt_factors[k mod len] (so the stage coefficient a varies), harvesting
    both implicit stages of steps 0 .. steps-1, or of the steps listed in sample_steps (the
    run then lasts until the last of them).  Returns float32 CUDA tensors X[rows, 19],
    T[rows, 7]."""
    import torch
    picked = sorted(set(sample_steps)) if sample_steps is not None else list(range(steps))
    rows = sum(2 * len(picked) * wl.cells for wl in workloads)
    X = torch.empty((rows, MLP_NIN), dtype=torch.float32, device="cuda")
    T = torch.empty((rows, MLP_NOUT), dtype=torch.float32, device="cuda")
    off = 0
    for wl in workloads:
        s = Solver.for_workload(wl)
        c, w = s.initial_state(wl.prims, wl.EB)
        dt = s.dt()
        for k in range(picked[-1] + 1):
            take = k in picked
            if take:
                s.set_harvest(X[off:], T[off:])
            s.step(dt * dt_factors[k % len(dt_factors)], c, w)
            if take:
                off += s.harvest_count()
                s.set_harvest(None, None)
        s.close()
    if off != rows:
        raise RmhdError(f"harvested {off} rows, expected {rows}")
    return X, T


def train_guess_network(train_n: int = 512, seeds=(1, 2, 3, 4), harvest_steps: int = 6,
                        dt_factors=(1.0, 0.5, 0.25), epochs: int = 8, batch: int = 16384, init_seed: int = 7,
                        shuffle_seed: int = 11, lr0: float = 3e-3, lr1: float = 1e-4,
                        sample_steps=(0, 1, 2, 10, 20, 40, 60, 90, 120, 150)):
    """The learned guess's network trained on the device: rows harvested from train_n^2
    two-fluid current sheets with per-cell conductivity 10^U[2, 6] at the given seeds (steps
    cycling through dt_factors of the CFL step; both stages of the steps in sample_steps, or
    of the first harvest_steps steps if it is None), normalisation fitted on them, then Adam.
    Rows from the whole run, not only its first steps: a network trained on steps 0-5 alone
    saved little at later times (2.27 against 2.39 Newton steps per cell after 20 steps of
    the 1024^2 sheet, against 2.07 for rows spread over steps 0-150).  Returns (network,
    info dict)."""
    import time

    import torch

    from . import workloads as WL
    t0 = time.perf_counter()
    X, T = harvest_stages([WL.learned_guess_sheet(train_n, seed=sd, steps=harvest_steps) for sd in seeds],
                          harvest_steps, dt_factors, sample_steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    net = Mlp(WL.mlp_initial_params(init_seed))
    net.fit_norm(X, T)
    hist = net.train(X, T, batch=batch, epochs=epochs, lr0=lr0, lr1=lr1, seed=shuffle_seed)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    picked = list(range(harvest_steps)) if sample_steps is None else sorted(set(sample_steps))
    info = {"rows": int(X.shape[0]),
            "harvest": f"{len(seeds)} seeds x steps {picked} x 2 stages of {train_n}x{train_n}, "
                       f"dt factors {list(dt_factors)}",
            "epochs": epochs, "batch": batch, "loss_first_epoch": float(hist[0]),
            "loss_last_epoch": float(hist[-1]), "harvest_s": t1 - t0, "train_s": t2 - t1}
    del X, T
    return net, info


class Mlp:
    """Owner of one guess network on the device."""

    def __init__(self, params, stream=None):
        self.m = rmhd_mlp_create(params, stream)

    def params(self) -> np.ndarray:
        return rmhd_mlp_get_params(self.m)

    def norm(self) -> np.ndarray:
        return rmhd_mlp_get_norm(self.m)

    def set_norm(self, norm):
        rmhd_mlp_set_norm(self.m, norm)

    def fit_norm(self, X, T):
        rmhd_mlp_fit_norm(self.m, X, T)

    def forward(self, X, precision: int = 1):
        import torch
        Y = torch.empty((X.shape[0], MLP_NOUT), dtype=torch.float32, device=X.device)
        rmhd_mlp_forward(self.m, X, Y, precision)
        return Y

    def loss_grad(self, X, T):
        import torch
        g = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=X.device)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        rmhd_mlp_loss_grad(self.m, X, T, g, loss)
        return float(loss.item()), g

    def train_step(self, X, T, first=0, stride=1, batch=None, lr=1e-3):
        import torch
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        rmhd_mlp_train_step(self.m, X, T, first, stride, batch or X.shape[0], lr, loss)
        return loss

    def train(self, X, T, batch=4096, epochs=10, lr0=3e-3, lr1=3e-4, seed=0) -> np.ndarray:
        return rmhd_mlp_train(self.m, X, T, batch, epochs, lr0, lr1, seed)

    def steps(self) -> int:
        return rmhd_mlp_steps(self.m)

    def close(self):
        if self.m is not None:
            rmhd_mlp_destroy(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


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
    return _stats_dict(s)


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

    def set_stats_detail(self, detail: bool = True):
        _bcheck(lib().rmhd_batch_set_stats_detail(self.b, int(detail)), self.b)

    def close(self):
        if self.b is not None:
            rmhd_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
