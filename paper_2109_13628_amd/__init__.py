"""Python binding of the MI355X IIM library (libiim.so, C ABI in include/iim.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch provides device memory (tensors on cuda:0) and the stream.
The library must have been built (paper_2109_13628_amd/build.py); importing
this module never falls back to another implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("IIM_LIBRARY") or os.path.join(HERE, "libiim.so")

IIM_OK, IIM_EINVAL, IIM_ENOMEM, IIM_EGEOM, IIM_ENOCONV, IIM_ENONFINITE, IIM_EDEVICE, IIM_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7
EXT = {"box": 0, "free": 1, "outflow": 2, "periodic": 3}
PREC_FP64, PREC_MIXED = 0, 1
GUESS_ZERO, GUESS_PREVIOUS, GUESS_EXTRAPOLATE, GUESS_NETWORK = 0, 1, 2, 3
NET_FEATURES = 10
SOLVER_KRYLOV, SOLVER_DIRECT = 0, 1
FFT_SIZES_TUNED, FFT_SIZES_COMPACT, FFT_SIZES_POW2 = 0, 1, 2

# every symbol declared in include/iim.h
EXPORTS = ["iim_abi_version", "iim_surface_loads", "iim_cv_terms", "iim_rhs_given_wb", "iim_set_body_motion", "iim_rk3_steps_moving", "iim_status_string", "iim_create", "iim_destroy", "iim_last_error", "iim_query",
           "iim_get_geometry", "iim_dt_max", "iim_lgf_table", "iim_poisson", "iim_poisson_fp32", "iim_reconstruct", "iim_rhs",
           "iim_rk3_step", "iim_rk3_steps", "iim_profile", "iim_profile_read", "iim_krylov_totals", "iim_profile_replay", "iim_solver_counters",
           "iim_net_create", "iim_net_destroy", "iim_net_num_params", "iim_net_get_params", "iim_net_set_params",
           "iim_net_forward", "iim_net_grad_mse", "iim_net_adam_step", "iim_net_save", "iim_net_load",
           "iim_set_warm_start", "iim_record_solves", "iim_warm_start_train", "iim_warm_start_stats",
           "iim_warm_start_sequences", "iim_reset_history", "iim_autotune", "iim_set_fft_shape",
           "iim_batch_create", "iim_batch_destroy", "iim_batch_last_error", "iim_batch_step", "iim_batch_info",
           "iim_dt_limit", "iim_set_speed_bound", "iim_net_train_step", "iim_net_forward_noalloc",
           "iim_warm_start_train_multi", "iim_warm_start_loss"]
KERNEL_NAMES = ["fft_rows_fwd", "fft_cols_conv", "fft_rows_inv", "transport", "arnoldi"]


class IIMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_status_name(code), code, msg))
        self.code = code


def _status_name(code):
    return {0: "IIM_OK", -1: "IIM_EINVAL", -2: "IIM_ENOMEM", -3: "IIM_EGEOM", -4: "IIM_ENOCONV",
            -5: "IIM_ENONFINITE", -6: "IIM_EDEVICE", -7: "IIM_EUNSUPPORTED"}.get(code, "?")


class GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("x0", C.c_double), ("y0", C.c_double), ("h", C.c_double),
                ("exterior", C.c_int32), ("u_inf", C.c_double * 2), ("nu", C.c_double)]


class BodyDesc(C.Structure):
    _fields_ = [("n_points", C.c_int32), ("xy_host", C.POINTER(C.c_double)), ("is_enclosure", C.c_int32),
                ("center", C.c_double * 2), ("u_rigid", C.c_double * 2), ("omega_rigid", C.c_double),
                ("rect", C.c_int32 * 4), ("bc_samples", C.POINTER(C.c_double))]


class SolverOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("krylov_tol", C.c_double), ("krylov_max_iter", C.c_int32),
                ("krylov_restart", C.c_int32), ("max_refine", C.c_int32), ("guess", C.c_int32),
                ("host_only", C.c_int32), ("solver", C.c_int32), ("fft_sizes", C.c_int32)]


class StepStats(C.Structure):
    _fields_ = [("iters", C.c_int32 * 3), ("refine_rounds", C.c_int32 * 3), ("res0", C.c_double * 3),
                ("res", C.c_double * 3), ("converged", C.c_int32)]

    def as_dict(self):
        return {"iters": list(self.iters), "refine_rounds": list(self.refine_rounds),
                "res0": list(self.res0), "res": list(self.res), "converged": bool(self.converged)}


class NetDesc(C.Structure):
    _fields_ = [("in_channels", C.c_int32), ("width", C.c_int32), ("layers", C.c_int32), ("bf16", C.c_int32),
                ("seed", C.c_uint64)]


class Counters(C.Structure):
    _fields_ = [("solves", C.c_int64), ("krylov_iterations", C.c_int64), ("fp32_products", C.c_int64),
                ("initial_residual_matvecs", C.c_int64), ("network_kept", C.c_int64),
                ("network_rejected", C.c_int64), ("recorded", C.c_int64)]


class BatchTuning(C.Structure):
    _fields_ = [("fft_mx", C.c_int32), ("fft_my", C.c_int32), ("tuned_on", C.c_int32), ("row_per", C.c_int32),
                ("col_per", C.c_int32), ("us_default", C.c_double), ("us_best", C.c_double)]


class BatchStats(C.Structure):
    _fields_ = [("steps", C.c_int32), ("cells_per_step", C.c_int64), ("ms_total", C.c_double),
                ("ms_p50", C.c_double), ("ms_p99", C.c_double), ("ms_max", C.c_double)]


class Info(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("n_control", C.c_int32), ("n_affected", C.c_int32),
                ("n_ghost", C.c_int32), ("n_circ", C.c_int32), ("n_special", C.c_int32), ("fft_mx", C.c_int32),
                ("fft_my", C.c_int32), ("win_j0", C.c_int32), ("win_j1", C.c_int32), ("device_bytes", C.c_int64)]


class GeometryView(C.Structure):
    _fields_ = [("n_control", C.c_int32), ("c_xy", C.POINTER(C.c_double)), ("c_theta", C.POINTER(C.c_double)),
                ("c_normal", C.POINTER(C.c_double)), ("c_int", C.POINTER(C.c_int32)),
                ("n_affected", C.c_int32), ("a_int", C.POINTER(C.c_int32)), ("cls", C.POINTER(C.c_int8)),
                ("n_circ", C.c_int32), ("rects", C.POINTER(C.c_int32)), ("circ_body", C.POINTER(C.c_int32)),
                ("c_ub", C.POINTER(C.c_double)), ("c_psib", C.POINTER(C.c_double))]


_lib = None


def lib():
    """Load libiim.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libiim.so is not built: run paper_2109_13628_amd/build.py (or __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.c_int
    L.iim_abi_version.restype = ip
    L.iim_status_string.restype = C.c_char_p
    L.iim_status_string.argtypes = [ip]
    L.iim_create.restype = ip
    L.iim_create.argtypes = [C.POINTER(GridDesc), C.c_int32, C.POINTER(BodyDesc), C.POINTER(SolverOpts), vp,
                             C.POINTER(vp)]
    L.iim_destroy.restype = ip
    L.iim_destroy.argtypes = [vp]
    L.iim_last_error.restype = C.c_char_p
    L.iim_last_error.argtypes = [vp]
    L.iim_query.restype = ip
    L.iim_query.argtypes = [vp, C.POINTER(Info)]
    L.iim_get_geometry.restype = ip
    L.iim_get_geometry.argtypes = [vp, C.POINTER(GeometryView)]
    L.iim_dt_max.restype = ip
    L.iim_dt_max.argtypes = [vp, C.c_double, dp]
    L.iim_dt_limit.restype = ip
    L.iim_dt_limit.argtypes = [vp, dp]
    L.iim_set_speed_bound.restype = ip
    L.iim_set_speed_bound.argtypes = [vp, C.c_double]
    L.iim_lgf_table.restype = ip
    L.iim_lgf_table.argtypes = [C.c_int32, C.c_int32, dp]
    L.iim_poisson.restype = ip
    L.iim_poisson.argtypes = [vp, vp, vp]
    L.iim_poisson_fp32.restype = ip
    L.iim_poisson_fp32.argtypes = [vp, vp, vp]
    L.iim_reconstruct.restype = ip
    L.iim_reconstruct.argtypes = [vp, vp, dp, vp, vp, vp, C.POINTER(StepStats)]
    L.iim_rhs.restype = ip
    L.iim_rhs.argtypes = [vp, vp, vp, vp, vp, dp, vp]
    L.iim_surface_loads.restype = ip
    L.iim_surface_loads.argtypes = [vp, vp, vp, vp, dp, dp]
    L.iim_cv_terms.restype = ip
    L.iim_rhs_given_wb.restype = ip
    L.iim_rhs_given_wb.argtypes = [vp, vp, vp, vp, vp, vp, dp]
    L.iim_set_body_motion.restype = ip
    L.iim_set_body_motion.argtypes = [vp, dp]
    L.iim_rk3_steps_moving.restype = ip
    L.iim_rk3_steps_moving.argtypes = [vp, vp, dp, C.c_double, C.c_int32, dp, vp]
    L.iim_cv_terms.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_int32), dp, dp]
    L.iim_rk3_step.restype = ip
    L.iim_rk3_step.argtypes = [vp, vp, dp, C.c_double, C.POINTER(StepStats)]
    L.iim_rk3_steps.restype = ip
    L.iim_rk3_steps.argtypes = [vp, vp, dp, C.c_double, C.c_int32, C.POINTER(StepStats)]
    L.iim_profile.restype = ip
    L.iim_profile.argtypes = [vp, C.c_int32]
    L.iim_profile_read.restype = ip
    L.iim_profile_read.argtypes = [vp, C.c_int32, dp, C.POINTER(C.c_int64), dp]
    L.iim_profile_replay.restype = ip
    L.iim_profile_replay.argtypes = [vp, C.c_int32, C.c_int32, dp, dp]
    L.iim_solver_counters.restype = ip
    L.iim_solver_counters.argtypes = [vp, C.POINTER(Counters)]
    L.iim_krylov_totals.restype = ip
    L.iim_krylov_totals.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    i64p = C.POINTER(C.c_int64)
    L.iim_net_create.restype = ip
    L.iim_net_create.argtypes = [C.POINTER(NetDesc), vp, C.POINTER(vp)]
    L.iim_net_destroy.restype = ip
    L.iim_net_destroy.argtypes = [vp]
    L.iim_net_num_params.restype = C.c_int64
    L.iim_net_num_params.argtypes = [vp]
    L.iim_net_get_params.restype = ip
    L.iim_net_get_params.argtypes = [vp, C.c_int32, vp, C.c_int64]
    L.iim_net_set_params.restype = ip
    L.iim_net_set_params.argtypes = [vp, vp, C.c_int64]
    L.iim_net_forward.restype = ip
    L.iim_net_forward.argtypes = [vp, vp, C.c_int32, C.c_int32, vp, vp]
    L.iim_net_forward_noalloc.restype = ip
    L.iim_net_forward_noalloc.argtypes = [vp, vp, C.c_int32, C.c_int32, vp, vp]
    L.iim_net_grad_mse.restype = ip
    L.iim_net_grad_mse.argtypes = [vp, vp, C.c_int32, C.c_int32, vp, vp, C.POINTER(C.c_float)]
    L.iim_net_adam_step.restype = ip
    L.iim_net_adam_step.argtypes = [vp, C.c_float]
    L.iim_net_train_step.restype = ip
    L.iim_net_train_step.argtypes = [vp, vp, C.c_int32, C.c_int32, vp, vp, C.c_float, C.POINTER(C.c_float)]
    L.iim_net_save.restype = ip
    L.iim_net_save.argtypes = [vp, C.c_char_p]
    L.iim_net_load.restype = ip
    L.iim_net_load.argtypes = [vp, C.c_char_p]
    L.iim_set_warm_start.restype = ip
    L.iim_set_warm_start.argtypes = [vp, C.c_int32, vp]
    L.iim_record_solves.restype = ip
    L.iim_record_solves.argtypes = [vp, C.c_int32]
    L.iim_warm_start_train.restype = ip
    L.iim_warm_start_train.argtypes = [vp, vp, C.c_int32, C.c_int32, C.c_float, C.c_uint64, vp]
    L.iim_warm_start_train_multi.restype = ip
    L.iim_warm_start_train_multi.argtypes = [C.POINTER(vp), C.c_int32, vp, C.c_int32, C.c_int32, C.c_float,
                                             C.c_uint64, vp]
    L.iim_warm_start_loss.restype = ip
    L.iim_warm_start_loss.argtypes = [vp, vp, C.c_int32, dp, i64p]
    L.iim_warm_start_stats.restype = ip
    L.iim_warm_start_stats.argtypes = [vp, i64p, i64p, i64p, i64p]
    L.iim_autotune.restype = ip
    L.iim_autotune.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), dp, dp]
    L.iim_set_fft_shape.restype = ip
    L.iim_set_fft_shape.argtypes = [vp, C.c_int32, C.c_int32]
    L.iim_batch_create.restype = ip
    L.iim_batch_create.argtypes = [C.c_int32, C.POINTER(GridDesc), C.POINTER(C.c_int32),
                                   C.POINTER(C.POINTER(BodyDesc)), C.POINTER(SolverOpts), vp, C.POINTER(vp)]
    L.iim_batch_destroy.restype = ip
    L.iim_batch_destroy.argtypes = [vp]
    L.iim_batch_last_error.restype = C.c_char_p
    L.iim_batch_last_error.argtypes = [vp]
    L.iim_batch_step.restype = ip
    L.iim_batch_step.argtypes = [vp, C.POINTER(vp), C.POINTER(C.POINTER(C.c_double)), dp, C.c_int32,
                                 C.POINTER(BatchStats)]
    L.iim_batch_info.restype = ip
    L.iim_batch_info.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(BatchTuning), dp]
    L.iim_reset_history.restype = ip
    L.iim_reset_history.argtypes = [vp]
    L.iim_warm_start_sequences.restype = ip
    L.iim_warm_start_sequences.argtypes = [vp, C.POINTER(C.c_int32), vp, vp, vp]
    _lib = L
    return L


def lgf_table(mx, my):
    out = np.zeros((my + 1, mx + 1))
    rc = lib().iim_lgf_table(mx, my, out.ctypes.data_as(C.POINTER(C.c_double)))
    if rc:
        raise IIMError(rc, "iim_lgf_table")
    return out


def _ptr(t):
    """Device pointer of a contiguous float64 CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def _sized(t, n, what):
    """_ptr of a tensor that must hold at least n values (None -> NULL)."""
    p = _ptr(t)
    if t is not None and t.numel() < n:
        raise ValueError("%s needs at least %d values, got %d" % (what, n, t.numel()))
    return p


def _gamma_array(Gamma, n_circ):
    """Host copy of the body circulations with room for the n_circ values the
    library reads and writes back (at least one element, so that the pointer
    is valid when there are none)."""
    G = np.ascontiguousarray(np.atleast_1d(np.asarray(Gamma, dtype=np.float64))).reshape(-1).copy()
    if G.size < n_circ:
        raise ValueError("expected %d body circulations, got %d" % (n_circ, G.size))
    return G if G.size else np.zeros(1)


class Context:
    """One IIM problem (grid + bodies) on the current device."""

    def __init__(self, grid, bodies, precision=PREC_FP64, tol=1e-13, max_iter=400, restart=40,
                 guess=GUESS_PREVIOUS, host_only=False, stream=None, solver=SOLVER_KRYLOV,
                 fft_sizes=FFT_SIZES_TUNED):
        L = lib()
        g = GridDesc(nx=grid.nx, ny=grid.ny, x0=grid.x0, y0=grid.y0, h=grid.h, exterior=EXT[grid.exterior],
                     nu=grid.nu)
        g.u_inf[0], g.u_inf[1] = grid.u_inf
        self.grid = grid
        self._pts = []
        arr = _body_array(bodies, self._pts)
        self.n_bodies = len(bodies)
        o = SolverOpts(precision=precision, krylov_tol=tol, krylov_max_iter=max_iter, krylov_restart=restart,
                       max_refine=8, guess=guess, host_only=int(host_only), solver=solver, fft_sizes=fft_sizes)
        if stream is None and not host_only:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        h = C.c_void_p()
        rc = L.iim_create(C.byref(g), len(bodies), arr, C.byref(o), C.c_void_p(stream or 0), C.byref(h))
        if rc:
            raise IIMError(rc, (L.iim_last_error(None) or b"").decode())
        self._h = h
        self.host_only = host_only
        info = Info()
        L.iim_query(h, C.byref(info))
        self.info = {f[0]: getattr(info, f[0]) for f in Info._fields_}
        self.n_circ = info.n_circ

    def close(self):
        if getattr(self, "_h", None):
            lib().iim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what, allow=()):
        if rc and rc not in allow:
            raise IIMError(rc, "%s: %s" % (what, (lib().iim_last_error(self._h) or b"").decode()))
        return rc

    # device arguments, checked against the sizes the kernels index
    def _grid(self, t):
        return _sized(t, self.grid.nx * self.grid.ny, "a grid field [ny][nx]")

    def _ring(self, t):
        return _sized(t, (self.grid.nx + 2) * (self.grid.ny + 2), "a ring field [ny+2][nx+2]")

    def _ctrl(self, t):
        return _sized(t, self.info["n_control"], "a control-point array")

    def geometry(self):
        v = GeometryView()
        self._check(lib().iim_get_geometry(self._h, C.byref(v)), "iim_get_geometry")
        nc, na = v.n_control, v.n_affected
        nx, ny = self.grid.nx, self.grid.ny
        a = lambda p, n: np.ctypeslib.as_array(p, shape=(n,)).copy() if n else np.zeros(0)
        out = {
            "c_xy": a(v.c_xy, 2 * nc).reshape(nc, 2), "c_theta": a(v.c_theta, nc),
            "c_normal": a(v.c_normal, 2 * nc).reshape(nc, 2), "c_int": a(v.c_int, 5 * nc).reshape(nc, 5),
            "a_int": a(v.a_int, 4 * na).reshape(na, 4), "cls": a(v.cls, nx * ny).reshape(ny, nx),
            "rects": a(v.rects, 4 * v.n_circ).reshape(v.n_circ, 4), "circ_body": a(v.circ_body, v.n_circ),
            "c_ub": a(v.c_ub, 2 * nc).reshape(nc, 2), "c_psib": a(v.c_psib, nc),
        }
        return out

    def dt_max(self, a_max):
        d = C.c_double()
        self._check(lib().iim_dt_max(self._h, a_max, C.byref(d)), "iim_dt_max")
        return d.value

    def dt_limit(self):
        """The step-size limit the RK3 steps enforce (iim_dt_limit)."""
        d = C.c_double()
        self._check(lib().iim_dt_limit(self._h, C.byref(d)), "iim_dt_limit")
        return d.value

    def set_speed_bound(self, a_max):
        self._check(lib().iim_set_speed_bound(self._h, a_max), "iim_set_speed_bound")

    def poisson(self, src, psi):
        self._check(lib().iim_poisson(self._h, self._grid(src), self._ring(psi)), "iim_poisson")

    def poisson_fp32(self, src, psi):
        self._check(lib().iim_poisson_fp32(self._h, self._grid(src), self._ring(psi)), "iim_poisson_fp32")

    def reconstruct(self, omega, Gamma, psi, u, v, allow_noconv=False):
        G = _gamma_array(Gamma, self.n_circ)
        st = StepStats()
        rc = lib().iim_reconstruct(self._h, self._grid(omega), G.ctypes.data_as(C.POINTER(C.c_double)),
                                   self._ring(psi), self._ring(u), self._ring(v), C.byref(st))
        self._check(rc, "iim_reconstruct", allow=(IIM_ENOCONV,) if allow_noconv else ())
        return st.as_dict()

    def surface_loads(self, omega, u, v):
        """Per control point (omega_b, tau, d omega/dn, relative pressure)
        and per body (F_x, F_y, torque); u, v: ring arrays from reconstruct."""
        nc = self.info["n_control"]
        pts = np.zeros((max(1, nc), 4))
        bod = np.zeros((max(1, self.n_bodies), 3))
        self._check(lib().iim_surface_loads(self._h, self._grid(omega), self._ring(u), self._ring(v),
                                            pts.ctypes.data_as(C.POINTER(C.c_double)),
                                            bod.ctypes.data_as(C.POINTER(C.c_double))), "iim_surface_loads")
        return {"omega_b": pts[:nc, 0].copy(), "tau": pts[:nc, 1].copy(), "dwdn": pts[:nc, 2].copy(),
                "p": pts[:nc, 3].copy(), "forces": bod[:self.n_bodies].copy()}

    def cv_terms(self, omega, u, v, box, origin=(0.0, 0.0)):
        """Control-volume parts on the box of nodes (i0, i1, j0, j1), x from
        origin: S_t, S_gamma (F = S_gamma - d S_t / dt) and I, S_lambda
        (M = d I / dt + S_lambda); the caller differences S_t and I in time.
        u, v: ring arrays from reconstruct."""
        b = (C.c_int32 * 4)(*[int(q) for q in box])
        o = np.ascontiguousarray(origin, dtype=np.float64)
        out = np.zeros(6)
        self._check(lib().iim_cv_terms(self._h, self._grid(omega), self._ring(u), self._ring(v), b,
                                       o.ctypes.data_as(C.POINTER(C.c_double)),
                                       out.ctypes.data_as(C.POINTER(C.c_double))), "iim_cv_terms")
        return {"S_t": out[:2].copy(), "S_gamma": out[2:4].copy(), "I": float(out[4]), "S_lambda": float(out[5])}

    def rhs(self, omega, u, v, domega, omega_b=None):
        dG = np.zeros(max(1, self.n_circ))
        self._check(lib().iim_rhs(self._h, self._grid(omega), self._ring(u), self._ring(v), self._grid(domega),
                                  dG.ctypes.data_as(C.POINTER(C.c_double)), self._ctrl(omega_b)), "iim_rhs")
        return dG[:self.n_circ]

    def rhs_given_wb(self, omega, u, v, omega_b, domega):
        """Transport right-hand side with the wall vorticity omega_b (device,
        per control point) given instead of computed from the velocity."""
        dG = np.zeros(max(1, self.n_circ))
        self._check(lib().iim_rhs_given_wb(self._h, self._grid(omega), self._ring(u), self._ring(v), self._ctrl(omega_b),
                                           self._grid(domega),
                                           dG.ctypes.data_as(C.POINTER(C.c_double))), "iim_rhs_given_wb")
        return dG[:self.n_circ]

    def profile(self, mask):
        self._check(lib().iim_profile(self._h, int(mask)), "iim_profile")

    def profile_read(self):
        out = {}
        for kid, name in enumerate(KERNEL_NAMES):
            ms, n, b = C.c_double(), C.c_int64(), C.c_double()
            self._check(lib().iim_profile_read(self._h, kid, C.byref(ms), C.byref(n), C.byref(b)),
                        "iim_profile_read")
            if n.value:
                avg = ms.value / n.value
                out[name] = {"launches": n.value, "total_ms": ms.value, "avg_us": 1e3 * avg,
                             "bytes_per_launch": b.value / n.value,
                             "GBps": (b.value / n.value) / (avg * 1e-3) / 1e9 if avg > 0 else None}
        return out

    def profile_replay(self, name, reps=200):
        ms, b = C.c_double(), C.c_double()
        self._check(lib().iim_profile_replay(self._h, KERNEL_NAMES.index(name), reps, C.byref(ms), C.byref(b)),
                    "iim_profile_replay")
        return {"avg_us": 1e3 * ms.value, "bytes_per_launch": b.value, "reps": reps,
                "GBps": b.value / (ms.value * 1e-3) / 1e9 if ms.value > 0 else None}

    def autotune(self, reps=5):
        r, c, d, b = C.c_int32(), C.c_int32(), C.c_double(), C.c_double()
        self._check(lib().iim_autotune(self._h, reps, C.byref(r), C.byref(c), C.byref(d), C.byref(b)),
                    "iim_autotune")
        return {"row_per": r.value, "col_per": c.value, "us_default": d.value, "us_best": b.value}

    def set_fft_shape(self, row_per, col_per):
        self._check(lib().iim_set_fft_shape(self._h, row_per, col_per), "iim_set_fft_shape")

    def counters(self):
        o = Counters()
        self._check(lib().iim_solver_counters(self._h, C.byref(o)), "iim_solver_counters")
        return {f[0]: getattr(o, f[0]) for f in Counters._fields_}

    def krylov_totals(self):
        s, m = C.c_int64(), C.c_int64()
        self._check(lib().iim_krylov_totals(self._h, C.byref(s), C.byref(m)), "iim_krylov_totals")
        return s.value, m.value

    def rk3_steps(self, omega, Gamma, dt, n_steps=1):
        G = _gamma_array(Gamma, self.n_circ)
        st = StepStats()
        self._check(lib().iim_rk3_steps(self._h, self._grid(omega), G.ctypes.data_as(C.POINTER(C.c_double)), dt,
                                        n_steps, C.byref(st)), "iim_rk3_steps")
        return G[:self.n_circ], st.as_dict()

    def set_body_motion(self, motion):
        """Rigid motion (u_x, u_y, omega) of every body from now on."""
        m = np.ascontiguousarray(motion, dtype=np.float64).reshape(-1)
        if m.size != 3 * self.n_bodies:
            raise ValueError("expected (u_x, u_y, omega) for each of %d bodies" % self.n_bodies)
        self._check(lib().iim_set_body_motion(self._h, m.ctypes.data_as(C.POINTER(C.c_double))),
                    "iim_set_body_motion")

    def rk3_steps_moving(self, omega, Gamma, dt, motion):
        """RK3 steps with the bodies' rigid motion at every stage's time:
        motion[n_steps][3][n_bodies][3] = (u_x, u_y, omega)."""
        m = np.ascontiguousarray(motion, dtype=np.float64)
        if m.ndim != 4 or m.shape[1:] != (3, self.n_bodies, 3):
            raise ValueError("expected motion of shape (n_steps, 3, %d, 3)" % self.n_bodies)
        G = _gamma_array(Gamma, self.n_circ)
        st = StepStats()
        self._check(lib().iim_rk3_steps_moving(self._h, self._grid(omega), G.ctypes.data_as(C.POINTER(C.c_double)), dt,
                                               m.shape[0], m.ctypes.data_as(C.POINTER(C.c_double)),
                                               C.byref(st)), "iim_rk3_steps_moving")
        return G[:self.n_circ], st.as_dict()

    # ---- learned initial guess
    def set_warm_start(self, guess, net=None):
        self._check(lib().iim_set_warm_start(self._h, int(guess), net._h if net is not None else None),
                    "iim_set_warm_start")
        self._net = net   # keep the network alive while the context uses it

    def reset_history(self):
        self._check(lib().iim_reset_history(self._h), "iim_reset_history")

    def record_solves(self, capacity):
        self._check(lib().iim_record_solves(self._h, int(capacity)), "iim_record_solves")

    def warm_start_train(self, net, iters, batch, lr, seed=0):
        losses = np.zeros(iters, dtype=np.float32)
        self._check(lib().iim_warm_start_train(self._h, net._h, iters, batch, lr, seed,
                                               losses.ctypes.data_as(C.c_void_p)), "iim_warm_start_train")
        return losses

    def warm_start_loss(self, net, batch=64):
        """Mean training loss of net over this context's qualifying records
        (forward passes only) and the number of records."""
        loss, n = C.c_double(), C.c_int64()
        self._check(lib().iim_warm_start_loss(self._h, net._h, batch, C.byref(loss), C.byref(n)),
                    "iim_warm_start_loss")
        return loss.value, n.value

    def warm_start_stats(self):
        v = [C.c_int64() for _ in range(4)]
        self._check(lib().iim_warm_start_stats(self._h, *[C.byref(x) for x in v]), "iim_warm_start_stats")
        return dict(zip(("recorded", "net_used", "net_rejected", "extra_matvecs"), (x.value for x in v)))

    def warm_start_sequences(self):
        P = C.c_int32()
        self._check(lib().iim_warm_start_sequences(self._h, C.byref(P), None, None, None), "iim_warm_start_sequences")
        n = P.value
        perm = np.zeros(n, dtype=np.int32)
        seq = np.zeros(3 * n, dtype=np.int32)
        geo = np.zeros(4 * n, dtype=np.float32)
        self._check(lib().iim_warm_start_sequences(self._h, C.byref(P), perm.ctypes.data_as(C.c_void_p),
                                                    seq.ctypes.data_as(C.c_void_p), geo.ctypes.data_as(C.c_void_p)),
                    "iim_warm_start_sequences")
        return perm, seq.reshape(3, n), geo.reshape(n, 4)


def _fptr(t, dtype_name="float32"):
    import torch
    want = {"float32": torch.float32, "int32": torch.int32}[dtype_name]
    if not (t.is_cuda and t.dtype == want and t.is_contiguous()):
        raise ValueError("expected a contiguous %s CUDA tensor" % dtype_name)
    return C.c_void_p(t.data_ptr())


def warm_start_train_multi(contexts, net, iters, batch, lr, seed=0):
    """Train net on the recorded solves of several contexts (one network for
    runs of different geometry or viscosity); the loss of every step."""
    if not contexts:
        raise ValueError("no contexts")
    arr = (C.c_void_p * len(contexts))(*[c._h for c in contexts])
    losses = np.zeros(iters, dtype=np.float32)
    contexts[0]._check(lib().iim_warm_start_train_multi(arr, len(contexts), net._h, iters, batch, lr, seed,
                                                        losses.ctypes.data_as(C.c_void_p)),
                       "iim_warm_start_train_multi")
    return losses


class Network:
    """Stack of circular 1D convolutions (kernel 5, GELU between layers, one
    output channel) run by the library's matrix-core kernels."""

    def __init__(self, in_channels=NET_FEATURES, width=128, layers=4, bf16=True, seed=0, stream=None):
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        d = NetDesc(in_channels=in_channels, width=width, layers=layers, bf16=int(bf16), seed=seed)
        h = C.c_void_p()
        rc = lib().iim_net_create(C.byref(d), C.c_void_p(stream or 0), C.byref(h))
        if rc:
            raise IIMError(rc, "iim_net_create")
        self._h = h
        self.shape = (in_channels, width, layers)
        self.nparam = lib().iim_net_num_params(h)

    def close(self):
        if getattr(self, "_h", None):
            lib().iim_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc:
            raise IIMError(rc, what)

    def get(self, which=0):
        out = np.zeros(self.nparam, dtype=np.float32)
        self._check(lib().iim_net_get_params(self._h, which, out.ctypes.data_as(C.c_void_p), self.nparam),
                    "iim_net_get_params")
        return out

    def set(self, flat):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        self._check(lib().iim_net_set_params(self._h, flat.ctypes.data_as(C.c_void_p), flat.size),
                    "iim_net_set_params")

    def _shapes(self, x, seq, out):
        """Batch and length from x [batch][P][in_channels]; seq must be
        [3][P] and the output or target [batch][P], so that no kernel reads
        or writes past a buffer."""
        if x.dim() != 3 or x.shape[2] != self.shape[0]:
            raise ValueError("x must be [batch][P][%d]" % self.shape[0])
        B, P = x.shape[0], x.shape[1]
        if tuple(seq.shape) != (3, P):
            raise ValueError("seq must be [3][%d]" % P)
        if out.numel() != B * P:
            raise ValueError("output and target must hold batch * P = %d values" % (B * P))
        return B, P

    def forward(self, x, seq, y):
        B, P = self._shapes(x, seq, y)
        self._check(lib().iim_net_forward(self._h, _fptr(x), B, P, _fptr(seq, "int32"), _fptr(y)), "iim_net_forward")

    def grad_mse(self, x, seq, target):
        B, P = self._shapes(x, seq, target)
        loss = C.c_float()
        self._check(lib().iim_net_grad_mse(self._h, _fptr(x), B, P, _fptr(seq, "int32"), _fptr(target),
                                           C.byref(loss)), "iim_net_grad_mse")
        return loss.value

    def adam_step(self, lr):
        self._check(lib().iim_net_adam_step(self._h, lr), "iim_net_adam_step")

    def train_step(self, x, seq, target, lr):
        """Gradients of the batch loss and one Adam step (iim_net_train_step);
        returns the loss before the update."""
        B, P = self._shapes(x, seq, target)
        loss = C.c_float()
        self._check(lib().iim_net_train_step(self._h, _fptr(x), B, P, _fptr(seq, "int32"), _fptr(target), lr,
                                             C.byref(loss)), "iim_net_train_step")
        return loss.value

    def save(self, path):
        self._check(lib().iim_net_save(self._h, path.encode()), "iim_net_save")

    def load(self, path):
        self._check(lib().iim_net_load(self._h, path.encode()), "iim_net_load")


def _grid_desc(grid):
    g = GridDesc(nx=grid.nx, ny=grid.ny, x0=grid.x0, y0=grid.y0, h=grid.h, exterior=EXT[grid.exterior], nu=grid.nu)
    g.u_inf[0], g.u_inf[1] = grid.u_inf
    return g


def _body_array(bodies, keep):
    arr = (BodyDesc * max(1, len(bodies)))()
    for k, b in enumerate(bodies):
        p = np.ascontiguousarray(b.points, dtype=np.float64)
        keep.append(p)
        arr[k].n_points = p.shape[0]
        arr[k].xy_host = p.ctypes.data_as(C.POINTER(C.c_double))
        arr[k].is_enclosure = int(b.is_enclosure)
        arr[k].center[0], arr[k].center[1] = b.center
        arr[k].u_rigid[0], arr[k].u_rigid[1] = b.u_rigid
        arr[k].omega_rigid = b.omega_rigid
        r = b.rect if b.rect is not None else (-1, -1, -1, -1)
        for q in range(4):
            arr[k].rect[q] = r[q]
        smp = getattr(b, "bc_samples", None)
        if smp is not None:
            smp = np.ascontiguousarray(smp, dtype=np.float64)
            if smp.shape != (p.shape[0], 3):
                raise ValueError("bc_samples must be shaped (n_points, 3)")
            keep.append(smp)
            arr[k].bc_samples = smp.ctypes.data_as(C.POINTER(C.c_double))
    return arr


class Batch:
    """Independent simulations advanced together, one HIP graph per batch
    step (dense FP64 Schur solver in every simulation)."""

    def __init__(self, workloads, stream=None, fft_sizes=FFT_SIZES_TUNED):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        n = len(workloads)
        grids = (GridDesc * n)(*[_grid_desc(w.grid) for w in workloads])
        self._keep = []
        arrs = [_body_array(w.bodies, self._keep) for w in workloads]
        self._arrs = arrs
        ptrs = (C.POINTER(BodyDesc) * n)(*[C.cast(a, C.POINTER(BodyDesc)) for a in arrs])
        nb = (C.c_int32 * n)(*[len(w.bodies) for w in workloads])
        o = SolverOpts(precision=PREC_FP64, krylov_tol=1e-13, krylov_max_iter=400, krylov_restart=40,
                       max_refine=8, guess=GUESS_PREVIOUS, host_only=0, solver=SOLVER_DIRECT, fft_sizes=fft_sizes)
        h = C.c_void_p()
        rc = lib().iim_batch_create(n, grids, nb, ptrs, C.byref(o), C.c_void_p(stream or 0), C.byref(h))
        if rc:
            raise IIMError(rc, (lib().iim_batch_last_error(None) or b"").decode())
        self._h = h
        self.n = n
        self.workloads = workloads

    def close(self):
        if getattr(self, "_h", None):
            lib().iim_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        nbr, nt = C.c_int32(), C.c_int32()
        tun = (BatchTuning * self.n)()
        bms = (C.c_double * 4)()
        rc = lib().iim_batch_info(self._h, C.byref(nbr), C.byref(nt), tun, bms)
        if rc:
            raise IIMError(rc, "iim_batch_info")
        tuning = [{f[0]: getattr(tun[i], f[0]) for f in BatchTuning._fields_} for i in range(nt.value)]
        tried = [c for c in (1, 2, 4, 8) if c <= min(8, self.n)]
        notes = (lib().iim_batch_last_error(self._h) or b"").decode()
        return {"branches": nbr.value, "tuning": tuning, "branch_ms": dict(zip(tried, list(bms)[:len(tried)])),
                "notes": notes or None}

    def step(self, omegas, gammas, dts, n_steps=1):
        """omegas: contiguous float64 CUDA tensors [ny][nx] (in place);
        gammas: list of float64 numpy arrays (in place); dts: per simulation."""
        n = self.n
        om = (C.c_void_p * n)(*[_sized(t, w.grid.nx * w.grid.ny, "a grid field [ny][nx]")
                                for t, w in zip(omegas, self.workloads)])
        if not (len(omegas) == len(gammas) == len(dts) == n):
            raise ValueError("expected %d vorticity fields, circulation arrays and time steps" % n)
        gs = [_gamma_array(g, len([b for b in w.bodies if not b.is_enclosure]))
              for g, w in zip(gammas, self.workloads)]
        gp = (C.POINTER(C.c_double) * n)(*[g.ctypes.data_as(C.POINTER(C.c_double)) for g in gs])
        dt = (C.c_double * n)(*dts)
        st = BatchStats()
        rc = lib().iim_batch_step(self._h, om, gp, dt, n_steps, C.byref(st))
        if rc:
            raise IIMError(rc, (lib().iim_batch_last_error(self._h) or b"").decode())
        for g_in, g_out in zip(gammas, gs):
            if np.size(g_in):
                g_in[...] = g_out[:np.size(g_in)]
        return {f[0]: getattr(st, f[0]) for f in BatchStats._fields_}
