"""Thin Python binding of libtrajam.so (the gfx950 AM projection).

Argument marshalling only: every step of the projection runs in the HIP kernels of
the library.  The functions keep the C names; `Solver` adds shape / dtype / device
checks around them for PyTorch tensors.  If the library is not built, or no GPU is
present, calls fail with an exception -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtrajam.so")

TRAJAM_OK = 0
TRAJAM_ERR_INVALID = -1
TRAJAM_ERR_UNSUPPORTED = -2
TRAJAM_ERR_NUMERIC = -3
TRAJAM_ERR_DEVICE = -4
TRAJAM_ERR_CAPACITY = -5

TRAJAM_FP64 = 0
TRAJAM_FP32 = 1
TRAJAM_BF16_REFINE = 2
PRECISIONS = {"fp64": TRAJAM_FP64, "fp32": TRAJAM_FP32, "bf16": TRAJAM_BF16_REFINE}

TRAJAM_ELLIPSOID = 0
TRAJAM_SPHERE = 1

TRAJAM_KERNEL_MULTIWAVE = 0
TRAJAM_KERNEL_WAVE = 1

FLAG_NONFINITE = 1
FLAG_GREW = 2
FLAG_COLD_FALLBACK = 4
MLP_MAX_LAYERS = 8
MLP_NOALLOC_SCRATCH_FLOATS = 2097152
MLP_MSE_LOSS_FLOATS = 513        # loss[0] and the partial sums of trajam_mlp_mse

# every symbol include/trajam.h declares
EXPORTS = [
    "trajam_init", "trajam_destroy", "trajam_project", "trajam_residuals",
    "trajam_fixed_matrices", "trajam_set_launch", "trajam_get_launch",
    "trajam_boundary_coefficients", "trajam_cem_sample", "trajam_cem_cost",
    "trajam_cem_select", "trajam_cem_update", "trajam_mlp_param_count", "trajam_mlp_forward",
    "trajam_mpc_shift", "trajam_normals", "trajam_mlp_backward", "trajam_mlp_backward_noalloc", "trajam_mlp_infer", "trajam_mlp_pack_infer", "trajam_mlp_mse", "trajam_mlp_adam", "trajam_warm_features",
    "trajam_warm_apply", "trajam_warm_fallback", "trajam_warm_pack_mfma", "trajam_warm_jump", "trajam_set_obstacles", "trajam_autotune",
    "trajam_ragged_plan_create", "trajam_ragged_launch", "trajam_ragged_plan_destroy", "trajam_polar",
    "trajam_qp_contraction", "trajam_set_continuation", "trajam_project_continuation",
    "trajam_heading_create", "trajam_heading_destroy", "trajam_heading_set_scene", "trajam_heading_project",
    "trajam_heading_last_error", "trajam_heading_shift",
    "trajam_status_string", "trajam_last_error",
]


class TrajamError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"trajam status {status}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int32),
        ("degree", ctypes.c_int32),
        ("n_steps", ctypes.c_int32),
        ("horizon", ctypes.c_double),
        ("v_max", ctypes.c_double),
        ("a_max", ctypes.c_double),
        ("rho", ctypes.c_double),
        ("n_obstacles", ctypes.c_int32),
        ("n_agents", ctypes.c_int32),
        ("agent_radius", ctypes.c_double),
        ("max_batch", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("obstacle_model", ctypes.c_int32),
        ("workspace", ctypes.c_int32),
        ("ws_lo", ctypes.c_double * 3),
        ("ws_hi", ctypes.c_double * 3),
    ]


class Continuation(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32),
        ("growth", ctypes.c_double),
        ("window", ctypes.c_int32),
        ("stall_ratio", ctypes.c_double),
        ("tol", ctypes.c_double),
    ]


CONT_MAX_LEVELS = 16


class MlpShape(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("width", ctypes.c_int32 * (8 + 1))]


HEADING_MAX_CIRCLES = 8


class HeadingProblem(ctypes.Structure):
    _fields_ = [
        ("degree", ctypes.c_int32),
        ("n_steps", ctypes.c_int32),
        ("horizon", ctypes.c_double),
        ("v_max", ctypes.c_double),
        ("a_max", ctypes.c_double),
        ("rho", ctypes.c_double),
        ("n_circles", ctypes.c_int32),
        ("radii", ctypes.c_double * HEADING_MAX_CIRCLES),
        ("n_obstacles", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
    ]


class RaggedItem(ctypes.Structure):
    _fields_ = [
        ("solver", ctypes.c_void_p),
        ("batch", ctypes.c_int32),
        ("xi", ctypes.c_void_p),
        ("boundary_host", ctypes.POINTER(ctypes.c_double)),
        ("xi_bar", ctypes.c_void_p),
        ("lam", ctypes.c_void_p),
        ("res_trace", ctypes.c_void_p),
        ("flags", ctypes.c_void_p),
    ]


def mlp_shape(widths) -> MlpShape:
    s = MlpShape()
    s.n_layers = len(widths) - 1
    for i, w in enumerate(widths):
        s.width[i] = int(w)
    return s


_lib = None


def load():
    """Load libtrajam.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        import torch  # noqa: F401  -- HIP runtime of the process comes from torch
    except ImportError:
        pass
    # TRAJAM_LIBRARY: another build of this library (the sanitizer test's instrumented
    # host code); the in-tree build otherwise
    path = os.environ.get("TRAJAM_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() first")
    L = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    L.trajam_init.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(vp)]
    L.trajam_init.restype = ctypes.c_int
    L.trajam_destroy.argtypes = [vp]
    L.trajam_destroy.restype = None
    L.trajam_project.argtypes = [vp, ctypes.c_int32, vp, dp, vp, vp, vp, vp, vp,
                                 ctypes.c_int32, vp, vp, vp]
    L.trajam_project.restype = ctypes.c_int
    L.trajam_residuals.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp]
    L.trajam_residuals.restype = ctypes.c_int
    L.trajam_polar.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.trajam_polar.restype = ctypes.c_int
    L.trajam_qp_contraction.argtypes = [ctypes.POINTER(Problem), dp]
    L.trajam_qp_contraction.restype = ctypes.c_int
    L.trajam_fixed_matrices.argtypes = [ctypes.POINTER(Problem), dp, dp, dp, dp, dp]
    L.trajam_fixed_matrices.restype = ctypes.c_int
    L.trajam_set_launch.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    L.trajam_set_launch.restype = ctypes.c_int
    L.trajam_get_launch.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    L.trajam_get_launch.restype = ctypes.c_int
    L.trajam_boundary_coefficients.argtypes = [ctypes.POINTER(Problem), dp, dp]
    L.trajam_boundary_coefficients.restype = ctypes.c_int
    L.trajam_cem_sample.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp]
    L.trajam_cem_sample.restype = ctypes.c_int
    L.trajam_mpc_shift.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, vp, vp, vp, vp, vp, vp]
    L.trajam_mpc_shift.restype = ctypes.c_int
    L.trajam_normals.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32, vp, vp]
    L.trajam_normals.restype = ctypes.c_int
    L.trajam_cem_cost.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_double, vp, vp, vp]
    L.trajam_cem_cost.restype = ctypes.c_int
    L.trajam_cem_select.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_int32, ctypes.c_int32,
                                    vp, vp, vp]
    L.trajam_cem_select.restype = ctypes.c_int
    L.trajam_cem_update.argtypes = [vp, ctypes.c_int32, vp, vp, vp, ctypes.c_double,
                                    ctypes.c_double, vp, vp, vp, vp]
    L.trajam_cem_update.restype = ctypes.c_int
    sp = ctypes.POINTER(MlpShape)
    i64 = ctypes.c_int64
    L.trajam_mlp_param_count.argtypes = [sp, ctypes.POINTER(i64)]
    L.trajam_mlp_forward.argtypes = [sp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp]
    L.trajam_mlp_backward.argtypes = [sp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp, vp,
                                      vp]
    L.trajam_mlp_backward_noalloc.argtypes = [sp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp,
                                              vp, vp]
    L.trajam_mlp_mse.argtypes = [i64, vp, vp, vp, vp, vp]
    L.trajam_mlp_adam.argtypes = [i64, vp, vp, vp, vp, ctypes.c_int32, ctypes.c_float,
                                  ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]
    L.trajam_warm_features.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp,
                                       vp, ctypes.c_float, vp, vp]
    L.trajam_warm_apply.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp,
                                    ctypes.c_float, vp, vp, vp, vp, vp, vp]
    L.trajam_mlp_infer.argtypes = [sp, ctypes.c_int32, vp, vp, vp, vp]
    L.trajam_mlp_infer.restype = ctypes.c_int
    L.trajam_mlp_pack_infer.argtypes = [sp, vp, vp, vp]
    L.trajam_mlp_pack_infer.restype = ctypes.c_int
    L.trajam_warm_fallback.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, vp,
                                       vp, vp, vp, vp, vp]
    L.trajam_set_obstacles.argtypes = [vp, vp, vp, vp, vp]
    i32p = ctypes.POINTER(ctypes.c_int32)
    L.trajam_autotune.argtypes = [vp, ctypes.c_int32, vp, dp, vp, vp, vp, vp, vp, ctypes.c_int32,
                                  i32p, i32p, vp]
    L.trajam_ragged_plan_create.argtypes = [ctypes.POINTER(RaggedItem), ctypes.c_int32,
                                            ctypes.c_int32, ctypes.POINTER(vp)]
    L.trajam_ragged_launch.argtypes = [vp, vp]
    L.trajam_warm_pack_mfma.argtypes = [sp, vp, vp, ctypes.POINTER(i64), vp]
    L.trajam_warm_pack_mfma.restype = ctypes.c_int
    L.trajam_warm_jump.argtypes = [sp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_float,
                                   ctypes.c_float, vp, vp, vp, vp, vp, vp]
    L.trajam_warm_jump.restype = ctypes.c_int
    L.trajam_set_continuation.argtypes = [vp, ctypes.POINTER(Continuation)]
    L.trajam_set_continuation.restype = ctypes.c_int
    L.trajam_project_continuation.argtypes = [vp, ctypes.c_int32, vp, dp, vp, vp, vp, vp, vp, vp,
                                              ctypes.c_int32, vp, vp, vp]
    L.trajam_project_continuation.restype = ctypes.c_int
    L.trajam_ragged_plan_destroy.argtypes = [vp]
    L.trajam_ragged_plan_destroy.restype = None
    for f in ("trajam_set_obstacles", "trajam_autotune", "trajam_ragged_plan_create",
              "trajam_ragged_launch"):
        getattr(L, f).restype = ctypes.c_int
    for f in ("trajam_mlp_param_count", "trajam_mlp_forward", "trajam_mlp_backward",
              "trajam_mlp_backward_noalloc",
              "trajam_mlp_mse", "trajam_mlp_adam", "trajam_warm_features", "trajam_warm_apply",
              "trajam_warm_fallback"):
        getattr(L, f).restype = ctypes.c_int
    L.trajam_heading_create.argtypes = [ctypes.POINTER(HeadingProblem), ctypes.POINTER(vp)]
    L.trajam_heading_create.restype = ctypes.c_int
    L.trajam_heading_destroy.argtypes = [vp]
    L.trajam_heading_destroy.restype = None
    L.trajam_heading_set_scene.argtypes = [vp, dp, dp, dp]
    L.trajam_heading_set_scene.restype = ctypes.c_int
    L.trajam_heading_project.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_int32, vp, vp]
    L.trajam_heading_project.restype = ctypes.c_int
    L.trajam_heading_shift.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, vp, vp, vp]
    L.trajam_heading_shift.restype = ctypes.c_int
    L.trajam_heading_last_error.argtypes = [vp]
    L.trajam_heading_last_error.restype = ctypes.c_char_p
    L.trajam_status_string.argtypes = [ctypes.c_int]
    L.trajam_status_string.restype = ctypes.c_char_p
    L.trajam_last_error.argtypes = [vp]
    L.trajam_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(st: int, handle=None):
    if st != TRAJAM_OK:
        L = load()
        msg = L.trajam_last_error(handle).decode()
        raise TrajamError(st, f"{L.trajam_status_string(st).decode()}: {msg}")


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ------------------------------------------------------------------ C names --


def trajam_init(problem: Problem) -> int:
    h = ctypes.c_void_p()
    _check(load().trajam_init(ctypes.byref(problem), ctypes.byref(h)))
    return h.value


def trajam_destroy(handle: int) -> None:
    load().trajam_destroy(handle)


def trajam_project(handle, batch, xi, boundary_host, obs_centre, obs_vel, obs_axes,
                   xi_bar, lam, iters, res_trace, flags, stream) -> None:
    """All array arguments are raw device pointers (ints) except boundary_host,
    a float64 numpy array [dims, 4]."""
    b = np.ascontiguousarray(boundary_host, dtype=np.float64)
    _check(load().trajam_project(handle, int(batch), xi, _dp(b), obs_centre, obs_vel,
                                 obs_axes, xi_bar, lam, int(iters), res_trace, flags, stream),
           handle)


def trajam_set_continuation(handle, cont) -> None:
    """cont: a Continuation, or None to switch the continuation off."""
    _check(load().trajam_set_continuation(handle, None if cont is None else ctypes.byref(cont)), handle)


def trajam_project_continuation(handle, batch, xi, boundary_host, obs_centre, obs_vel, obs_axes,
                                xi_bar, lam, state, iters, res_trace, flags, stream) -> None:
    b = np.ascontiguousarray(boundary_host, dtype=np.float64)
    _check(load().trajam_project_continuation(handle, int(batch), xi, _dp(b), obs_centre, obs_vel,
                                              obs_axes, xi_bar, lam, state, int(iters), res_trace,
                                              flags, stream), handle)


def trajam_residuals(handle, batch, xi_bar, obs_centre, obs_vel, obs_axes, res_l2, res_max,
                     stream) -> None:
    _check(load().trajam_residuals(handle, int(batch), xi_bar, obs_centre, obs_vel, obs_axes,
                                   res_l2, res_max, stream), handle)


def trajam_polar(handle, batch, xi_bar, obs_centre, obs_vel, obs_axes, obs_alpha, obs_beta, obs_d, kin,
                 stream) -> None:
    _check(load().trajam_polar(handle, int(batch), xi_bar, obs_centre, obs_vel, obs_axes, obs_alpha,
                               obs_beta, obs_d, kin, stream), handle)


def trajam_qp_contraction(problem: Problem) -> float:
    """Spectral radius of I - W~ H_ff for the problem's precision (host only)."""
    out = ctypes.c_double(0.0)
    _check(load().trajam_qp_contraction(ctypes.byref(problem), ctypes.byref(out)), None)
    return float(out.value)


def trajam_fixed_matrices(problem: Problem):
    """(P, Pd, Pdd, H, W) in float64, computed on the host (no GPU needed)."""
    nv = problem.degree + 1
    P = np.zeros((problem.n_steps, nv)); Pd = np.zeros_like(P); Pdd = np.zeros_like(P)
    H = np.zeros((nv, nv)); W = np.zeros((max(nv - 4, 0), nv))
    _check(load().trajam_fixed_matrices(ctypes.byref(problem), _dp(P), _dp(Pd), _dp(Pdd),
                                        _dp(H), _dp(W) if W.size else None))
    return P, Pd, Pdd, H, W


def trajam_set_launch(handle, kernel: int, samples_per_workgroup: int) -> None:
    _check(load().trajam_set_launch(handle, int(kernel), int(samples_per_workgroup)), handle)


def trajam_get_launch(handle):
    k = ctypes.c_int32(); t = ctypes.c_int32()
    _check(load().trajam_get_launch(handle, ctypes.byref(k), ctypes.byref(t)), handle)
    return int(k.value), int(t.value)


def trajam_boundary_coefficients(problem: Problem, b4) -> np.ndarray:
    b = np.ascontiguousarray(b4, dtype=np.float64)
    out = np.zeros(4)
    _check(load().trajam_boundary_coefficients(ctypes.byref(problem), _dp(b), _dp(out)))
    return out


def trajam_mpc_shift(handle, batch, delta, keep_lambda, xi_bar, lam, xi_next, xi_bar_next, lam_next,
                     stream) -> None:
    _check(load().trajam_mpc_shift(handle, int(batch), float(delta), int(bool(keep_lambda)), xi_bar, lam,
                                   xi_next, xi_bar_next, lam_next, stream), handle)


def trajam_normals(count, key, counter, fp64, z, stream) -> None:
    _check(load().trajam_normals(int(count), int(key) & (2 ** 64 - 1), int(counter) & (2 ** 64 - 1),
                                 int(bool(fp64)), z, stream))


def trajam_cem_sample(handle, n, mu, chol, z, xi, xi_bar, lam, stream) -> None:
    _check(load().trajam_cem_sample(handle, int(n), mu, chol, z, xi, xi_bar, lam, stream), handle)


def trajam_cem_cost(handle, n, xi_bar, res, quantum, c_aug, res_key, stream) -> None:
    _check(load().trajam_cem_cost(handle, int(n), xi_bar, res, float(quantum), c_aug, res_key,
                                  stream), handle)


def trajam_cem_select(handle, n, res_key, c_aug, n_proj, n_elite, proj_idx, elite_idx,
                      stream) -> None:
    _check(load().trajam_cem_select(handle, int(n), res_key, c_aug, int(n_proj), int(n_elite),
                                    proj_idx, elite_idx, stream), handle)


def trajam_cem_update(handle, n_elite, elite_idx, xi_bar, c_aug, sigma, gamma, mu, Sigma, chol,
                      stream) -> None:
    _check(load().trajam_cem_update(handle, int(n_elite), elite_idx, xi_bar, c_aug, float(sigma),
                                    float(gamma), mu, Sigma, chol, stream), handle)


def trajam_mlp_param_count(shape: MlpShape) -> int:
    n = ctypes.c_int64()
    _check(load().trajam_mlp_param_count(ctypes.byref(shape), ctypes.byref(n)))
    return int(n.value)


def trajam_mlp_forward(shape, batch, precision, params, x, acts, y, stream) -> None:
    _check(load().trajam_mlp_forward(ctypes.byref(shape), int(batch), int(precision), params, x,
                                     acts, y, stream))


def trajam_mlp_backward(shape, batch, precision, params, x, acts, dy, grads, scratch,
                        stream) -> None:
    _check(load().trajam_mlp_backward(ctypes.byref(shape), int(batch), int(precision), params, x,
                                      acts, dy, grads, scratch, stream))


def trajam_mlp_backward_noalloc(shape, batch, precision, params, x, acts, dy, grads,
                                stream) -> None:
    _check(load().trajam_mlp_backward_noalloc(ctypes.byref(shape), int(batch), int(precision),
                                              params, x, acts, dy, grads, stream))


def trajam_warm_pack_mfma(shape, params, packed, stream) -> int:
    """Packs the flat fp32 parameters for trajam_warm_jump; packed None: size query.
    Returns the packed size in bytes."""
    n = ctypes.c_int64()
    _check(load().trajam_warm_pack_mfma(ctypes.byref(shape), params, packed, ctypes.byref(n), stream))
    return int(n.value)


def trajam_warm_jump(shape, batch, dims, nv, packed, in_scale, out_scale, xi, xb, lam, xb_out, lam_out,
                     stream) -> None:
    _check(load().trajam_warm_jump(ctypes.byref(shape), int(batch), int(dims), int(nv), packed,
                                   float(in_scale), float(out_scale), xi, xb, lam, xb_out, lam_out, stream))


def trajam_mlp_mse(count, y, target, dy, loss, stream) -> None:
    _check(load().trajam_mlp_mse(int(count), y, target, dy, loss, stream))


def trajam_mlp_adam(n, params, grads, m, v, step, lr, beta1, beta2, eps, stream) -> None:
    _check(load().trajam_mlp_adam(int(n), params, grads, m, v, int(step), float(lr), float(beta1),
                                  float(beta2), float(eps), stream))


def trajam_warm_features(batch, dims, n_coeffs, xi, xb, lam, inv_scale, x, stream) -> None:
    _check(load().trajam_warm_features(int(batch), int(dims), int(n_coeffs), xi, xb, lam,
                                       float(inv_scale), x, stream))


def trajam_warm_apply(batch, dims, n_coeffs, y, out_scale, xi, xb, lam, xb_out, lam_out,
                      stream) -> None:
    _check(load().trajam_warm_apply(int(batch), int(dims), int(n_coeffs), y, float(out_scale), xi,
                                    xb, lam, xb_out, lam_out, stream))


def trajam_mlp_infer(shape: MlpShape, batch, packed, x, y, stream) -> None:
    _check(load().trajam_mlp_infer(ctypes.byref(shape), int(batch), packed, x, y, stream))


def trajam_mlp_pack_infer(shape: MlpShape, params, packed, stream) -> None:
    _check(load().trajam_mlp_pack_infer(ctypes.byref(shape), params, packed, stream))


def trajam_warm_fallback(batch, dims, n_coeffs, res_warm, res_cold, xb_src, lam_src, xb, lam,
                         flags, stream) -> None:
    _check(load().trajam_warm_fallback(int(batch), int(dims), int(n_coeffs), res_warm, res_cold,
                                       xb_src, lam_src, xb, lam, flags, stream))


def trajam_set_obstacles(handle, obs_centre, obs_vel, obs_axes, stream) -> None:
    _check(load().trajam_set_obstacles(handle, obs_centre, obs_vel, obs_axes, stream), handle)


def trajam_autotune(handle, batch, xi, boundary_host, obs_centre, obs_vel, obs_axes, xi_bar,
                    lam, probe_iters, stream):
    b = np.ascontiguousarray(boundary_host, dtype=np.float64)
    k, t = ctypes.c_int32(), ctypes.c_int32()
    _check(load().trajam_autotune(handle, batch, xi, _dp(b), obs_centre, obs_vel, obs_axes, xi_bar,
                                  lam, probe_iters, ctypes.byref(k), ctypes.byref(t), stream),
           handle)
    return k.value, t.value


def trajam_ragged_plan_create(items, iters) -> int:
    arr = (RaggedItem * len(items))(*items)
    out = ctypes.c_void_p()
    _check(load().trajam_ragged_plan_create(arr, len(items), iters, ctypes.byref(out)))
    return out.value


def trajam_ragged_launch(plan, stream) -> None:
    _check(load().trajam_ragged_launch(plan, stream))


def trajam_ragged_plan_destroy(plan) -> None:
    load().trajam_ragged_plan_destroy(plan)


def make_problem(dims, degree, n_steps, horizon, v_max, a_max, rho, n_obstacles,
                 max_batch, precision="fp64", sphere=True, n_agents=1,
                 agent_radius=0.0, workspace=None) -> Problem:
    """workspace: None, or (lo [D], hi [D]) bounds on every position coordinate."""
    pr = Problem(int(dims), int(degree), int(n_steps), float(horizon), float(v_max),
                 float(a_max), float(rho), int(n_obstacles), int(n_agents),
                 float(agent_radius), int(max_batch), PRECISIONS.get(precision, precision),
                 TRAJAM_SPHERE if sphere else TRAJAM_ELLIPSOID)
    if workspace is not None:
        lo, hi = (np.asarray(x, dtype=np.float64) for x in workspace)
        pr.workspace = 1
        for ax in range(int(dims)):
            pr.ws_lo[ax], pr.ws_hi[ax] = float(lo[ax]), float(hi[ax])
    return pr


class Solver:
    """Owns one trajam_solver handle; methods take torch tensors on the GPU."""

    def __init__(self, problem: Problem):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("trajam needs a ROCm GPU; torch.cuda.is_available() is False")
        self.problem = problem
        self.dims = problem.dims
        self.nv = problem.degree + 1
        self.n_agents = problem.n_agents
        # per-sample layout: [D, n_v], or [N, D, n_v] for a joint sample of N agents
        self.sample_shape = ((self.n_agents, self.dims, self.nv) if self.n_agents > 1
                             else (self.dims, self.nv))
        self.dtype = torch.float64 if problem.precision == TRAJAM_FP64 else torch.float32
        self.handle = trajam_init(problem)

    @classmethod
    def for_workload(cls, w, max_batch=None, precision=None, sphere=None):
        prec = precision or w.precision
        if sphere is None:
            sphere = bool(np.all(w.obs_axes == w.obs_axes[:, :1]))
        return cls(make_problem(w.dims, w.degree, w.n_steps, w.horizon, w.v_max, w.a_max,
                                w.rho, w.n_obs, max_batch or w.batch, prec, sphere,
                                n_agents=w.n_agents, agent_radius=w.agent_radius,
                                workspace=getattr(w, "workspace", None)))

    def close(self):
        if getattr(self, "handle", None):
            trajam_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _t(self, x, shape, name):
        import torch
        if x.dtype != self.dtype or not x.is_cuda or not x.is_contiguous():
            raise TypeError(f"{name} must be a contiguous {self.dtype} CUDA tensor")
        if tuple(x.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(x.shape)}, expected {tuple(shape)}")
        return x.data_ptr()

    def obstacles(self, centre=None, vel=None, axes=None):
        """Device pointers of the obstacles; all None reuses the ones packed last."""
        n = self.problem.n_obstacles
        if n == 0 or (centre is None and vel is None and axes is None):
            return None, None, None
        c = self._t(centre, (n, self.dims), "obs_centre")
        v = None if vel is None else self._t(vel, (n, self.dims), "obs_vel")
        a = self._t(axes, (n, self.dims), "obs_axes")
        return c, v, a

    def project(self, xi, boundary, obs, xi_bar, lam, iters, res_trace=None, flags=None,
                stream=None):
        import torch
        B = xi.shape[0]
        shape = (B,) + self.sample_shape
        c, v, a = self.obstacles(*(obs or ()))
        rt = None if res_trace is None else self._t(res_trace, (iters, B), "res_trace")
        fl = None
        if flags is not None:
            if flags.dtype != torch.int32 or not flags.is_cuda or flags.numel() != B:
                raise TypeError("flags must be an int32 CUDA tensor of length batch")
            fl = flags.data_ptr()
        st = (stream or torch.cuda.current_stream()).cuda_stream
        trajam_project(self.handle, B, self._t(xi, shape, "xi"), boundary, c, v, a,
                       self._t(xi_bar, shape, "xi_bar"), self._t(lam, shape, "lambda"),
                       iters, rt, fl, st)

    def residuals(self, xi_bar, obs, res_l2, res_max=None, stream=None):
        import torch
        B = xi_bar.shape[0]
        c, v, a = self.obstacles(*(obs or ()))
        st = (stream or torch.cuda.current_stream()).cuda_stream
        trajam_residuals(self.handle, B, self._t(xi_bar, (B,) + self.sample_shape, "xi_bar"),
                         c, v, a, self._t(res_l2, (B,), "res_l2"),
                         None if res_max is None else self._t(res_max, (B,), "res_max"), st)

    def polar(self, xi_bar, obs, kinematic=True, stream=None, beta=True):
        """Polar variables of step (a) at xi_bar: (alpha, beta, d) tensors [B, n_o, n_steps]
        (None without obstacles; beta None when `beta` is false) and, with kinematic,
        [B, 6, n_steps] (alpha_v, beta_v, d_v, alpha_a, beta_a, d_a)."""
        import torch
        if self.n_agents != 1:
            raise ValueError("polar variables are single-robot")
        B = xi_bar.shape[0]
        n_p = self.problem.n_steps
        n_o = self.problem.n_obstacles
        c, v, a = self.obstacles(*(obs or ()))
        st = (stream or torch.cuda.current_stream()).cuda_stream
        kw = dict(dtype=self.dtype, device=xi_bar.device)
        al = be = d = None
        if n_o:
            al, d = (torch.empty((B, n_o, n_p), **kw) for _ in range(2))
            if beta:
                be = torch.empty((B, n_o, n_p), **kw)
        kin = torch.empty((B, 6, n_p), **kw) if kinematic else None
        ptr = lambda t: None if t is None else t.data_ptr()
        trajam_polar(self.handle, B, self._t(xi_bar, (B,) + self.sample_shape, "xi_bar"), c, v, a,
                     ptr(al), ptr(be), ptr(d), ptr(kin), st)
        return al, be, d, kin

    def set_continuation(self, levels, growth, window, stall_ratio, tol):
        """Penalty ladder rho * growth^l (l < levels) with the per-sample stall check;
        levels = 0 switches it off."""
        if levels == 0:
            trajam_set_continuation(self.handle, None)
        else:
            trajam_set_continuation(self.handle, Continuation(int(levels), float(growth), int(window),
                                                              float(stall_ratio), float(tol)))

    @staticmethod
    def cont_state(batch, device="cuda"):
        """Zeroed per-sample continuation state: [batch, 2] float64 (16 bytes a sample:
        int32 level, int32 count, then the float64 reference residual)."""
        import torch
        return torch.zeros((batch, 2), dtype=torch.float64, device=device)

    @staticmethod
    def cont_levels(state):
        """(level, count, reference) of a state tensor, on the host."""
        import torch
        raw = state.detach().cpu().contiguous()
        ints = raw.view(torch.int32).reshape(raw.shape[0], 4)
        return ints[:, 0].numpy().copy(), ints[:, 1].numpy().copy(), raw[:, 1].numpy().copy()

    def project_continuation(self, xi, boundary, obs, xi_bar, lam, state, iters, res_trace=None,
                             flags=None, stream=None):
        import torch
        B = xi.shape[0]
        shape = (B,) + self.sample_shape
        c, v, a = self.obstacles(*(obs or ()))
        if state.dtype != torch.float64 or tuple(state.shape) != (B, 2) or not state.is_cuda:
            raise ValueError("state must be a [batch, 2] float64 CUDA tensor (Solver.cont_state)")
        st = (stream or torch.cuda.current_stream()).cuda_stream
        trajam_project_continuation(self.handle, B, self._t(xi, shape, "xi"), boundary, c, v, a,
                                    self._t(xi_bar, shape, "xi_bar"), self._t(lam, shape, "lambda"),
                                    state.data_ptr(), iters,
                                    None if res_trace is None else self._t(res_trace, (iters, B), "res_trace"),
                                    None if flags is None else flags.data_ptr(), st)

    def set_launch(self, kernel: int, samples_per_workgroup: int):
        trajam_set_launch(self.handle, kernel, samples_per_workgroup)

    def set_obstacles(self, obs, stream=None):
        import torch
        if self.problem.n_obstacles and (obs is None or obs[0] is None or obs[2] is None):
            raise ValueError("set_obstacles needs centre and axes tensors")
        c, v, a = self.obstacles(*obs)
        st = (stream or torch.cuda.current_stream()).cuda_stream
        trajam_set_obstacles(self.handle, c, v, a, st)

    def autotune(self, xi, boundary, obs, xi_bar, lam, probe_iters=20, stream=None):
        """Time every launch shape, apply the fastest; returns (kernel, samples/WG)."""
        import torch
        B = xi.shape[0]
        shape = (B,) + self.sample_shape
        c, v, a = self.obstacles(*(obs or ()))
        st = (stream or torch.cuda.current_stream()).cuda_stream
        return trajam_autotune(self.handle, B, self._t(xi, shape, "xi"), boundary, c, v, a,
                               self._t(xi_bar, shape, "xi_bar"), self._t(lam, shape, "lambda"),
                               probe_iters, st)

    def launch(self):
        return trajam_get_launch(self.handle)


class RaggedPlan:
    """Many problems (FP32 solvers with obstacles set) in one persistent launch.

    `items` holds (solver, xi, boundary, xi_bar, lam[, res_trace]) tuples of torch
    tensors; the plan keeps references to them, since the device table points at
    their memory."""

    def __init__(self, items, iters):
        keep, cit = [], []
        for it in items:
            solver, xi, boundary, xb, lam = it[:5]
            rt = it[5] if len(it) > 5 else None
            B = xi.shape[0]
            shape = (B,) + solver.sample_shape
            b = np.ascontiguousarray(boundary, dtype=np.float64)
            keep.append((solver, xi, xb, lam, rt, b))
            cit.append(RaggedItem(solver.handle, B, solver._t(xi, shape, "xi"), _dp(b),
                                  solver._t(xb, shape, "xi_bar"), solver._t(lam, shape, "lambda"),
                                  None if rt is None else solver._t(rt, (iters, B), "res_trace"),
                                  None))
        self._keep = keep
        self.iters = iters
        self.handle = trajam_ragged_plan_create(cit, iters)

    def launch(self, stream=None):
        import torch
        trajam_ragged_launch(self.handle, (stream or torch.cuda.current_stream()).cuda_stream)

    def close(self):
        if getattr(self, "handle", None):
            trajam_ragged_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_workload(w, dtype, device="cuda", static=None):
    """Upload a workload's arrays; returns (xi, obs=(centre, vel|None, axes))."""
    import torch
    xi = torch.as_tensor(w.xi, dtype=dtype, device=device).contiguous()
    c = torch.as_tensor(w.obs_centre, dtype=dtype, device=device).contiguous()
    a = torch.as_tensor(w.obs_axes, dtype=dtype, device=device).contiguous()
    if static is None:
        static = not np.any(w.obs_vel)
    v = None if static else torch.as_tensor(w.obs_vel, dtype=dtype, device=device).contiguous()
    return xi, (c, v, a)


# ------------------------------------------------------- heading variant --


def _hcheck(st: int, handle=None):
    if st != TRAJAM_OK:
        L = load()
        msg = (L.trajam_heading_last_error(handle) if handle else L.trajam_last_error(None)).decode()
        raise TrajamError(st, f"{L.trajam_status_string(st).decode()}: {msg}")


def trajam_heading_create(problem: HeadingProblem):
    h = ctypes.c_void_p()
    _hcheck(load().trajam_heading_create(ctypes.byref(problem), ctypes.byref(h)))
    return h


def trajam_heading_destroy(handle) -> None:
    load().trajam_heading_destroy(handle)


def trajam_heading_set_scene(handle, boundary, x_des, obstacles) -> None:
    b = np.ascontiguousarray(boundary, dtype=np.float64).reshape(-1)
    xd = np.ascontiguousarray(x_des, dtype=np.float64)
    ob = np.ascontiguousarray(obstacles, dtype=np.float64).reshape(-1)
    if b.size != 10:
        raise ValueError("boundary needs 10 values")
    _hcheck(load().trajam_heading_set_scene(handle, _dp(b), _dp(xd), _dp(ob) if ob.size else None), handle)


def trajam_heading_project(handle, batch, state, lam, iters, res_trace, stream) -> None:
    _hcheck(load().trajam_heading_project(handle, int(batch), state, lam, int(iters), res_trace, stream), handle)


def trajam_heading_shift(handle, batch, delta, keep_lambda, state, lam, stream) -> None:
    _hcheck(load().trajam_heading_shift(handle, int(batch), float(delta), int(bool(keep_lambda)), state, lam,
                                        stream), handle)


def make_heading_problem(degree, n_steps, horizon, v_max, a_max, rho, radii, n_obstacles, max_batch,
                         precision="fp32") -> HeadingProblem:
    p = HeadingProblem()
    p.degree, p.n_steps = int(degree), int(n_steps)
    p.horizon, p.v_max, p.a_max, p.rho = float(horizon), float(v_max), float(a_max), float(rho)
    r = np.asarray(radii, dtype=np.float64).reshape(-1)
    if not 1 <= r.size <= HEADING_MAX_CIRCLES:
        raise ValueError("1..8 footprint circles")
    p.n_circles = int(r.size)
    for m, v in enumerate(r):
        p.radii[m] = float(v)
    p.n_obstacles = int(n_obstacles)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.max_batch = int(max_batch)
    return p


class HeadingSolver:
    """One trajam_heading handle (Paper II's heading / multi-circle variant): the scene
    is set from a HeadingWorkload; `project` runs Alg 2 in place on torch tensors
    state, lam [B, 5, n_v] (rows x, c, y, s, psi)."""

    def __init__(self, w, precision="fp32", max_batch=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("trajam needs a ROCm GPU; torch.cuda.is_available() is False")
        self.problem = make_heading_problem(w.degree, w.n_steps, w.horizon, w.v_max, w.a_max, w.rho, w.radii,
                                            w.n_obs, max_batch or max(w.batch, 1), precision)
        self.dtype = torch.float64 if self.problem.precision == TRAJAM_FP64 else torch.float32
        self.nv = w.degree + 1
        self.handle = trajam_heading_create(self.problem)
        self.set_scene(w)

    def set_scene(self, w):
        bnd = np.concatenate([np.asarray(w.boundary, dtype=np.float64).reshape(-1),
                              np.asarray(w.boundary_psi, dtype=np.float64).reshape(-1)])
        obs = np.concatenate([w.obs_centre, w.obs_vel, w.obs_axes], axis=1) if w.n_obs else np.zeros((0, 6))
        trajam_heading_set_scene(self.handle, bnd, w.x_des, obs)

    def project(self, state, lam, iters, res_trace=None):
        import torch
        for t in (state, lam) + ((res_trace,) if res_trace is not None else ()):
            if t.dtype != self.dtype or not t.is_cuda or not t.is_contiguous():
                raise ValueError("contiguous device tensors of the solver's precision required")
        B = state.shape[0]
        if tuple(state.shape[1:]) != (5, self.nv) or lam.shape != state.shape:
            raise ValueError("state and lam must be [B, 5, n_v]")
        if res_trace is not None and tuple(res_trace.shape) != (int(iters), B, 2):
            raise ValueError("res_trace must be [iters, B, 2]")
        st = torch.cuda.current_stream().cuda_stream
        trajam_heading_project(self.handle, B, state.data_ptr(), lam.data_ptr(), iters,
                               res_trace.data_ptr() if res_trace is not None else None, st)

    def shift(self, state, lam, delta, keep_lambda=True):
        """Receding horizon: state and lam [B, 5, n_v] re-expressed in place on the window
        moved on by delta (the multipliers kept or cleared)."""
        import torch
        st = torch.cuda.current_stream().cuda_stream
        trajam_heading_shift(self.handle, state.shape[0], delta, keep_lambda, state.data_ptr(), lam.data_ptr(), st)

    def close(self):
        if getattr(self, "handle", None):
            trajam_heading_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
