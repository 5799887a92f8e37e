"""CPU FP64 oracle of the batched alternating-minimization projection.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg
of the benchmark may import this package.  The product path never does, and the
oracle never imports the product package: the two share no code.  Both sides only
consume the same host arrays drawn by the seeded input generator.

`trajam_oracle.c` holds the projection (basis, KKT LU, polar steps, multiplier,
residual) for one robot and for N agents with pairwise avoidance; `mlp.py` and `cem.py` hold the numpy FP64 oracles of the learned warm
start and of the sampling loop.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "trajam_oracle.c")
_LIB = os.path.join(_HERE, "_trajam_oracle.so")
_lib = None


class Problem(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int),
        ("degree", ctypes.c_int),
        ("n_steps", ctypes.c_int),
        ("horizon", ctypes.c_double),
        ("v_max", ctypes.c_double),
        ("a_max", ctypes.c_double),
        ("rho", ctypes.c_double),
        ("n_obs", ctypes.c_int),
        ("workspace", ctypes.c_int),
        ("ws_lo", ctypes.c_double * 3),
        ("ws_hi", ctypes.c_double * 3),
    ]


class Cont(ctypes.Structure):
    """Penalty continuation parameters (see orc_project_cont)."""
    _fields_ = [
        ("n_levels", ctypes.c_int),
        ("growth", ctypes.c_double),
        ("window", ctypes.c_int),
        ("stall", ctypes.c_double),
        ("tol", ctypes.c_double),
    ]


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, no fast-math, OpenMP over trajectories)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp",
                               "-fPIC", "-shared", "-Wall", "-Wno-unused-variable",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        # TRAJAM_ORACLE_LIB: a separately built copy of this oracle (the sanitizer test's
        # instrumented build), loaded as it is
        path = os.environ.get("TRAJAM_ORACLE_LIB")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(Problem)
        L.orc_bernstein.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp, dp]
        L.orc_constraint_matrices.argtypes = [pp, dp, dp]
        L.orc_kkt_matrix.argtypes = [pp, dp]
        L.orc_kkt_solve.argtypes = [pp, dp, dp, dp]
        L.orc_qp_nullspace.argtypes = [pp, dp, dp, dp]
        L.orc_polar_obstacle.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp, dp]
        L.orc_polar_obstacle.restype = None
        L.orc_polar_bound.argtypes = [ctypes.c_int, dp, ctypes.c_double, dp]
        L.orc_polar_bound.restype = None
        L.orc_project.argtypes = [pp, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, ctypes.c_int,
                                  dp, dp, ctypes.c_int, ctypes.c_int]
        L.orc_residuals.argtypes = [pp, ctypes.c_int, dp, dp, dp, dp, dp, dp, ctypes.c_int]
        L.orc_polar_products.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_agents_kkt_matrix.argtypes = [pp, ctypes.c_int, dp]
        L.orc_agents_qp.argtypes = [pp, ctypes.c_int, dp, dp, dp]
        L.orc_agents_polar_products.argtypes = [pp, ctypes.c_int, ctypes.c_double, dp, dp, dp,
                                                dp, dp, dp, dp]
        L.orc_project_agents.argtypes = [pp, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp,
                                         dp, dp, dp, dp, dp, dp, ctypes.c_int, dp, dp,
                                         ctypes.c_int]
        L.orc_residuals_agents.argtypes = [pp, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp,
                                           dp, dp, dp, dp, dp, ctypes.c_int]
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_project_cont.argtypes = [pp, ctypes.POINTER(Cont), ctypes.c_int, dp, dp, dp, dp, dp, dp, dp,
                                       ip, ip, dp, ctypes.c_int, dp, ip, ctypes.c_int]
        L.orc_set_fault.argtypes = [ctypes.c_int]
        L.orc_set_fault.restype = None
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def problem(dims, degree, n_steps, horizon, v_max, a_max, rho, n_obs, workspace=None) -> Problem:
    """workspace: None, or (lo [D], hi [D]) bounds on every position coordinate."""
    pr = Problem(int(dims), int(degree), int(n_steps), float(horizon), float(v_max),
                 float(a_max), float(rho), int(n_obs))
    if workspace is not None:
        lo, hi = (np.asarray(x, dtype=np.float64) for x in workspace)
        pr.workspace = 1
        for ax in range(int(dims)):
            pr.ws_lo[ax], pr.ws_hi[ax] = float(lo[ax]), float(hi[ax])
    return pr


def problem_of(w) -> Problem:
    """Problem struct from a workload object (duck-typed: any object with the fields)."""
    return problem(w.dims, w.degree, w.n_steps, w.horizon, w.v_max, w.a_max, w.rho,
                   w.obs_centre.shape[0], getattr(w, "workspace", None))


def set_fault(code: int) -> None:
    """Plant a deliberate mistake (mutation tests only); 0 restores the oracle."""
    lib().orc_set_fault(int(code))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def bernstein(n: int, n_p: int, T: float):
    nv = n + 1
    P = np.zeros((n_p, nv)); Pd = np.zeros((n_p, nv)); Pdd = np.zeros((n_p, nv))
    if lib().orc_bernstein(n, n_p, T, _p(P), _p(Pd), _p(Pdd)) != 0:
        raise ValueError("invalid basis parameters")
    return P, Pd, Pdd


def constraint_matrices(pr: Problem):
    nv = pr.degree + 1
    A = np.zeros((4, nv)); H = np.zeros((nv, nv))
    if lib().orc_constraint_matrices(ctypes.byref(pr), _p(A), _p(H)) != 0:
        raise ValueError("invalid problem")
    return A, H


def kkt_matrix(pr: Problem):
    N = pr.degree + 5
    K = np.zeros((N, N))
    if lib().orc_kkt_matrix(ctypes.byref(pr), _p(K)) != 0:
        raise ValueError("invalid problem")
    return K


def kkt_solve(pr: Problem, q, b):
    q = _f64(q); b = _f64(b); out = np.zeros(pr.degree + 1)
    if lib().orc_kkt_solve(ctypes.byref(pr), _p(q), _p(b), _p(out)) != 0:
        raise ValueError("singular KKT")
    return out


def qp_nullspace(pr: Problem, q, b):
    q = _f64(q); b = _f64(b); out = np.zeros(pr.degree + 1)
    if lib().orc_qp_nullspace(ctypes.byref(pr), _p(q), _p(b), _p(out)) != 0:
        raise ValueError("nullspace solve failed")
    return out


def polar_obstacle(xt, s):
    xt = _f64(xt); s = _f64(s); D = xt.shape[0]
    al = np.zeros(1); be = np.zeros(1); d = np.zeros(1); off = np.zeros(D)
    lib().orc_polar_obstacle(D, _p(xt), _p(s), _p(al), _p(be), _p(d), _p(off))
    return float(al[0]), float(be[0]), float(d[0]), off


def polar_bound(v, bound):
    v = _f64(v); e = np.zeros(v.shape[0])
    lib().orc_polar_bound(v.shape[0], _p(v), float(bound), _p(e))
    return e


def project(w, xi_bar=None, lam=None, iters=None, freeze_lambda=False, n_threads=0,
            xi=None):
    """Run the AM projection on workload `w`.

    Returns (xi_bar [B,D,n_v], lam [B,D,n_v], res_trace [K,B], resmax_trace [K,B]).
    Cold start by default: xi_bar = xi, lam = 0.
    """
    pr = problem_of(w)
    xi = _f64(w.xi if xi is None else xi)
    B = xi.shape[0]
    xb = _f64(xi if xi_bar is None else xi_bar).copy()
    lm = np.zeros_like(xi) if lam is None else _f64(lam).copy()
    K = int(w.iters if iters is None else iters)
    tr = np.zeros((max(K, 1), B)); tm = np.zeros((max(K, 1), B))
    oc = _f64(w.obs_centre).reshape(-1, w.dims)
    ow = _f64(w.obs_vel).reshape(-1, w.dims)
    os_ = _f64(w.obs_axes).reshape(-1, w.dims)
    bnd = _f64(w.boundary)
    rc = lib().orc_project(ctypes.byref(pr), B, _p(xi), _p(oc), _p(ow), _p(os_), _p(bnd),
                           _p(xb), _p(lm), K, _p(tr), _p(tm), int(bool(freeze_lambda)),
                           int(n_threads))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return xb, lm, tr[:K], tm[:K]


def residuals(w, xi_bar, n_threads=0):
    """(res_l2 [B], res_max [B]) of the polar step evaluated at xi_bar."""
    pr = problem_of(w)
    xb = _f64(xi_bar)
    B = xb.shape[0]
    r2 = np.zeros(B); mx = np.zeros(B)
    rc = lib().orc_residuals(ctypes.byref(pr), B, _p(xb), _p(_f64(w.obs_centre)),
                             _p(_f64(w.obs_vel)), _p(_f64(w.obs_axes)), _p(r2), _p(mx),
                             int(n_threads))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return r2, mx


def polar_products(w, xb_one):
    """(F^T e [D,n_v], F^T r [D,n_v], |r|^2) at one coefficient array [D, n_v]."""
    pr = problem_of(w)
    xb = _f64(xb_one)
    fte = np.zeros_like(xb); ftr = np.zeros_like(xb); r2 = np.zeros(1)
    lib().orc_polar_products(ctypes.byref(pr), _p(xb), _p(_f64(w.obs_centre)),
                             _p(_f64(w.obs_vel)), _p(_f64(w.obs_axes)), _p(fte), _p(ftr),
                             _p(r2))
    return fte, ftr, float(r2[0])


# ------------------------------------------------------------ multi-agent --


def _combined_radius(w):
    return 2.0 * float(w.agent_radius)


def agents_kkt_matrix(pr: Problem, n_agents: int):
    S = n_agents * (pr.degree + 5)
    K = np.zeros((S, S))
    if lib().orc_agents_kkt_matrix(ctypes.byref(pr), int(n_agents), _p(K)) != 0:
        raise ValueError("invalid problem")
    return K


def agents_qp(pr: Problem, q, b):
    """Joint QP of one axis: q [N, n_v], b [N, 4] -> [N, n_v]."""
    q = _f64(q); b = _f64(b); out = np.zeros_like(q)
    if lib().orc_agents_qp(ctypes.byref(pr), q.shape[0], _p(q), _p(b), _p(out)) != 0:
        raise ValueError("singular joint KKT")
    return out


def agents_polar_products(w, xb_joint):
    """(F^T e, F^T r [N, D, n_v], |r|^2) of the joint problem at one joint sample."""
    pr = problem_of(w)
    xb = _f64(xb_joint)
    fte = np.zeros_like(xb); ftr = np.zeros_like(xb); r2 = np.zeros(1)
    lib().orc_agents_polar_products(ctypes.byref(pr), xb.shape[0], _combined_radius(w), _p(xb),
                                    _p(_f64(w.obs_centre)), _p(_f64(w.obs_vel)),
                                    _p(_f64(w.obs_axes)), _p(fte), _p(ftr), _p(r2))
    return fte, ftr, float(r2[0])


def project_agents(w, xi_bar=None, lam=None, iters=None, n_threads=0):
    """Joint AM projection of workload `w` (xi [B, N, D, n_v], boundary [N, D, 4]).

    Returns (xi_bar, lam [B, N, D, n_v], res_trace [K, B], resmax_trace [K, B])."""
    pr = problem_of(w)
    xi = _f64(w.xi)
    B, N = xi.shape[0], xi.shape[1]
    xb = _f64(xi if xi_bar is None else xi_bar).copy()
    lm = np.zeros_like(xi) if lam is None else _f64(lam).copy()
    K = int(w.iters if iters is None else iters)
    tr = np.zeros((max(K, 1), B)); tm = np.zeros((max(K, 1), B))
    rc = lib().orc_project_agents(ctypes.byref(pr), N, _combined_radius(w), B, _p(xi),
                                  _p(_f64(w.obs_centre)), _p(_f64(w.obs_vel)),
                                  _p(_f64(w.obs_axes)), _p(_f64(w.boundary)), _p(xb), _p(lm), K,
                                  _p(tr), _p(tm), int(n_threads))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return xb, lm, tr[:K], tm[:K]


def residuals_agents(w, xi_bar, n_threads=0):
    """(res_l2 [B], res_max [B]) of the joint polar step at xi_bar [B, N, D, n_v]."""
    pr = problem_of(w)
    xb = _f64(xi_bar)
    B, N = xb.shape[0], xb.shape[1]
    r2 = np.zeros(B); mx = np.zeros(B)
    rc = lib().orc_residuals_agents(ctypes.byref(pr), N, _combined_radius(w), B, _p(xb),
                                    _p(_f64(w.obs_centre)), _p(_f64(w.obs_vel)),
                                    _p(_f64(w.obs_axes)), _p(r2), _p(mx), int(n_threads))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return r2, mx


# ------------------------------------------------------- rho-continuation --


def project_cont(w, n_levels, growth, window, stall, tol, iters=None, xi_bar=None, lam=None,
                 state=None, n_threads=0, xi=None):
    """AM projection with penalty continuation (orc_project_cont).  state: None (cold:
    level 0, count 0, no reference) or (level [B] int, count [B] int, ref [B] float).
    Returns (xi_bar, lam, res_trace [K, B], level_trace [K, B], (level, count, ref))."""
    pr = problem_of(w)
    xi = _f64(w.xi if xi is None else xi)
    B = xi.shape[0]
    xb = _f64(xi if xi_bar is None else xi_bar).copy()
    lm = np.zeros_like(xi) if lam is None else _f64(lam).copy()
    K = int(w.iters if iters is None else iters)
    if state is None:
        lev, cnt, ref = np.zeros(B, np.int32), np.zeros(B, np.int32), np.zeros(B)
    else:
        lev, cnt, ref = (np.ascontiguousarray(state[0], np.int32).copy(),
                         np.ascontiguousarray(state[1], np.int32).copy(), _f64(state[2]).copy())
    tr = np.zeros((max(K, 1), B)); lt = np.zeros((max(K, 1), B), np.int32)
    cc = Cont(int(n_levels), float(growth), int(window), float(stall), float(tol))
    ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    rc = lib().orc_project_cont(ctypes.byref(pr), ctypes.byref(cc), B, _p(xi),
                                _p(_f64(w.obs_centre).reshape(-1, w.dims)),
                                _p(_f64(w.obs_vel).reshape(-1, w.dims)),
                                _p(_f64(w.obs_axes).reshape(-1, w.dims)), _p(_f64(w.boundary)),
                                _p(xb), _p(lm), ip(lev), ip(cnt), _p(ref), K, _p(tr), ip(lt),
                                int(n_threads))
    if rc != 0:
        raise ValueError("oracle rejected the problem or the continuation")
    return xb, lm, tr[:K], lt[:K], (lev, cnt, ref)
