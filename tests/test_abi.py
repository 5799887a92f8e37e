"""CPU checks of the C-ABI library: it loads, exports every declared symbol, rejects
invalid problems on the host, and its FP64 host precompute agrees with the oracle.
No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2408_10731_amd import trajam as tj
from paper_2408_10731_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "trajam.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(trajam_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = tj.load()
    decl = declared_symbols()
    assert len(decl) >= 10
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(tj.EXPORTS) == decl


def test_status_strings():
    L = tj.load()
    for st in (0, -1, -2, -3, -4, -5):
        assert L.trajam_status_string(st)
    assert L.trajam_status_string(99) == b"unknown status"


def _problem(**kw):
    base = dict(dims=2, degree=10, n_steps=100, horizon=10.0, v_max=1.5, a_max=2.0, rho=1.0,
                n_obstacles=10, max_batch=64, precision="fp64", sphere=True)
    base.update(kw)
    return tj.make_problem(**base)


@pytest.mark.parametrize("kw,status", [
    (dict(dims=4), tj.TRAJAM_ERR_INVALID),
    (dict(degree=2), tj.TRAJAM_ERR_INVALID),
    (dict(degree=16), tj.TRAJAM_ERR_INVALID),
    (dict(n_steps=5), tj.TRAJAM_ERR_INVALID),
    (dict(n_steps=257), tj.TRAJAM_ERR_INVALID),
    (dict(horizon=0.0), tj.TRAJAM_ERR_INVALID),
    (dict(rho=-1.0), tj.TRAJAM_ERR_INVALID),
    (dict(n_obstacles=-1), tj.TRAJAM_ERR_INVALID),
    (dict(max_batch=0), tj.TRAJAM_ERR_INVALID),
    (dict(precision=7), tj.TRAJAM_ERR_INVALID),
    (dict(v_max=float("nan")), tj.TRAJAM_ERR_INVALID),
    (dict(n_agents=0), tj.TRAJAM_ERR_INVALID),
    (dict(n_agents=65, agent_radius=0.3), tj.TRAJAM_ERR_INVALID),
    (dict(n_agents=3, agent_radius=0.0), tj.TRAJAM_ERR_INVALID),
    (dict(n_agents=3, agent_radius=float("inf")), tj.TRAJAM_ERR_INVALID),
    (dict(n_agents=3, agent_radius=0.3, precision="bf16"), tj.TRAJAM_ERR_UNSUPPORTED),
    (dict(n_agents=3, agent_radius=0.3, degree=12, n_steps=100), tj.TRAJAM_ERR_UNSUPPORTED),
])
def test_invalid_problems_rejected_on_host(kw, status):
    L = tj.load()
    h = ctypes.c_void_p(123)
    st = L.trajam_init(ctypes.byref(_problem(**kw)), ctypes.byref(h))
    assert st == status
    assert h.value is None
    assert L.trajam_last_error(None)


def test_null_handles_are_rejected():
    L = tj.load()
    assert L.trajam_project(None, 1, None, None, None, None, None, None, None, 1, None, None,
                            None) == tj.TRAJAM_ERR_INVALID
    assert L.trajam_residuals(None, 1, None, None, None, None, None, None, None) == \
        tj.TRAJAM_ERR_INVALID
    assert L.trajam_polar(None, 1, None, None, None, None, None, None, None, None, None) == \
        tj.TRAJAM_ERR_INVALID
    assert L.trajam_init(None, None) == tj.TRAJAM_ERR_INVALID
    L.trajam_destroy(None)
    assert L.trajam_set_launch(None, 0, 1) == tj.TRAJAM_ERR_INVALID
    assert L.trajam_get_launch(None, None, None) == tj.TRAJAM_ERR_INVALID


@pytest.mark.parametrize("dims,degree,n_steps,T,n_obs,vm,am", [
    (2, 10, 100, 10.0, 10, 1.5, 2.0), (3, 15, 150, 20.0, 200, 1.5, 2.0),
    (2, 5, 9, 4.0, 2, 0.0, 2.0), (3, 7, 64, 3.0, 0, 1.0, 0.0), (2, 3, 4, 1.0, 1, 1.0, 1.0)])
def test_host_precompute_matches_oracle(dims, degree, n_steps, T, n_obs, vm, am):
    pr = _problem(dims=dims, degree=degree, n_steps=n_steps, horizon=T, n_obstacles=n_obs,
                  v_max=vm, a_max=am)
    P, Pd, Pdd, H, W = tj.trajam_fixed_matrices(pr)
    oP, oPd, oPdd = oracle.bernstein(degree, n_steps, T)
    np.testing.assert_allclose(P, oP, atol=1e-14)
    np.testing.assert_allclose(Pd, oPd, atol=1e-12 * degree / T)
    np.testing.assert_allclose(Pdd, oPdd, atol=1e-11 * degree ** 2 / T ** 2)
    opr = oracle.problem(dims, degree, n_steps, T, vm, am, 1.0, n_obs)
    _, oH = oracle.constraint_matrices(opr)
    np.testing.assert_allclose(H, oH, rtol=1e-12, atol=1e-12)
    # the delta-form operator reproduces the oracle's KKT solve: for any q and
    # boundary b, xb = xb0 + W z with z = (q - H xb0) on free, (xb*_b - xb0_b) on boundary
    rng = np.random.default_rng(1)
    n = degree
    for _ in range(3):
        q = rng.normal(size=n + 1) * 10
        b = rng.normal(size=4)
        x0 = rng.normal(size=n + 1)
        ref = oracle.kkt_solve(opr, q, b)
        cb = tj.trajam_boundary_coefficients(pr, b)
        z = q - H @ x0
        bidx = [0, 1, 2, n]
        z[bidx] = cb - x0[bidx]
        x = x0.copy()
        x[3:n] += W @ z
        x[bidx] = cb
        np.testing.assert_allclose(x, ref, atol=1e-9 * max(1, np.abs(ref).max()))


def test_boundary_coefficients_reach_boundary_rows():
    pr = _problem(degree=10, horizon=7.0)
    opr = oracle.problem(2, 10, 100, 7.0, 1.5, 2.0, 1.0, 10)
    A, _ = oracle.constraint_matrices(opr)
    b = np.array([1.0, -0.3, 0.2, 4.0])
    c = tj.trajam_boundary_coefficients(pr, b)
    x = np.zeros(11)
    x[[0, 1, 2, 10]] = c
    np.testing.assert_allclose(A @ x, b, atol=1e-12)


def _bf16_round(x32):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float32."""
    u = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32)


@pytest.mark.parametrize("dims,degree,n_steps,T,n_obs,prec,agents", [
    (2, 10, 100, 30.0, 50, tj.TRAJAM_FP64, 1),
    (2, 10, 100, 30.0, 50, tj.TRAJAM_FP32, 1),
    (3, 15, 150, 20.0, 200, tj.TRAJAM_FP32, 1),
    (3, 15, 150, 20.0, 200, tj.TRAJAM_BF16_REFINE, 1),
    (2, 10, 100, 30.0, 50, tj.TRAJAM_BF16_REFINE, 1),
    (3, 10, 100, 10.0, 20, tj.TRAJAM_FP32, 16),
    (2, 3, 20, 4.0, 2, tj.TRAJAM_FP32, 1),      # no free coefficient: nothing to contract
])
def test_qp_contraction_is_the_spectral_radius(dims, degree, n_steps, T, n_obs, prec, agents):
    """The library's contraction estimate against numpy's eigenvalues of I - W~ H_ff,
    built here from the oracle's Hessian with the rounding each precision applies."""
    pr = _problem(dims=dims, degree=degree, n_steps=n_steps, horizon=T, n_obstacles=n_obs,
                  v_max=1.5, a_max=2.0, precision=prec, n_agents=agents,
                  agent_radius=0.3 if agents > 1 else 0.0)
    rho = tj.trajam_qp_contraction(pr)
    opr = oracle.problem(dims, degree, n_steps, T, 1.5, 2.0, 1.0, n_obs)
    _, H = oracle.constraint_matrices(opr)
    Hs = [H]
    if agents > 1:
        P, _, _ = oracle.bernstein(degree, n_steps, T)
        Hs.append(H + agents * 1.0 * P.T @ P)
    ref = 0.0
    for Hm in Hs:
        Hff = Hm[3:degree, 3:degree]
        if Hff.size == 0:
            continue
        W = np.linalg.inv(Hff)
        if prec == tj.TRAJAM_FP32:
            Wt = W.astype(np.float32).astype(np.float64)
        elif prec == tj.TRAJAM_BF16_REFINE:
            w32 = W.astype(np.float32)
            hi = _bf16_round(w32)
            lo = _bf16_round(w32 - hi)
            Wt = hi.astype(np.float64) + lo.astype(np.float64)
        else:
            Wt = W
        E = np.eye(Hff.shape[0]) - Wt @ Hff
        ref = max(ref, np.abs(np.linalg.eigvals(E)).max())
    if prec == tj.TRAJAM_FP64 or degree == 3:
        assert rho < 1e-10
    else:
        # an upper estimate within n_f^(1/512) of the radius
        assert ref * (1 - 1e-9) <= rho <= ref * 1.01 + 1e-300, (rho, ref)
    assert rho < 0.5


def test_qp_contraction_rejects_a_null_output():
    pr = _problem()
    assert tj.load().trajam_qp_contraction(ctypes.byref(pr), None) == tj.TRAJAM_ERR_INVALID


def test_header_constants_match_the_binding():
    src = open(os.path.join(ROOT, "include", "trajam.h")).read()
    defs = {k: int(v) for k, v in re.findall(r"#define TRAJAM_([A-Z_0-9]+) (\d+)u?\b", src)}
    for name in ("FLAG_NONFINITE", "FLAG_GREW", "FLAG_COLD_FALLBACK", "MLP_MAX_LAYERS",
                 "MLP_NOALLOC_SCRATCH_FLOATS", "MLP_MSE_LOSS_FLOATS", "CONT_MAX_LEVELS"):
        assert defs[name] == getattr(tj, name), name
