"""Pins of the oracle's workspace bounds (Paper III, eq bound_con: G xb <= tau with
G = [-P; P], through the slack step s = max(0, -G xb + tau) of its AM list): the
residual against the textbook distance to a box, the fixed matrix against an explicit
stacking of G, KKT stationarity of the QP with F and e built independently, and
convergence into the box of a workspace-only problem.  A planted sign mistake in the
slack step must fail them."""
import dataclasses
from math import comb

import numpy as np
import pytest

import oracle
from paper_2408_10731_amd import workloads as wl


def basis(n, n_p, T):
    """P, Pd, Pdd by the definition (math.comb), independent of the oracle's basis."""
    tau = np.arange(n_p) / (n_p - 1)
    P = np.array([[comb(n, k) * u ** k * (1 - u) ** (n - k) for k in range(n + 1)] for u in tau])

    def deriv(B, m):   # Bernstein derivative on [0, T] of degree m
        D = np.zeros((m + 1, m))
        for k in range(m):
            D[k, k], D[k + 1, k] = -1.0, 1.0
        return D * (m / T)
    Pm1 = np.array([[comb(n - 1, k) * u ** k * (1 - u) ** (n - 1 - k) for k in range(n)] for u in tau])
    Pm2 = np.array([[comb(n - 2, k) * u ** k * (1 - u) ** (n - 2 - k) for k in range(n - 1)] for u in tau])
    Pd = Pm1 @ deriv(None, n).T
    Pdd = Pm2 @ deriv(None, n - 1).T @ deriv(None, n).T
    return P, Pd, Pdd


def ws_scene(batch=3, seed=5, box=((-1.0, 14.8), (31.0, 15.2)), n_obs=2, loose=False):
    """A config-2 style scene whose samples leave the box |y - 15| <= 0.2."""
    w = wl.config2(batch=batch, seed=seed)
    w = dataclasses.replace(w, obs_centre=w.obs_centre[:n_obs], obs_vel=w.obs_vel[:n_obs],
                            obs_axes=w.obs_axes[:n_obs], workspace=np.array(box, dtype=np.float64),
                            precision="fp64")
    if loose:
        w = dataclasses.replace(w, v_max=0.0, a_max=0.0)
    return w


def box_distance2(pos, lo, hi):
    """Squared Euclidean distance of every point to the box (textbook clip)."""
    return ((pos - np.clip(pos, lo, hi)) ** 2).sum()


def test_workspace_residual_is_the_distance_to_the_box():
    w = ws_scene(n_obs=0, loose=True)
    P, _, _ = basis(w.degree, w.n_steps, w.horizon)
    lo, hi = w.workspace
    res, mx = oracle.residuals(w, w.xi)
    for i in range(w.batch):
        pos = P @ w.xi[i].T
        d2 = box_distance2(pos, lo, hi)
        assert d2 > 1e-2
        assert abs(res[i] ** 2 - d2) <= 1e-10 * (1 + d2)
        assert abs(mx[i] - np.abs(pos - np.clip(pos, lo, hi)).max()) <= 1e-12
    # inside the box: no residual
    w_in = dataclasses.replace(w, workspace=np.array([[-1e3, -1e3], [1e3, 1e3]]))
    # (the slack form tau - (tau - g) leaves rounding of the bound's size)
    np.testing.assert_allclose(oracle.residuals(w_in, w.xi)[0], 0.0, atol=1e-11)


def test_fixed_matrix_gains_two_copies_of_P():
    w = ws_scene()
    P, Pd, Pdd = basis(w.degree, w.n_steps, w.horizon)
    K1 = oracle.kkt_matrix(oracle.problem_of(w))
    K0 = oracle.kkt_matrix(oracle.problem_of(dataclasses.replace(w, workspace=None)))
    nv = w.n_v
    G = np.vstack([-P, P])
    np.testing.assert_allclose(K1[:nv, :nv] - K0[:nv, :nv], w.rho * G.T @ G, atol=1e-10)
    np.testing.assert_allclose(K1[nv:, :], K0[nv:, :], atol=0)


def _explicit_FtR(w, xb_one):
    """F^T (F xb - e) with F = [P x n_o; G; Pd; Pdd] stacked explicitly and e from the
    characterizations: nearest surface point for circles, ball clip for the bounds,
    and for the workspace rows the projection onto each half-space."""
    P, Pd, Pdd = basis(w.degree, w.n_steps, w.horizon)
    t = np.arange(w.n_steps) * w.horizon / (w.n_steps - 1)
    pos, vel, acc = P @ xb_one.T, Pd @ xb_one.T, Pdd @ xb_one.T
    lo, hi = w.workspace

    def clip(v, bnd):
        nv = np.linalg.norm(v, axis=1, keepdims=True)
        return np.where(nv > bnd, v * bnd / np.maximum(nv, 1e-300), v)
    out = np.zeros_like(xb_one)
    for ax in range(w.dims):
        Fb, eb = [], []
        for j in range(w.obs_centre.shape[0]):
            c = w.obs_centre[j] + t[:, None] * w.obs_vel[j]
            xt = pos - c
            r = w.obs_axes[j, 0]
            nx = np.linalg.norm(xt, axis=1, keepdims=True)
            Fb.append(P)
            eb.append(np.where(nx >= r, pos, c + r * xt / nx)[:, ax])
        # G = [-P; P]: -p <= -lo projects to min(-p, -lo); p <= hi to min(p, hi)
        Fb += [-P, P]
        eb += [np.minimum(-pos[:, ax], -lo[ax]), np.minimum(pos[:, ax], hi[ax])]
        if w.v_max > 0:
            Fb.append(Pd); eb.append(clip(vel, w.v_max)[:, ax])
        if w.a_max > 0:
            Fb.append(Pdd); eb.append(clip(acc, w.a_max)[:, ax])
        F, e = np.vstack(Fb), np.concatenate(eb)
        out[ax] = F.T @ (F @ xb_one[ax] - e)
    return out


def _stationarity_holds(w):
    P, Pd, Pdd = basis(w.degree, w.n_steps, w.horizon)
    n_o = w.obs_centre.shape[0]
    F = np.vstack([P] * n_o + [-P, P] + ([Pd] if w.v_max > 0 else []) + ([Pdd] if w.a_max > 0 else []))
    FtF = F.T @ F
    xb0, lam0, _, _ = oracle.project(w, iters=1)
    xb1, lam1, _, _ = oracle.project(w, xi_bar=xb0, lam=lam0, iters=1)
    free = list(range(3, w.degree))
    ok = True
    for i in range(w.batch):
        ftr0 = _explicit_FtR(w, xb0[i])
        for ax in range(w.dims):
            fte1 = FtF @ xb0[i, ax] - ftr0[ax]
            stat = (xb1[i, ax] - w.xi[i, ax]) + w.rho * (FtF @ xb1[i, ax] - fte1)
            ok &= np.allclose(lam1[i, ax, free], stat[free], atol=1e-9)
            ok &= np.allclose(lam1[i, ax], lam0[i, ax] - w.rho * ftr0[ax], atol=1e-9)
    return ok


def test_qp_stationarity_with_the_workspace_rows():
    """KKT stationarity of one iteration's QP on the free coefficients with F (obstacle
    copies of P, G = [-P; P], Pd, Pdd) and e built here: the multiplier is
    lambda^{k+1} = lambda^k - rho F^T r^k and the QP meets
    lambda^{k+1}_f = (xb^{k+1} - xi)_f + rho [F^T F xb^{k+1} - F^T e^{k+1}]_f."""
    w = ws_scene()
    xb0 = oracle.project(w, iters=1)[0]
    assert max(np.abs(_explicit_FtR(w, xb0[i])).max() for i in range(w.batch)) > 1e-2   # rows active
    assert _stationarity_holds(w)


def test_workspace_only_problem_converges_into_the_box():
    w = ws_scene(n_obs=0, loose=True)
    lo, hi = w.workspace
    xb, _, tr, _ = oracle.project(w, iters=300)
    assert tr[0].min() > 1e-2
    assert tr[-1].max() <= 1e-4
    P, _, _ = basis(w.degree, w.n_steps, w.horizon)
    for i in range(w.batch):
        pos = P @ xb[i].T
        assert (pos >= lo - 1e-4).all() and (pos <= hi + 1e-4).all()


def test_planted_slack_sign_mistake_is_caught():
    w = ws_scene()
    assert _stationarity_holds(w)
    oracle.set_fault(10)
    try:
        w0 = ws_scene(n_obs=0, loose=True)
        P, _, _ = basis(w0.degree, w0.n_steps, w0.horizon)
        res = oracle.residuals(w0, w0.xi)[0]
        d2 = box_distance2(P @ w0.xi[0].T, *w0.workspace)
        assert (not _stationarity_holds(w)) or abs(res[0] ** 2 - d2) > 1e-6
    finally:
        oracle.set_fault(0)
