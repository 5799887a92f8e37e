"""Pins of the CPU oracle against facts fixed by the thesis and by mathematics.

None of these re-types the oracle's formulas: each compares it with an independent
route (de Casteljau evaluation, explicit stacking of F, brute-force grids, a second
linear solver, closed forms derived by hand, invariants of the AM iteration).
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2408_10731_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def de_casteljau(coef, tau):
    """Evaluate a Bernstein polynomial by repeated linear interpolation."""
    b = np.array(coef, dtype=np.float64)
    for r in range(1, len(b)):
        b = (1.0 - tau) * b[:-1] + tau * b[1:]
    return b[0]


def stacked_F(P, Pd, Pdd, n_obs, use_v=True, use_a=True):
    """F for one axis built by literally stacking the blocks (eq f_e)."""
    blocks = [P] * n_obs + ([Pd] if use_v else []) + ([Pdd] if use_a else [])
    return np.vstack(blocks) if blocks else np.zeros((0, P.shape[1]))


# --------------------------------------------------------------------- basis


def test_basis_golden_by_hand():
    g = json.load(open(os.path.join(GOLD, "bernstein_n3_np3_T2.json")))
    P, Pd, Pdd = oracle.bernstein(g["degree"], g["n_steps"], g["horizon"])
    np.testing.assert_allclose(P, g["P"], atol=1e-15)
    np.testing.assert_allclose(Pd, g["Pd"], atol=1e-14)
    np.testing.assert_allclose(Pdd, g["Pdd"], atol=1e-14)


@pytest.mark.parametrize("n,n_p,T", [(10, 100, 10.0), (15, 150, 20.0), (5, 9, 4.0)])
def test_basis_identities(n, n_p, T):
    P, Pd, Pdd = oracle.bernstein(n, n_p, T)
    tau = np.arange(n_p) / (n_p - 1)
    # partition of unity and its derivatives
    np.testing.assert_allclose(P.sum(1), 1.0, atol=1e-13)
    np.testing.assert_allclose(Pd.sum(1), 0.0, atol=1e-11)
    np.testing.assert_allclose(Pdd.sum(1), 0.0, atol=1e-9)
    # linear precision: coefficients m/n reproduce tau; derivative 1/T, second 0
    lin = np.arange(n + 1) / n
    np.testing.assert_allclose(P @ lin, tau, atol=1e-13)
    np.testing.assert_allclose(Pd @ lin, 1.0 / T, atol=1e-11)
    np.testing.assert_allclose(Pdd @ lin, 0.0, atol=1e-9)
    # endpoint interpolation
    e0 = np.zeros(n + 1); e0[0] = 1
    en = np.zeros(n + 1); en[-1] = 1
    np.testing.assert_allclose(P[0], e0, atol=1e-15)
    np.testing.assert_allclose(P[-1], en, atol=1e-15)


def test_basis_against_de_casteljau_and_differences():
    n, n_p, T = 10, 37, 7.0
    P, Pd, Pdd = oracle.bernstein(n, n_p, T)
    rng = np.random.default_rng(3)
    c = rng.normal(size=n + 1)
    h = 1e-4
    for k in range(1, n_p - 1):
        t = k * T / (n_p - 1)
        f = lambda tt: de_casteljau(c, tt / T)
        assert abs(P[k] @ c - f(t)) < 1e-12
        d1 = (f(t + h) - f(t - h)) / (2 * h)
        d2 = (f(t + h) - 2 * f(t) + f(t - h)) / (h * h)
        assert abs(Pd[k] @ c - d1) < 1e-6 * max(1, abs(d1))
        assert abs(Pdd[k] @ c - d2) < 1e-3 * max(1, abs(d2))


# ------------------------------------------------------------ fixed matrices


def test_boundary_rows_structure_and_closed_form():
    pr = oracle.problem(2, 10, 100, 10.0, 1.5, 2.0, 1.0, 10)
    A, H = oracle.constraint_matrices(pr)
    n = pr.degree
    nz = [set(np.nonzero(np.abs(A[r]) > 0)[0]) for r in range(4)]
    assert nz == [{0}, {0, 1}, {0, 1, 2}, {n}]
    # boundary values reached exactly by the hand-derived coefficients
    T = pr.horizon
    x0, v0, a0, xf = 1.25, -0.5, 0.75, 7.0
    xi = np.zeros(n + 1)
    xi[0] = x0
    xi[1] = x0 + v0 * T / n
    xi[2] = x0 + 2 * v0 * T / n + a0 * T * T / (n * (n - 1))
    xi[n] = xf
    np.testing.assert_allclose(A @ xi, [x0, v0, a0, xf], atol=1e-12)


@pytest.mark.parametrize("use_v,use_a,n_obs", [(True, True, 10), (True, False, 3),
                                                (False, False, 0), (False, True, 50)])
def test_H_equals_stacked_F(use_v, use_a, n_obs):
    pr = oracle.problem(2, 10, 40, 10.0, 1.5 if use_v else 0.0, 2.0 if use_a else -1.0,
                        0.7, n_obs)
    A, H = oracle.constraint_matrices(pr)
    P, Pd, Pdd = oracle.bernstein(10, 40, 10.0)
    F = stacked_F(P, Pd, Pdd, n_obs, use_v, use_a)
    np.testing.assert_allclose(H, np.eye(11) + 0.7 * F.T @ F, rtol=1e-12, atol=1e-9)


def test_kkt_lu_vs_nullspace_vs_numpy_and_stationarity():
    pr = oracle.problem(3, 15, 150, 20.0, 1.5, 2.0, 1.0, 200)
    rng = np.random.default_rng(5)
    K = oracle.kkt_matrix(pr)
    A, H = oracle.constraint_matrices(pr)
    for _ in range(5):
        q = rng.normal(size=16) * 100
        b = rng.normal(size=4)
        x1 = oracle.kkt_solve(pr, q, b)
        x2 = oracle.qp_nullspace(pr, q, b)
        x3 = np.linalg.solve(K, np.concatenate([q, b]))[:16]
        scale = np.abs(x1).max()
        assert np.abs(x1 - x2).max() <= 1e-12 * max(scale, 1) * 100
        assert np.abs(x1 - x3).max() <= 1e-12 * max(scale, 1) * 100
        np.testing.assert_allclose(A @ x1, b, atol=1e-10)
        # stationarity: H x - q lies in range(A^T)
        g = H @ x1 - q
        nu = np.linalg.lstsq(A.T, -g, rcond=None)[0]
        assert np.abs(g + A.T @ nu).max() <= 1e-10 * np.abs(q).max()


def test_no_F_rows_gives_overwrite_projection():
    """With no obstacles and no kinematic blocks F is empty: one QP is the Euclidean
    projection onto {A xi = b}, i.e. the sample with its 4 boundary coefficients
    overwritten."""
    w = wl.tiny(dims=2, batch=4, n_obs=0)
    w.v_max = 0.0
    w.a_max = 0.0
    xb, lam, tr, _ = oracle.project(w, iters=1)
    n, T = w.degree, w.horizon
    for i in range(w.batch):
        for ax in range(2):
            x0, v0, a0, xf = w.boundary[ax]
            exp = w.xi[i, ax].copy()
            exp[0] = x0
            exp[1] = x0 + v0 * T / n
            exp[2] = x0 + 2 * v0 * T / n + a0 * T * T / (n * (n - 1))
            exp[n] = xf
            np.testing.assert_allclose(xb[i, ax], exp, atol=1e-12)
    assert np.all(tr == 0) and np.all(lam == 0)


# --------------------------------------------------------------- polar steps


def test_polar_golden_by_hand():
    g = json.load(open(os.path.join(GOLD, "polar_worked_examples.json")))
    for c in g["obstacle"]:
        al, be, d, off = oracle.polar_obstacle(c["xt"], c["s"])
        assert abs(al - c["alpha"]) < 1e-15
        if "beta" in c:
            assert abs(be - c["beta"]) < 1e-15
        assert abs(d - c["d"]) < 1e-15
        np.testing.assert_allclose(off, c["offset"], atol=1e-15)
    for c in g["bound"]:
        np.testing.assert_allclose(oracle.polar_bound(c["v"], c["bound"]), c["e"], atol=1e-15)


def test_polar_circle_is_exact_projection_bruteforce():
    """Over a fine grid of angles (and the exact best d >= 1 for each angle) no point
    s.d.dir(alpha) is closer to x~ than the closed form's."""
    rng = np.random.default_rng(11)
    al_grid = np.linspace(-np.pi, np.pi, 100001)
    for _ in range(40):
        r = rng.uniform(0.3, 1.0)
        xt = rng.uniform(-1.5, 1.5, size=2)
        _, _, d, off = oracle.polar_obstacle(xt, [r, r])
        best_closed = np.linalg.norm(xt - off)
        dirs = np.stack([np.cos(al_grid), np.sin(al_grid)], 1)
        dstar = np.maximum(1.0, dirs @ xt / r)
        dist = np.linalg.norm(xt[None] - r * dstar[:, None] * dirs, axis=1)
        assert best_closed <= dist.min() + 1e-12
        # a grid angle misses the exact one by at most h/2: first order off the ray
        assert dist.min() <= best_closed + np.linalg.norm(xt) * (al_grid[1] - al_grid[0])
        # characterization: e = p outside, nearest surface point inside
        nx = np.linalg.norm(xt)
        exp = xt if nx >= r else r * xt / nx
        np.testing.assert_allclose(off, exp, atol=1e-12)


def test_polar_sphere_is_exact_projection_bruteforce():
    rng = np.random.default_rng(12)
    a = np.linspace(-np.pi, np.pi, 721)
    b = np.linspace(0, np.pi, 361)
    A_, B_ = np.meshgrid(a, b, indexing="ij")
    dirs = np.stack([np.cos(A_) * np.sin(B_), np.sin(A_) * np.sin(B_), np.cos(B_)], -1)
    dirs = dirs.reshape(-1, 3)
    h = a[1] - a[0]
    for _ in range(15):
        r = rng.uniform(0.3, 1.0)
        xt = rng.uniform(-1.2, 1.2, size=3)
        _, _, d, off = oracle.polar_obstacle(xt, [r, r, r])
        best = np.linalg.norm(xt - off)
        dstar = np.maximum(1.0, dirs @ xt / r)
        dist = np.linalg.norm(xt[None] - r * dstar[:, None] * dirs, axis=1)
        assert best <= dist.min() + 1e-12
        assert dist.min() <= best + 2 * h * np.linalg.norm(xt)


def test_polar_ellipsoid_properties():
    rng = np.random.default_rng(13)
    for D in (2, 3):
        for _ in range(200):
            s = rng.uniform(0.3, 1.0, size=D)
            xt = rng.uniform(-1.5, 1.5, size=D)
            _, _, d, off = oracle.polar_obstacle(xt, s)
            rn = np.linalg.norm(xt / s)
            if rn >= 1:
                np.testing.assert_allclose(off, xt, atol=1e-12)   # feasible: zero residual
            else:
                assert abs(np.linalg.norm(off / s) - 1.0) < 1e-12  # pushed onto the surface
                # along the ray from the centre through the point
                assert abs(np.dot(off, xt) - np.linalg.norm(off) * np.linalg.norm(xt)) < 1e-12
        # equal semi-axes reduce to the circle/sphere characterization
        r = 0.55
        xt = rng.uniform(-0.3, 0.3, size=D)
        _, _, _, off = oracle.polar_obstacle(xt, [r] * D)
        np.testing.assert_allclose(off, r * xt / np.linalg.norm(xt), atol=1e-12)


def test_polar_bound_is_ball_projection_bruteforce():
    rng = np.random.default_rng(14)
    al = np.linspace(-np.pi, np.pi, 20001)
    dirs = np.stack([np.cos(al), np.sin(al)], 1)
    for _ in range(40):
        bound = rng.uniform(0.5, 2.0)
        v = rng.normal(size=2) * 2
        e = oracle.polar_bound(v, bound)
        nv = np.linalg.norm(v)
        exp = v if nv <= bound else bound * v / nv
        np.testing.assert_allclose(e, exp, atol=1e-12)
        dstar = np.clip(dirs @ v / bound, 0.0, 1.0)
        dist = np.linalg.norm(v[None] - bound * dstar[:, None] * dirs, axis=1)
        assert np.linalg.norm(v - e) <= dist.min() + 1e-12
    for _ in range(20):
        bound = rng.uniform(0.5, 2.0)
        v = rng.normal(size=3) * 2
        nv = np.linalg.norm(v)
        exp = v if nv <= bound else bound * v / nv
        np.testing.assert_allclose(oracle.polar_bound(v, bound), exp, atol=1e-12)


# ----------------------------------------------------------- whole iteration


def feasible_workload():
    """A straight, slow, boundary-consistent line far from every obstacle."""
    w = wl.tiny(dims=2, batch=2, n_obs=2)
    w.obs_centre = np.array([[2.0, 3.0], [1.0, -4.0]])
    w.obs_axes = np.full((2, 2), 0.5)
    w.obs_vel = np.zeros((2, 2))
    n = w.degree
    line = np.stack([np.linspace(0, 4, n + 1), np.zeros(n + 1)])
    w.xi = np.stack([line, line])
    # boundary rows consistent with the line: constant speed 4 m / T along x
    w.boundary = np.array([[0.0, 4.0 / w.horizon, 0.0, 4.0], [0.0, 0.0, 0.0, 0.0]])
    return w


def test_feasible_sample_is_fixed_point():
    w = feasible_workload()
    xb, lam, tr, _ = oracle.project(w, iters=3)
    np.testing.assert_allclose(xb, w.xi, atol=1e-10)
    assert np.abs(lam).max() < 1e-10
    assert tr.max() < 1e-10


def test_obstacle_free_converges_to_overwrite_at_closed_form_rate():
    w = wl.tiny(dims=2, batch=3, n_obs=0)
    w.v_max = 1e6
    w.a_max = 1e6
    n, T = w.degree, w.horizon
    P, Pd, Pdd = oracle.bernstein(n, w.n_steps, T)
    F = stacked_F(P, Pd, Pdd, 0)
    H = np.eye(n + 1) + w.rho * F.T @ F
    free = list(range(3, n))
    lam_max = np.linalg.eigvalsh(H[np.ix_(free, free)]).max()
    rate = 1 - 1 / lam_max
    target = w.xi.copy()
    for ax in range(2):
        x0, v0, a0, xf = w.boundary[ax]
        target[:, ax, 0] = x0
        target[:, ax, 1] = x0 + v0 * T / n
        target[:, ax, 2] = x0 + 2 * v0 * T / n + a0 * T * T / (n * (n - 1))
        target[:, ax, n] = xf
    xb = w.xi.copy()
    lam = np.zeros_like(xb)
    errs = []
    for k in range(60):
        xb, lam, tr, _ = oracle.project(w, xi_bar=xb, lam=lam, iters=1)
        errs.append(np.linalg.norm((xb - target).reshape(3, -1), axis=1))
    errs = np.array(errs)
    for k in range(1, len(errs) - 1):
        assert np.all(errs[k + 1] <= rate * errs[k] + 1e-13)
    assert np.abs(lam).max() < 1e-12


def _one_circle_grazing(batch=1, n_steps=60):
    w = wl.tiny(dims=2, batch=batch, n_obs=1, n_steps=n_steps)
    w.obs_centre = np.array([[2.0, 0.3]])
    w.obs_axes = np.array([[0.5, 0.5]])
    w.obs_vel = np.zeros((1, 2))
    n = w.degree
    line = np.stack([np.linspace(0, 4, n + 1), np.zeros(n + 1)])
    w.xi = np.repeat(line[None], batch, 0)
    return w


def test_frozen_lambda_objective_non_increasing():
    """With lam = 0 every AM block is an exact minimization of
    J = 1/2|xb - xi|^2 + rho/2 |F xb - e|^2 (circles), so J(xb^k, e^{k+1}) cannot grow
    once xb satisfies the boundary rows (k >= 1)."""
    for seed in (1, 2, 3):
        w = wl.tiny(dims=2, batch=4, n_obs=3, seed=seed, n_steps=30)
        xb = w.xi.copy()
        lam = np.zeros_like(xb)
        J = []
        for k in range(25):
            xnew, lam, tr, _ = oracle.project(w, xi_bar=xb, lam=lam, iters=1,
                                              freeze_lambda=True)
            J.append(0.5 * np.sum((xb - w.xi) ** 2, axis=(1, 2)) + 0.5 * w.rho * tr[0] ** 2)
            xb = xnew
        J = np.array(J)
        assert np.all(J[2:] <= J[1:-1] + 1e-10)


def test_worked_case_residual_non_increasing_and_small():
    """One circle (centre (2, 0.3), r 0.5) grazing the straight line y = 0.  Chosen in
    advance as an empirical check: the residual decreases monotonically until it first
    vanishes (rounding level).  The multiplier then keeps pulling xb towards xi + lam,
    so the residual can rise again for a while (a primal-dual transient of the
    augmented Lagrangian); after enough iterations it is back at rounding level."""
    w = _one_circle_grazing()
    xb, lam, tr, _ = oracle.project(w, iters=400)
    res = tr[:, 0]
    first = int(np.argmax(res <= 1e-12))
    assert res[first] <= 1e-12 and first <= 40
    assert np.all(res[1:first + 1] <= res[:first] + 1e-12)
    assert np.all(res[-100:] <= 1e-12)
    r_final, _ = oracle.residuals(w, xb)
    assert r_final[0] < 1e-12


def test_tie_case_line_through_centre_stays_on_axis():
    """Symmetric case: the straight line passes through the obstacle centre.  Every
    push is along +-x, so the y coefficients stay zero up to the rounding of
    sin(pi) in the angle form (deterministic tie)."""
    w = _one_circle_grazing()
    w.obs_centre = np.array([[2.0, 0.0]])
    xb, lam, tr, _ = oracle.project(w, iters=20)
    assert np.abs(xb[:, 1, :]).max() < 1e-9
    assert np.abs(lam[:, 1, :]).max() < 1e-9
    assert np.abs(xb[:, 0, :] - w.xi[:, 0, :]).max() > 0.1   # x was pushed


def _algebraic_residual_products(w, xb_one):
    """F^T r by an independent route: explicit stacked F, and e from the
    characterization of the projections (nearest surface point / ball clip)."""
    P, Pd, Pdd = oracle.bernstein(w.degree, w.n_steps, w.horizon)
    F = stacked_F(P, Pd, Pdd, w.n_obs)
    t = np.arange(w.n_steps) * w.horizon / (w.n_steps - 1)
    out = np.zeros_like(xb_one)
    pos = P @ xb_one.T
    vel = Pd @ xb_one.T
    acc = Pdd @ xb_one.T
    def clip(v, bnd):
        nv = np.linalg.norm(v, axis=1, keepdims=True)
        return np.where(nv > bnd, v * bnd / np.maximum(nv, 1e-300), v)
    ev, ea = clip(vel, w.v_max), clip(acc, w.a_max)
    for ax in range(w.dims):
        e_parts = []
        for j in range(w.n_obs):
            c = w.obs_centre[j] + t[:, None] * w.obs_vel[j]
            xt = pos - c
            r = w.obs_axes[j, 0]
            nx = np.linalg.norm(xt, axis=1, keepdims=True)
            e = np.where(nx >= r, pos, c + r * xt / nx)
            e_parts.append(e[:, ax])
        e_parts += [ev[:, ax], ea[:, ax]]
        evec = np.concatenate(e_parts)
        out[ax] = F.T @ (F @ xb_one[ax] - evec)
    return out


def test_multiplier_telescopes():
    w = wl.tiny(dims=2, batch=2, n_obs=3, seed=4, n_steps=25)
    xb = w.xi.copy()
    lam = np.zeros_like(xb)
    total = np.zeros_like(xb)
    for k in range(12):
        for i in range(w.batch):
            total[i] += _algebraic_residual_products(w, xb[i])
        xb, lam, _, _ = oracle.project(w, xi_bar=xb, lam=lam, iters=1)
    np.testing.assert_allclose(lam, -w.rho * total, atol=1e-9)


def test_batch_and_thread_invariance():
    w = wl.config1(batch=6)
    a = oracle.project(w, iters=5, n_threads=1)
    b = oracle.project(w, iters=5, n_threads=4)
    c = oracle.project(w.subset(3), iters=5, n_threads=2)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    np.testing.assert_array_equal(a[0][:3], c[0])


def _golden_two_iterates():
    from fractions import Fraction
    with open(os.path.join(GOLD, "am_two_iterates.json")) as f:
        g = json.load(f)
    pr = g["problem"]
    w = wl.tiny(dims=2, batch=1, n_obs=1, degree=pr["degree"], n_steps=pr["n_steps"])
    w.horizon = pr["horizon"]
    w.v_max, w.a_max, w.rho = pr["v_max"], pr["a_max"], pr["rho"]
    w.obs_centre = np.array(pr["obs_centre"], dtype=np.float64)
    w.obs_axes = np.array(pr["obs_axes"], dtype=np.float64)
    w.obs_vel = np.zeros((1, 2))
    w.boundary = np.array(pr["boundary"], dtype=np.float64)
    xi = np.zeros((1, 2, pr["degree"] + 1))
    xi[0, 0] = pr["xi_x"]
    w.xi = xi
    fr = lambda v: float(Fraction(v))
    return w, g, fr


def test_two_iterates_golden_by_hand():
    """The first two iterates of a tiny one-obstacle problem (degree 4, five time
    samples, a point inside the circle at k = 0 and k = 1), worked by hand in exact
    rational arithmetic: waypoints, residual, multiplier lambda^{k+1} = lambda^k - rho
    F^T r^k (eq lag) and the QP taking that fresh multiplier (eqs affine_trans /
    matrix_vec, the AM step list's order).  The QP's value with lambda^k instead is
    recorded beside it and must not match."""
    w, g, fr = _golden_two_iterates()
    xb = w.xi.copy()
    lam = np.zeros_like(xb)
    P, _, _ = oracle.bernstein(w.degree, w.n_steps, w.horizon)
    for it, want in enumerate(g["iterates"]):
        np.testing.assert_allclose(P @ xb[0, 0], [fr(v) for v in want["waypoints_x"]],
                                   atol=1e-14)
        xb, lam, tr, _ = oracle.project(w, xi_bar=xb, lam=lam, iters=1)
        assert abs(tr[0, 0] ** 2 - fr(want["residual_sq"])) <= 1e-14
        np.testing.assert_allclose(xb[0, 0], [fr(v) for v in want["xi_bar_x"]], atol=1e-13)
        np.testing.assert_allclose(lam[0, 0], [fr(v) for v in want["lambda_x"]], atol=1e-13)
        assert np.abs(xb[0, 1]).max() < 1e-13 and np.abs(lam[0, 1]).max() < 1e-13
        wrong = [fr(v) for v in g["wrong_order"][it]["xi_bar_x"]]
        if it == 0:
            assert abs(xb[0, 0, 3] - wrong[3]) > 1e-3
    # the same two iterates in one call
    xb2, lam2, tr2, _ = oracle.project(w, iters=2)
    np.testing.assert_array_equal(xb2, xb)
    np.testing.assert_array_equal(lam2, lam)


def test_qp_stationarity_takes_fresh_multiplier():
    """KKT stationarity of the QP of one iteration (eqs affine_trans / matrix_vec) with
    the multiplier of eq lag from the same iteration: on the free coefficients, where
    the boundary rows' A^T nu vanishes,
        lambda^{k+1}_f = (xb^{k+1} - xi)_f + rho [F^T F xb^{k+1} - F^T e^{k+1}]_f,
    with F stacked explicitly and F^T e^{k+1} = F^T F xb^k - F^T r^k taken from the
    characterization of the polar projections (independent of the oracle's angle
    form).  Starts from a non-zero multiplier and a state that meets the boundary."""
    w = wl.tiny(dims=2, batch=2, n_obs=3, seed=9, n_steps=25)
    P, Pd, Pdd = oracle.bernstein(w.degree, w.n_steps, w.horizon)
    F = stacked_F(P, Pd, Pdd, w.n_obs)
    FtF = F.T @ F
    xb0, lam0, _, _ = oracle.project(w, iters=3)
    assert np.abs(lam0).max() > 1e-3
    xb1, lam1, _, _ = oracle.project(w, xi_bar=xb0, lam=lam0, iters=1)
    free = list(range(3, w.degree))
    for i in range(w.batch):
        ftr0 = _algebraic_residual_products(w, xb0[i])
        assert np.abs(ftr0).max() > 1e-3
        for ax in range(w.dims):
            fte1 = FtF @ xb0[i, ax] - ftr0[ax]
            stat = (xb1[i, ax] - w.xi[i, ax]) + w.rho * (FtF @ xb1[i, ax] - fte1)
            np.testing.assert_allclose(lam1[i, ax, free], stat[free], atol=1e-10)
            np.testing.assert_allclose(lam1[i, ax], lam0[i, ax] - w.rho * ftr0[ax], atol=1e-10)


# ------------------------------------------------------------- mutation tests


def _pins_pass():
    """The cheap pins, as one predicate: True when all hold."""
    try:
        test_feasible_sample_is_fixed_point()
        test_multiplier_telescopes()
        test_polar_circle_is_exact_projection_bruteforce()
        test_worked_case_residual_non_increasing_and_small()
        test_two_iterates_golden_by_hand()
        test_qp_stationarity_takes_fresh_multiplier()
    except AssertionError:
        return False
    return True


@pytest.mark.parametrize("fault", [1, 2, 3, 4, 5, 8])
def test_planted_mistakes_are_caught(fault):
    """Each plausible mistake (printed sign of rho F^T e, a dropped kinematic term,
    reversed basis columns, a flipped multiplier sign, a dropped d >= 1 bound, the QP
    taking lambda^k instead of the fresh lambda^{k+1}) planted in the oracle makes at
    least one pin fail."""
    assert _pins_pass()
    oracle.set_fault(fault)
    try:
        assert not _pins_pass()
    finally:
        oracle.set_fault(0)


def test_stale_multiplier_fault_is_caught_by_the_order_pins():
    """The step-order mistake (the QP reads lambda^k) passes the older pins, so each of
    the two order pins must catch it on its own."""
    oracle.set_fault(8)
    try:
        for pin in (test_two_iterates_golden_by_hand, test_qp_stationarity_takes_fresh_multiplier):
            with pytest.raises(AssertionError):
                pin()
    finally:
        oracle.set_fault(0)
