"""Pins of the heading / multi-circle oracle (oracle/heading.py) to what Paper II and the
mathematics fix, independently of its own matrices:

* step 1 and step 2 are the minimisers of the printed objectives (reform_formulation
  restricted to xi, and eq compute_convex_surrogate), written here as sums over the time
  steps with scipy's own Bernstein polynomials and minimised exactly over the affine set
  of the boundary rows (a quadratic's Hessian from exact central differences);
* the polar steps are the brute-force minimisers of eqs compute_zeta_33 .. compute_da;
* without obstacles the desired constant-velocity line is reached (closed form), and the
  line with a level heading is a fixed point of the iteration;
* the iteration is covariant under a mirror about the x axis, a translation and (for
  circular obstacles) a rotation of the whole scene, which fixes the signs and the
  sin / cos pairings of every row and of the heading coupling r_m (cos psi, sin psi).
"""
import dataclasses

import numpy as np
import pytest
import scipy.interpolate as si
import scipy.linalg as sl

from oracle import heading as oh
from paper_2408_10731_amd import workloads as wl


def tiny(seed=0, n_obs=2, n_c=2, batch=3, degree=5, n_steps=12, flow="static"):
    w = wl.heading_scene(seed, n_obs=n_obs, n_circles=n_c, batch=batch, flow=flow,
                         degree=degree, n_steps=n_steps)
    rng = np.random.default_rng(seed + 100)
    # obstacles near the line so that several collision rows are active
    if n_obs:
        w.obs_centre[:, 0] = rng.uniform(5.0, 15.0, n_obs)
        w.obs_centre[:, 1] = rng.uniform(-0.5, 0.5, n_obs)
        w.obs_axes[:] = rng.uniform(0.5, 1.5, (n_obs, 2))
    return w


def bpoly(coef, T, nu=0):
    """Values (or the nu-th derivative) at the time steps of the Bernstein polynomial with
    coefficients coef on [0, T], by scipy."""
    p = si.BPoly(np.asarray(coef, dtype=np.float64)[:, None], [0.0, T])
    return p.derivative(nu) if nu else p


def quad_min(J, Aeq, beq, n):
    """Exact minimiser of a quadratic J over {z : Aeq z = beq}."""
    z0 = np.linalg.lstsq(Aeq, beq, rcond=None)[0]
    Z = sl.null_space(Aeq)
    k = Z.shape[1]
    f = lambda u: J(z0 + Z @ u)
    h = 1.0
    H = np.zeros((k, k))
    g = np.zeros(k)
    E = np.eye(k) * h
    f0 = f(np.zeros(k))
    for i in range(k):
        g[i] = (f(E[i]) - f(-E[i])) / (2 * h)
        for j in range(i, k):
            H[i, j] = H[j, i] = (f(E[i] + E[j]) - f(E[i] - E[j]) - f(-E[i] + E[j]) + f(-E[i] - E[j])) / (4 * h * h)
    u = np.linalg.solve(H, -g)
    return z0 + Z @ u


def boundary_rows(w, n_v):
    T = w.horizon
    rows = []
    for nu, t in ((0, 0.0), (1, 0.0), (2, 0.0), (0, T)):
        rows.append(np.array([bpoly(np.eye(n_v)[k], T, nu)(t) for k in range(n_v)]))
    return np.array(rows)


def test_xi_step_minimises_the_printed_objective():
    w = tiny(1)
    ops = oh.operators(w)
    T, t, nv, rho = w.horizon, ops.t, w.n_v, w.rho
    rng = np.random.default_rng(7)
    xi0 = w.xi0[0]
    pol = oh.polar_step(w, ops, xi0[:4], xi0[4])
    gx, gy = oh.g_vectors(w, ops, pol)
    lam = rng.normal(0.0, 2.0, (4, nv))
    got = oh.xi_step(w, ops, lam, gx, gy)
    xo, yo = w.obs_centre[:, 0:1] + w.obs_vel[:, 0:1] * t, w.obs_centre[:, 1:2] + w.obs_vel[:, 1:2] * t
    a, b = w.obs_axes[:, 0], w.obs_axes[:, 1]
    psi = bpoly(xi0[4], T)(t)

    def J(z):   # z = (xi_x, xi_c, xi_y, xi_s), the objective summed over the time steps
        cx, cc, cy, cs = z.reshape(4, nv)
        x, y, c, s = (bpoly(v, T)(t) for v in (cx, cy, cc, cs))
        vx, vy = bpoly(cx, T, 1)(t), bpoly(cy, T, 1)(t)
        ax, ay = bpoly(cx, T, 2)(t), bpoly(cy, T, 2)(t)
        cost = 0.5 * np.sum(ax ** 2 + ay ** 2 + (x - w.x_des[0]) ** 2 + (y - w.x_des[1]) ** 2)
        cost -= np.sum(lam.reshape(-1) * z)
        pen = np.sum((vx - pol["d_v"] * w.v_max * np.cos(pol["al_v"])) ** 2
                     + (vy - pol["d_v"] * w.v_max * np.sin(pol["al_v"])) ** 2)
        pen += np.sum((ax - pol["d_a"] * w.a_max * np.cos(pol["al_a"])) ** 2
                      + (ay - pol["d_a"] * w.a_max * np.sin(pol["al_a"])) ** 2)
        for m, r in enumerate(w.radii):
            for j in range(w.n_obs):
                d, al = pol["d_o"][m, j], pol["al_o"][m, j]
                pen += np.sum((x + r * c - xo[j] - a[j] * d * np.cos(al)) ** 2
                              + (y + r * s - yo[j] - b[j] * d * np.sin(al)) ** 2)
        pen += np.sum((c - np.cos(psi)) ** 2 + (s - np.sin(psi)) ** 2)
        return cost + 0.5 * rho * pen

    Ab = boundary_rows(w, nv)
    Aeq = np.zeros((8, 4 * nv))
    Aeq[0:4, 0:nv] = Ab
    Aeq[4:8, 2 * nv:3 * nv] = Ab
    beq = np.concatenate([w.boundary[0], w.boundary[1]])
    ref = quad_min(J, Aeq, beq, 4 * nv).reshape(4, nv)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-7 * max(1.0, np.abs(ref).max()))


def test_psi_step_minimises_the_surrogate():
    w = tiny(2)
    ops = oh.operators(w)
    T, t, nv, rho = w.horizon, ops.t, w.n_v, w.rho
    rng = np.random.default_rng(8)
    lam_psi = rng.normal(0.0, 1.0, nv)
    target = rng.normal(0.0, 0.5, w.n_steps)
    got = oh.psi_step(w, ops, lam_psi, target)

    def J(z):
        return (0.5 * np.sum(bpoly(z, T, 2)(t) ** 2) - lam_psi @ z
                + 0.5 * rho * np.sum((target - bpoly(z, T)(t)) ** 2))

    Aeq = np.array([[bpoly(np.eye(nv)[k], T)(tt) for k in range(nv)] for tt in (0.0, T)])
    ref = quad_min(J, Aeq, w.boundary_psi, nv)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-8 * max(1.0, np.abs(ref).max()))


def test_psi_target_is_atan2_on_the_nearest_branch():
    w = tiny(3)
    ops = oh.operators(w)
    rng = np.random.default_rng(9)
    xi = rng.normal(0.0, 1.0, (4, w.n_v))
    prev = rng.uniform(-10.0, 10.0, w.n_steps)
    pt = oh.psi_target(ops, xi, prev)
    c, s = bpoly(xi[1], w.horizon)(ops.t), bpoly(xi[3], w.horizon)(ops.t)
    np.testing.assert_allclose(np.cos(pt), c / np.hypot(c, s), atol=1e-12)
    np.testing.assert_allclose(np.sin(pt), s / np.hypot(c, s), atol=1e-12)
    assert np.all(np.abs(pt - prev) <= np.pi + 1e-12)


def test_polar_steps_are_brute_force_minimisers():
    """Collision rows with circles (a = b: the scaled angle is the exact minimiser),
    velocity and acceleration rows: the printed objectives minimised on a fine grid of
    angles (d in closed form per angle, then clipped to its bound)."""
    w = tiny(4, n_obs=3, n_c=3)
    w.obs_axes[:] = np.array([[0.7, 0.7], [1.1, 1.1], [0.4, 0.4]])
    w.v_max, w.a_max = 1.2, 0.05
    ops = oh.operators(w)
    xi = w.xi0[1]
    T, t = w.horizon, ops.t
    x, y, psi = bpoly(xi[0], T)(t), bpoly(xi[2], T)(t), bpoly(xi[4], T)(t)
    # obstacle 0 sits on the path at step 6, so the bound d >= 1 is active there
    w.obs_centre[0] = (x[6] + 0.1, y[6] - 0.05)
    w.obs_vel[0] = 0.0
    pol = oh.polar_step(w, ops, xi[:4], xi[4])
    assert pol["d_o"].min() >= 1.0 and pol["d_o"][:, 0, 6].min() == 1.0
    ang = np.linspace(-np.pi, np.pi, 200001)
    ca, sa = np.cos(ang), np.sin(ang)

    def brute(u, v, scale, lo, hi):
        d = np.clip((u * ca + v * sa) / scale, lo, hi)
        f = (u - scale * d * ca) ** 2 + (v - scale * d * sa) ** 2
        i = np.argmin(f)
        return f[i], ang[i], d[i]

    for k in range(0, w.n_steps, 3):
        for m, r in enumerate(w.radii):
            for j in range(w.n_obs):
                a = w.obs_axes[j, 0]
                u = x[k] + r * np.cos(psi[k]) - (w.obs_centre[j, 0] + w.obs_vel[j, 0] * t[k])
                v = y[k] + r * np.sin(psi[k]) - (w.obs_centre[j, 1] + w.obs_vel[j, 1] * t[k])
                fb, ab, db = brute(u, v, a, 1.0, np.inf)
                al, d = pol["al_o"][m, j, k], pol["d_o"][m, j, k]
                f = (u - a * d * np.cos(al)) ** 2 + (v - a * d * np.sin(al)) ** 2
                assert f <= fb + 1e-9 and abs(d - db) < 1e-4
        for nu, key, bound in ((1, "v", w.v_max), (2, "a", w.a_max)):
            u, v = bpoly(xi[0], T, nu)(t[k]), bpoly(xi[2], T, nu)(t[k])
            fb, _, db = brute(u, v, bound, 0.0, 1.0)
            al, d = pol["al_" + key][k], pol["d_" + key][k]
            f = (u - bound * d * np.cos(al)) ** 2 + (v - bound * d * np.sin(al)) ** 2
            assert f <= fb + 1e-9 and abs(d - db) < 1e-4


def test_without_obstacles_the_desired_line_is_reached():
    """No obstacles and velocity / acceleration bounds that the line keeps: the tracking
    QP's minimiser is the desired constant-velocity line itself (zero tracking error and
    zero acceleration), and every boundary row holds after every iteration."""
    w = wl.heading_scene(4, n_obs=0, n_circles=4, batch=3)
    st, _, tr = oh.iterate(w, 200)
    ops = oh.operators(w)
    assert np.abs(ops.P @ st[:, 0].T - w.x_des[0][:, None]).max() <= 1e-9
    assert np.abs(ops.P @ st[:, 2].T - w.x_des[1][:, None]).max() <= 1e-9
    psi = ops.P @ st[:, 4].T
    np.testing.assert_allclose(ops.P @ st[:, 1].T, np.cos(psi), atol=1e-4)
    np.testing.assert_allclose(ops.P @ st[:, 3].T, np.sin(psi), atol=1e-4)
    assert tr[-1].max() < 1e-4
    for k in (1, 7, 50):
        s_k, _, _ = oh.iterate(w, k)
        for grp in range(2):
            assert np.abs(ops.A[:, :w.n_v] @ s_k[:, 2 * grp].T - w.boundary[grp][:, None]).max() <= 1e-9
        assert np.abs(ops.Apsi @ s_k[:, 4].T - w.boundary_psi[:, None]).max() <= 1e-10


def test_the_line_with_level_heading_is_a_fixed_point():
    w = wl.heading_scene(5, n_obs=0, n_circles=3, batch=1)
    nv = w.n_v
    st = np.zeros((1, 5, nv))
    st[0, 0] = np.linspace(0.0, 20.0, nv)
    st[0, 1] = 1.0
    st2, lam2, tr = oh.iterate(w, 5, state=st)
    np.testing.assert_allclose(st2, st, atol=1e-11)
    assert np.abs(lam2).max() < 1e-10 and tr.max() < 1e-10


def _mirror(w):
    m = dataclasses.replace(w)
    m.obs_centre = w.obs_centre * [1, -1]
    m.obs_vel = w.obs_vel * [1, -1]
    m.boundary = w.boundary * np.array([[1.0], [-1.0]])
    m.boundary_psi = -w.boundary_psi
    m.x_des = w.x_des * np.array([[1.0], [-1.0]])
    m.xi0 = w.xi0 * np.array([1, 1, -1, -1, -1])[None, :, None]
    return m


def test_mirror_about_the_x_axis():
    w = tiny(6, n_obs=3, n_c=3, flow="same")
    w.obs_axes[:, 1] = w.obs_axes[:, 0] * 0.7      # ellipses: a mirror keeps them
    a, la, ta = oh.iterate(w, 12)
    b, lb, tb = oh.iterate(_mirror(w), 12)
    sign = np.array([1, 1, -1, -1, -1])[None, :, None]
    np.testing.assert_allclose(b, a * sign, atol=1e-9)
    np.testing.assert_allclose(lb, la * sign, atol=1e-8)
    np.testing.assert_allclose(tb, ta, atol=1e-9)


def test_translation():
    w = tiny(7, n_obs=3, n_c=2, flow="opposite")
    d = np.array([3.5, -2.25])
    v = dataclasses.replace(w)
    v.obs_centre = w.obs_centre + d
    v.boundary = w.boundary.copy()
    v.boundary[:, 0] += d
    v.boundary[:, 3] += d
    v.x_des = w.x_des + d[:, None]
    v.xi0 = w.xi0.copy()
    v.xi0[:, 0] += d[0]
    v.xi0[:, 2] += d[1]
    a, la, ta = oh.iterate(w, 10)
    b, lb, tb = oh.iterate(v, 10)
    a[:, 0] += d[0]
    a[:, 2] += d[1]
    np.testing.assert_allclose(b, a, atol=1e-8)
    np.testing.assert_allclose(tb, ta, atol=1e-8)


def test_rotation_with_circular_obstacles():
    """Rotating positions, velocities, the desired path, the obstacles and (c, s) by phi
    and adding phi to the heading leaves every residual unchanged and rotates the result."""
    w = tiny(8, n_obs=3, n_c=3, flow="same")
    w.obs_axes[:, 1] = w.obs_axes[:, 0]
    phi = 0.6
    R = np.array([[np.cos(phi), -np.sin(phi)], [np.sin(phi), np.cos(phi)]])
    v = dataclasses.replace(w)
    v.obs_centre = w.obs_centre @ R.T
    v.obs_vel = w.obs_vel @ R.T
    v.boundary = R @ w.boundary
    v.boundary_psi = w.boundary_psi + phi
    v.x_des = R @ w.x_des

    def rot(st):
        out = st.copy()
        out[:, [0, 2]] = np.einsum("ij,bjk->bik", R, st[:, [0, 2]])
        out[:, [1, 3]] = np.einsum("ij,bjk->bik", R, st[:, [1, 3]])
        out[:, 4] = st[:, 4] + phi
        return out

    v.xi0 = rot(w.xi0)
    a, la, ta = oh.iterate(w, 10)
    b, lb, tb = oh.iterate(v, 10)
    np.testing.assert_allclose(b, rot(a), atol=1e-8)
    np.testing.assert_allclose(tb, ta, atol=1e-8)


def test_residuals_fall_on_a_crowd():
    """The thesis's convergence figure: both residuals of the best sample fall."""
    w = wl.heading_scene(9, n_obs=30, n_circles=4, batch=6)
    _, _, tr = oh.iterate(w, 60)
    best = np.argmin(tr[-1, :, 0])
    assert tr[-1, best, 0] < 0.5 * tr[0, best, 0]
    assert tr[-1, :, 1].max() < 0.2 * tr[0, :, 1].max()


def test_initial_state_meets_the_boundary_rows():
    """The initialization reading: the coefficients the boundary rows involve are solved
    for (checked with scipy's polynomials), the others are the input's."""
    w = tiny(10)
    ops = oh.operators(w)
    st = w.xi0[0] + 0.3
    out = oh.meet_boundary(w, ops, st)
    T, nv = w.horizon, w.n_v
    for row, grp in ((0, 0), (2, 1)):
        got = [bpoly(out[row], T, nu)(t) for nu, t in ((0, 0.0), (1, 0.0), (2, 0.0), (0, T))]
        np.testing.assert_allclose(got, w.boundary[grp], atol=1e-12)
        np.testing.assert_array_equal(out[row, 3:nv - 1], st[row, 3:nv - 1])
    np.testing.assert_allclose([bpoly(out[4], T)(0.0), bpoly(out[4], T)(T)], w.boundary_psi, atol=1e-12)
    np.testing.assert_array_equal(out[4, 1:nv - 1], st[4, 1:nv - 1])
    np.testing.assert_array_equal(out[[1, 3]], st[[1, 3]])


def test_receding_horizon_cycle_hands_over_the_executed_state():
    """One cycle of the heading MPC oracle: the next start rows are the executed sample's
    position, velocity, acceleration and heading at delta, and the next cycle's samples
    are the results' polynomials moved on by delta (both checked with scipy's
    polynomials); the first cycle is Alg 2 from the input state."""
    w = tiny(11, n_obs=3, n_c=2, batch=4, flow="same")
    T, d = w.horizon, 0.8
    cyc = oh.mpc(w, 2, d, 5)
    first = oh.iterate(w, 5)
    np.testing.assert_array_equal(cyc[0].result, first[0])
    res, i = cyc[0].result, cyc[0].executed
    assert i == int(np.argmin(np.floor(cyc[0].trace[-1, :, 0] / 1e-6)))
    for grp, row in ((0, 0), (1, 2)):
        got = [bpoly(res[i, row], T, nu)(d) for nu in (0, 1, 2)]
        np.testing.assert_allclose(cyc[1].boundary[grp, :3], got, atol=1e-10)
        assert cyc[1].boundary[grp, 3] == w.boundary[grp, 3]
    assert abs(cyc[1].boundary_psi[0] - bpoly(res[i, 4], T)(d)) < 1e-10
    tq = np.linspace(0.0, T - d, 7)
    for b in range(w.batch):
        for r in range(5):
            np.testing.assert_allclose(bpoly(cyc[1].state[b, r], T)(tq), bpoly(res[b, r], T)(tq + d), atol=1e-9)
    # the second cycle is Alg 2 from the shifted samples with the first cycle's multipliers
    wc = dataclasses.replace(w, xi0=cyc[1].state, boundary=cyc[1].boundary, boundary_psi=cyc[1].boundary_psi,
                             obs_centre=w.obs_centre + w.obs_vel * d, x_des=wl.desired_window(w, d))
    again = oh.iterate(wc, 5, state=cyc[1].state, lam=cyc[0].lam)
    np.testing.assert_array_equal(again[0], cyc[1].result)
    np.testing.assert_array_equal(again[1], cyc[1].lam)
