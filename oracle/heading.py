"""FP64 oracle of the heading / multi-circle variant of the batch optimizer (thesis
ch. 5, Paper II: Problem Formulation, the reformulated problem (reform_cost)-(d_bound),
its augmented Lagrangian (reform_formulation) and Alg 2).  TEST INFRASTRUCTURE ONLY:
only tests/, the smoke check and the benchmark's CPU leg may call it.

The robot is a rectangle modelled by n_c circles at offsets r_m on its heading axis;
obstacle j is an axis-aligned ellipse (semi-axes a_j, b_j, inflated by the circles'
radius) moving at constant velocity.  Per sample the variables are the Bernstein
coefficients xi = (xi_x, xi_c, xi_y, xi_s) and xi_psi; c and s are slack copies of
cos psi and sin psi.

The matrices are formed explicitly here (eq Q_matrix and the F / g stacking):
  group x acts on (xi_x, xi_c), rows in this order
      [Pd 0] (velocity), [Pdd 0] (acceleration),
      [P  r_m P] for m = 1..n_c, j = 1..n_o (collision), [0 P] (c = cos psi);
  group y acts on (xi_y, xi_s) with the same rows;
  Q = blockdiag(Pdd'Pdd + P'P, 0) per group, q = (-P' x_des, 0);
  A = the rows P[0], Pd[0], Pdd[0], P[-1] on the position block; A_psi = P[0], P[-1].
One iteration (Alg 2, in its order):
  1. xi     <- argmin 1/2 xi'Q xi + q'xi - <lam, xi> + rho/2 |F xi - g|^2,  A xi = b
  2. psi_t  <- atan2(P xi_s, P xi_c);
     xi_psi <- argmin 1/2 xi_psi'Pdd'Pdd xi_psi - <lam_psi, xi_psi>
                      + rho/2 |psi_t - P xi_psi|^2,  A_psi xi_psi = b_psi  (eq compute_convex_surrogate)
  3. alpha  <- the angles of every collision, velocity and acceleration row (eqs zeta_2, alpha_v, alpha_a)
  4. d      <- the radii (eqs compute_d_mij, compute_dv, compute_da)
  5. lam     <- lam - rho F'(F xi - g);  lam_psi <- lam_psi - rho P'(P xi_psi - psi_t)
Residuals of an iterate (the two plotted in the thesis's convergence figure):
|F xi - g| over both groups and |psi_t - P xi_psi|.

Readings (each listed in the design notes):
  - the collision step's offset uses cos and sin of the new heading P xi_psi (as the
    printed alpha step does), the collision rows of F use the slack c, s;
  - psi_t is taken on the branch of atan2 nearest the heading before the psi step:
    psi_t = theta + 2 pi rint((psi_prev - theta) / (2 pi)), theta = atan2(s, c);
  - the printed lam_psi update repeats lam's residual; here it is the multiplier of the
    surrogate's own constraint P xi_psi = psi_t;
  - the printed d_v, d_a steps say max over d <= 1; the minimiser of the printed
    objective is min(1, |v| / v_max), which is taken;
  - angles of an ellipse in coordinates scaled by its semi-axes, d = max(1, |scaled|)
    (as in the main path); a point at an obstacle's centre takes atan2(+0, +0) = 0;
  - the input state is first made to satisfy the boundary rows (its coefficients that
    the rows involve, 0, 1, 2 and n of x and y, 0 and n of psi, are solved for; the
    others are kept); initial alpha, d come from the polar step of that state;
    lam = lam_psi = 0 unless given; one rho for every block;
  - boundary rows: position, velocity, acceleration at t = 0 and position at T for x
    and y; heading at t = 0 and T.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import bernstein

X, C, Y, S, PSI = range(5)


@dataclasses.dataclass
class Ops:
    P: np.ndarray
    Pd: np.ndarray
    Pdd: np.ndarray
    t: np.ndarray
    F: np.ndarray      # [rows, 2 n_v] one group's rows (the same for x and y)
    Qg: np.ndarray     # [2 n_v, 2 n_v] Q of one group
    A: np.ndarray      # [4, 2 n_v]
    Apsi: np.ndarray   # [2, n_v]
    K: np.ndarray      # [2 n_v + 4, 2 n_v + 4] KKT matrix of one group's QP (step 1)
    Kpsi: np.ndarray   # [n_v + 2, n_v + 2] KKT matrix of the heading QP (step 2)


def operators(w) -> Ops:
    n, nt, T = w.degree, w.n_steps, w.horizon
    nv = n + 1
    P, Pd, Pdd = bernstein(n, nt, T)
    Z = np.zeros_like(P)
    rows = [np.hstack([Pd, Z]), np.hstack([Pdd, Z])]
    for r in w.radii:
        for _ in range(w.n_obs):
            rows.append(np.hstack([P, r * P]))
    rows.append(np.hstack([Z, P]))
    F = np.vstack(rows)
    Qg = np.zeros((2 * nv, 2 * nv))
    Qg[:nv, :nv] = Pdd.T @ Pdd + P.T @ P
    A = np.zeros((4, 2 * nv))
    A[0, :nv], A[1, :nv], A[2, :nv], A[3, :nv] = P[0], Pd[0], Pdd[0], P[-1]
    Apsi = np.vstack([P[0], P[-1]])
    Qbar = Qg + w.rho * F.T @ F
    K = np.block([[Qbar, A.T], [A, np.zeros((4, 4))]])
    Kpsi = np.block([[Pdd.T @ Pdd + w.rho * P.T @ P, Apsi.T], [Apsi, np.zeros((2, 2))]])
    return Ops(P, Pd, Pdd, np.linspace(0.0, T, nt), F, Qg, A, Apsi, K, Kpsi)


def obstacle_paths(w, t):
    """[n_o, n_t] x and y of every obstacle centre at the time steps."""
    xo = w.obs_centre[:, 0:1] + w.obs_vel[:, 0:1] * t[None, :]
    yo = w.obs_centre[:, 1:2] + w.obs_vel[:, 1:2] * t[None, :]
    return xo, yo


def polar_step(w, ops, xi, xi_psi):
    """Steps 3 and 4 for one sample: angles and radii of every row, from the position
    coefficients xi [4, n_v] and the heading xi_psi [n_v]."""
    P, Pd, Pdd = ops.P, ops.Pd, ops.Pdd
    x, y = P @ xi[0], P @ xi[2]
    psi = P @ xi_psi
    xo, yo = obstacle_paths(w, ops.t)
    a, b = w.obs_axes[:, 0:1], w.obs_axes[:, 1:2]
    al_o = np.zeros((w.n_circles, w.n_obs, w.n_steps))
    d_o = np.zeros_like(al_o)
    for m, r in enumerate(w.radii):
        xt = x[None, :] + r * np.cos(psi)[None, :] - xo
        yt = y[None, :] + r * np.sin(psi)[None, :] - yo
        al_o[m] = np.arctan2(yt / b, xt / a)
        d_o[m] = np.maximum(1.0, np.hypot(xt / a, yt / b))
    vx, vy = Pd @ xi[0], Pd @ xi[2]
    ax, ay = Pdd @ xi[0], Pdd @ xi[2]
    al_v, d_v = np.arctan2(vy, vx), np.minimum(1.0, np.hypot(vx, vy) / w.v_max)
    al_a, d_a = np.arctan2(ay, ax), np.minimum(1.0, np.hypot(ax, ay) / w.a_max)
    return dict(al_o=al_o, d_o=d_o, al_v=al_v, d_v=d_v, al_a=al_a, d_a=d_a, psi=psi)


def g_vectors(w, ops, pol):
    """The right-hand sides g of the x and y groups, row blocks in F's order."""
    xo, yo = obstacle_paths(w, ops.t)
    a, b = w.obs_axes[:, 0], w.obs_axes[:, 1]
    gx = [pol["d_v"] * w.v_max * np.cos(pol["al_v"]), pol["d_a"] * w.a_max * np.cos(pol["al_a"])]
    gy = [pol["d_v"] * w.v_max * np.sin(pol["al_v"]), pol["d_a"] * w.a_max * np.sin(pol["al_a"])]
    for m in range(w.n_circles):
        for j in range(w.n_obs):
            gx.append(xo[j] + a[j] * pol["d_o"][m, j] * np.cos(pol["al_o"][m, j]))
            gy.append(yo[j] + b[j] * pol["d_o"][m, j] * np.sin(pol["al_o"][m, j]))
    gx.append(np.cos(pol["psi"]))
    gy.append(np.sin(pol["psi"]))
    return np.concatenate(gx), np.concatenate(gy)


def xi_step(w, ops, lam, gx, gy):
    """Step 1: the equality-constrained QP of each group, solved through its KKT system."""
    nv = w.n_v
    rho = w.rho
    out = np.zeros((4, nv))
    for grp, (g, des) in enumerate(((gx, w.x_des[0]), (gy, w.x_des[1]))):
        q = np.zeros(2 * nv)
        q[:nv] = -ops.P.T @ des
        lg = np.concatenate([lam[2 * grp], lam[2 * grp + 1]])
        rhs = np.concatenate([lg - q + rho * ops.F.T @ g, w.boundary[grp]])
        sol = np.linalg.solve(ops.K, rhs)   # [Q + rho F'F, A'; A, 0]
        out[2 * grp], out[2 * grp + 1] = sol[:nv], sol[nv:2 * nv]
    return out


def psi_target(ops, xi, psi_prev):
    """atan2(s, c) at the time steps, on the branch nearest psi_prev."""
    th = np.arctan2(ops.P @ xi[3], ops.P @ xi[1])
    return th + 2.0 * np.pi * np.rint((psi_prev - th) / (2.0 * np.pi))


def psi_step(w, ops, lam_psi, psi_t):
    """Step 2: the surrogate QP (eq compute_convex_surrogate) through its KKT system."""
    rhs = np.concatenate([lam_psi + w.rho * ops.P.T @ psi_t, w.boundary_psi])
    return np.linalg.solve(ops.Kpsi, rhs)[:w.n_v]   # [Pdd'Pdd + rho P'P, A_psi'; A_psi, 0]


def group_rows(ops, xi):
    """F xi of the x and y groups."""
    return ops.F @ np.concatenate([xi[0], xi[1]]), ops.F @ np.concatenate([xi[2], xi[3]])


def meet_boundary(w, ops, st):
    """The state with the coefficients that the boundary rows involve solved for, so
    that A xi = b and A_psi xi_psi = b_psi hold; the other coefficients unchanged."""
    nv = w.n_v
    out = np.array(st, dtype=np.float64).copy()
    fixed = [0, 1, 2, nv - 1]
    other = [k for k in range(nv) if k not in fixed]
    Ab = ops.A[:, :nv]
    for row, grp in ((0, 0), (2, 1)):
        rhs = w.boundary[grp] - Ab[:, other] @ out[row, other]
        out[row, fixed] = np.linalg.solve(Ab[:, fixed], rhs)
    fp, op = [0, nv - 1], list(range(1, nv - 1))
    out[4, fp] = np.linalg.solve(ops.Apsi[:, fp], w.boundary_psi - ops.Apsi[:, op] @ out[4, op])
    return out


def iterate(w, iters=None, state=None, lam=None):
    """Alg 2 on every sample.  state, lam [B, 5, n_v] (rows x, c, y, s, psi) default to
    w.xi0 and zeros.  Returns (state, lam, trace [iters, B, 2]) with trace[k, b] the two
    residuals of iterate k + 1."""
    ops = operators(w)
    K = w.iters if iters is None else int(iters)
    st = np.array(w.xi0 if state is None else state, dtype=np.float64).copy()
    lm = np.zeros_like(st) if lam is None else np.array(lam, dtype=np.float64).copy()
    B = st.shape[0]
    trace = np.zeros((K, B, 2))
    nv = w.n_v
    for i in range(B):
        st[i] = meet_boundary(w, ops, st[i])
        xi, xps = st[i, :4].copy(), st[i, 4].copy()
        la, lps = lm[i, :4].copy(), lm[i, 4].copy()
        gx, gy = g_vectors(w, ops, polar_step(w, ops, xi, xps))
        for k in range(K):
            xi = xi_step(w, ops, la, gx, gy)                       # step 1
            pt = psi_target(ops, xi, ops.P @ xps)                  # step 2
            xps = psi_step(w, ops, lps, pt)
            gx, gy = g_vectors(w, ops, polar_step(w, ops, xi, xps))  # steps 3, 4
            fx, fy = group_rows(ops, xi)
            ex, ey = fx - gx, fy - gy
            gxe, gye = w.rho * ops.F.T @ ex, w.rho * ops.F.T @ ey   # step 5
            la[0], la[1] = la[0] - gxe[:nv], la[1] - gxe[nv:]
            la[2], la[3] = la[2] - gye[:nv], la[3] - gye[nv:]
            dpsi = ops.P @ xps - pt
            lps = lps - w.rho * ops.P.T @ dpsi
            trace[k, i, 0] = np.sqrt(ex @ ex + ey @ ey)
            trace[k, i, 1] = np.sqrt(dpsi @ dpsi)
        st[i, :4], st[i, 4] = xi, xps
        lm[i, :4], lm[i, 4] = la, lps
    return st, lm, trace


def residuals(w, state):
    """|F xi - g| after the polar step of each sample of `state` [B, 5, n_v] (the
    heading residual needs the step's psi_t and is not defined here)."""
    ops = operators(w)
    out = np.zeros(state.shape[0])
    for i in range(state.shape[0]):
        xi, xps = state[i, :4], state[i, 4]
        gx, gy = g_vectors(w, ops, polar_step(w, ops, xi, xps))
        fx, fy = group_rows(ops, xi)
        out[i] = np.sqrt(np.sum((fx - gx) ** 2) + np.sum((fy - gy) ** 2))
    return out


@dataclasses.dataclass
class Cycle:
    state: np.ndarray     # [B, 5, n_v] the cycle's starting state
    result: np.ndarray    # [B, 5, n_v] after K iterations
    lam: np.ndarray       # [B, 5, n_v]
    trace: np.ndarray     # [K, B, 2]
    boundary: np.ndarray  # [2, 4] the cycle's boundary rows of x and y
    boundary_psi: np.ndarray
    executed: int


def mpc(w, n_cycles, delta, iters, keep_lambda=True, redraw_seed=None):
    """Paper II's receding-horizon loop on the heading variant (Implementation Details:
    each control cycle starts from the preceding one's solution, lam and lam_psi
    included).  One cycle: Alg 2 for `iters` iterations; the executed sample is the one
    of lowest final |F xi - g| at a 1e-6 resolution (ties: the lowest index); its
    position, velocity, acceleration (x, y) and heading at delta become the next start
    rows (the final rows stay); the obstacles move on by delta; the desired path is the
    window `delta` later (workloads.desired_window, an input); every row of every sample
    is re-expressed on the shifted window, xi_next = S(delta) xi per row, and the
    multipliers are carried over or cleared.  Readings as in oracle/mpc.py.
    redraw_seed: the next cycle's samples are drawn afresh instead (workloads.heading_samples
    around the line from the new start to the goal, heading about the new start's, from
    numpy's PCG64 seeded with redraw_seed; an input), the multipliers still carried over."""
    from . import mpc as om
    from paper_2408_10731_amd.workloads import desired_window, heading_samples
    S = om.shift_matrix(w.degree, w.horizon, delta)
    rng = np.random.Generator(np.random.PCG64(redraw_seed)) if redraw_seed is not None else None
    st = np.array(w.xi0, dtype=np.float64)
    lam = np.zeros_like(st)
    bnd = np.array(w.boundary, dtype=np.float64)
    bpsi = np.array(w.boundary_psi, dtype=np.float64)
    centre = np.array(w.obs_centre, dtype=np.float64)
    out = []
    for c in range(n_cycles):
        wc = dataclasses.replace(w, xi0=st, boundary=bnd, boundary_psi=bpsi, obs_centre=centre,
                                 x_des=desired_window(w, c * delta))
        res, lam2, tr = iterate(wc, iters, state=st, lam=lam)
        i = om.executed_sample(tr[-1, :, 0])
        out.append(Cycle(st, res, lam2, tr, bnd, bpsi, i))
        p, v, a = om.state_at(res[i][[0, 2]], w.horizon, delta)
        psi = om.state_at(res[i][[4]], w.horizon, delta)[0][0]
        bnd = bnd.copy()
        bnd[:, 0], bnd[:, 1], bnd[:, 2] = p, v, a
        bpsi = np.array([psi, bpsi[1]])
        centre = centre + np.array(w.obs_vel, dtype=np.float64) * delta
        st = np.einsum("jk,brk->brj", S, res)
        if rng is not None:
            st = heading_samples(rng, st.shape[0], bnd[:, 0], w.boundary[:, 3], w.degree, bpsi[0])
        lam = lam2.copy() if keep_lambda else np.zeros_like(lam2)
    return out
