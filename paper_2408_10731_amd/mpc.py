"""Receding-horizon loop around the projection (thesis ch. 5, Paper II, Implementation
Details: an MPC on the batch optimizer whose every control cycle starts from the
preceding cycle's solution, multipliers included).

One cycle: project the batch (K AM iterations); follow the sample whose result has the
lowest residual (compared at a 1e-6 resolution, ties by the lowest index) for delta
seconds, so its position, velocity and acceleration at delta become the next cycle's
start rows (the goal row stays); move the obstacles on by delta; re-express every
sample on the shifted window with trajam_mpc_shift, which also carries the
multipliers over (or clears them).  The next cycle projects those shifted samples.

The alternative start of a cycle is the learned warm start (warmstart.WarmContext):
probe, jump and fallback from the shifted samples with zero multipliers.

Marshalling and control logic only: the projection, the residuals and the shift run in
the library; the host evaluates one trajectory's state at delta (de Casteljau on the
coefficients and their differences) to set the next boundary rows.
"""
from __future__ import annotations

import numpy as np

from . import trajam as tj

QUANTUM = 1e-6


def _de_casteljau(c: np.ndarray, u: float) -> np.ndarray:
    """Value at u in [0, 1] (or beyond) of the Bernstein polynomials with coefficients
    c [..., m] (last axis)."""
    b = np.array(c, dtype=np.float64)
    while b.shape[-1] > 1:
        b = (1.0 - u) * b[..., :-1] + u * b[..., 1:]
    return b[..., 0]


def trajectory_state(coeffs: np.ndarray, horizon: float, t: float):
    """(position, velocity, acceleration) [D] at time t of the trajectories with degree-n
    Bernstein coefficients coeffs [D, n + 1] on [0, horizon]."""
    c = np.asarray(coeffs, dtype=np.float64)
    n = c.shape[-1] - 1
    u = t / horizon
    p = _de_casteljau(c, u)
    d1 = (c[..., 1:] - c[..., :-1]) * (n / horizon)
    v = _de_casteljau(d1, u)
    d2 = (d1[..., 1:] - d1[..., :-1]) * ((n - 1) / horizon)
    a = _de_casteljau(d2, u)
    return p, v, a


class MPC:
    """The loop on one solver.  xi0 [B, D, n_v] (device): the first cycle's samples,
    projected from a cold start; boundary [D, 4] host rows (x0, v0, a0, xf);
    obstacles (centre, velocity, semi-axes) host arrays [n_o, D] at time 0.
    keep_lambda: carry the multipliers over (the thesis); warm: a WarmContext of the
    same solver, used from the second cycle on instead (learned warm start, zero
    multipliers)."""

    def __init__(self, solver: "tj.Solver", xi0, boundary, obstacles, iters: int, delta: float,
                 keep_lambda: bool = True, warm=None):
        import torch
        self.torch = torch
        self.s = solver
        self.K, self.delta = int(iters), float(delta)
        self.keep_lambda = bool(keep_lambda)
        self.warm = warm
        if warm is not None and not (warm.solver is solver and 0 < warm.k0 < self.K):
            raise ValueError("warm start: a context of this solver with 0 < k0 < iters")
        self.xi = xi0.clone().contiguous()
        self.xb = self.xi.clone()
        self.lam = torch.zeros_like(self.xi)
        self.B = self.xi.shape[0]
        self.res = torch.zeros(self.B, dtype=self.xi.dtype, device=self.xi.device)
        self.trace = torch.zeros((self.K, self.B), dtype=self.xi.dtype, device=self.xi.device)
        self.boundary = np.array(boundary, dtype=np.float64)
        c, v, a = (np.array(x, dtype=np.float64) for x in obstacles)
        self.centre, self.vel, self.axes = c, v, a
        self.dynamic = bool(np.any(v))
        self.cycles = 0

    def _obstacles(self):
        t = self.torch
        dt = self.xi.dtype
        c = t.as_tensor(self.centre, dtype=dt, device="cuda")
        v = t.as_tensor(self.vel, dtype=dt, device="cuda") if self.dynamic else None
        a = t.as_tensor(self.axes, dtype=dt, device="cuda")
        return c, v, a

    def cycle(self):
        """Run one control cycle; returns a dict with the executed sample, the batch's
        residual trace [K, B] (device) and the residuals of the result [B] (device)."""
        s = self.s
        s.set_obstacles(self._obstacles())
        if self.warm is not None and self.cycles > 0:
            k0 = self.warm.k0
            self.warm.run(self.xi, self.boundary, None, xb_out=self.xb, lam_out=self.lam,
                          trace_out=self.trace[:k0])
            s.project(self.xi, self.boundary, None, self.xb, self.lam, self.K - k0, res_trace=self.trace[k0:])
        else:
            s.project(self.xi, self.boundary, None, self.xb, self.lam, self.K, res_trace=self.trace)
        s.residuals(self.xb, None, self.res)
        res = self.res.double().cpu().numpy()
        i = int(np.argmin(np.floor(res / QUANTUM)))
        p, v, a = trajectory_state(self.xb[i].double().cpu().numpy(), s.problem.horizon, self.delta)
        out = {"executed": i, "trace": self.trace, "res": self.res, "boundary": self.boundary.copy()}
        self.boundary = self.boundary.copy()
        self.boundary[:, 0], self.boundary[:, 1], self.boundary[:, 2] = p, v, a
        self.centre = self.centre + self.vel * self.delta
        st = self.torch.cuda.current_stream().cuda_stream
        tj.trajam_mpc_shift(s.handle, self.B, self.delta, self.keep_lambda, self.xb.data_ptr(),
                            self.lam.data_ptr(), self.xi.data_ptr(), self.xb.data_ptr(), self.lam.data_ptr(), st)
        self.cycles += 1
        return out


class HeadingMPC:
    """The receding-horizon loop of the heading / multi-circle variant (Paper II,
    Implementation Details: every control cycle starts from the preceding one's state
    with both multipliers, lam and lam_psi, carried over).  One cycle: the scene of the
    window (start rows, desired path, obstacles moved on), `iters` iterations of Alg 2
    in the library, the executed sample (lowest final |F xi - g| at a 1e-6 resolution,
    ties by the lowest index), its state at delta as the next start rows (x, y: position,
    velocity, acceleration; psi), and trajam_heading_shift of every sample.  Marshalling
    and control logic only; the host evaluates the executed sample at delta."""

    def __init__(self, w, iters: int, delta: float, keep_lambda: bool = True, precision: str = "fp32",
                 redraw_seed=None):
        import torch
        from . import workloads as wl
        self.torch, self.wl = torch, wl
        self.w = w
        self.K, self.delta, self.keep_lambda = int(iters), float(delta), bool(keep_lambda)
        self.s = tj.HeadingSolver(w, precision=precision)
        dt = self.s.dtype
        self.state = torch.as_tensor(w.xi0, dtype=dt, device="cuda").contiguous()
        self.lam = torch.zeros_like(self.state)
        self.trace = torch.zeros((self.K, self.state.shape[0], 2), dtype=dt, device="cuda")
        self.boundary = np.array(w.boundary, dtype=np.float64)
        self.boundary_psi = np.array(w.boundary_psi, dtype=np.float64)
        self.centre = np.array(w.obs_centre, dtype=np.float64)
        # redraw_seed: each next cycle starts from samples drawn afresh around the line
        # from the new start to the goal (an input), the multipliers still carried over
        self.rng = np.random.Generator(np.random.PCG64(redraw_seed)) if redraw_seed is not None else None
        self.cycles = 0

    def cycle(self):
        """Run one control cycle; returns the executed sample, its coefficients [5, n_v]
        (host), the cycle's boundary rows, obstacle centres at its start and residual
        trace [K, B, 2] (device)."""
        import dataclasses
        w = self.w
        elapsed = self.cycles * self.delta
        wc = dataclasses.replace(w, boundary=self.boundary, boundary_psi=self.boundary_psi,
                                 obs_centre=self.centre, x_des=self.wl.desired_window(w, elapsed))
        self.s.set_scene(wc)
        self.s.project(self.state, self.lam, self.K, self.trace)
        r = self.trace[-1, :, 0].double().cpu().numpy()
        i = int(np.argmin(np.floor(r / QUANTUM)))
        coef = self.state[i].double().cpu().numpy()
        out = {"executed": i, "coefficients": coef, "boundary": self.boundary.copy(),
               "boundary_psi": self.boundary_psi.copy(), "obs_centre": self.centre.copy(), "trace": self.trace}
        p, v, a = trajectory_state(coef[[0, 2]], w.horizon, self.delta)
        psi = float(trajectory_state(coef[[4]], w.horizon, self.delta)[0][0])
        self.boundary = self.boundary.copy()
        self.boundary[:, 0], self.boundary[:, 1], self.boundary[:, 2] = p, v, a
        self.boundary_psi = np.array([psi, self.boundary_psi[1]])
        self.centre = self.centre + np.asarray(w.obs_vel, dtype=np.float64) * self.delta
        self.s.shift(self.state, self.lam, self.delta, self.keep_lambda)
        if self.rng is not None:
            fresh = self.wl.heading_samples(self.rng, self.state.shape[0], self.boundary[:, 0], w.boundary[:, 3],
                                            w.degree, self.boundary_psi[0])
            self.state.copy_(self.torch.as_tensor(fresh, dtype=self.state.dtype, device="cuda"))
        self.cycles += 1
        return out

    def close(self):
        self.s.close()
