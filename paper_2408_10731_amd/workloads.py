"""Seeded synthetic inputs for the batched alternating-minimization projection.

This module only draws random numbers and lays them out.  It holds none of the
method's arithmetic, so both the CPU oracle (through the tests) and the HIP path
consume exactly the same host arrays.

The thesis evaluates on BARN, crowd simulations and real robots, none of which is
available; the recipes below stand in for them with the shapes and value
distributions of the five evaluation configurations (2D/3D point robot, circular or
ellipsoidal obstacles, Bernstein trajectories with a fixed horizon):

* samples: the straight start-goal line written as Bernstein coefficients
  (coefficient m at s + (m/n)(g - s)) plus i.i.d. N(0, sigma^2) per coefficient;
* obstacles: centres uniform in a box, semi-axes uniform in a range (one radius for
  circles/spheres, independent per axis for ellipsoids), optional constant velocity
  with each component uniform in [-v, v];  an obstacle whose centre lies within
  (largest semi-axis + 0.5 m) of the start or the goal is redrawn;
* boundary: start and goal positions, zero initial velocity and acceleration.

Arrays use float64; the HIP path casts to its own precision on upload.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

MASTER_SEED = 240810731


@dataclasses.dataclass
class Workload:
    """One projection problem plus a batch of samples to project."""

    name: str
    dims: int
    degree: int
    n_steps: int
    horizon: float
    v_max: float
    a_max: float
    rho: float
    obs_centre: np.ndarray  # [n_o, D]
    obs_vel: np.ndarray  # [n_o, D]
    obs_axes: np.ndarray  # [n_o, D]
    boundary: np.ndarray  # [D, 4] = (x0, v0, a0, xf) per axis
    xi: np.ndarray  # [B, D, n_v]
    iters: int
    precision: str = "fp64"
    n_agents: int = 1
    agent_radius: float = 0.0
    workspace: Optional[np.ndarray] = None  # [2, D] (lo, hi) bounds on every position, or None

    @property
    def n_v(self) -> int:
        return self.degree + 1

    @property
    def n_obs(self) -> int:
        return int(self.obs_centre.shape[0])

    @property
    def batch(self) -> int:
        return int(self.xi.shape[0])

    def rounded(self, dtype=np.float32) -> "Workload":
        """Same problem with every array rounded to `dtype` (kept as float64), i.e.
        exactly the values a reduced-precision device path receives."""
        r = lambda a: np.asarray(a, dtype=dtype).astype(np.float64)
        return dataclasses.replace(self, obs_centre=r(self.obs_centre), obs_vel=r(self.obs_vel),
                                   obs_axes=r(self.obs_axes), xi=r(self.xi))

    def subset(self, batch: int) -> "Workload":
        """Same problem, the first `batch` samples."""
        return dataclasses.replace(self, xi=np.ascontiguousarray(self.xi[:batch]))


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def draw_obstacles(rng, n_o, dims, lo, hi, axes_range, per_axis, start, goal,
                   speed=0.0, clearance=0.5):
    """Rejection-sampled obstacles; returns centre, velocity, semi-axes [n_o, D]."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    start = np.asarray(start, dtype=np.float64)
    goal = np.asarray(goal, dtype=np.float64)
    centre = np.zeros((n_o, dims))
    axes = np.zeros((n_o, dims))
    for j in range(n_o):
        while True:
            c = rng.uniform(lo, hi)
            if per_axis:
                s = rng.uniform(axes_range[0], axes_range[1], size=dims)
            else:
                s = np.full(dims, rng.uniform(axes_range[0], axes_range[1]))
            reach = s.max() + clearance
            if np.linalg.norm(c - start) > reach and np.linalg.norm(c - goal) > reach:
                break
        centre[j] = c
        axes[j] = s
    if speed > 0.0:
        vel = rng.uniform(-speed, speed, size=(n_o, dims))
    else:
        vel = np.zeros((n_o, dims))
    return centre, vel, axes


def line_samples(rng, batch, degree, start, goal, sigma):
    """Straight start-goal line as Bernstein coefficients plus Gaussian noise."""
    start = np.asarray(start, dtype=np.float64)
    goal = np.asarray(goal, dtype=np.float64)
    dims = start.shape[0]
    frac = np.arange(degree + 1, dtype=np.float64) / degree
    line = start[:, None] + frac[None, :] * (goal - start)[:, None]  # [D, n_v]
    noise = rng.normal(0.0, sigma, size=(batch, dims, degree + 1))
    return np.ascontiguousarray(line[None] + noise)


def boundary_rows(start, goal):
    start = np.asarray(start, dtype=np.float64)
    goal = np.asarray(goal, dtype=np.float64)
    b = np.zeros((start.shape[0], 4))
    b[:, 0] = start
    b[:, 3] = goal
    return b


def config1(batch: int = 64, seed: Optional[int] = None) -> Workload:
    """2D, degree 10, 100 steps over 10 s, 10 circles r~U(0.4,0.6) in [0,10]^2, FP64."""
    rng = _rng(MASTER_SEED + 1 if seed is None else seed)
    start, goal = (0.0, 5.0), (10.0, 5.0)
    c, w, s = draw_obstacles(rng, 10, 2, (0, 0), (10, 10), (0.4, 0.6), False, start, goal)
    xi = line_samples(rng, batch, 10, start, goal, 0.5)
    return Workload("cfg1-2d-fp64", 2, 10, 100, 10.0, 1.5, 2.0, 1.0, c, w, s,
                    boundary_rows(start, goal), xi, 100, "fp64")


def config2(batch: int = 1024, seed: Optional[int] = None) -> Workload:
    """2D, degree 10, 100 steps over 30 s, 50 circles r~U(0.3,0.8) in [0,30]^2, FP32."""
    rng = _rng(MASTER_SEED + 2 if seed is None else seed)
    start, goal = (0.0, 15.0), (30.0, 15.0)
    c, w, s = draw_obstacles(rng, 50, 2, (0, 0), (30, 30), (0.3, 0.8), False, start, goal)
    xi = line_samples(rng, batch, 10, start, goal, 0.5)
    return Workload("cfg2-2d-fp32", 2, 10, 100, 30.0, 1.5, 2.0, 1.0, c, w, s,
                    boundary_rows(start, goal), xi, 50, "fp32")


def config3(batch: int = 4096, seed: Optional[int] = None) -> Workload:
    """3D, degree 15, 150 steps over 20 s, 200 ellipsoids (semi-axes U(0.3,1.0) each)."""
    rng = _rng(MASTER_SEED + 3 if seed is None else seed)
    start, goal = (0.0, 10.0, 3.0), (20.0, 10.0, 3.0)
    c, w, s = draw_obstacles(rng, 200, 3, (0, 0, 0), (20, 20, 6), (0.3, 1.0), True,
                             start, goal)
    xi = line_samples(rng, batch, 15, start, goal, 0.5)
    return Workload("cfg3-3d-bf16", 3, 15, 150, 20.0, 1.5, 2.0, 1.0, c, w, s,
                    boundary_rows(start, goal), xi, 50, "bf16")


def config4_scene(seed: int, n_obs: int = 100, batch: int = 2000) -> Workload:
    """2D, degree 10, 100 steps over 30 s, 100 moving circles (velocity U(-1,1) m/s)."""
    rng = _rng(seed)
    start, goal = (0.0, 15.0), (30.0, 15.0)
    c, w, s = draw_obstacles(rng, n_obs, 2, (0, 0), (30, 30), (0.3, 0.8), False,
                             start, goal, speed=1.0)
    xi = line_samples(rng, batch, 10, start, goal, 0.5)
    return Workload("cfg4-2d-dynamic", 2, 10, 100, 30.0, 1.5, 2.0, 1.0, c, w, s,
                    boundary_rows(start, goal), xi, 15, "fp32")


def config4(batch: int = 2000, seed: Optional[int] = None) -> Workload:
    return config4_scene(MASTER_SEED + 4 if seed is None else seed, batch=batch)


def tiny(dims: int = 2, batch: int = 3, n_obs: int = 2, degree: int = 5,
         n_steps: int = 9, seed: int = 7, speed: float = 0.0,
         per_axis: bool = False) -> Workload:
    """A very small problem for brute-force and by-hand checks."""
    rng = _rng(seed)
    start = (0.0,) * (dims - 1) + (0.0,)
    goal = (4.0,) + (0.0,) * (dims - 1)
    lo = (0.5,) + (-1.0,) * (dims - 1)
    hi = (3.5,) + (1.0,) * (dims - 1)
    c, w, s = draw_obstacles(rng, n_obs, dims, lo, hi, (0.3, 0.7), per_axis, start, goal,
                             speed=speed, clearance=0.1)
    xi = line_samples(rng, batch, degree, start, goal, 0.4)
    return Workload(f"tiny-{dims}d", dims, degree, n_steps, 4.0, 1.5, 2.0, 1.0, c, w, s,
                    boundary_rows(start, goal), xi, 5, "fp64")


def problem2d(seed: int, n_obs: int, batch: int, iters: int = 50) -> Workload:
    """The 2D single-robot geometry of config 2 with n_obs circles and `batch` samples."""
    rng = _rng(seed)
    start, goal = (0.0, 15.0), (30.0, 15.0)
    c, w, s = draw_obstacles(rng, n_obs, 2, (0, 0), (30, 30), (0.3, 0.8), False, start, goal)
    xi = line_samples(rng, batch, 10, start, goal, 0.5)
    return Workload(f"2d-n{n_obs}-b{batch}", 2, 10, 100, 30.0, 1.5, 2.0, 1.0, c, w, s,
                    boundary_rows(start, goal), xi, iters, "fp32")


def problem3d(seed: int, n_obs: int, batch: int, iters: int = 50) -> Workload:
    """3D single robot: static spheres r~U(0.3,1.0) in [-10,10]^2 x [0,6], from a point
    of the radius-8 m circle at z = 3 to its antipode in 10 s, degree 10, 100 steps,
    v_max = a_max = 3 (the straight line needs 1.6 m/s)."""
    rng = _rng(seed)
    ang = rng.uniform(0.0, 2.0 * np.pi)
    start = (8.0 * np.cos(ang), 8.0 * np.sin(ang), 3.0)
    goal = (-start[0], -start[1], 3.0)
    c, w, s = draw_obstacles(rng, n_obs, 3, (-10, -10, 0), (10, 10, 6), (0.3, 1.0), False,
                             start, goal)
    xi = line_samples(rng, batch, 10, start, goal, 0.5)
    return Workload(f"3d-n{n_obs}-b{batch}", 3, 10, 100, 10.0, 3.0, 3.0, 1.0, c, w, s,
                    boundary_rows(start, goal), xi, iters, "fp32")


def _far_from(c, s, points, clearance):
    reach = s.max() + clearance
    return bool(np.min(np.linalg.norm(points - c[None], axis=1)) > reach)


def agents3d(seed: int, n_agents: int, n_obs: int, batch: int, iters: int = 50,
             radius: float = 8.0, agent_radius: float = 0.3, sigma: float = 0.5) -> Workload:
    """N agents in 3D: evenly spaced on a horizontal circle (radius 8 m, z = 3, random
    phase), each flying to its antipode in 10 s; agent radius 0.3 m (pair clearance
    0.6 m); static spheres r~U(0.3,1.0) in [-10,10]^2 x [0,6], kept 0.5 m clear of
    every start and goal; degree 10, 100 steps, v_max = a_max = 3.  xi [B, N, 3, 11]:
    each agent's straight line plus N(0, sigma^2) per coefficient; boundary [N, 3, 4]."""
    rng = _rng(seed)
    phase = rng.uniform(0.0, 2.0 * np.pi)
    ang = phase + 2.0 * np.pi * np.arange(n_agents) / n_agents
    starts = np.stack([radius * np.cos(ang), radius * np.sin(ang), np.full(n_agents, 3.0)], 1)
    goals = starts * np.array([-1.0, -1.0, 1.0])
    pts = np.concatenate([starts, goals])
    centre = np.zeros((n_obs, 3))
    axes = np.zeros((n_obs, 3))
    for j in range(n_obs):
        while True:
            c = rng.uniform((-10, -10, 0), (10, 10, 6))
            s = np.full(3, rng.uniform(0.3, 1.0))
            if _far_from(c, s, pts, 0.5):
                break
        centre[j] = c
        axes[j] = s
    xi = np.stack([line_samples(rng, batch, 10, starts[a], goals[a], sigma)
                   for a in range(n_agents)], 1)
    bnd = np.stack([boundary_rows(starts[a], goals[a]) for a in range(n_agents)])
    return Workload(f"agents3d-N{n_agents}-n{n_obs}-b{batch}", 3, 10, 100, 10.0, 3.0, 3.0, 1.0,
                    centre, np.zeros((n_obs, 3)), axes, bnd, np.ascontiguousarray(xi), iters,
                    "fp32", n_agents, agent_radius)


def tiny_agents(dims: int = 2, n_agents: int = 3, batch: int = 2, n_obs: int = 1,
                degree: int = 5, n_steps: int = 9, seed: int = 11,
                agent_radius: float = 0.4, speed: float = 0.0,
                per_axis: bool = False) -> Workload:
    """A few agents crossing a small square (each to the opposite corner region) for
    brute-force and by-hand checks of the joint projection."""
    rng = _rng(seed)
    ang = rng.uniform(0, 2 * np.pi) + 2 * np.pi * np.arange(n_agents) / n_agents
    ring = np.stack([2.0 * np.cos(ang), 2.0 * np.sin(ang)], 1)
    if dims == 3:
        ring = np.concatenate([ring, rng.uniform(-0.3, 0.3, size=(n_agents, 1))], 1)
    starts, goals = ring, -ring
    pts = np.concatenate([starts, goals])
    centre = np.zeros((n_obs, dims))
    axes = np.zeros((n_obs, dims))
    for j in range(n_obs):
        while True:
            c = rng.uniform(-1.5, 1.5, size=dims)
            if per_axis:
                s = rng.uniform(0.2, 0.4, size=dims)
            else:
                s = np.full(dims, rng.uniform(0.2, 0.4))
            if _far_from(c, s, pts, 0.1):
                break
        centre[j] = c
        axes[j] = s
    vel = rng.uniform(-speed, speed, size=(n_obs, dims)) if speed > 0 else np.zeros((n_obs, dims))
    xi = np.stack([line_samples(rng, batch, degree, starts[a], goals[a], 0.3)
                   for a in range(n_agents)], 1)
    bnd = np.stack([boundary_rows(starts[a], goals[a]) for a in range(n_agents)])
    return Workload(f"tiny-agents-{dims}d", dims, degree, n_steps, 4.0, 3.0, 4.0, 1.0, centre,
                    vel, axes, bnd, np.ascontiguousarray(xi), 5, "fp64", n_agents, agent_radius)


def ragged_set(n_problems: int = 256, seed: Optional[int] = None, n_obs=(5, 300),
               batch=(32, 2048), iters: int = 50, dims3_every: int = 2):
    """Many independent problems: n_obs ~ U{n_obs}, batch ~ U{batch} per problem;
    every `dims3_every`-th problem is 3D (problem3d), the rest 2D (problem2d)."""
    base = MASTER_SEED + 5 if seed is None else seed
    pick = _rng(base)
    out = []
    for k in range(n_problems):
        no = int(pick.integers(n_obs[0], n_obs[1] + 1))
        b = int(pick.integers(batch[0], batch[1] + 1))
        gen = problem3d if (dims3_every and k % dims3_every == dims3_every - 1) else problem2d
        out.append(gen(base + 1000 + k, no, b, iters))
    return out


def config5(n_problems: int = 256, seed: Optional[int] = None, iters: int = 50,
            n_obs=(5, 300), batch=(32, 2048), agents=(16, 64)):
    """Ragged set: n_obs ~ U{n_obs} and batch ~ U{batch} per problem; even problems are
    2D single robots in the config-2 geometry (problem2d), odd ones 3D multi-agent
    problems with N ~ U{agents} agents (agents3d; a batch entry is a joint sample)."""
    base = MASTER_SEED + 50 if seed is None else seed
    pick = _rng(base)
    out = []
    for k in range(n_problems):
        no = int(pick.integers(n_obs[0], n_obs[1] + 1))
        b = int(pick.integers(batch[0], batch[1] + 1))
        na = int(pick.integers(agents[0], agents[1] + 1))
        if k % 2 == 0:
            out.append(problem2d(base + 1000 + k, no, b, iters))
        else:
            out.append(agents3d(base + 1000 + k, na, no, b, iters))
    return out


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


@dataclasses.dataclass
class HeadingWorkload:
    """A problem of the heading / multi-circle variant (Paper II: a rectangular robot
    modelled by circles on its heading axis, a tracking-and-smoothness cost, crowds of
    elliptical obstacles) plus a batch of initial states.

    xi0 [B, 5, n_v]: per sample the initial coefficients of x, c, y, s, psi (c and s:
    the slack copies of cos psi and sin psi).  x_des [2, n_steps]: the desired
    positions at the time steps t_k = k T / (n_steps - 1)."""

    name: str
    degree: int
    n_steps: int
    horizon: float
    v_max: float
    a_max: float
    rho: float
    radii: np.ndarray        # [n_c] circle offsets along the heading axis
    obs_centre: np.ndarray   # [n_o, 2] at t = 0
    obs_vel: np.ndarray      # [n_o, 2] constant velocity
    obs_axes: np.ndarray     # [n_o, 2] semi-axes (inflated by the footprint circles' radius)
    boundary: np.ndarray     # [2, 4] rows (p0, v0, a0, pf) of x and y
    boundary_psi: np.ndarray  # [2] (psi(0), psi(T))
    x_des: np.ndarray        # [2, n_steps]
    xi0: np.ndarray          # [B, 5, n_v]
    iters: int

    @property
    def n_v(self) -> int:
        return self.degree + 1

    @property
    def n_obs(self) -> int:
        return int(self.obs_centre.shape[0])

    @property
    def n_circles(self) -> int:
        return int(self.radii.shape[0])

    @property
    def batch(self) -> int:
        return int(self.xi0.shape[0])


def heading_samples(rng, batch: int, start, goal, degree: int, psi0: float = 0.0) -> np.ndarray:
    """Initial states [batch, 5, n_v] of the heading variant around the line from start
    to goal: x along the line plus N(0, 0.3^2) per coefficient, y with a lateral bump of
    amplitude N(0, 1.5^2) plus N(0, 0.3^2), heading coefficients psi0 + N(0, 0.2^2), c and
    s their cosines and sines."""
    start, goal = np.asarray(start, dtype=np.float64), np.asarray(goal, dtype=np.float64)
    nv = degree + 1
    frac = np.arange(nv) / degree
    bump = np.sin(np.pi * frac)
    xi0 = np.zeros((batch, 5, nv))
    xi0[:, 0] = start[0] + frac * (goal[0] - start[0]) + rng.normal(0.0, 0.3, (batch, nv))
    xi0[:, 2] = (start[1] + frac * (goal[1] - start[1]) + rng.normal(0.0, 1.5, (batch, 1)) * bump
                 + rng.normal(0.0, 0.3, (batch, nv)))
    psi = psi0 + rng.normal(0.0, 0.2, (batch, nv))
    xi0[:, 4] = psi
    xi0[:, 1] = np.cos(psi)
    xi0[:, 3] = np.sin(psi)
    return xi0


def heading_scene(seed: int, n_obs: int = 30, n_circles: int = 4, batch: int = 1000,
                  iters: int = 10, flow: str = "static", degree: int = 10, n_steps: int = 100) -> HeadingWorkload:
    """Paper II's crowd benchmarks as synthetic scenes: a 1.2 m x 0.6 m robot (n_circles
    circles of radius 0.3 m spread along its length) tracks the straight line from
    (0, 0) to (20, 0) at 1 m/s over T = 20 s through a crowd of n_obs people (radius
    0.25 m, so the semi-axes are 0.55 m) placed in [3, 17] x [-3, 3].  flow: "static"
    (benchmark 1), "same" (the crowd walks along +x at up to 0.3 m/s, benchmark 2) or
    "opposite" (along -x at up to 1 m/s, benchmark 3).  v_max = 2 m/s, a_max = 2 m/s^2.
    Initial states: the line with lateral offsets drawn per sample (a smooth bump of
    amplitude ~ N(0, 1.5) m plus coefficient noise N(0, 0.3)), the heading coefficients
    N(0, 0.2) rad with psi fixed to 0 at both ends, c and s the cosine and sine of the
    heading coefficients."""
    rng = _rng(seed)
    T = 20.0
    start, goal = np.array([0.0, 0.0]), np.array([20.0, 0.0])
    radii = (np.linspace(-0.45, 0.45, n_circles) if n_circles > 1 else np.zeros(1))
    centre = np.zeros((max(n_obs, 0), 2))
    for j in range(n_obs):
        while True:
            c = rng.uniform((3.0, -3.0), (17.0, 3.0))
            if np.linalg.norm(c - start) > 2.0 and np.linalg.norm(c - goal) > 2.0:
                break
        centre[j] = c
    vel = np.zeros_like(centre)
    if flow == "same":
        vel[:, 0] = rng.uniform(0.0, 0.3, n_obs)
    elif flow == "opposite":
        vel[:, 0] = -rng.uniform(0.0, 1.0, n_obs)
    elif flow != "static":
        raise ValueError(flow)
    axes = np.full((n_obs, 2), 0.55)
    xi0 = heading_samples(rng, batch, start, goal, degree)
    psi = xi0[:, 4]
    psi[:, 0] = psi[:, -1] = 0.0
    xi0[:, 1] = np.cos(psi)
    xi0[:, 3] = np.sin(psi)
    bnd = np.zeros((2, 4))
    bnd[:, 0], bnd[:, 3] = start, goal
    bnd[:, 1] = (goal - start) / T
    t = np.linspace(0.0, T, n_steps)
    x_des = start[:, None] + (goal - start)[:, None] * (t / T)[None, :]
    return HeadingWorkload(f"heading-{flow}-n{n_obs}-c{n_circles}-b{batch}", degree, n_steps, T, 2.0, 2.0,
                           1.0, radii, centre, vel, axes, bnd, np.zeros(2), x_des, xi0, iters)


def desired_window(w: HeadingWorkload, elapsed: float) -> np.ndarray:
    """The desired positions [2, n_steps] of the window that starts `elapsed` seconds
    after w's: the straight line from w.x_des's first point to its last at w's constant
    speed, held at the last point once reached."""
    t = np.linspace(0.0, w.horizon, w.n_steps)
    p0, pf = w.x_des[:, 0], w.x_des[:, -1]
    frac = np.minimum(1.0, (elapsed + t) / w.horizon)
    return p0[:, None] + (pf - p0)[:, None] * frac[None, :]
