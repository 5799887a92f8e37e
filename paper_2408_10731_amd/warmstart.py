"""Learned warm start of the projection (no thesis counterpart; its future-work
chapter names learning-based methods).  Marshalling around the library's kernels:
the network is trained and evaluated by trajam_mlp_* and applied by trajam_warm_*.

What the network predicts.  For a scene (obstacles, start, goal) and a sample xi it
predicts delta = xb* - xi on the free coefficients, the correction of the converged
projection (the boundary coefficients of xb* are known exactly from the boundary
conditions, so they are not learned).  At a converged fixed point the residual is
zero, so the QP's stationarity leaves lambda* = xb* - xi on the free coefficients;
the warm start is therefore
    xb0 = xi + delta_hat (free), the exact boundary coefficients (boundary);
    lambda0 = delta_hat (free), 0 (boundary),
from which the first polar step recovers the polar variables.  A sample starts cold
(xb0 = xi, lambda0 = 0) when the prediction is not finite or when the warm start's
residual exceeds the cold start's.

Scene encoding (host, once per scene): obstacles sorted by distance of their t = 0
centre to the start, each (centre - start) / L, velocity, radius, padded with zeros
to `k_obs` obstacles; then start / L and goal / L (L = |goal - start|).  The sample
part of the input, (xi - straight line) / in_scale, is built on the device.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

from . import trajam as tj
from . import workloads as wl

IN_SCALE = 0.5
OUT_SCALE = 0.5


def scene_features(w, k_obs: int) -> np.ndarray:
    start, goal = w.boundary[:, 0], w.boundary[:, 3]
    L = max(float(np.linalg.norm(goal - start)), 1e-9)
    c = np.asarray(w.obs_centre, dtype=np.float64)
    order = np.argsort(np.linalg.norm(c - start[None], axis=1), kind="stable")[:k_obs]
    D = w.dims
    feat = np.zeros((k_obs, 2 * D + 1))
    feat[:len(order), :D] = (c[order] - start[None]) / L
    feat[:len(order), D:2 * D] = np.asarray(w.obs_vel)[order]
    feat[:len(order), 2 * D] = np.asarray(w.obs_axes)[order, 0]
    return np.concatenate([feat.reshape(-1), start / L, goal / L]).astype(np.float32)


def straight_line(w) -> np.ndarray:
    start, goal = w.boundary[:, 0], w.boundary[:, 3]
    frac = np.arange(w.degree + 1) / w.degree
    return (start[:, None] + frac[None, :] * (goal - start)[:, None]).astype(np.float32)


def init_params(widths, seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (float32, the library's flat layout)."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(len(widths) - 1):
        fan_in, out = widths[l], widths[l + 1]
        bound = math.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-bound, bound, size=out * fan_in))
        parts.append(np.zeros(out))
    return np.concatenate(parts).astype(np.float32)


class Net:
    """Device parameters, Adam state and work buffers of one network."""

    def __init__(self, widths, seed: int = 0, precision: int = 0, max_batch: int = 4096):
        import torch
        self.torch = torch
        self.widths = list(widths)
        self.shape = tj.mlp_shape(self.widths)
        self.n = tj.trajam_mlp_param_count(self.shape)
        self.precision = int(precision)
        dev = "cuda"
        self.params = torch.as_tensor(init_params(self.widths, seed), device=dev)
        assert self.params.numel() == self.n
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grads = torch.zeros_like(self.params)
        self.step_count = 0
        self.max_batch = int(max_batch)
        hid = sum(self.widths[1:-1])
        maxw = max(self.widths[1:-1]) if len(self.widths) > 2 else 1
        self.acts = torch.zeros(max(hid, 1) * self.max_batch, device=dev)
        self.scratch = torch.zeros(2 * maxw * self.max_batch, device=dev)
        self.y = torch.zeros((self.max_batch, self.widths[-1]), device=dev)
        self.dy = torch.zeros_like(self.y)
        self.loss = torch.zeros(1, device=dev)

    def _st(self):
        return self.torch.cuda.current_stream().cuda_stream

    def forward(self, x):
        B = x.shape[0]
        assert B <= self.max_batch and x.is_contiguous() and x.shape[1] == self.widths[0]
        tj.trajam_mlp_forward(self.shape, B, self.precision, self.params.data_ptr(), x.data_ptr(),
                              self.acts.data_ptr(), self.y.data_ptr(), self._st())
        return self.y[:B]

    def backward(self, x, dy):
        B = x.shape[0]
        tj.trajam_mlp_backward(self.shape, B, self.precision, self.params.data_ptr(),
                               x.data_ptr(), self.acts.data_ptr(), dy.data_ptr(),
                               self.grads.data_ptr(), self.scratch.data_ptr(), self._st())
        return self.grads

    def train_step(self, x, target, lr=1e-3):
        B = x.shape[0]
        y = self.forward(x)
        tj.trajam_mlp_mse(B * self.widths[-1], y.data_ptr(), target.data_ptr(),
                          self.dy.data_ptr(), self.loss.data_ptr(), self._st())
        self.backward(x, self.dy[:B])
        self.step_count += 1
        tj.trajam_mlp_adam(self.n, self.params.data_ptr(), self.grads.data_ptr(),
                           self.m.data_ptr(), self.v.data_ptr(), self.step_count, lr, 0.9, 0.999,
                           1e-8, self._st())
        return self.loss


@dataclasses.dataclass
class Dataset:
    x: object       # [N, n_in] device float32
    t: object       # [N, dim] device float32 (delta / OUT_SCALE)
    n_scenes: int


def build_inputs(w, xi, k_obs, out=None):
    """Network inputs for the samples xi (device [B, D, nv]) of scene w."""
    import torch
    scene = torch.as_tensor(scene_features(w, k_obs), device="cuda")
    line = torch.as_tensor(straight_line(w), device="cuda")
    B = xi.shape[0]
    n_in = scene.numel() + w.dims * w.n_v
    x = out if out is not None else torch.zeros((B, n_in), device="cuda")
    tj.trajam_warm_features(B, w.dims, w.n_v, scene.numel(), scene.data_ptr(), xi.data_ptr(),
                            line.data_ptr(), 1.0 / IN_SCALE, x.data_ptr(),
                            torch.cuda.current_stream().cuda_stream)
    return x


def boundary_coeffs(solver: "tj.Solver", w) -> np.ndarray:
    """[D][4] Bernstein coefficients (xi_0, xi_1, xi_2, xi_n) fixed by the boundary rows."""
    return np.stack([tj.trajam_boundary_coefficients(solver.problem, w.boundary[ax])
                     for ax in range(w.dims)])


def generate(scene_fn, seeds, samples_per_scene, k_obs, iters=300, tol=1e-3, chunk=256):
    """Solver-generated pairs.  The scenes (one obstacle count per family) are taken
    `chunk` at a time: a fixed pool of solvers and device buffers is refilled with the
    chunk's obstacles and samples, all samples are projected `iters` AM iterations from
    a cold start in one ragged launch, and converged samples (residual <= tol) are
    kept."""
    import torch
    seeds = [int(x) for x in seeds]
    B = int(samples_per_scene)
    w0 = scene_fn(seeds[0], B)
    n = min(chunk, len(seeds))
    D, nv, no = w0.dims, w0.n_v, w0.n_obs
    solvers = [tj.Solver.for_workload(w0, precision="fp32", max_batch=B) for _ in range(n)]
    xi = torch.zeros((n, B, D, nv), device="cuda")
    xb, lam = torch.zeros_like(xi), torch.zeros_like(xi)
    oc = torch.zeros((n, max(no, 1), D), device="cuda")
    ov, oa = torch.zeros_like(oc), torch.zeros_like(oc)
    res = torch.zeros((n, B), device="cuda")
    plan, plan_key = None, None
    xs, ts = [], []
    for c0 in range(0, len(seeds), n):
        ws = [scene_fn(sd, B) for sd in seeds[c0:c0 + n]]
        m = len(ws)
        for w in ws:
            if w.n_obs != no or w.dims != D or w.n_v != nv:
                raise ValueError("generate: scenes of one family must share dims, degree and n_obs")
        bnd = ws[0].boundary
        if any(not np.array_equal(w.boundary, bnd) for w in ws):
            raise ValueError("generate: scenes of one chunk must share the boundary conditions")
        xi[:m].copy_(torch.from_numpy(np.stack([w.xi for w in ws]).astype(np.float32)))
        dynamic = any(np.any(w.obs_vel) for w in ws)
        if no:
            oc[:m].copy_(torch.from_numpy(np.stack([w.obs_centre for w in ws]).astype(np.float32)))
            ov[:m].copy_(torch.from_numpy(np.stack([w.obs_vel for w in ws]).astype(np.float32)))
            oa[:m].copy_(torch.from_numpy(np.stack([w.obs_axes for w in ws]).astype(np.float32)))
        obs = [(oc[i], ov[i] if dynamic else None, oa[i]) for i in range(m)]
        for i in range(m):
            solvers[i].set_obstacles(obs[i])
        key = (m, dynamic, bnd.tobytes())   # a plan bakes these in
        if key != plan_key:
            if plan is not None:
                plan.close()
            plan = tj.RaggedPlan([(solvers[i], xi[i], bnd, xb[i], lam[i]) for i in range(m)],
                                 iters)
            plan_key = key
        xb[:m].copy_(xi[:m])
        lam[:m].zero_()
        plan.launch()
        xs_c = []
        for i, w in enumerate(ws):
            solvers[i].residuals(xb[i], obs[i], res[i])
            xs_c.append(build_inputs(w, xi[i], k_obs))
        keep = (res[:m] <= tol).reshape(-1)
        # the warm start writes the boundary coefficients exactly, so only the free
        # coefficients' correction is learned
        delta = xb[:m] - xi[:m]
        delta[:, :, :, [0, 1, 2, nv - 1]] = 0.0
        xs.append(torch.cat(xs_c)[keep])
        ts.append((delta / OUT_SCALE).reshape(m * B, -1)[keep])
    torch.cuda.synchronize()
    plan.close()
    for s_ in solvers:
        s_.close()
    return Dataset(torch.cat(xs).contiguous(), torch.cat(ts).contiguous(), len(seeds))


def train(net: Net, data: Dataset, epochs: int, batch: int = 1024, lr: float = 1e-3,
          seed: int = 0):
    """Minibatch Adam on the mean squared error; returns the per-epoch mean loss."""
    import torch
    N = data.x.shape[0]
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    curve = []
    for _ in range(epochs):
        perm = torch.randperm(N, device="cuda", generator=g)
        tot = torch.zeros(1, device="cuda")
        nb = 0
        for i in range(0, N - batch + 1, batch):
            idx = perm[i:i + batch]
            loss = net.train_step(data.x[idx].contiguous(), data.t[idx].contiguous(), lr)
            tot += loss
            nb += 1
        curve.append(float(tot.item()) / max(nb, 1))
    return curve


class WarmContext:
    """Per-scene state of the warm start: scene features, reference line and boundary
    coefficients on the device, and every work buffer, allocated once.  `run` only
    launches kernels (features, the network, apply, two residuals, fallback), so it
    can be captured in a graph together with the projection that follows."""

    def __init__(self, solver: "tj.Solver", net: Net, w, k_obs: int, max_batch: int):
        import torch
        self.solver, self.net, self.w, self.k_obs = solver, net, w, k_obs
        self.scene = torch.as_tensor(scene_features(w, k_obs), device="cuda")
        self.line = torch.as_tensor(straight_line(w), device="cuda")
        self.bc = boundary_coeffs(solver, w)
        n_in = self.scene.numel() + w.dims * w.n_v
        assert n_in == net.widths[0] and max_batch <= net.max_batch
        self.x = torch.zeros((max_batch, n_in), device="cuda")
        shape = (max_batch, w.dims, w.n_v)
        self.xb0 = torch.zeros(shape, device="cuda")
        self.lam0 = torch.zeros(shape, device="cuda")
        self.rw = torch.zeros(max_batch, device="cuda")
        self.rc = torch.zeros(max_batch, device="cuda")
        self.flags = torch.zeros(max_batch, dtype=torch.int32, device="cuda")

    def run(self, xi, obs):
        """(xb0, lam0, flags) views for the samples xi [B, D, n_v]."""
        import torch
        w, B = self.w, xi.shape[0]
        st = torch.cuda.current_stream().cuda_stream
        x = self.x[:B]
        tj.trajam_warm_features(B, w.dims, w.n_v, self.scene.numel(), self.scene.data_ptr(),
                                xi.data_ptr(), self.line.data_ptr(), 1.0 / IN_SCALE, x.data_ptr(),
                                st)
        y = self.net.forward(x)
        xb0, lam0, fl = self.xb0[:B], self.lam0[:B], self.flags[:B]
        tj.trajam_warm_apply(B, w.dims, w.n_v, y.data_ptr(), xi.data_ptr(), OUT_SCALE, self.bc,
                             xb0.data_ptr(), lam0.data_ptr(), fl.data_ptr(), st)
        rw, rc = self.rw[:B], self.rc[:B]
        self.solver.residuals(xb0, obs, rw)
        self.solver.residuals(xi, obs, rc)
        tj.trajam_warm_fallback(B, w.dims, w.n_v, rw.data_ptr(), rc.data_ptr(), xi.data_ptr(),
                                xb0.data_ptr(), lam0.data_ptr(), fl.data_ptr(), st)
        return xb0, lam0, fl


def warm_start(solver: "tj.Solver", net: Net, w, xi, obs, k_obs):
    """(xb0, lam0, flags): network prediction with the per-sample cold fallback."""
    ctx = WarmContext(solver, net, w, k_obs, xi.shape[0])
    xb0, lam0, fl = ctx.run(xi, obs)
    return xb0.clone(), lam0.clone(), fl.clone()


def family_scene(family: str):
    """Scene generators for training / evaluation families (seeded, synthetic)."""
    if family == "cfg2":
        return lambda seed, batch: wl.config2(batch=batch, seed=seed)
    if family == "cfg4":
        return lambda seed, batch: wl.config4_scene(seed, batch=batch)
    raise ValueError(family)


def widths_for(w, k_obs: int, hidden: int = 256):
    n_in = k_obs * (2 * w.dims + 1) + 2 * w.dims + w.dims * w.n_v
    return [n_in, hidden, hidden, w.dims * w.n_v]
