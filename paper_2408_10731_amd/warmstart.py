"""Learned warm start of the projection (no thesis counterpart; its future-work
chapter names learning-based methods).  Marshalling around the library's kernels:
the network is trained and evaluated by trajam_mlp_* and applied by trajam_warm_*.

What the network predicts.  For a scene (obstacles, start, goal) and a sample xi it
predicts delta = xb* - xi, the correction of the converged projection.  At a
converged fixed point the residual is zero, so the QP's stationarity leaves
lambda* = xb* - xi on the free coefficients; the warm start is therefore
    xb0 = xi + delta_hat,   lambda0 = delta_hat (free coefficients), 0 (boundary ones),
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


def generate(scene_fn, seeds, samples_per_scene, k_obs, iters=300, tol=1e-3):
    """Solver-generated pairs: each scene's samples projected `iters` AM iterations
    from a cold start on the GPU; converged samples (residual <= tol) are kept."""
    import torch
    xs, ts = [], []
    for seed in seeds:
        w = scene_fn(int(seed), samples_per_scene)
        solver = tj.Solver.for_workload(w, precision="fp32")
        xi, obs = tj.device_workload(w, torch.float32)
        xb = xi.clone()
        lam = torch.zeros_like(xi)
        solver.project(xi, w.boundary, obs, xb, lam, iters)
        res = torch.zeros(w.batch, device="cuda")
        solver.residuals(xb, obs, res)
        keep = res <= tol
        x = build_inputs(w, xi, k_obs)
        t = ((xb - xi) / OUT_SCALE).reshape(w.batch, -1)
        xs.append(x[keep])
        ts.append(t[keep])
        solver.close()
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


def warm_start(solver: "tj.Solver", net: Net, w, xi, obs, k_obs, flags=None):
    """(xb0, lam0, flags): network prediction with the per-sample cold fallback."""
    import torch
    st = torch.cuda.current_stream().cuda_stream
    B = xi.shape[0]
    x = build_inputs(w, xi, k_obs)
    y = net.forward(x)
    xb0 = torch.empty_like(xi)
    lam0 = torch.empty_like(xi)
    fl = flags if flags is not None else torch.zeros(B, dtype=torch.int32, device="cuda")
    tj.trajam_warm_apply(B, w.dims, w.n_v, y.data_ptr(), xi.data_ptr(), OUT_SCALE,
                         xb0.data_ptr(), lam0.data_ptr(), fl.data_ptr(), st)
    rw = torch.empty(B, device="cuda")
    rc = torch.empty(B, device="cuda")
    solver.residuals(xb0, obs, rw)
    solver.residuals(xi, obs, rc)
    tj.trajam_warm_fallback(B, w.dims, w.n_v, rw.data_ptr(), rc.data_ptr(), xi.data_ptr(),
                            xb0.data_ptr(), lam0.data_ptr(), fl.data_ptr(), st)
    return xb0, lam0, fl


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
