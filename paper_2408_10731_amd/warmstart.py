"""Learned warm start of the projection (no thesis counterpart; its future-work
chapter names learning-based methods).  Marshalling around the library's kernels:
the network is trained and evaluated by trajam_mlp_*, and the warm start is built by
trajam_project, trajam_warm_* and trajam_residuals.

Why a jump of the AM state.  The multiplier of the projection lives in coefficient
space, so every feasible xb with lam = xb - xi is a fixed point of the iteration:
where the iteration lands depends on its path, and the converged state is not a
function of the scene and the sample that a network could learn.  What is a smooth
function is the map from an early state of the cold iteration to the state at which
the cold iteration first reaches the residual tolerance.  So the warm start is

    probe:  k0 cold AM iterations from (xi, 0)            -> (xb_p, lam_p)
    jump:   xb_w = xb_p + network(xb_p - xi, lam_p) on the free coefficients,
            lam_w = xb_w - xi there (the multiplier of a fixed point)
    check:  per sample, keep the probe state unless the jump lowers the residual

and the projection continues from (xb_w, lam_w).  With the fixed-point multiplier a
feasible jump is a fixed point, and an almost feasible one settles nearby instead of
following the cold iteration's oscillations.  The network is trained on
solver-generated pairs (probe state -> coefficients of the first state with
residual <= tol); the boundary coefficients are untouched (exact after the first
iteration).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import trajam as tj
from . import workloads as wl

K0 = 3          # cold iterations of the probe
IN_SCALE = 1.0
OUT_SCALE = 1.0


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


def widths_for(w, hidden: int = 256):
    """[2 D n_v, hidden, hidden, D n_v]: probe state in, coefficient jump out."""
    dim = w.dims * w.n_v
    return [2 * dim, hidden, hidden, dim]


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
        self.loss = torch.zeros(tj.MLP_MSE_LOSS_FLOATS, device=dev)   # [0] is the loss

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
        return self.loss[:1]


@dataclasses.dataclass
class Dataset:
    x: object       # [N, 2 dim] device float32: probe features
    t: object       # [N, dim] device float32: (coefficients at first hit - probe) / OUT_SCALE
    n_scenes: int


def generate(scene_fn, seeds, samples_per_scene, k0=K0, cap=150, tol=1e-3, chunk=256):
    """Solver-generated pairs.  The scenes of one family are taken `chunk` at a time:
    a fixed pool of solvers and device buffers is refilled with the chunk's obstacles
    and samples, and the cold iteration runs one AM iteration per ragged launch over
    the whole chunk; the probe state after k0 iterations is kept, and each sample's
    first state (after the probe) whose residual is <= tol is recorded.  Samples that
    reach tol within `cap` iterations give one pair each."""
    import torch
    seeds = [int(x) for x in seeds]
    B = int(samples_per_scene)
    w0 = scene_fn(seeds[0], B)
    n = min(chunk, len(seeds))
    D, nv, no = w0.dims, w0.n_v, w0.n_obs
    dim = D * nv
    solvers = [tj.Solver.for_workload(w0, precision="fp32", max_batch=B) for _ in range(n)]
    xi = torch.zeros((n, B, D, nv), device="cuda")
    xb, lam = torch.zeros_like(xi), torch.zeros_like(xi)
    tr = torch.zeros((n, 1, B), device="cuda")
    oc = torch.zeros((n, max(no, 1), D), device="cuda")
    ov, oa = torch.zeros_like(oc), torch.zeros_like(oc)
    x_all = torch.zeros((n * B, 2 * dim), device="cuda")
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
        for i in range(m):
            solvers[i].set_obstacles((oc[i], ov[i] if dynamic else None, oa[i]))
        key = (m, dynamic, bnd.tobytes())   # a plan bakes these in
        if key != plan_key:
            if plan is not None:
                plan.close()
            plan = tj.RaggedPlan([(solvers[i], xi[i], bnd, xb[i], lam[i], tr[i]) for i in range(m)], 1)
            plan_key = key
        xb[:m].copy_(xi[:m])
        lam[:m].zero_()
        for _ in range(k0):
            plan.launch()
        xp, lp = xb[:m].clone(), lam[:m].clone()
        hx = torch.zeros_like(xp)
        hit = torch.zeros((m, B), dtype=torch.bool, device="cuda")
        for k in range(k0, cap):
            px = xb[:m].clone()
            plan.launch()   # the trace holds the residual of the state before the launch
            new = (~hit) & (tr[:m, 0] <= tol)
            sel = new[:, :, None, None]
            hx = torch.where(sel, px, hx)
            hit |= new
            if (k - k0) % 16 == 15 and bool(hit.all()):
                break
        x = x_all[:m * B]
        tj.trajam_warm_features(m * B, D, nv, xi[:m].data_ptr(), xp.data_ptr(), lp.data_ptr(),
                                1.0 / IN_SCALE, x.data_ptr(), torch.cuda.current_stream().cuda_stream)
        t = (hx - xp).reshape(m * B, dim) / OUT_SCALE
        keep = hit.reshape(-1)
        xs.append(x[keep].clone())
        ts.append(t[keep])
    torch.cuda.synchronize()
    plan.close()
    for s_ in solvers:
        s_.close()
    return Dataset(torch.cat(xs).contiguous(), torch.cat(ts).contiguous(), len(seeds))


def generate_mixed(scene_fns, seeds, samples_per_scene, k0=K0, cap=150, tol=1e-3, chunk=256):
    """Pairs from several scene families that differ in their obstacle count (each
    family on its own pool of solvers, `generate`), the seeds dealt out round-robin;
    one dataset."""
    import torch
    seeds = [int(x) for x in seeds]
    parts = [generate(fn, seeds[i::len(scene_fns)], samples_per_scene, k0, cap, tol, chunk)
             for i, fn in enumerate(scene_fns) if seeds[i::len(scene_fns)]]
    return Dataset(torch.cat([d.x for d in parts]).contiguous(), torch.cat([d.t for d in parts]).contiguous(),
                   len(seeds))


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
    """The warm start of one solver: every buffer allocated once, `run` only launches
    kernels (probe projection; features, network and jump fused in one matrix-core
    launch; residual; check), so it can be captured in a graph together with the
    projection that continues from it."""

    def __init__(self, solver: "tj.Solver", net: Net, max_batch: int, k0: int = K0):
        import torch
        self.solver, self.net, self.k0 = solver, net, int(k0)
        D, nv = solver.dims, solver.nv
        self.dim = D * nv
        assert net.widths[0] == 2 * self.dim and net.widths[-1] == self.dim
        assert max(net.widths) <= 256
        assert max_batch <= net.max_batch
        shape = (max_batch, D, nv)
        self.xp = torch.zeros(shape, device="cuda")
        self.lp = torch.zeros(shape, device="cuda")
        self.xw = torch.zeros(shape, device="cuda")
        self.lw = torch.zeros(shape, device="cuda")
        nbytes = tj.trajam_warm_pack_mfma(net.shape, None, None, None)
        self.packed = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
        self.refresh()
        self.trace = torch.zeros((self.k0, max_batch), device="cuda")
        self.rw = torch.zeros(max_batch, device="cuda")
        self.flags = torch.zeros(max_batch, dtype=torch.int32, device="cuda")

    def refresh(self):
        """Re-pack the network's parameters for the matrix-core jump (after training)."""
        import torch
        tj.trajam_warm_pack_mfma(self.net.shape, self.net.params.data_ptr(), self.packed.data_ptr(),
                                 torch.cuda.current_stream().cuda_stream)

    def run(self, xi, boundary, obs, xb_out=None, lam_out=None, trace_out=None):
        """(xb_w, lam_w, flags, probe_trace) for the samples xi [B, D, n_v]: the state
        after the probe and the jump; the projection continues from it.  xb_out, lam_out
        [B, D, n_v] and trace_out [k0, B] (contiguous device tensors) receive the state
        and the probe's residual trace in place of the context's own buffers."""
        import torch
        s = self.solver
        B = xi.shape[0]
        D, nv = s.dims, s.nv
        st = torch.cuda.current_stream().cuda_stream
        xp, lp = self.xp[:B], self.lp[:B]
        xw = self.xw[:B] if xb_out is None else xb_out
        lw = self.lw[:B] if lam_out is None else lam_out
        tr = self.trace[:, :B] if trace_out is None else trace_out
        assert xw.is_contiguous() and lw.is_contiguous() and tr.is_contiguous()
        xp.copy_(xi)
        lp.zero_()
        s.project(xi, boundary, obs, xp, lp, self.k0, res_trace=tr)
        tj.trajam_warm_jump(self.net.shape, B, D, nv, self.packed.data_ptr(), 1.0 / IN_SCALE, OUT_SCALE,
                            xi.data_ptr(), xp.data_ptr(), lp.data_ptr(), xw.data_ptr(), lw.data_ptr(), st)
        rw = self.rw[:B]
        s.residuals(xw, obs, rw)
        fl = self.flags[:B]
        tj.trajam_warm_fallback(B, D, nv, rw.data_ptr(), tr[self.k0 - 1].data_ptr(),
                                xp.data_ptr(), lp.data_ptr(), xw.data_ptr(), lw.data_ptr(),
                                fl.data_ptr(), st)
        return xw, lw, fl, tr


def iterations_to(trace, tol=1e-3):
    """1-based index of the first iteration whose batch-median residual is <= tol."""
    med = np.median(np.asarray(trace), axis=1)
    hit = np.nonzero(med <= tol)[0]
    return int(hit[0]) + 1 if hit.size else None


def family_scene(family: str):
    """Scene generators for training / evaluation families (seeded, synthetic)."""
    if family == "cfg2":
        return lambda seed, batch: wl.config2(batch=batch, seed=seed)
    if family == "cfg4":
        return lambda seed, batch: wl.config4_scene(seed, batch=batch)
    if family.startswith("2d-n"):
        # the config-2 geometry with a given number of circles (the single-robot
        # problems of the ragged set draw it from 5..300)
        n_obs = int(family[4:])
        return lambda seed, batch: wl.problem2d(seed, n_obs, batch)
    raise ValueError(family)


class RaggedWarmStart:
    """The learned warm start for the single-robot problems of a ragged set (all of one
    family: the network's dims and n_v), with the per-sample cold fallback:

        probe:    one ragged launch of k0 iterations over every problem from (xi, 0);
        jump:     one fused launch over all the problems' samples;
        check:    per problem the residual of the jumped state against the probe's last
                  residual (trajam_residuals, trajam_warm_fallback);
        continue: one ragged launch of iters - k0 iterations from the checked state.

    The problems' samples and states live in shared buffers, problem after problem, so
    the jump is one launch; `states()` gives each problem's (xi_bar, lambda) views.  A
    cold plan of `iters` iterations over the same problems is built beside it for
    comparison (`run_cold`).  Every method only launches kernels (capturable)."""

    def __init__(self, solvers, xis, boundaries, net: Net, iters: int, k0: int = K0, trace: bool = True):
        import torch
        self.solvers, self.net, self.k0, self.K = list(solvers), net, int(k0), int(iters)
        D, nv = self.solvers[0].dims, self.solvers[0].nv
        if any(s.dims != D or s.nv != nv or s.n_agents != 1 for s in self.solvers):
            raise ValueError("one family of single-robot problems")
        if not 0 < self.k0 < self.K:
            raise ValueError("0 < k0 < iters")
        self.D, self.nv = D, nv
        sizes = [int(x.shape[0]) for x in xis]
        self.off = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
        Bt = int(self.off[-1])
        dev = "cuda"
        self.X = torch.cat([x.reshape(-1, D, nv) for x in xis]).contiguous()
        self.XB, self.LAM = torch.zeros_like(self.X), torch.zeros_like(self.X)
        self.XW, self.LW = torch.zeros_like(self.X), torch.zeros_like(self.X)
        self.RW = torch.zeros(Bt, device=dev)
        self.FL = torch.zeros(Bt, dtype=torch.int32, device=dev)
        # per problem: the probe's trace [k0][B_i], the continuation's [K - k0][B_i] and
        # the cold plan's [K][B_i], each a contiguous chunk
        self.TP = torch.zeros(self.k0 * Bt, device=dev)
        self.TC = torch.zeros((self.K - self.k0) * Bt if trace else 1, device=dev)
        self.TK = torch.zeros(self.K * Bt if trace else 1, device=dev)
        self.boundaries = [np.asarray(b, dtype=np.float64) for b in boundaries]
        v = self._views
        self.probe = tj.RaggedPlan([(s, v(self.X, i), self.boundaries[i], v(self.XB, i), v(self.LAM, i),
                                     self._trace(self.TP, self.k0, i)) for i, s in enumerate(self.solvers)],
                                   self.k0)
        self.rest = tj.RaggedPlan([(s, v(self.X, i), self.boundaries[i], v(self.XW, i), v(self.LW, i))
                                   + ((self._trace(self.TC, self.K - self.k0, i),) if trace else ())
                                   for i, s in enumerate(self.solvers)], self.K - self.k0)
        self.cold = tj.RaggedPlan([(s, v(self.X, i), self.boundaries[i], v(self.XB, i), v(self.LAM, i))
                                   + ((self._trace(self.TK, self.K, i),) if trace else ())
                                   for i, s in enumerate(self.solvers)], self.K)
        nbytes = tj.trajam_warm_pack_mfma(net.shape, None, None, None)
        self.packed = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
        tj.trajam_warm_pack_mfma(net.shape, net.params.data_ptr(), self.packed.data_ptr(),
                                 torch.cuda.current_stream().cuda_stream)

    def _views(self, T, i):
        return T[self.off[i]:self.off[i + 1]]

    def _trace(self, T, k, i):
        B0, B1 = int(self.off[i]), int(self.off[i + 1])
        return T[k * B0:k * B1].view(k, B1 - B0)

    def traces(self, cold: bool = False):
        """Per problem, the residual trace [K, B_i] of the last run (warm: probe rows then
        the continuation's)."""
        import torch
        out = []
        for i in range(len(self.solvers)):
            if cold:
                out.append(self._trace(self.TK, self.K, i))
            else:
                out.append(torch.cat([self._trace(self.TP, self.k0, i), self._trace(self.TC, self.K - self.k0, i)]))
        return out

    def states(self, cold: bool = False):
        v = self._views
        return [(v(self.XB, i), v(self.LAM, i)) if cold else (v(self.XW, i), v(self.LW, i))
                for i in range(len(self.solvers))]

    def run(self):
        import torch
        st = torch.cuda.current_stream().cuda_stream
        self.XB.copy_(self.X)
        self.LAM.zero_()
        self.probe.launch()
        Bt = int(self.off[-1])
        tj.trajam_warm_jump(self.net.shape, Bt, self.D, self.nv, self.packed.data_ptr(), 1.0 / IN_SCALE, OUT_SCALE,
                            self.X.data_ptr(), self.XB.data_ptr(), self.LAM.data_ptr(), self.XW.data_ptr(),
                            self.LW.data_ptr(), st)
        for i, s in enumerate(self.solvers):
            xw, lw = self._views(self.XW, i), self._views(self.LW, i)
            rw, fl = self._views(self.RW, i), self._views(self.FL, i)
            s.residuals(xw, None, rw)
            rc = self._trace(self.TP, self.k0, i)[self.k0 - 1]
            tj.trajam_warm_fallback(int(rw.shape[0]), self.D, self.nv, rw.data_ptr(), rc.data_ptr(),
                                    self._views(self.XB, i).data_ptr(), self._views(self.LAM, i).data_ptr(),
                                    xw.data_ptr(), lw.data_ptr(), fl.data_ptr(), st)
        self.rest.launch()

    def run_cold(self):
        self.XB.copy_(self.X)
        self.LAM.zero_()
        self.cold.launch()

    def close(self):
        for p in (self.probe, self.rest, self.cold):
            p.close()
