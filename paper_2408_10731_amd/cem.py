"""Projection-guided sampling loop on the GPU (thesis ch. 6, Alg 3), driving the
C-ABI kernels on one stream: the obstacles are packed once per call, then sample
(with the projection's cold start) -> project -> residuals -> cost -> select ->
update, N times.  Marshalling only; every step runs in the library.

The standard normal draws z [N, N_b, dim] are an input.  All iterations can be
captured into one HIP graph (`capture=True`): the loop never synchronizes with the
host, so a replay re-runs the whole planning call with one launch.
"""
from __future__ import annotations

import numpy as np

from . import trajam as tj


def draw(n_iterations: int, n_samples: int, dim: int, key: int, counter: int = 0, fp64: bool = False):
    """The loop's standard normal draws z [n_iterations, n_samples, dim] from the
    library's counter-based generator (one stream, iteration after iteration)."""
    import torch
    z = torch.empty((n_iterations, n_samples, dim), dtype=torch.float64 if fp64 else torch.float32,
                    device="cuda")
    tj.trajam_normals(z.numel(), key, counter, fp64, z.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return z


class Planner:
    """warm: a warmstart.WarmContext of the same solver (max batch >= n_samples).  With
    it every projection starts from the learned warm start -- its probe's k0 cold
    iterations, the network's jump and the per-sample cold fallback -- and continues
    for am_iters - k0 iterations, so a projection still costs am_iters AM iterations."""

    def __init__(self, solver: "tj.Solver", n_samples: int, n_proj: int, n_elite: int,
                 am_iters: int, sigma: float = 0.5, gamma: float = 1.0, quantum: float = 1e-6,
                 warm=None):
        import torch
        self.s = solver
        self.torch = torch
        self.N_b, self.n_proj, self.n_elite = int(n_samples), int(n_proj), int(n_elite)
        self.K = int(am_iters)
        self.warm = warm
        if warm is not None and not (warm.solver is solver and 0 < warm.k0 < self.K):
            raise ValueError("warm start: a context of this solver with 0 < k0 < am_iters")
        self.sigma, self.gamma, self.quantum = float(sigma), float(gamma), float(quantum)
        D, nv, dt = solver.dims, solver.nv, solver.dtype
        self.dim = D * nv
        dev = "cuda"
        self.xi = torch.zeros((self.N_b, D, nv), dtype=dt, device=dev)
        self.xb = torch.zeros_like(self.xi)
        self.lam = torch.zeros_like(self.xi)
        self.res = torch.zeros(self.N_b, dtype=dt, device=dev)
        self.caug = torch.zeros_like(self.res)
        self.rkey = torch.zeros(self.N_b, dtype=torch.int32, device=dev)
        self.proj = torch.zeros(self.n_proj, dtype=torch.int32, device=dev)
        self.elite = torch.zeros(self.n_elite, dtype=torch.int32, device=dev)
        self.mu = torch.zeros(self.dim, dtype=dt, device=dev)
        self.Sigma = torch.zeros((self.dim, self.dim), dtype=dt, device=dev)
        self.chol = torch.zeros_like(self.Sigma)
        self.trace = torch.zeros((self.K, self.N_b), dtype=dt, device=dev)  # residual per AM iteration
        self.flags = None   # warm start: the last projection's fallback flags
        self.graph = None

    def set_distribution(self, mu0, Sigma0, chol0):
        """Initial distribution: mean, covariance and its lower Cholesky factor."""
        t = self.torch
        self.mu.copy_(t.as_tensor(np.asarray(mu0).reshape(-1), dtype=self.mu.dtype))
        self.Sigma.copy_(t.as_tensor(np.asarray(Sigma0), dtype=self.mu.dtype))
        self.chol.copy_(t.as_tensor(np.asarray(chol0), dtype=self.mu.dtype))

    def _iteration(self, z_l, boundary, obs, stream, record=None):
        h, st = self.s.handle, stream.cuda_stream
        tj.trajam_cem_sample(h, self.N_b, self.mu.data_ptr(), self.chol.data_ptr(),
                             z_l.data_ptr(), self.xi.data_ptr(), self.xb.data_ptr(),
                             self.lam.data_ptr(), st)
        # obstacles were packed once for the whole call (None reuses them)
        if self.warm is None:
            self.s.project(self.xi, boundary, None, self.xb, self.lam, self.K, res_trace=self.trace,
                           stream=stream)
        else:
            k0 = self.warm.k0
            _, _, fl, _ = self.warm.run(self.xi, boundary, None, xb_out=self.xb, lam_out=self.lam,
                                        trace_out=self.trace[:k0])
            self.s.project(self.xi, boundary, None, self.xb, self.lam, self.K - k0, res_trace=self.trace[k0:],
                           stream=stream)
            self.flags = fl
        self.s.residuals(self.xb, None, self.res, stream=stream)
        tj.trajam_cem_cost(h, self.N_b, self.xb.data_ptr(), self.res.data_ptr(), self.quantum,
                           self.caug.data_ptr(), self.rkey.data_ptr(), st)
        tj.trajam_cem_select(h, self.N_b, self.rkey.data_ptr(), self.caug.data_ptr(),
                             self.n_proj, self.n_elite, self.proj.data_ptr(),
                             self.elite.data_ptr(), st)
        if record is not None:
            record.append((self.proj.clone(), self.elite.clone(), self.res.clone(),
                           self.caug.clone(), self.rkey.clone()))
        tj.trajam_cem_update(h, self.n_elite, self.elite.data_ptr(), self.xb.data_ptr(),
                             self.caug.data_ptr(), self.sigma, self.gamma, self.mu.data_ptr(),
                             self.Sigma.data_ptr(), self.chol.data_ptr(), st)
        if record is not None:
            record[-1] = record[-1] + (self.mu.clone(), self.Sigma.clone(), self.xb.clone(), self.trace.clone())

    def autotune(self, z0, boundary, obs):
        """Pick the projection's launch shape for this planner's batch: draws one batch
        from the current distribution with the draws z0 [N_b, dim] and times every
        shape on it with the planner's iteration count.  Returns (kernel, samples/WG)."""
        st = self.torch.cuda.current_stream()
        tj.trajam_cem_sample(self.s.handle, self.N_b, self.mu.data_ptr(), self.chol.data_ptr(),
                             z0.data_ptr(), self.xi.data_ptr(), self.xb.data_ptr(),
                             self.lam.data_ptr(), st.cuda_stream)
        return self.s.autotune(self.xi, boundary, obs, self.xb, self.lam, probe_iters=self.K)

    def best(self):
        """The returned trajectory of Alg 3: the projected sample of the last elite
        set with the lowest c_aug (elite_idx[0]); gathered on the device."""
        return self.torch.index_select(self.xb, 0, self.elite[:1].long())[0]

    def run(self, z, boundary, obs, record=None, stream=None):
        """z: [N, N_b, dim] device tensor.  Returns best() after the N iterations."""
        self._loop(z, boundary, obs, record, stream)
        return self.best()

    def _loop(self, z, boundary, obs, record=None, stream=None):
        stream = stream or self.torch.cuda.current_stream()
        if self.s.problem.n_obstacles:
            self.s.set_obstacles(obs, stream=stream)
        for l in range(z.shape[0]):
            self._iteration(z[l], boundary, obs, stream, record)

    def capture(self, z, boundary, obs):
        """Capture all N iterations into one HIP graph (replay with `replay`)."""
        t = self.torch
        s = t.cuda.Stream()
        s.wait_stream(t.cuda.current_stream())
        with t.cuda.stream(s):  # warm-up outside capture
            self._loop(z, boundary, obs, stream=s)
        t.cuda.current_stream().wait_stream(s)
        g = t.cuda.CUDAGraph()
        with t.cuda.graph(g):
            self._loop(z, boundary, obs)
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()
        return self.best()
