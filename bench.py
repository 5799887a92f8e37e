"""Benchmark of the MI355X AM projection (one JSON line on stdout).

Workload (one "step"): one full projection of the 2D point-robot problem with
50 static circles (radius U(0.3, 0.8) m in a 30 x 30 m box), Bernstein degree 10,
100 time samples over 30 s, batch 1024 samples, 50 AM iterations, FP32, cold start
(xb = xi, lambda = 0).  Inputs are seeded and synthetic and already resident in
HBM when the timed region starts.

metric: traj-iters/s = batch * iterations / (wall time of one projection).
Also reported: time until the batch-median residual first reaches 1e-3 (cold
start; learned warm start when a trained network is available), the roofline of
the fused AM kernel (VALU-bound: algorithmic lane-ops / kernel time against the
chip's 256 CU x 64 lanes x 2.4 GHz), and the FP64 CPU oracle timed on a bounded
sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_VALU_OPS = 256 * 64 * 2.4e9  # lane-ops/s, one FMA = one op (no packed FP32)


def algorithmic_ops_per_traj_iter(w) -> float:
    """VALU lane-ops one trajectory-iteration needs at minimum.

    * obstacle inside test per (obstacle, time): per axis one subtraction and one
      FMA (plus one FMA per axis for moving obstacles), i.e. 2D static circle = 4;
    * waypoint map p, v, a: 3 D n_v FMAs per time sample;
    * F^T r contraction: 3 D n_v FMAs per time sample;
    * kinematic tests: 2 (D + 1) per time sample;
    * multiplier, defect and QP: D n_v (3 + (n_v - 4)).
    """
    D, nv, np_, no = w.dims, w.n_v, w.n_steps, w.n_obs
    dyn = bool(np.any(w.obs_vel))
    per_obs = D * (3 if dyn else 2) + (0 if np.all(w.obs_axes == w.obs_axes[:, :1]) else D)
    return (no * np_ * per_obs + np_ * (6 * D * nv + 2 * (D + 1)) + D * nv * (3 + max(nv - 4, 0)))


def median_time_to_residual(trace: np.ndarray, tol: float = 1e-3):
    med = np.median(trace, axis=1)
    hit = np.nonzero(med <= tol)[0]
    return (int(hit[0]) if hit.size else None), med


def cpu_baseline(w, iters_sample: int):
    import oracle
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.project(w, iters=iters_sample, n_threads=threads)
    dt = time.perf_counter() - t0
    return {"value": w.batch * iters_sample / dt, "unit": "traj-iters/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{w.batch} trajectories x {iters_sample} AM iterations of the same "
                      f"workload, FP64 C oracle, OpenMP over trajectories ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--ttr-cap", type=int, default=300)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(samples are independent: a multi-GPU run shards the batch "
                                   "with no communication)"}))
        sys.exit(2)

    import torch
    from paper_2408_10731_amd import trajam as tj
    from paper_2408_10731_amd import workloads as wl

    w = wl.config2(batch=args.batch)
    K = args.iters
    solver = tj.Solver.for_workload(w, precision="fp32")
    xi, obs = tj.device_workload(w, torch.float32)
    xb = xi.clone()
    lam = torch.zeros_like(xi)
    trace = torch.zeros((K, w.batch), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        xb.copy_(xi)
        lam.zero_()
        solver.project(xi, w.boundary, obs, xb, lam, K, res_trace=trace)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # per-launch kernel time (events on the launch stream), then the timed region
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for i in range(args.steps):
        xb.copy_(xi)
        lam.zero_()
        ev[i][0].record(stream)
        solver.project(xi, w.boundary, obs, xb, lam, K, res_trace=trace)
        ev[i][1].record(stream)
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_start.elapsed_time(t_end)
    launch_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    ms_per_step = total_ms / args.steps
    value = w.batch * K / (ms_per_step * 1e-3)

    ops = algorithmic_ops_per_traj_iter(w) * w.batch * K
    achieved = ops / (launch_ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_OPS / 1e12,
                "unit": "Tops/s", "frac": achieved / PEAK_VALU_OPS, "traffic": None,
                "kernel": "am_project_kernel<float,2,12>",
                "ops_per_traj_iter": algorithmic_ops_per_traj_iter(w),
                "launch_ms": launch_ms}

    # time to batch-median residual <= 1e-3, cold start
    cap = args.ttr_cap
    tr_long = torch.zeros((cap, w.batch), dtype=torch.float32, device="cuda")
    xb.copy_(xi); lam.zero_()
    solver.project(xi, w.boundary, obs, xb, lam, cap, res_trace=tr_long)
    torch.cuda.synchronize()
    hit, med = median_time_to_residual(tr_long.cpu().numpy())
    ttr = {"cold_iters": None if hit is None else hit + 1, "cold_ms": None, "cap": cap}
    if hit is not None:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        xb.copy_(xi); lam.zero_()
        torch.cuda.synchronize()
        e0.record(stream)
        solver.project(xi, w.boundary, obs, xb, lam, hit + 1)
        e1.record(stream)
        torch.cuda.synchronize()
        ttr["cold_ms"] = e0.elapsed_time(e1)

    out = {
        "metric": "traj-iters/s & time-to-residual<=1e-3, learned warm-start vs cold, 1 MI355X",
        "value": value, "unit": "traj-iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "2D point robot, 50 static circles r~U(0.3,0.8) m in 30x30 m, "
                               "Bernstein degree 10, 100 steps over 30 s, batch 1024, "
                               "50 AM iterations, cold start",
                   "batch": w.batch, "iterations": K, "obstacles": w.n_obs,
                   "timesteps": w.n_steps, "degree": w.degree, "precision": "fp32"},
        "roofline": roofline,
        "time_to_residual": ttr,
        "wall_s_timed_region": wall,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, 20)
    print(json.dumps(out), flush=True)
    solver.close()


if __name__ == "__main__":
    main()
