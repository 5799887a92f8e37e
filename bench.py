"""Benchmark of the MI355X AM projection (one JSON line on stdout).

Workload (one "step"): one full projection of config 3 -- the 3D point robot among
200 static ellipsoids (semi-axes U(0.3, 1.0) m each, centres in 20 x 20 x 6 m),
Bernstein degree 15, 150 time samples over 20 s, batch 4096 samples, 50 AM
iterations, FP32, cold start (xb = xi, lambda = 0), the residual trace written.
Inputs are seeded and synthetic and already resident in HBM when the timed region
starts; the scene's obstacles are packed into the solver once before it.

metric: traj-iters/s = batch * iterations / (wall time of one projection).
The roofline of the projection kernel counts the algorithmic work of one
trajectory-iteration (every obstacle and kinematic element at the lower end of its
VALU cost, the waypoint map, the F^T contraction and the QP) against the chip's
non-packed VALU rate; beside it, the VALU issue fraction and the HBM traffic that
hardware counters (rocprofv3 --pmc, in child processes of this run) give for one
launch of the same kernel.  Also reported: config 2 (2D, the former headline) with
the same roofline, the time until the batch-median residual first reaches 1e-3 from
a cold start and from the learned warm start (network trained here first, untimed),
the ragged set of 256 problems (half of them multi-agent) in one plan, one
graph-replayed planning call of the sampling loop, config 3 in FP64 / FP32 / BF16
with the reduced precisions' deviation from FP64, the materialised polar variables
against the HBM peak, and the FP64 CPU oracle timed on a bounded sample of the
headline workload (median of 5 runs) on the host cores and on one thread, with its
time to the residual tolerance.
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

PEAK_VALU_OPS = 256 * 64 * 2.4e9   # lane-ops/s, one FMA = one op (no packed FP32)
PEAK_VALU_INSTS = 256 * 2.4e9      # wave64 VALU instructions/s: 4 SIMDs x 16 lanes per CU per clock
PEAK_HBM = 8.0e12                  # bytes/s


def survey_ops_per_unit(w) -> int:
    """Algorithmic VALU lane-ops of one trajectory-iteration, counted the way the work
    is specified, not the way the kernel does it: every (obstacle, time) and every
    kinematic (block, time) element at the lower end of its cost (12 ops for a 2D
    circle, 20 for a 3D ellipsoid), the waypoint map plus the F^T contraction
    (2 D 3 n_p n_v FMAs) and the QP (D n_v (n_v + 4) FMAs); an FMA counts once.  The
    kernel skips every inside test that exact culling proves zero, so it can do this
    work faster than the VALU peak allows (frac > 1)."""
    D, nv, np_, no = w.dims, w.n_v, w.n_steps, w.n_obs
    kin = (w.v_max > 0) + (w.a_max > 0)
    elements = no * np_ + kin * np_
    per_el = 20 if D == 3 else 12
    return elements * per_el + 2 * D * 3 * np_ * nv + D * nv * (nv + 4)


def state_bytes_per_launch(w, K, word=4) -> int:
    """Bytes one launch must move: xi, xb, lambda read, xb, lambda written, the
    residual trace written."""
    return 5 * w.batch * w.dims * w.n_v * word + K * w.batch * word


def median_time_to_residual(trace: np.ndarray, tol: float = 1e-3):
    med = np.median(trace, axis=1)
    hit = np.nonzero(med <= tol)[0]
    return (int(hit[0]) if hit.size else None), med


def _graph(fn):
    """Capture fn() (after a warm-up run on a side stream) into a graph."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


def _time(fn, reps, stream):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def train_warm_start(w, scenes, epochs, seed0=20_000, batch=512):
    """Network of the learned warm start, trained on the GPU on solver-generated pairs
    (probe state -> state at the first residual <= 1e-3) of the workload's family,
    with scene seeds disjoint from the benchmark scene's."""
    import torch
    from paper_2408_10731_amd import warmstart as ws
    t0 = time.perf_counter()
    data = ws.generate(ws.family_scene("cfg2"), list(range(seed0, seed0 + scenes)), 64,
                       k0=ws.K0, cap=150)
    net = ws.Net(ws.widths_for(w), seed=0, precision=1, max_batch=max(batch, w.batch))
    curve = ws.train(net, data, epochs=epochs, batch=batch, lr=1e-3)
    torch.cuda.synchronize()
    info = {"pairs": int(data.x.shape[0]), "scenes": scenes, "epochs": epochs, "precision": "bf16 matrix cores",
            "loss_first": curve[0], "loss_last": curve[-1],
            "seconds": time.perf_counter() - t0}
    return net, info


def ttr_scene(w, solver, xi, obs, net, cap, stream, tol=1e-3, reps=20):
    """Cold vs learned warm start on one scene: AM iterations until the batch-median
    residual first reaches tol (the warm start's 3-iteration probe included) and the
    time of that work, per replay of a captured graph (cold: resets + projection;
    warm: probe, features, fused network, jump, residual, check + projection) and
    launched eagerly."""
    import torch
    from paper_2408_10731_amd import warmstart as ws

    out = {}
    solver.set_obstacles(obs)   # packed once for the scene; the calls below reuse them
    obs = None
    tr = torch.zeros((cap, w.batch), dtype=torch.float32, device="cuda")
    xb, lam = xi.clone(), torch.zeros_like(xi)
    solver.project(xi, w.boundary, obs, xb, lam, cap, res_trace=tr)
    torch.cuda.synchronize()
    ic = ws.iterations_to(tr.cpu().numpy(), tol)
    out["cold_iters"] = ic
    ctx = ws.WarmContext(solver, net, w.batch)
    xw, lw, fl, trp = ctx.run(xi, w.boundary, obs)
    trw = torch.zeros((cap - ws.K0, w.batch), dtype=torch.float32, device="cuda")
    solver.project(xi, w.boundary, obs, xw, lw, cap - ws.K0, res_trace=trw)
    torch.cuda.synchronize()
    iw = ws.iterations_to(np.concatenate([trp.cpu().numpy(), trw.cpu().numpy()]), tol)
    out["warm_iters"] = iw
    out["warm_fallbacks"] = int(((fl.cpu().numpy() & 4) != 0).sum())
    # a start that never reaches tol within the cap is timed over the whole cap (a
    # lower bound of its time to tol) and marked as not reached
    out["cold_reached"], out["warm_reached"] = ic is not None, iw is not None
    n_cold = ic if ic is not None else cap
    n_warm = iw if iw is not None else cap
    if n_cold > 0:
        def cold():
            xb.copy_(xi)
            lam.zero_()
            solver.project(xi, w.boundary, obs, xb, lam, n_cold)
        out["cold_ms_eager"] = _time(cold, reps, stream)
        g = _graph(cold)
        out["cold_ms"] = _time(g.replay, reps, stream)
        del g
    if n_warm > 0:
        rest = max(n_warm - ws.K0, 0)

        def warm():
            b0, l0, _, _ = ctx.run(xi, w.boundary, obs)
            solver.project(xi, w.boundary, obs, b0, l0, rest)
        out["warm_ms_eager"] = _time(warm, reps, stream)
        g = _graph(warm)
        out["warm_ms"] = _time(g.replay, reps, stream)
        del g
    return out


CONTINUATION = (10, 2.0, 10, 0.9, 1e-3)   # levels, growth, window, stall ratio, tol


def continuation_leg(w, cap, stream, tol=1e-3, reps=10):
    """The benchmark scene from a cold start, plain and with the penalty continuation
    (a ladder of 10 penalties rho 2^l, a check every 10 iterations raising a sample's
    penalty while its residual is above tol and above 0.9 x its residual at the
    previous check): the first iteration at which the batch-median residual is <= tol,
    the iteration from which it stays <= tol up to the cap, the fraction of samples
    within tol at the cap, and the graph-replayed time of the projection to the cap."""
    import torch
    from paper_2408_10731_amd import trajam as tj
    solver = tj.Solver.for_workload(w, precision="fp32")
    xi, obs = tj.device_workload(w, torch.float32)
    solver.set_launch(1, 1)
    solver.set_obstacles(obs)
    solver.set_continuation(*CONTINUATION)
    xb, lam = xi.clone(), torch.zeros_like(xi)
    state = solver.cont_state(w.batch)
    tr = torch.zeros((cap, w.batch), dtype=torch.float32, device="cuda")

    def metrics(trace):
        med = np.median(trace, axis=1)
        hit = np.nonzero(med <= tol)[0]
        bad = np.nonzero(med > tol)[0]
        stay = (None if bad.size and bad[-1] == len(med) - 1 else (int(bad[-1]) + 2 if bad.size else 1))
        return {"first": int(hit[0]) + 1 if hit.size else None, "stays_from": stay,
                "frac_within_tol_at_cap": float(np.mean(trace[-1] <= tol)),
                "median_at_cap": float(med[-1])}

    out = {"ladder": dict(zip(("levels", "growth", "window", "stall_ratio", "tol"), CONTINUATION)), "cap": cap}
    for name, cont in (("plain", False), ("continuation", True)):
        def run():
            xb.copy_(xi)
            lam.zero_()
            if cont:
                state.zero_()
                solver.project_continuation(xi, w.boundary, None, xb, lam, state, cap, res_trace=tr)
            else:
                solver.project(xi, w.boundary, None, xb, lam, cap, res_trace=tr)
        run()
        torch.cuda.synchronize()
        m = metrics(tr.cpu().numpy())
        g = _graph(run)
        m["ms_to_cap"] = _time(g.replay, reps, stream)
        del g
        if cont:
            m["levels_at_cap"] = np.bincount(solver.cont_levels(state)[0], minlength=CONTINUATION[0]).tolist()
        out[name] = m
    solver.close()
    return out


def time_to_residual(args, w, solver, xi, obs, stream, tol=1e-3, net=None, info=None):
    """The learned warm start against the cold start: on the benchmark scene, and summed
    over the 16 held-out scenes 90,001-90,016 of the same family (scene seeds disjoint from the training
    ones); a scene whose median never reaches tol within the cap counts the cap, in
    iterations and in time."""
    import torch
    from paper_2408_10731_amd import trajam as tj
    from paper_2408_10731_amd import warmstart as ws
    from paper_2408_10731_amd import workloads as wl

    cap = args.ttr_cap
    if net is None:
        net, info = train_warm_start(w, args.ws_scenes, args.ws_epochs)
    out = {"tol": tol, "cap": cap, "probe_iters": ws.K0, "warm_training": info,
           "scene": ttr_scene(w, solver, xi, obs, net, cap, stream, tol)}
    per, tot = [], {"cold_iters": 0, "warm_iters": 0, "cold_ms": 0.0, "warm_ms": 0.0}
    for seed in range(90_001, 90_017):
        ws_ = wl.config2(batch=w.batch, seed=seed)
        s = tj.Solver.for_workload(ws_, precision="fp32")
        x_, o_ = tj.device_workload(ws_, torch.float32)
        r = ttr_scene(ws_, s, x_, o_, net, cap, stream, tol, reps=10)
        s.close()
        per.append({"seed": seed, **{k: r.get(k) for k in ("cold_iters", "warm_iters", "cold_ms",
                                                           "warm_ms", "cold_reached", "warm_reached")}})
        tot["cold_iters"] += r["cold_iters"] if r["cold_iters"] is not None else cap
        tot["warm_iters"] += r["warm_iters"] if r["warm_iters"] is not None else cap
        tot["cold_ms"] += r.get("cold_ms", 0.0)
        tot["warm_ms"] += r.get("warm_ms", 0.0)
    out["held_out"] = {"scenes": per, "total": tot}
    return out


def warm_cfg4_bench(args, tol=1e-3):
    """The learned warm start where config 4 uses it: inside the sampling loop among
    moving obstacles.  A network is trained (bf16, matrix cores) on solver-generated
    pairs of config-4 scenes (seeds from 40,000, disjoint from the held-out ones); then
      - time to residual, cold against warm, on the 16 held-out config-4 scenes
        90,001-90,016 (2000 samples each, the planner's first-iteration distribution:
        straight line plus N(0, 0.5^2) per coefficient; a scene whose median never
        reaches tol within the cap counts the cap, in iterations and in time);
      - one planning call of the loop (30 iterations x 2000 samples x 15 AM
        iterations) on the benchmark scene, cold and with the warm start (3-iteration
        probe, jump, fallback, 12 more iterations: the same 15 AM iterations a
        projection), on the same draws: time per call (graph replay), and per CEM
        iteration the batch-median residual after the 15 iterations and the first
        iteration at which it is <= tol."""
    import torch
    from paper_2408_10731_amd import cem
    from paper_2408_10731_amd import trajam as tj
    from paper_2408_10731_amd import warmstart as ws
    from paper_2408_10731_amd import workloads as wl

    stream = torch.cuda.current_stream()
    cap = args.ttr_cap
    t0 = time.perf_counter()
    data = ws.generate(ws.family_scene("cfg4"), list(range(40_000, 40_000 + args.ws4_scenes)), 64,
                       k0=ws.K0, cap=150)
    t_gen = time.perf_counter() - t0
    w4 = wl.config4(batch=2000)
    net = ws.Net(ws.widths_for(w4), seed=0, precision=1, max_batch=2000)
    curve = ws.train(net, data, epochs=args.ws_epochs, batch=512, lr=1e-3)
    torch.cuda.synchronize()
    out = {"tol": tol, "cap": cap, "probe_iters": ws.K0,
           "training": {"family": "config 4 (100 moving circles)", "scenes": args.ws4_scenes,
                        "pairs": int(data.x.shape[0]), "epochs": args.ws_epochs, "precision": "bf16 matrix cores",
                        "loss_first": curve[0], "loss_last": curve[-1], "generate_s": t_gen,
                        "seconds": time.perf_counter() - t0}}
    per, tot = [], {"cold_iters": 0, "warm_iters": 0, "cold_ms": 0.0, "warm_ms": 0.0, "warm_wins_iters": 0,
                    "warm_wins_time": 0}
    for seed in range(90_001, 90_017):
        w_ = wl.config4_scene(seed, batch=2000)
        s_ = tj.Solver.for_workload(w_, precision="fp32")
        x_, o_ = tj.device_workload(w_, torch.float32)
        r = ttr_scene(w_, s_, x_, o_, net, cap, stream, tol, reps=10)
        s_.close()
        ci = r["cold_iters"] if r["cold_iters"] is not None else cap
        wi = r["warm_iters"] if r["warm_iters"] is not None else cap
        per.append({"seed": seed, **{k: r.get(k) for k in ("cold_iters", "warm_iters", "cold_ms", "warm_ms",
                                                           "cold_reached", "warm_reached", "warm_fallbacks")}})
        tot["cold_iters"] += ci
        tot["warm_iters"] += wi
        tot["cold_ms"] += r.get("cold_ms", 0.0)
        tot["warm_ms"] += r.get("warm_ms", 0.0)
        tot["warm_wins_iters"] += int(wi < ci)
        tot["warm_wins_time"] += int(r.get("warm_ms", 0.0) < r.get("cold_ms", 0.0))
    out["held_out"] = {"scenes": per, "total": tot}

    # one planning call, cold and warm, on the same draws
    w = wl.config4(batch=4)
    D, nv = w.dims, w.n_v
    N, Nb, Np, Ne, K = 30, 2000, 1454, 363, 15
    mu0 = wl.line_samples(np.random.default_rng(0), 1, w.degree, w.boundary[:, 0],
                          w.boundary[:, 3], 0.0)[0].reshape(-1)
    S0 = 0.25 * np.eye(D * nv)
    L0 = np.linalg.cholesky(S0 + 1e-10 * np.eye(D * nv))
    z = cem.draw(N, Nb, D * nv, key=1)
    calls = {}
    for arm in ("cold", "warm"):
        solver = tj.Solver.for_workload(w, precision="fp32", max_batch=Nb)
        _, obs = tj.device_workload(w, torch.float32)
        ctx = ws.WarmContext(solver, net, Nb) if arm == "warm" else None
        planner = cem.Planner(solver, Nb, Np, Ne, K, warm=ctx)
        planner.set_distribution(mu0, S0, L0)
        rec = []
        planner.run(z, w.boundary, obs, record=rec)
        torch.cuda.synchronize()
        med = np.array([np.median(r[8].cpu().numpy(), axis=1) for r in rec])   # [N, K]
        first = [int(np.nonzero(m <= tol)[0][0]) + 1 if np.any(m <= tol) else None for m in med]
        best_cost = float(rec[-1][3].cpu().numpy()[int(rec[-1][1][0])])
        planner.set_distribution(mu0, S0, L0)
        planner.capture(z, w.boundary, obs)

        def call():
            planner.set_distribution(mu0, S0, L0)
            planner.replay()
        ms = _time(call, args.cem_calls, stream)
        calls[arm] = {"ms_per_planning_call": ms,
                      "median_residual_after_15": [float(m[-1]) for m in med],
                      "cem_iterations_reaching_tol": int(sum(f is not None for f in first)),
                      "first_iteration_at_tol": first,
                      "best_c_aug": best_cost}
        if arm == "warm":
            calls[arm]["fallbacks_last_iteration"] = int(((planner.flags.cpu().numpy() & 4) != 0).sum())
        del planner
        solver.close()
    out["planning_call"] = {"config": "30 CEM iterations x 2000 samples x 15 AM iterations, 100 moving "
                                      "circles, 1454 projected / 363 elite, fp32, same draws for both arms",
                            **calls}
    return out, net


def mpc_bench(args, net=None, tol=1e-3):
    """Receding-horizon loop on the config-4 benchmark scene (100 moving circles):
    1000 samples, 10 AM iterations a control cycle (the thesis's MPC budget), the time
    origin moving 1 s a cycle, 20 cycles.  Three starts of a cycle: the multipliers
    carried over from the preceding cycle (the thesis), cleared, and the learned warm
    start (network of the config-4 leg).  Per arm: the batch-median residual after each
    cycle, the cycles whose median reaches tol, and the wall time of a cycle (host
    included: the executed state is read back every cycle)."""
    import torch
    from paper_2408_10731_amd import mpc
    from paper_2408_10731_amd import trajam as tj
    from paper_2408_10731_amd import warmstart as ws
    from paper_2408_10731_amd import workloads as wl

    w = wl.config4(batch=1000)
    K, delta, n_cyc = 10, 1.0, args.mpc_cycles
    arms = [("reuse_multipliers", True, False), ("clear_multipliers", False, False)]
    if net is not None:
        arms.append(("learned_warm_start", False, True))
    out = {"config": f"config-4 scene, {w.batch} samples, {K} AM iterations a cycle, delta {delta} s, "
                     f"{n_cyc} cycles, fp32", "tol": tol}
    for name, keep, learned in arms:
        s = tj.Solver.for_workload(w, precision="fp32")
        xi0 = torch.as_tensor(w.xi, dtype=torch.float32, device="cuda")
        ctx = ws.WarmContext(s, net, w.batch) if learned else None
        m = mpc.MPC(s, xi0, w.boundary, (w.obs_centre, w.obs_vel, w.obs_axes), K, delta, keep_lambda=keep,
                    warm=ctx)
        med, wall = [], []
        for _ in range(n_cyc):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = m.cycle()
            torch.cuda.synchronize()
            wall.append(time.perf_counter() - t0)
            med.append(float(np.median(r["res"].cpu().numpy())))
        out[name] = {"median_residual_per_cycle": med, "cycles_at_tol": int(sum(x <= tol for x in med)),
                     "mean_median_residual": float(np.mean(med)),
                     "ms_per_cycle": 1e3 * float(np.median(wall[1:] if len(wall) > 1 else wall))}
        s.close()
    return out


PEAK_BF16_MFMA = 2.5e15   # dense bf16 matrix-core FLOP/s of MI355X


def mfma_bench(args):
    """The matrix-core kernels of the warm start at sizes where their products are
    large enough to time: one training step (forward, backward, Adam) of the network
    [44, 256, 256, 22] in bf16 at batch 16384, and the fused warm jump at batch 4096.
    Algorithmic FLOPs: 2 B sum(in out) forward, twice that backward (weight and input
    gradients); achieved FLOP/s against the dense bf16 peak."""
    import torch
    from paper_2408_10731_amd import trajam as tj
    from paper_2408_10731_amd import warmstart as ws
    widths = [44, 256, 256, 22]
    macs = sum(widths[l] * widths[l + 1] for l in range(len(widths) - 1))
    st = torch.cuda.current_stream()
    out = {"network": widths, "peak_TFLOPs": PEAK_BF16_MFMA / 1e12}
    B = 16384
    net = ws.Net(widths, seed=0, precision=1, max_batch=B)
    g = torch.Generator(device="cuda").manual_seed(2)
    x = torch.randn((B, widths[0]), device="cuda", generator=g)
    t = torch.randn((B, widths[-1]), device="cuda", generator=g)
    ms = _time(lambda: net.train_step(x, t, 1e-4), args.mfma_steps, st)
    fl = 6.0 * B * macs
    # bytes each product must move with fp32 activations in HBM: forward reads its
    # input and writes its output; the loss reads y, t and writes dy; the weight
    # gradient reads d and the layer input, the input gradient reads d and the mask and
    # writes the new d
    w = widths
    per_row = sum(w[l] + w[l + 1] for l in range(len(w) - 1)) + 3 * w[-1]
    per_row += sum(w[l + 1] + w[l] + (3 * w[l] + w[l + 1] if l > 0 else 0) for l in range(len(w) - 1))
    nbytes = 4.0 * B * per_row
    out["train_step"] = {"batch": B, "ms": ms, "gflop": fl / 1e9, "achieved_TFLOPs": fl / (ms * 1e-3) / 1e12,
                         "frac_of_peak": fl / (ms * 1e-3) / PEAK_BF16_MFMA, "algorithmic_MB": nbytes / 1e6,
                         "hbm_GBs": nbytes / (ms * 1e-3) / 1e9, "hbm_frac": nbytes / (ms * 1e-3) / 8e12}
    Bj, D, nv = 4096, 2, 11
    shape = tj.mlp_shape(widths)
    n = tj.trajam_warm_pack_mfma(shape, None, None, st.cuda_stream)
    packed = torch.zeros(n, dtype=torch.uint8, device="cuda")
    tj.trajam_warm_pack_mfma(shape, net.params.data_ptr(), packed.data_ptr(), st.cuda_stream)
    xi = torch.randn((Bj, D, nv), device="cuda", generator=g)
    xb, lam = xi + 0.1, torch.zeros_like(xi)
    xo, lo = torch.empty_like(xi), torch.empty_like(xi)

    def jump():
        tj.trajam_warm_jump(shape, Bj, D, nv, packed.data_ptr(), 1.0, 1.0, xi.data_ptr(), xb.data_ptr(),
                            lam.data_ptr(), xo.data_ptr(), lo.data_ptr(), st.cuda_stream)
    ms = _time(jump, args.mfma_steps, st)
    fl = 2.0 * Bj * macs
    out["warm_jump"] = {"batch": Bj, "ms": ms, "gflop": fl / 1e9, "achieved_TFLOPs": fl / (ms * 1e-3) / 1e12,
                        "frac_of_peak": fl / (ms * 1e-3) / PEAK_BF16_MFMA}
    return out


def ragged_bench(args, net=None):
    """Ragged set of many independent problems in one plan: n_obs ~ U{5..300}, batch ~
    U{32..2048}; even problems are 2D single robots (config-2 geometry), odd ones 3D
    multi-agent problems with N ~ U{16..64} agents (pair clearance 0.6 m; a batch entry
    is a joint sample).  Times the eager launch and the same launch replayed from a
    captured graph; reports trajectory-iterations per second over the whole set (a
    joint sample of N agents counts N trajectories)."""
    import torch
    from paper_2408_10731_amd import trajam as tj
    from paper_2408_10731_amd import workloads as wl

    ws = wl.config5(args.ragged_problems, iters=args.iters)
    K = args.iters
    solvers, items, keep = [], [], []
    for w in ws:
        s = tj.Solver.for_workload(w, precision="fp32")
        xi, obs = tj.device_workload(w, torch.float32)
        s.set_obstacles(obs)
        xb, lam = xi.clone(), torch.zeros_like(xi)
        solvers.append(s)
        items.append((s, xi, w.boundary, xb, lam))
        keep.append((xi, xb, lam))
    plan = tj.RaggedPlan(items, K)
    stream = torch.cuda.current_stream()

    def reset():
        for xi, xb, lam in keep:
            xb.copy_(xi)
            lam.zero_()

    reset()
    plan.launch()
    torch.cuda.synchronize()
    launch_ms = []
    for _ in range(args.ragged_steps):
        reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.launch()
        e1.record(stream)
        torch.cuda.synchronize()
        launch_ms.append(e0.elapsed_time(e1))
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        reset()
        plan.launch()
    stream.wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        reset()
        plan.launch()
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.ragged_steps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / args.ragged_steps
    trajs = sum(w.batch * w.n_agents for w in ws)
    kern = float(np.mean(launch_ms))
    elements = sum(w.batch * (w.n_agents * w.n_obs + w.n_agents * (w.n_agents - 1) // 2)
                   * w.n_steps for w in ws)
    out = {"problems": len(ws), "multi_agent_problems": sum(w.n_agents > 1 for w in ws),
           "joint_samples": sum(w.batch for w in ws), "trajectories": trajs,
           "iterations": K, "launch_ms": kern, "graph_step_ms": graph_ms,
           "traj_iters_per_s": trajs * K / (graph_ms * 1e-3),
           "polar_elements_per_s": elements * K / (kern * 1e-3),
           "mix": "even problems 2D single robot (config-2 geometry), odd 3D multi-agent "
                  "N~U{16..64}; n_obs~U{5..300}, batch~U{32..2048}; graph step includes "
                  "the resets"}
    del g
    plan.close()
    # the learned warm start on the single-robot half, with the cold fallback, against
    # the cold plan of the same problems: the config-2 network (one obstacle count) and
    # one trained on the half's own family (circle counts 5..300, held-out seeds)
    if net is not None:
        out["warm_single_robot"] = ragged_warm(args, ws, items, K, net)
    # the multi-agent half alone (its own plan): the agents kernel's time and roofline
    agent_items = [it for it, w in zip(items, ws) if w.n_agents > 1]
    agent_ws = [w for w in ws if w.n_agents > 1]
    if agent_items:
        aplan = tj.RaggedPlan(agent_items, K)
        reset()
        aplan.launch()
        torch.cuda.synchronize()
        ams = []
        for _ in range(args.ragged_steps):
            reset()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            aplan.launch()
            e1.record(stream)
            torch.cuda.synchronize()
            ams.append(e0.elapsed_time(e1))
        aplan.close()
        a_ms = float(np.mean(ams))
        ops = sum(w.batch * agents_ops_per_unit(w) for w in agent_ws) * K
        out["multi_agent"] = {
            "problems": len(agent_ws), "joint_samples": sum(w.batch for w in agent_ws),
            "agents_mean": float(np.mean([w.n_agents for w in agent_ws])), "launch_ms": a_ms,
            "roofline": {"bound": "alu", "achieved": ops / (a_ms * 1e-3) / 1e12, "peak": PEAK_VALU_OPS / 1e12,
                         "unit": "Tlane-ops/s", "frac": ops / (a_ms * 1e-3) / PEAK_VALU_OPS,
                         "ops_per_launch": ops}}
        if not args.no_counters:
            _, c = hw_counters(["--probe", "ragged", "--ragged-problems", str(args.ragged_problems),
                                "--iters", str(K)], "am_ragged_kernel", a_ms, 1)
            out["multi_agent"]["counters"] = {k: c.get(k) for k in ("sq", "valu_insts", "valu_issue_frac",
                                                                    "valu_insts_per_wave", "error")}
    for s in solvers:
        s.close()
    return out




def ragged_warm(args, ws, items, K, net_cfg2):
    import torch
    from paper_2408_10731_amd import warmstart as ws_mod
    two = [(w, it) for w, it in zip(ws, items) if w.n_agents == 1]
    t0 = time.perf_counter()
    fams = [ws_mod.family_scene(f"2d-n{n}") for n in (5, 40, 80, 120, 160, 200, 250, 300)]
    data = ws_mod.generate_mixed(fams, list(range(60_000, 60_000 + args.ws_scenes)), 64, k0=ws_mod.K0, cap=150)
    net_mix = ws_mod.Net(ws_mod.widths_for(two[0][0]), seed=0, precision=1, max_batch=512)
    curve = ws_mod.train(net_mix, data, epochs=args.ws_epochs, batch=512, lr=1e-3)
    torch.cuda.synchronize()
    training = {"pairs": int(data.x.shape[0]), "scenes": args.ws_scenes, "epochs": args.ws_epochs,
                "circle_counts": [5, 40, 80, 120, 160, 200, 250, 300], "scene_seeds": [60_000, 60_000 + args.ws_scenes - 1],
                "loss_first": curve[0], "loss_last": curve[-1], "seconds": time.perf_counter() - t0}
    del data

    def first(tr):
        med = np.median(tr, axis=1)
        hit = np.nonzero(med <= 1e-3)[0]
        return int(hit[0]) + 1 if hit.size else None

    res = {"problems": len(two), "samples": int(sum(w.batch for w, _ in two)), "iterations": K,
           "tol": 1e-3, "ragged_family_training": training}
    cold = None
    for name, net in (("cfg2_network", net_cfg2), ("ragged_family_network", net_mix)):
        rws = ws_mod.RaggedWarmStart([it[0] for _, it in two], [it[1] for _, it in two],
                                     [w.boundary for w, _ in two], net, K)
        t_w, t_c = [], []
        for _ in range(max(2, args.ragged_steps)):
            for fn, acc in ((rws.run, t_w), (rws.run_cold, t_c)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                acc.append(time.perf_counter() - t0)
        rws.run()
        torch.cuda.synchronize()
        wtr = [t.cpu().numpy() for t in rws.traces()]
        fl = rws.FL.cpu().numpy()
        if cold is None:
            rws.run_cold()
            torch.cuda.synchronize()
            ctr = [t.cpu().numpy() for t in rws.traces(cold=True)]
            fc = [first(t) for t in ctr]
            cold = {"problems_at_tol": int(sum(f is not None for f in fc)),
                    "iterations_to_tol_capped": int(sum(f if f is not None else K for f in fc)),
                    "mean_final_median_residual": float(np.mean([np.median(t[-1]) for t in ctr])),
                    "ms_per_set": 1e3 * float(np.median(t_c))}
            res["cold"] = cold
        fw = [first(t) for t in wtr]
        res[name] = {
            "problems_at_tol": int(sum(f is not None for f in fw)),
            "iterations_to_tol_capped": int(sum(f if f is not None else K for f in fw)),
            "fewer_iterations_than_cold": int(sum((a if a is not None else K) < (b if b is not None else K)
                                                  for a, b in zip(fw, fc))),
            "more_iterations_than_cold": int(sum((a if a is not None else K) > (b if b is not None else K)
                                                 for a, b in zip(fw, fc))),
            "mean_final_median_residual": float(np.mean([np.median(t[-1]) for t in wtr])),
            "fallbacks": int(((fl & 4) != 0).sum()),
            "ms_per_set": 1e3 * float(np.median(t_w))}
        rws.close()
    return res

def heading_ops_per_unit(w) -> int:
    """Algorithmic VALU lane-ops of one sample's iteration of the heading / multi-circle
    variant.  Every (circle, obstacle, time) row enters F (no pair can be skipped), so
    each takes the whole polar step: the obstacle's position (2), the offset and its
    scaling (4), the norm, its reciprocal square root, the radius and d (5), the
    direction (2), the target (4), the residual (2) and the sums F'(F xi - g) and
    |F xi - g|^2 need (6): 25 ops.  The two kinematic rows take 12 each, the two heading
    rows 4 (cos, sin, two residuals); per time step the evaluation of x, c, y, s, psi
    and the derivatives (10 n_v FMAs) and the contractions over time (15 n_v); both QP
    products once per sample.  An FMA counts once."""
    nv, npt = w.n_v, w.n_steps
    nfx = 2 * nv - 4
    per_t = w.n_circles * w.n_obs * 25 + 2 * 12 + 4 + 25 * nv
    return npt * per_t + 2 * nfx * nfx + (nv - 2) ** 2


def heading_bench(args):
    """Paper II's setting for the heading / multi-circle variant: one control cycle of
    10 iterations over 1000 samples in a crowd of 30 (4 footprint circles), FP32, HIP
    events around the launch on the current stream; the per-iteration time over a grid
    of circle and obstacle counts (the thesis's computation-time scaling figure); the
    two residuals of the best sample (its convergence figure)."""
    import torch
    from paper_2408_10731_amd import trajam as tj
    from paper_2408_10731_amd import workloads as wl

    stream = torch.cuda.current_stream()
    out = {"config": "Paper II crowd: 1000 samples, 30 people (semi-axes 0.55 m), 4 circles on a 1.2 m "
                     "robot, degree 10, 100 steps over 20 s, 10 iterations a call, FP32"}

    def timed(w, iters, reps):
        s = tj.HeadingSolver(w, precision="fp32")
        x0 = torch.as_tensor(w.xi0, dtype=torch.float32, device="cuda").contiguous()
        st, lm = x0.clone(), torch.zeros_like(x0)

        def call():
            s.project(st, lm, iters)
        ms = _time(call, reps, stream)
        st.copy_(x0)
        lm.zero_()
        tr = torch.zeros((iters, w.batch, 2), dtype=torch.float32, device="cuda")
        s.project(st, lm, iters, tr)
        torch.cuda.synchronize()
        s.close()
        return ms, tr.cpu().numpy()

    w = wl.heading_scene(20_001, n_obs=30, n_circles=4, batch=1000, flow="static")
    ms, tr = timed(w, 10, args.heading_reps)
    ops = w.batch * 10 * heading_ops_per_unit(w)
    out["ms_per_call"] = ms
    out["ms_per_iteration"] = ms / 10
    out["traj_iters_per_s"] = w.batch * 10 / (ms * 1e-3)
    out["roofline"] = {"bound": "alu", "achieved": ops / (ms * 1e-3) / 1e12, "peak": PEAK_VALU_OPS / 1e12,
                       "unit": "Tlane-ops/s", "frac": ops / (ms * 1e-3) / PEAK_VALU_OPS,
                       "ops_per_unit": heading_ops_per_unit(w)}
    _, tr50 = timed(w, 50, 1)
    best = int(np.argmin(tr50[-1, :, 0]))
    out["best_sample_residuals"] = {f"iter_{k}": [float(tr50[k - 1, best, 0]), float(tr50[k - 1, best, 1])]
                                    for k in (1, 5, 10, 20, 50)}
    grid = {}
    for nc in (1, 2, 4, 8):
        for no in (10, 30, 50):
            wg = wl.heading_scene(20_002, n_obs=no, n_circles=nc, batch=1000)
            mg, _ = timed(wg, 10, max(3, args.heading_reps // 4))
            grid[f"c{nc}_o{no}"] = mg / 10
    out["ms_per_iteration_grid"] = grid
    # the thesis's batch sweep of its batch optimizer (batch 5 .. 1000; its GPU, JAX and
    # obstacle count are not ours: context, not a target)
    sweep = {}
    for B in (5, 200, 400, 600, 800, 1000):
        wb = wl.heading_scene(20_003, n_obs=30, n_circles=4, batch=B)
        mb, _ = timed(wb, 10, max(3, args.heading_reps // 2))
        sweep[str(B)] = mb / 10
    out["ms_per_iteration_by_batch"] = sweep
    out["thesis_ms_per_iteration_by_batch"] = {"5": 1.6, "200": 1.7, "400": 2.6, "600": 3.3, "800": 3.9, "1000": 4.5,
                                               "note": "printed table of the thesis; GPU model not stated, Python + "
                                                       "JAX, obstacle count not stated"}
    return out


def heading_mpc_bench(args, delta=0.5, iters=10, horizon_s=20.0):
    """Paper II's MPC over batch sizes (its batch-size table, on synthetic crowds): per
    batch size, the same scenes (static crowd of 30, 4 circles, seeds 21,001 ..), the
    robot executing delta = 0.5 s of the chosen sample each control cycle (10 AM
    iterations, multipliers carried over) for 20 s.  A run succeeds when no footprint
    circle of the executed motion (checked every 0.05 s) enters a person's ellipse.
    Reports the success rate, the tracking error against the desired line and the
    acceleration of the executed motion, and the time per cycle, for next samples moved
    on from the cycle's results and for samples drawn afresh each cycle; the latter also
    with 30 and 100 iterations a cycle (the thesis's budget is 40 ms a cycle)."""
    from paper_2408_10731_amd import mpc as mp
    from paper_2408_10731_amd import workloads as wl

    n_cyc = int(round(horizon_s / delta))
    seeds = list(range(21_001, 21_001 + args.heading_mpc_scenes))
    out = {"config": f"static crowd of 30, 4 circles, {len(seeds)} scenes, {n_cyc} cycles of {delta} s, "
                     f"{iters} iterations a cycle, FP32, multipliers carried over",
           "by_batch": {}}
    ts = np.linspace(0.0, delta, 11)[:-1]
    runs = ([("moved_on", b, iters) for b in (1, 200, 1000)] + [("redrawn", b, iters) for b in (1, 50, 200, 1000)]
            + [("redrawn", b, k) for k in (30, 100) for b in (200, 1000)])
    for mode, B, its in runs:
        ok_runs, errs, accs, cyc_ms = 0, [], [], []
        for sd in seeds:
            w = wl.heading_scene(sd, n_obs=30, n_circles=4, batch=B, flow="static")
            m = mp.HeadingMPC(w, its, delta, redraw_seed=(sd + 7) if mode == "redrawn" else None)
            ok = True
            t0 = time.perf_counter()
            for c in range(n_cyc):
                o = m.cycle()
                coef, centre = o["coefficients"], o["obs_centre"]
                for t in ts:
                    p, _, a = mp.trajectory_state(coef[[0, 2]], w.horizon, t)
                    psi = float(mp.trajectory_state(coef[[4]], w.horizon, t)[0][0])
                    oc = centre + w.obs_vel * t
                    for r in w.radii:
                        q = p + r * np.array([np.cos(psi), np.sin(psi)])
                        if np.any(np.sum(((q[None] - oc) / w.obs_axes) ** 2, axis=1) < 1.0):
                            ok = False
                    tk = c * delta + t
                    line = w.x_des[:, 0] + (w.x_des[:, -1] - w.x_des[:, 0]) * min(1.0, tk / w.horizon)
                    errs.append(float(np.linalg.norm(p - line)))
                    accs.append(float(np.linalg.norm(a)))
            cyc_ms.append(1e3 * (time.perf_counter() - t0) / n_cyc)
            ok_runs += ok
            m.close()
        key = mode if its == iters else f"{mode}_{its}_iterations"
        out["by_batch"].setdefault(key, {})[str(B)] = {"success_rate": ok_runs / len(seeds),
                                   "tracking_error_m": [float(np.mean(errs)), float(np.max(errs)), float(np.min(errs))],
                                   "acceleration": [float(np.mean(accs)), float(np.max(accs)), float(np.min(accs))],
                                   "ms_per_cycle": float(np.median(cyc_ms))}
    out["thesis_success_rate_by_batch"] = {"1": 0.016, "200": 0.8, "400": 0.88, "600": 0.9, "800": 0.95, "1000": 1.0,
                                           "note": "printed table of the thesis; its simulator and crowds, not these"}
    return out


def agents_ops_per_unit(w) -> int:
    """Algorithmic VALU lane-ops of one joint sample's AM iteration in a multi-agent
    problem, at the lower end of each element's cost: every (agent, obstacle, time) and
    every unordered (agent pair, time) clearance test at 2 D + 1 ops (a difference, a
    squared norm, a compare), the two kinematic bounds of every agent at D + 1, the
    waypoint map and the F^T contraction (2 D 3 n_v FMAs per agent and time) and the QP
    (D n_v (n_v + 4) per agent); an FMA counts once."""
    D, nv, npt, no, N = w.dims, w.n_v, w.n_steps, w.n_obs, w.n_agents
    per_t = (N * no + N * (N - 1) // 2) * (2 * D + 1) + 2 * N * (D + 1) + 2 * D * 3 * nv * N
    return npt * per_t + N * D * nv * (nv + 4)


def precision_bench(args):
    """Config 3 (3D, degree 15, 150 steps over 20 s, 200 ellipsoids, 4096 samples, 50 AM
    iterations, cold start) in each precision: FP64, FP32, and BF16 (the QP product on
    the matrix cores with hi/lo split, fp32 accumulation and one refinement pass).
    Reports each precision's time per projection (autotuned shape; the cold-start
    resets included) and the FP32 / BF16 results' deviation from the FP64 run on the
    same inputs: the largest waypoint difference over every sample and time step and
    the largest difference of the final residual."""
    import torch
    from paper_2408_10731_amd import trajam as tj
    from paper_2408_10731_amd import workloads as wl

    w = wl.config3()
    K = w.iters
    out, final = {"config": "config 3: 3D, degree 15, 150 steps, 200 ellipsoids, 4096 samples, "
                            f"{K} AM iterations, cold start"}, {}
    stream = torch.cuda.current_stream()
    P = None
    for prec in ("fp64", "fp32", "bf16"):
        solver = tj.Solver.for_workload(w, precision=prec, sphere=False)
        if P is None:
            P = tj.trajam_fixed_matrices(solver.problem)[0]
        dt = solver.dtype
        xi, obs = tj.device_workload(w, dt)
        xb, lam = xi.clone(), torch.zeros_like(xi)
        shape = solver.autotune(xi, w.boundary, obs, xb, lam, probe_iters=K)
        solver.set_obstacles(obs)
        tr = torch.zeros((K, w.batch), dtype=dt, device="cuda")

        def run():
            xb.copy_(xi)
            lam.zero_()
            solver.project(xi, w.boundary, None, xb, lam, K, res_trace=tr)
        ms = _time(run, args.precision_steps, stream)
        run()
        torch.cuda.synchronize()
        final[prec] = (np.einsum("tm,bdm->btd", P, xb.double().cpu().numpy()), tr[-1].double().cpu().numpy())
        out[prec] = {"ms_per_projection": ms, "traj_iters_per_s": w.batch * K / (ms * 1e-3),
                     "launch_shape": list(shape)}
        solver.close()
    for prec in ("fp32", "bf16"):
        out[prec]["vs_fp64"] = {
            "waypoint_max_m": float(np.abs(final[prec][0] - final["fp64"][0]).max()),
            "residual_max": float(np.abs(final[prec][1] - final["fp64"][1]).max())}
    return out


def cem_bench(args):
    """One planning call of the projection-guided sampling loop at config-4 sizes:
    30 iterations, each drawing 2000 samples, projecting them with 15 AM iterations
    (100 moving circles), selecting 1454 by residual and 363 elites by cost, and
    updating the Gaussian; the whole call replayed from one captured graph."""
    import torch
    from paper_2408_10731_amd import cem
    from paper_2408_10731_amd import trajam as tj
    from paper_2408_10731_amd import workloads as wl

    w = wl.config4(batch=4)
    D, nv = w.dims, w.n_v
    N, Nb, Np, Ne, K = 30, 2000, 1454, 363, 15
    solver = tj.Solver.for_workload(w, precision="fp32", max_batch=Nb)
    _, obs = tj.device_workload(w, torch.float32)
    planner = cem.Planner(solver, Nb, Np, Ne, K)
    mu0 = wl.line_samples(np.random.default_rng(0), 1, w.degree, w.boundary[:, 0],
                          w.boundary[:, 3], 0.0)[0].reshape(-1)
    S0 = 0.25 * np.eye(D * nv)
    L0 = np.linalg.cholesky(S0 + 1e-10 * np.eye(D * nv))
    z = cem.draw(N, Nb, D * nv, key=1)   # the library's counter-based generator
    planner.set_distribution(mu0, S0, L0)
    shape = planner.autotune(z[0], w.boundary, obs)
    planner.set_distribution(mu0, S0, L0)
    planner.capture(z, w.boundary, obs)
    stream = torch.cuda.current_stream()

    def call():
        planner.set_distribution(mu0, S0, L0)
        planner.replay()

    ms = _time(call, args.cem_calls, stream)
    out = {"config": "30 CEM iterations x 2000 samples x 15 AM iterations, 100 moving "
                     "circles, 1454 projected / 363 elite, fp32, one graph replay per call; draws from "
                     "the library's Philox4x64-10 stream (key 1)",
           "ms_per_planning_call": ms, "traj_iters_per_s": N * Nb * K / (ms * 1e-3),
           "launch_shape": list(shape)}
    solver.close()
    return out


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, iters: int, tol: float = 1e-3, cap: int = 300):
    """The FP64 C oracle (untuned) on the host cores, on a bounded sample of the
    headline workload: 128 of its trajectories x its AM iterations on all threads, and
    4 trajectories x 10 iterations on one thread, each the median of 5 runs; and its
    time to the residual tolerance on 32 trajectories (iterated 10 at a time until the
    batch-median residual first reaches tol, capped like the GPU run), median of 3."""
    import oracle
    threads = oracle.max_threads()

    def rate(wk, k, n_threads, runs=5):
        vals = []
        for _ in range(runs):
            t0 = time.perf_counter()
            oracle.project(wk, iters=k, n_threads=n_threads)
            vals.append(wk.batch * k / (time.perf_counter() - t0))
        return float(np.median(vals))

    ws = w.subset(128)
    value = rate(ws, iters, threads)
    value_1t = rate(w.subset(4), 10, 1)
    wt = w.subset(32)
    ttr_s, ttr_it = [], None
    for _ in range(3):
        xb, lam = wt.xi.copy(), np.zeros_like(wt.xi)
        t0, done, it = time.perf_counter(), None, 0
        while it < cap and done is None:
            xb, lam, tr, _ = oracle.project(wt, xi_bar=xb, lam=lam, iters=10, n_threads=threads)
            hit = np.nonzero(np.median(tr, axis=1) <= tol)[0]
            if hit.size:
                done = it + int(hit[0]) + 1
            it += 10
        ttr_s.append(time.perf_counter() - t0)
        ttr_it = done
    return {"value": value, "unit": "traj-iters/s", "cores": threads, "kind": "oracle",
            "sample": f"{ws.batch} of the {w.batch} trajectories x {iters} AM iterations, FP64 C oracle, "
                      f"OpenMP over trajectories on {threads} threads, median of 5 runs",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "value_1thread": value_1t,
            "sample_1thread": "4 trajectories x 10 AM iterations on one thread, median of 5 runs",
            "time_to_residual": {"tol": tol, "cap": cap, "trajectories": wt.batch,
                                 "iterations": ttr_it, "reached": ttr_it is not None,
                                 "seconds": float(np.median(ttr_s)),
                                 "note": "batch-median residual, checked every 10 iterations (the time "
                                         "runs to the end of the 10-iteration block that reaches tol)"}}


def polar_bench(args):
    """The materialised polar variables (trajam_polar, unpadded [batch][n_o][n_steps]
    rows) against the HBM peak: config 3 (3D: alpha, beta and d of 4096 samples x 200
    ellipsoids x 150 steps, 1.47 GB, plus the kinematic blocks) and config 2 (2D:
    alpha and d of 1024 x 50 x 100 -- beta is the constant pi/2 in 2D and is not
    written), FP32, the latter also at batches 2048-8192.  Useful bytes are the
    arrays' entries that carry information (in 2D the kinematic beta rows are
    constant and not counted); the bytes the kernel writes, those rows included, and
    a plain fill of the same size are reported beside them."""
    import torch
    from paper_2408_10731_amd import trajam as tj
    from paper_2408_10731_amd import workloads as wl

    kw = dict(dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()

    def measure(w):
        solver = tj.Solver.for_workload(w, precision="fp32", sphere=False if w.dims == 3 else None)
        xi, obs = tj.device_workload(w, torch.float32)
        solver.set_obstacles(obs)
        n = w.batch * w.n_obs * w.n_steps
        al, d = torch.empty(n, **kw), torch.empty(n, **kw)
        be = torch.empty(n, **kw) if w.dims == 3 else None
        kin = torch.empty((w.batch, 6, w.n_steps), **kw)
        ptr = lambda t: None if t is None else t.data_ptr()

        def run():
            tj.trajam_polar(solver.handle, w.batch, xi.data_ptr(), None, None, None, al.data_ptr(),
                            ptr(be), d.data_ptr(), kin.data_ptr(), st.cuda_stream)
        ms = _time(run, args.polar_steps, st)
        arrays = 3 if w.dims == 3 else 2
        kin_rows = 6 if w.dims == 3 else 4
        useful = 4 * (arrays * n + kin_rows * w.batch * w.n_steps)
        written = 4 * (arrays * n + kin.numel())
        read = 4 * (xi.numel() + 3 * w.n_steps * 16)
        solver.close()
        del al, be, d, kin
        gbs = useful / (ms * 1e-3) / 1e9
        # a plain write stream of the same size on this chip: torch's fill kernel
        buf = torch.empty(written // 4, **kw)
        fill_ms = _time(lambda: buf.fill_(1.0), args.polar_steps, st)
        del buf
        fill_gbs = written / (fill_ms * 1e-3) / 1e9
        return {"ms_per_call": ms, "useful_bytes": useful, "written_bytes": written, "read_bytes": read,
                "achieved_GBps": gbs, "peak_GBps": PEAK_HBM / 1e9, "frac_useful": gbs * 1e9 / PEAK_HBM,
                "written_GBps": (written + read) / (ms * 1e-3) / 1e9,
                "fill_same_bytes_GBps": fill_gbs, "frac_of_fill": (written / (ms * 1e-3) / 1e9) / fill_gbs}

    out = {"cfg3": {"config": "config 3: 4096 samples x 200 ellipsoids x 150 steps, alpha, beta, d "
                              "+ kinematic blocks, fp32", **measure(wl.config3())},
           "cfg2": {"config": "config 2: 1024 samples x 50 circles x 100 steps, alpha and d (beta = pi/2 "
                              "not written) + kinematic blocks, fp32", **measure(wl.config2())}}
    # the same 2D geometry at larger batches: how much of a call is the launch's fixed cost
    out["cfg2"]["by_batch"] = [dict(batch=b, **measure(wl.problem2d(20240, 50, b))) for b in (2048, 4096, 8192)]
    return out


COUNTER_PASSES = (
    ("FETCH_SIZE",),
    ("WRITE_SIZE",),
    ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES",
     "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_SMEM"),
)
PROBE_COPY_MIB = 64


def _read_counters(outdir):
    """{(kernel name, dispatch id): {counter: value}} from rocprofv3's CSV output."""
    import csv
    import glob
    rows = {}
    for path in glob.glob(os.path.join(outdir, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            for r in csv.DictReader(f):
                key = (r["Kernel_Name"], int(r["Dispatch_Id"]))
                rows.setdefault(key, {})[r["Counter_Name"]] = float(r["Counter_Value"])
    return rows


def _last(rows, pred):
    keys = sorted((k for k in rows if pred(k[0])), key=lambda k: k[1])
    return rows[keys[-1]] if keys else None


def hw_counters(probe_args, kernel_prefix, launch_ms, algorithmic_bytes, timeout=150):
    """HBM traffic and VALU issue of one launch of the projection kernel, measured in
    this run: three rocprofv3 --pmc passes (FETCH_SIZE; WRITE_SIZE; eight SQ counters),
    each over a child process that repeats the timed step's launch twice and then
    copies PROBE_COPY_MIB MiB once.  The byte counters are scaled by what they read
    for that copy of known size; the last dispatch of the kernel is the one reported.
    Returns (traffic bytes or None, details)."""
    import shutil
    import subprocess
    import tempfile
    prof = shutil.which("rocprofv3")
    if prof is None:
        return None, {"error": "rocprofv3 not found"}
    vals, copy = {}, {}
    env = dict(os.environ, TMPDIR="/tmp")
    for counters in COUNTER_PASSES:
        d = tempfile.mkdtemp(prefix="trajam_pmc_", dir="/tmp")
        cmd = ["timeout", "-s", "KILL", str(timeout), prof, "--pmc", *counters, "--output-format", "csv",
               "-d", d, "-o", "p", "--", sys.executable, os.path.abspath(__file__), *probe_args]
        print("bench: counter pass " + " ".join(counters), file=sys.stderr, flush=True)
        r = subprocess.run(cmd, cwd="/tmp", env=env, capture_output=True, text=True)
        rows = _read_counters(d)
        shutil.rmtree(d, ignore_errors=True)
        # names read "void trajam::(anonymous namespace)::am_wave_kernel<float, 3, ...>(...)"
        k = _last(rows, lambda n: f"::{kernel_prefix}<" in n or n.startswith(kernel_prefix + "<"))
        c = _last(rows, lambda n: "copyBuffer" in n)
        if k is None:
            return None, {"error": f"no {kernel_prefix} dispatch in the {counters[0]} pass "
                                   f"(rocprofv3 exit {r.returncode}): {r.stderr[-300:]}"}
        vals.update(k)
        if c is not None:
            copy.update(c)
    out = {"kernel": kernel_prefix, "passes": [list(c) for c in COUNTER_PASSES]}
    traffic = None
    nbytes = PROBE_COPY_MIB << 20
    if copy.get("FETCH_SIZE") and copy.get("WRITE_SIZE"):
        fs = nbytes / (copy["FETCH_SIZE"] * 1024.0)
        wsc = nbytes / (copy["WRITE_SIZE"] * 1024.0)
        rd = vals["FETCH_SIZE"] * 1024.0 * fs
        wr = vals["WRITE_SIZE"] * 1024.0 * wsc
        traffic = rd + wr
        out.update({"fetch_KiB": vals["FETCH_SIZE"], "write_KiB": vals["WRITE_SIZE"],
                    "copy_fetch_KiB": copy["FETCH_SIZE"], "copy_write_KiB": copy["WRITE_SIZE"],
                    "fetch_scale": fs, "write_scale": wsc, "read_bytes": rd, "written_bytes": wr,
                    "algorithmic_bytes": algorithmic_bytes,
                    "traffic_over_algorithmic": traffic / algorithmic_bytes})
    else:
        out["error_traffic"] = "no copy dispatch to calibrate the byte counters"
    sq = {k: v for k, v in vals.items() if k.startswith("SQ_")}
    out["sq"] = sq
    if sq.get("SQ_INSTS_VALU"):
        out["valu_insts"] = sq["SQ_INSTS_VALU"]
        out["valu_issue_frac"] = sq["SQ_INSTS_VALU"] / (launch_ms * 1e-3 * PEAK_VALU_INSTS)
        if sq.get("SQ_WAVES"):
            out["valu_insts_per_wave"] = sq["SQ_INSTS_VALU"] / sq["SQ_WAVES"]
    return traffic, out


MFMA_COUNTERS = ("SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE")
N_SIMD = 1024   # 256 CUs x 4 SIMDs


def mfma_counters(child_args, families, calls, timeout=150):
    """Matrix-core counters measured in this run: one rocprofv3 --pmc pass over a
    child `bench.py <child_args>` that makes `calls` calls of each measured operation.
    Per kernel family (a name fragment -> a label): bf16 matrix-core FLOPs issued per
    call (MOPS x 512, including the zero padding of edge tiles) and the matrix cores'
    busy fraction while the family's dispatches run (busy cycles over GRBM_GUI_ACTIVE
    per XCD x 1024 SIMDs)."""
    import shutil
    import subprocess
    import tempfile
    prof = shutil.which("rocprofv3")
    if prof is None:
        return {"error": "rocprofv3 not found"}
    d = tempfile.mkdtemp(prefix="trajam_mfma_", dir="/tmp")
    cmd = ["timeout", "-s", "KILL", str(timeout), prof, "--pmc", *MFMA_COUNTERS, "--output-format", "csv",
           "-d", d, "-o", "p", "--", sys.executable, os.path.abspath(__file__), *child_args]
    print("bench: matrix-core counter pass " + " ".join(child_args), file=sys.stderr, flush=True)
    r = subprocess.run(cmd, cwd="/tmp", env=dict(os.environ, TMPDIR="/tmp"), capture_output=True, text=True)
    rows = _read_counters(d)
    shutil.rmtree(d, ignore_errors=True)
    out = {"counters": list(MFMA_COUNTERS), "calls": calls}
    for fam, label in families:
        ks = [v for (n, _), v in rows.items() if f"::{fam}" in n]
        if not ks:
            out[label] = {"error": f"no {fam} dispatch (rocprofv3 exit {r.returncode}): {r.stderr[-300:]}"}
            continue
        mops = sum(v.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0) for v in ks)
        busy = sum(v.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) for v in ks)
        gui = sum(v.get("GRBM_GUI_ACTIVE", 0.0) for v in ks) / 8.0
        out[label] = {"kernel": fam, "dispatches": len(ks), "mfma_gflop_per_call": mops * 512 / calls / 1e9,
                      "mfma_busy_frac": busy / (gui * N_SIMD) if gui > 0 else None}
    return out


def probe_ragged(args):
    """Child of hw_counters for the multi-agent half of the ragged set: its plan
    launched twice, then the copy of known size."""
    import torch
    from paper_2408_10731_amd import trajam as tj
    from paper_2408_10731_amd import workloads as wl
    ws = [w for w in wl.config5(args.ragged_problems, iters=args.iters) if w.n_agents > 1]
    items, solvers = [], []
    for w in ws:
        s = tj.Solver.for_workload(w, precision="fp32")
        xi, obs = tj.device_workload(w, torch.float32)
        s.set_obstacles(obs)
        items.append((s, xi, w.boundary, xi.clone(), torch.zeros_like(xi)))
        solvers.append(s)
    plan = tj.RaggedPlan(items, args.iters)
    for _ in range(2):
        for it in items:
            it[3].copy_(it[1])
            it[4].zero_()
        plan.launch()
    torch.cuda.synchronize()
    a = torch.ones(PROBE_COPY_MIB << 18, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    plan.close()
    for s in solvers:
        s.close()


def probe(args):
    """Child of hw_counters: the headline step's launch twice, then a copy of known
    size (the byte counters' calibration).  Prints nothing on stdout."""
    import torch
    from paper_2408_10731_amd import trajam as tj
    from paper_2408_10731_amd import workloads as wl
    if args.probe == "ragged":
        probe_ragged(args)
        return
    k, spw = (int(x) for x in args.probe_launch.split(","))
    w = wl.config3() if args.probe == "cfg3" else wl.config2(batch=args.batch)
    K = args.iters
    solver = tj.Solver.for_workload(w, precision=args.probe_precision,
                                    sphere=False if args.probe == "cfg3" else None)
    xi, obs = tj.device_workload(w, solver.dtype)
    solver.set_launch(k, spw)
    solver.set_obstacles(obs)
    xb, lam = xi.clone(), torch.zeros_like(xi)
    tr = torch.zeros((K, w.batch), dtype=solver.dtype, device="cuda")
    for _ in range(2):
        xb.copy_(xi)
        lam.zero_()
        solver.project(xi, w.boundary, None, xb, lam, K, res_trace=tr)
    torch.cuda.synchronize()
    a = torch.ones(PROBE_COPY_MIB << 18, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    solver.close()


def projection_leg(w, K, steps, warmup, sphere=None):
    """Times one workload's projection (autotuned launch shape, obstacles packed once,
    cold-start resets inside the step): returns the timing and the solver state."""
    import torch
    from paper_2408_10731_amd import trajam as tj
    solver = tj.Solver.for_workload(w, precision="fp32", sphere=sphere)
    xi, obs = tj.device_workload(w, torch.float32)
    xb = xi.clone()
    lam = torch.zeros_like(xi)
    trace = torch.zeros((K, w.batch), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    # launch shape from the autotuner (setup, untimed), then the scene's obstacles,
    # packed once before timing
    kern, spw = solver.autotune(xi, w.boundary, obs, xb, lam, probe_iters=K)
    solver.set_obstacles(obs)
    for _ in range(warmup):
        xb.copy_(xi)
        lam.zero_()
        solver.project(xi, w.boundary, None, xb, lam, K, res_trace=trace)
    torch.cuda.synchronize()
    # per-launch kernel time (events on the launch stream), then the timed region
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for i in range(steps):
        xb.copy_(xi)
        lam.zero_()
        ev[i][0].record(stream)
        solver.project(xi, w.boundary, None, xb, lam, K, res_trace=trace)
        ev[i][1].record(stream)
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_per_step = t_start.elapsed_time(t_end) / steps
    launch_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    kname = "am_project_kernel" if kern == 0 else "am_wave_kernel"
    ops = survey_ops_per_unit(w)
    achieved = ops * w.batch * K / (launch_ms * 1e-3)
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_OPS / 1e12,
            "unit": "Tlane-ops/s", "frac": achieved / PEAK_VALU_OPS, "traffic": None,
            "kernel": f"{kname}<float,{w.dims},...>, {spw} sample(s)/workgroup",
            "ops_per_traj_iter": ops, "units_per_launch": w.batch * K, "launch_ms": launch_ms}
    return {"solver": solver, "xi": xi, "obs": obs, "xb": xb, "lam": lam, "ms_per_step": ms_per_step,
            "launch_ms": launch_ms, "wall": wall, "kern": kern, "spw": spw, "kname": kname,
            "roofline": roof, "value": w.batch * K / (ms_per_step * 1e-3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-counters", action="store_true",
                    help="skip the rocprofv3 counter passes (traffic and VALU issue become null)")
    ap.add_argument("--probe", choices=["cfg3", "cfg2", "ragged"], default=None,
                    help="internal: the counter passes' child process")
    ap.add_argument("--probe-launch", default="1,1", help="internal: kernel,samples-per-workgroup")
    ap.add_argument("--probe-precision", choices=["fp32", "bf16"], default="fp32", help="internal")
    ap.add_argument("--ttr-cap", type=int, default=300)
    ap.add_argument("--heading-reps", type=int, default=20,
                    help="timed calls of the heading / multi-circle leg (0 skips it)")
    ap.add_argument("--heading-mpc-scenes", type=int, default=20,
                    help="crowd scenes of the heading variant's receding-horizon leg (0 skips it)")
    ap.add_argument("--ws-scenes", type=int, default=2048)
    ap.add_argument("--ws-epochs", type=int, default=20)
    ap.add_argument("--ragged-problems", type=int, default=256, help="0 skips the ragged set")
    ap.add_argument("--ragged-steps", type=int, default=3)
    ap.add_argument("--cem-calls", type=int, default=5, help="0 skips the sampling loop")
    ap.add_argument("--precision-steps", type=int, default=3,
                    help="timed projections per precision of config 3; 0 skips that leg")
    ap.add_argument("--polar-steps", type=int, default=10,
                    help="timed calls of the materialised polar variables; 0 skips that leg")
    ap.add_argument("--cem-only", action="store_true",
                    help="run only the sampling-loop leg and print its JSON (profiling)")
    ap.add_argument("--mpc-cycles", type=int, default=20, help="control cycles of the MPC leg; 0 skips it")
    ap.add_argument("--ws4-scenes", type=int, default=8192,
                    help="config-4 training scenes of the warm start in the sampling loop; 0 skips that leg")
    ap.add_argument("--mfma-steps", type=int, default=10, help="timed calls of the matrix-core leg; 0 skips it")
    ap.add_argument("--mfma-only", action="store_true",
                    help="run only the matrix-core leg and print its JSON (profiling)")
    ap.add_argument("--polar-only", action="store_true",
                    help="run only the materialised-polar leg and print its JSON (profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB buffer 3 times (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 4 * n, "launches": 3}), flush=True)
        return
    if args.probe:
        probe(args)
        return
    if args.cem_only:
        print(json.dumps(cem_bench(args)), flush=True)
        return
    if args.polar_only:
        print(json.dumps(polar_bench(args)), flush=True)
        return
    if args.mfma_only:
        print(json.dumps(mfma_bench(args)), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(samples are independent: a multi-GPU run shards the batch "
                                   "with no communication)"}))
        sys.exit(2)

    import torch
    from paper_2408_10731_amd import workloads as wl

    K = args.iters
    # headline: config 3 (the largest single-problem configuration), FP32
    w3 = wl.config3()
    h = projection_leg(w3, K, args.steps, args.warmup, sphere=False)
    roofline = h["roofline"]
    counters = None
    if not args.no_counters:
        probe_args = ["--probe", "cfg3", "--probe-launch", f"{h['kern']},{h['spw']}", "--iters", str(K)]
        traffic, counters = hw_counters(probe_args, h["kname"], h["launch_ms"],
                                        state_bytes_per_launch(w3, K))
        roofline["traffic"] = traffic
        if counters.get("valu_issue_frac") is not None:
            roofline["valu_issue_frac"] = counters["valu_issue_frac"]

    # config 2 (2D, 1024 samples, 50 circles, 50 iterations): the former headline
    w2 = wl.config2(batch=args.batch)
    c2 = projection_leg(w2, K, args.steps, args.warmup)
    cfg2 = {"workload": "2D point robot, 50 static circles r~U(0.3,0.8) m in 30x30 m, Bernstein degree 10, "
                        f"100 steps over 30 s, batch {w2.batch}, {K} AM iterations, cold start, fp32",
            "value": c2["value"], "ms_per_step": c2["ms_per_step"], "roofline": c2["roofline"]}

    # config 2 inside the workspace band |y - 15| <= 1.2 (rows G = [-P; P] with slack)
    import dataclasses
    w2b = dataclasses.replace(w2, workspace=np.array(((-1.0, 13.8), (31.0, 16.2))))
    c2b = projection_leg(w2b, K, args.steps, args.warmup)
    c2b["solver"].close()
    cfg2["workspace_band"] = {"workload": "config 2 with workspace bounds x in [-1, 31], y in [13.8, 16.2]",
                              "value": c2b["value"], "ms_per_step": c2b["ms_per_step"],
                              "launch_ms": c2b["launch_ms"]}

    net2, info2 = (train_warm_start(w2, args.ws_scenes, args.ws_epochs) if args.ttr_cap > 0 else (None, None))
    ttr = (time_to_residual(args, w2, c2["solver"], c2["xi"], c2["obs"], torch.cuda.current_stream(),
                            net=net2, info=info2)
           if args.ttr_cap > 0 else None)
    cont = continuation_leg(w2, args.ttr_cap, torch.cuda.current_stream()) if args.ttr_cap > 0 else None
    c2["solver"].close()
    ragged = ragged_bench(args, net2) if args.ragged_problems > 0 else None
    cem_out = cem_bench(args) if args.cem_calls > 0 else None
    warm4, net4 = ((warm_cfg4_bench(args) if args.ws4_scenes > 0 and args.cem_calls > 0 and args.ttr_cap > 0
                    else (None, None)))
    mpc_out = mpc_bench(args, net4) if args.mpc_cycles > 0 else None
    heading_out = heading_bench(args) if args.heading_reps > 0 else None
    if heading_out is not None and args.heading_mpc_scenes > 0:
        heading_out["receding_horizon"] = heading_mpc_bench(args)
    prec_out = precision_bench(args) if args.precision_steps > 0 else None
    polar_out = polar_bench(args) if args.polar_steps > 0 else None
    mfma_out = mfma_bench(args) if args.mfma_steps > 0 else None
    if mfma_out is not None and not args.no_counters:
        # one untimed and two timed calls of each in the child
        mfma_out["counters"] = mfma_counters(["--mfma-only", "--mfma-steps", "2"],
                                             [("gemm_mfma_kernel", "train_step"), ("warm_jump_kernel", "warm_jump")], 3)
    if prec_out is not None and not args.no_counters:
        k, spw = prec_out["bf16"]["launch_shape"][:2]
        fam = "am_project_kernel" if k == 0 else "am_wave_kernel"
        c = mfma_counters(["--probe", "cfg3", "--probe-precision", "bf16", "--probe-launch", f"{k},{spw}",
                           "--iters", str(wl.config3().iters)], [(fam, "projection")], 2)
        proj = c.get("projection", {})
        if "mfma_gflop_per_call" in proj:
            ms = prec_out["bf16"]["ms_per_projection"]
            proj["achieved_TFLOPs"] = proj["mfma_gflop_per_call"] * 1e9 / (ms * 1e-3) / 1e12
            proj["frac_of_bf16_peak"] = proj["achieved_TFLOPs"] * 1e12 / PEAK_BF16_MFMA
        prec_out["bf16"]["matrix_cores"] = c

    out = {
        "metric": "traj-iters/s & time-to-residual<=1e-3, learned warm-start vs cold, 1 MI355X",
        "value": h["value"], "unit": "traj-iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": h["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "config 3: 3D point robot, 200 static ellipsoids (semi-axes U(0.3,1.0) m "
                               "each) in 20x20x6 m, Bernstein degree 15, 150 steps over 20 s, batch 4096, "
                               f"{K} AM iterations, cold start, fp32",
                   "batch": w3.batch, "iterations": K, "obstacles": w3.n_obs,
                   "timesteps": w3.n_steps, "degree": w3.degree, "precision": "fp32"},
        "roofline": roofline,
        "counters": counters,
        "config2": cfg2,
        "time_to_residual": ttr,
        "continuation": cont,
        "ragged": ragged,
        "cem": cem_out,
        "precision_cfg3": prec_out,
        "polar_materialised": polar_out,
        "matrix_cores": mfma_out,
        "warm_start_config4": warm4,
        "mpc": mpc_out,
        "heading_multi_circle": heading_out,
        "wall_s_timed_region": h["wall"],
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w3, K)
    print(json.dumps(out), flush=True)
    h["solver"].close()


if __name__ == "__main__":
    main()
