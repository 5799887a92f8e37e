"""Ragged persistent launches (many problems, one kernel) and the autotuner.

* A ragged launch runs, per sample, the same arithmetic as the single-problem
  wave-per-sample kernel: its results are compared with those launches element by
  element (and reported bitwise), and with the FP64 oracle to the FP32 bar (final
  waypoints within 1e-3 m, residual within 1e-4).
* The launch captured in a graph replays to the eager result, with eager work and
  synchronizations between replays.
* The autotuner picks a valid launch shape, caches it by problem key, and the tuned
  launch stays within the FP32 bar of the oracle.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2408_10731_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _tj():
    from paper_2408_10731_amd import trajam as tj
    return tj


class Set:
    """Solvers and device buffers of a list of workloads."""

    def __init__(self, ws, iters):
        tj = _tj()
        self.ws, self.iters = ws, iters
        self.solvers, self.bufs = [], []
        for w in ws:
            s = tj.Solver.for_workload(w, precision="fp32", max_batch=max(w.batch, 1))
            xi, obs = tj.device_workload(w, torch.float32)
            s.set_obstacles(obs)
            xb, lam = xi.clone(), torch.zeros_like(xi)
            tr = torch.zeros((iters, w.batch), dtype=torch.float32, device="cuda")
            self.solvers.append(s)
            self.bufs.append((xi, obs, xb, lam, tr))

    def reset(self):
        for xi, _, xb, lam, tr in self.bufs:
            xb.copy_(xi)
            lam.zero_()
            tr.zero_()

    def plan(self):
        tj = _tj()
        return tj.RaggedPlan([(s, b[0], w.boundary, b[2], b[3], b[4])
                              for s, w, b in zip(self.solvers, self.ws, self.bufs)], self.iters)

    def single(self):
        """Each problem on its own with the wave-per-sample kernel."""
        for s, w, (xi, obs, xb, lam, tr) in zip(self.solvers, self.ws, self.bufs):
            s.set_launch(1, 1)
            s.project(xi, w.boundary, obs, xb, lam, self.iters, res_trace=tr)

    def results(self):
        torch.cuda.synchronize()
        return [(b[2].double().cpu().numpy(), b[3].double().cpu().numpy(),
                 b[4].double().cpu().numpy()) for b in self.bufs]

    def close(self):
        for s in self.solvers:
            s.close()


def _mixed(n, seed, n_obs, batch, iters=25):
    ws = wl.ragged_set(n, seed=seed, n_obs=n_obs, batch=batch, iters=iters)
    return [w.rounded(np.float32) for w in ws]


def test_ragged_matches_single_problem_launches():
    ws = _mixed(20, 777, (0, 80), (1, 300))
    ws.append(wl.problem2d(31, 7, 1).rounded(np.float32))       # batch 1
    ws.append(wl.problem3d(32, 0, 5).rounded(np.float32))       # no obstacles
    ws.append(wl.problem2d(33, 3, 0).rounded(np.float32))       # empty batch
    say("case: ragged vs single launches,", len(ws), "problems,",
        sum(w.batch for w in ws), "samples")
    S = Set(ws, 25)
    plan = S.plan()
    S.reset()
    plan.launch()
    rag = S.results()
    S.reset()
    S.single()
    one = S.results()
    bitwise = True
    for w, r, o in zip(ws, rag, one):
        for a, b in zip(r, o):
            bitwise &= bool(np.array_equal(a, b))
            scale = max(1.0, float(np.abs(b).max()) if b.size else 1.0)
            np.testing.assert_allclose(a, b, rtol=0, atol=1e-5 * scale, err_msg=w.name)
    say("  ragged == single-problem launches bitwise:", bitwise)
    plan.close()
    S.close()


def test_ragged_oracle_parity():
    ws = _mixed(6, 4242, (3, 40), (5, 24), iters=30)
    say("case: ragged vs oracle,", [(w.dims, w.n_obs, w.batch) for w in ws])
    S = Set(ws, 30)
    plan = S.plan()
    S.reset()
    plan.launch()
    res = S.results()
    for w, (xb_g, _, _) in zip(ws, res):
        xb_o, _, _, _ = oracle.project(w, iters=30)
        P, _, _ = oracle.bernstein(w.degree, w.n_steps, w.horizon)
        wp = np.abs(np.einsum("tm,bdm->btd", P, xb_g - xb_o)).max()
        dr = np.abs(oracle.residuals(w, xb_g)[0] - oracle.residuals(w, xb_o)[0]).max()
        say(f"  {w.name}: waypoint err {wp:.2e} m, residual err {dr:.2e}")
        assert wp <= 1e-3 and dr <= 1e-4
        for ax in range(w.dims):
            assert np.abs(xb_g[:, ax, 0] - w.boundary[ax, 0]).max() <= 1e-5
            assert np.abs(xb_g[:, ax, -1] - w.boundary[ax, 3]).max() <= 1e-5
    plan.close()
    S.close()


def test_ragged_config5_shapes_sampled_oracle_parity():
    """The largest shapes of the ragged set in one plan: a 2D problem with 300 circles
    and 2048 samples and a 3D joint problem with 64 agents and 300 spheres (64 joint
    samples), 50 iterations.  Sampled samples of the full launch against the FP64
    oracle: final waypoints within 1e-3 m, the residual the oracle recomputes from the
    GPU's coefficients within 1e-4 of its own, boundary rows within 1e-5 (FP32 state)."""
    import dataclasses
    iters = 50
    w2 = wl.problem2d(5002, 300, 2048, iters).rounded(np.float32)
    wa = wl.agents3d(5001, 64, 300, 64, iters).rounded(np.float32)
    say("case: ragged config-5 shapes: 2D n_o 300 B 2048; 3D N 64 n_o 300 B 64")
    S = Set([w2, wa], iters)
    plan = S.plan()
    S.reset()
    plan.launch()
    (xb2, _, _), (xba, _, _) = S.results()
    plan.close()
    S.close()
    P, _, _ = oracle.bernstein(w2.degree, w2.n_steps, w2.horizon)
    idx = np.arange(3, 2048, 128)
    xo, _, _, _ = oracle.project(w2, iters=iters, xi=w2.xi[idx])
    ws = w2.subset(2048)
    ws = dataclasses.replace(ws, xi=np.ascontiguousarray(w2.xi[idx]))
    wp = np.abs(np.einsum("tm,bdm->btd", P, xb2[idx] - xo)).max()
    dr = np.abs(oracle.residuals(ws, xb2[idx])[0] - oracle.residuals(ws, xo)[0]).max()
    say(f"  2D, {idx.size} samples: waypoint err {wp:.2e} m, residual err {dr:.2e}")
    assert wp <= 1e-3 and dr <= 1e-4
    for ax in range(2):
        assert np.abs(xb2[idx, ax, 0] - w2.boundary[ax, 0]).max() <= 1e-5
        assert np.abs(xb2[idx, ax, -1] - w2.boundary[ax, 3]).max() <= 1e-5
    ida = np.arange(5, 64, 8)
    wsa = dataclasses.replace(wa, xi=np.ascontiguousarray(wa.xi[ida]))
    xoa, _, _, _ = oracle.project_agents(wsa, iters=iters)
    P, _, _ = oracle.bernstein(wa.degree, wa.n_steps, wa.horizon)
    wp = np.abs(np.einsum("tm,badm->batd", P, xba[ida] - xoa)).max()
    dr = np.abs(oracle.residuals_agents(wsa, xba[ida])[0] - oracle.residuals_agents(wsa, xoa)[0]).max()
    say(f"  3D 64 agents, {ida.size} joint samples: waypoint err {wp:.2e} m, residual err {dr:.2e}")
    assert wp <= 1e-3 and dr <= 1e-4
    for a in range(wa.n_agents):
        assert np.abs(xba[ida, a, :, 0] - wa.boundary[a, :, 0]).max() <= 1e-5
        assert np.abs(xba[ida, a, :, -1] - wa.boundary[a, :, 3]).max() <= 1e-5


def test_ragged_graph_replays_match_eager():
    ws = _mixed(12, 99, (5, 60), (16, 200), iters=20)
    say("case: ragged graph capture,", len(ws), "problems")
    S = Set(ws, 20)
    plan = S.plan()
    S.reset()
    plan.launch()
    ref = S.results()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        S.reset()
        plan.launch()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        S.reset()
        plan.launch()
    for rep in range(3):
        for _, _, xb, lam, _ in S.bufs:   # eager work between replays
            xb.mul_(0.5)
            lam.add_(1.0)
        torch.cuda.synchronize()
        g.replay()
        got = S.results()
        for r, o in zip(got, ref):
            for a, b in zip(r, o):
                assert np.array_equal(a, b), f"replay {rep}"
    say("  3 replays bitwise equal to the eager launch")
    del g
    plan.close()
    S.close()


def test_ragged_plan_validation():
    tj = _tj()
    w = wl.problem2d(5, 4, 8).rounded(np.float32)
    xi, obs = tj.device_workload(w, torch.float32)
    xb, lam = xi.clone(), torch.zeros_like(xi)
    s64 = tj.Solver.for_workload(w, precision="fp64")
    xi64, obs64 = tj.device_workload(w, torch.float64)
    s64.set_obstacles(obs64)
    with pytest.raises(tj.TrajamError) as e:
        tj.RaggedPlan([(s64, xi64, w.boundary, xi64.clone(), torch.zeros_like(xi64))], 5)
    assert e.value.status == tj.TRAJAM_ERR_UNSUPPORTED
    s32 = tj.Solver.for_workload(w, precision="fp32")
    with pytest.raises(tj.TrajamError) as e:   # obstacles never set
        tj.RaggedPlan([(s32, xi, w.boundary, xb, lam)], 5)
    assert e.value.status == tj.TRAJAM_ERR_INVALID
    s32.set_obstacles(obs)
    bad = w.boundary.copy()
    bad[0, 0] = np.nan
    with pytest.raises(tj.TrajamError) as e:
        tj.RaggedPlan([(s32, xi, bad, xb, lam)], 5)
    assert e.value.status == tj.TRAJAM_ERR_INVALID
    small = tj.Solver.for_workload(w, precision="fp32", max_batch=4)
    small.set_obstacles(obs)
    with pytest.raises(tj.TrajamError):
        tj.RaggedPlan([(small, xi, w.boundary, xb, lam)], 5)
    s64.close()
    s32.close()
    small.close()


def test_autotune_picks_cached_valid_launch(tmp_path):
    tj = _tj()
    cache = tmp_path / "tune.txt"
    os.environ["TRAJAM_AUTOTUNE_CACHE"] = str(cache)
    try:
        w = wl.config2(batch=256).rounded(np.float32)
        say("case: autotune cfg2 B=256")
        s = tj.Solver.for_workload(w, precision="fp32")
        xi, obs = tj.device_workload(w, torch.float32)
        xb, lam = xi.clone(), torch.zeros_like(xi)
        k, t = s.autotune(xi, w.boundary, obs, xb, lam, probe_iters=10)
        say("  picked kernel", k, "samples/WG", t)
        assert (k, t) == s.launch()
        assert k in (0, 1) and t >= 1
        assert cache.exists() and len(cache.read_text().split()) == 3
        s.set_launch(0 if k else 1, 1)
        assert s.autotune(xi, w.boundary, obs, xb, lam, probe_iters=10) == (k, t)  # cached
        xb.copy_(xi)
        lam.zero_()
        s.project(xi, w.boundary, obs, xb, lam, 30)
        torch.cuda.synchronize()
        ws = w.subset(64)
        xb_o, _, _, _ = oracle.project(ws, iters=30)
        xg = xb.double().cpu().numpy()[:64]
        P, _, _ = oracle.bernstein(w.degree, w.n_steps, w.horizon)
        wp = np.abs(np.einsum("tm,bdm->btd", P, xg - xb_o)).max()
        dr = np.abs(oracle.residuals(ws, xg)[0] - oracle.residuals(ws, xb_o)[0]).max()
        say(f"  tuned launch vs oracle: waypoint {wp:.2e} m, residual {dr:.2e}")
        assert wp <= 1e-3 and dr <= 1e-4
        s.close()
    finally:
        os.environ.pop("TRAJAM_AUTOTUNE_CACHE", None)


@pytest.mark.gpu
def test_ragged_warm_start_composes_the_library_calls():
    """The ragged set's learned warm start: one probe launch over every problem, one
    fused jump over all samples, per problem the residual check and fallback, one
    continuation launch -- equal (bitwise) to the same steps made problem by problem
    with single launches; the cold plan equals single cold launches; fallback flags
    are 0 or TRAJAM_FLAG_COLD_FALLBACK."""
    import torch
    from paper_2408_10731_amd import trajam as tj
    from paper_2408_10731_amd import warmstart as ws
    print("case: ragged warm start", flush=True)
    problems = [wl.problem2d(700 + k, n_obs, b, 10) for k, (n_obs, b) in
                enumerate([(5, 40), (60, 300), (200, 77), (13, 129), (300, 33)])]
    K = 10
    solvers, xis = [], []
    for w in problems:
        s = tj.Solver.for_workload(w, precision="fp32")
        xi, obs = tj.device_workload(w, torch.float32)
        s.set_obstacles(obs)
        solvers.append(s)
        xis.append(xi)
    Bt = sum(w.batch for w in problems)
    net = ws.Net(ws.widths_for(problems[0]), seed=5, precision=1, max_batch=Bt)
    rw = ws.RaggedWarmStart(solvers, xis, [w.boundary for w in problems], net, K)
    rw.run()
    torch.cuda.synchronize()
    warm = [(a.clone(), b.clone()) for a, b in rw.states()]
    warm_tr = [t.clone() for t in rw.traces()]
    fl = rw.FL.cpu().numpy()
    assert set(np.unique(fl)) <= {0, tj.FLAG_COLD_FALLBACK}
    rw.run_cold()
    torch.cuda.synchronize()
    cold = [(a.clone(), b.clone()) for a, b in rw.states(cold=True)]
    # by hand, problem by problem
    nbytes = tj.trajam_warm_pack_mfma(net.shape, None, None, None)
    packed = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    tj.trajam_warm_pack_mfma(net.shape, net.params.data_ptr(), packed.data_ptr(), st)
    for i, (w, s, xi) in enumerate(zip(problems, solvers, xis)):
        s.set_launch(1, 1)   # the wave-per-sample kernel, whose arithmetic the ragged kernel runs
        xb, lam = xi.clone(), torch.zeros_like(xi)
        trp = torch.zeros((ws.K0, w.batch), device="cuda")
        s.project(xi, w.boundary, None, xb, lam, ws.K0, res_trace=trp)
        xw, lw = torch.empty_like(xb), torch.empty_like(lam)
        tj.trajam_warm_jump(net.shape, w.batch, 2, w.n_v, packed.data_ptr(), 1.0, 1.0, xi.data_ptr(),
                            xb.data_ptr(), lam.data_ptr(), xw.data_ptr(), lw.data_ptr(), st)
        r = torch.zeros(w.batch, device="cuda")
        s.residuals(xw, None, r)
        f = torch.zeros(w.batch, dtype=torch.int32, device="cuda")
        tj.trajam_warm_fallback(w.batch, 2, w.n_v, r.data_ptr(), trp[ws.K0 - 1].data_ptr(), xb.data_ptr(),
                                lam.data_ptr(), xw.data_ptr(), lw.data_ptr(), f.data_ptr(), st)
        trc = torch.zeros((K - ws.K0, w.batch), device="cuda")
        s.project(xi, w.boundary, None, xw, lw, K - ws.K0, res_trace=trc)
        xc, lc = xi.clone(), torch.zeros_like(xi)
        s.project(xi, w.boundary, None, xc, lc, K)
        torch.cuda.synchronize()
        assert torch.equal(warm[i][0], xw) and torch.equal(warm[i][1], lw), i
        assert torch.equal(warm_tr[i], torch.cat([trp, trc])), i
        assert np.array_equal(fl[rw.off[i]:rw.off[i + 1]], f.cpu().numpy()), i
        assert torch.equal(cold[i][0], xc) and torch.equal(cold[i][1], lc), i
    rw.close()
    for s in solvers:
        s.close()
