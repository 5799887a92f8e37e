"""GPU parity of the HIP AM projection against the FP64 CPU oracle.

Tolerances:
* FP64 path: every iterate (xb^k, lam^k) and every residual of the trace within
  1e-9 of the oracle (the thesis fixes no precision; rounding-order differences of
  the two implementations are ~1e-13 here).
* FP32 path: final waypoints P xb^K within 1e-3 m of the oracle's, and the residual
  the oracle recomputes from the GPU's xb^K within 1e-4 of the oracle's own final
  residual; boundary rows met to 1e-10 with the boundary values of these workloads
  (exactly representable in float).
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2408_10731_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _tj():
    from paper_2408_10731_amd import trajam as tj
    return tj


def say(*a):
    print(*a, flush=True)


def run_gpu(w, iters, precision="fp64", xi_bar=None, lam=None, tb=None, sphere=None,
            static=None, split=None, kernel=None):
    """kernel: None (library default), 0 multi-wave, 1 wave-per-sample; tb: samples
    per workgroup (default 1 when a kernel is named)."""
    tj = _tj()
    solver = tj.Solver.for_workload(w, precision=precision, sphere=sphere)
    if kernel is not None or tb is not None:
        solver.set_launch(1 if kernel is None else kernel, 1 if tb is None else tb)
    dt = solver.dtype
    xi, obs = tj.device_workload(w, dt, static=static)
    xb = (xi.clone() if xi_bar is None else torch.as_tensor(xi_bar, dtype=dt, device="cuda").contiguous())
    lm = (torch.zeros_like(xi) if lam is None else torch.as_tensor(lam, dtype=dt, device="cuda").contiguous())
    B = w.batch
    traces = []
    flags = torch.zeros(B, dtype=torch.int32, device="cuda")
    chunks = [iters] if split is None else split
    for k in chunks:
        tr = torch.zeros((max(k, 1), B), dtype=dt, device="cuda")
        solver.project(xi, w.boundary, obs, xb, lm, k, res_trace=tr[:k] if k else None,
                       flags=flags)
        traces.append(tr[:k])
    torch.cuda.synchronize()
    out = (xb.double().cpu().numpy(), lm.double().cpu().numpy(),
           torch.cat(traces).double().cpu().numpy(), flags.cpu().numpy())
    solver.close()
    return out


def waypoints(w, xb):
    P, _, _ = oracle.bernstein(w.degree, w.n_steps, w.horizon)
    return np.einsum("tm,bdm->btd", P, xb)


# ------------------------------------------------------------------ FP64 --


def test_fp64_config1_every_iterate():
    """Config 1 (2D, degree 10, 100 steps, 10 circles, B = 64): the first 12 iterates
    one call at a time, each compared with the oracle's iterate."""
    w = wl.config1()
    say("case: cfg1 fp64 per-iterate, B", w.batch)
    xb_o, lam_o = w.xi.copy(), np.zeros_like(w.xi)
    xb_g, lam_g = w.xi.copy(), np.zeros_like(w.xi)
    for k in range(12):
        xb_o, lam_o, tr_o, _ = oracle.project(w, xi_bar=xb_o, lam=lam_o, iters=1)
        xb_g, lam_g, tr_g, _ = run_gpu(w, 1, xi_bar=xb_g, lam=lam_g)
        assert np.abs(xb_g - xb_o).max() <= 1e-9, k
        assert np.abs(lam_g - lam_o).max() <= 1e-9, k
        assert np.abs(tr_g - tr_o).max() <= 1e-9, k


def test_fp64_config1_full_run():
    """Config 1 at its full size in one launch: 100 iterations, trace and final state."""
    w = wl.config1()
    say("case: cfg1 fp64 100 iterations")
    xb_o, lam_o, tr_o, _ = oracle.project(w)
    xb_g, lam_g, tr_g, fl = run_gpu(w, w.iters)
    assert np.abs(tr_g - tr_o).max() <= 1e-9
    assert np.abs(xb_g - xb_o).max() <= 1e-9
    assert np.abs(lam_g - lam_o).max() <= 1e-9
    assert not np.any(fl & 1)
    r_g = oracle.residuals(w, xb_g)[0]
    r_o = oracle.residuals(w, xb_o)[0]
    assert np.abs(r_g - r_o).max() <= 1e-9


def test_fp64_config2_full_size_every_iterate():
    """Config 2 at its full size (2D, degree 10, 100 steps over 30 s, 50 circles,
    B = 1024) in FP64: all 50 iterates, one call at a time, each against the oracle's
    iterate; then the same 50 iterations in one launch (trace and final state)."""
    w = dataclasses.replace(wl.config2(), precision="fp64")
    say("case: cfg2 fp64 per-iterate, B", w.batch, "K", w.iters)
    xb_o, lam_o = w.xi.copy(), np.zeros_like(w.xi)
    xb_g, lam_g = w.xi.copy(), np.zeros_like(w.xi)
    traces = []
    worst = 0.0
    for k in range(w.iters):
        xb_o, lam_o, tr_o, _ = oracle.project(w, xi_bar=xb_o, lam=lam_o, iters=1)
        xb_g, lam_g, tr_g, _ = run_gpu(w, 1, xi_bar=xb_g, lam=lam_g)
        err = max(np.abs(xb_g - xb_o).max(), np.abs(lam_g - lam_o).max(),
                  np.abs(tr_g - tr_o).max())
        worst = max(worst, err)
        assert err <= 1e-9, (k, err)
        traces.append(tr_o[0])
    say(f"  worst per-iterate error {worst:.2e}")
    xb_1, lam_1, tr_1, fl = run_gpu(w, w.iters)
    assert np.abs(tr_1 - np.array(traces)).max() <= 1e-9
    assert np.abs(xb_1 - xb_o).max() <= 1e-9
    assert np.abs(lam_1 - lam_o).max() <= 1e-9
    assert not np.any(fl & 1)


@pytest.mark.parametrize("dims,degree,n_steps,n_obs,batch,speed,per_axis", [
    (2, 5, 9, 2, 3, 0.0, False),      # nvp 8, one partial wave
    (2, 7, 64, 3, 5, 0.5, False),     # exactly one wave, moving obstacles
    (2, 10, 65, 5, 7, 0.0, True),     # ellipses, two waves with a 1-lane tail
    (3, 11, 100, 4, 6, 0.0, True),    # ellipsoids, nvp 12
    (3, 15, 150, 6, 5, 0.3, True),    # nvp 16, three waves, moving ellipsoids
    (3, 4, 200, 1, 4, 0.0, False),    # spheres, four waves
    (2, 3, 30, 9, 2, 0.0, False),     # no free coefficient (degree 3)
    (2, 10, 100, 150, 6, 0.5, False), # three obstacle chunks, candidate masks kept across iterations
    (3, 9, 80, 100, 4, 0.4, True),    # two chunks of moving ellipsoids
    (2, 8, 70, 300, 4, 0.0, False),   # five chunks: past the masks kept, rebuilt every iteration
])
def test_fp64_shapes_and_obstacle_models(dims, degree, n_steps, n_obs, batch, speed, per_axis):
    w = wl.tiny(dims=dims, batch=batch, n_obs=n_obs, degree=degree, n_steps=n_steps,
                speed=speed, per_axis=per_axis, seed=dims * 100 + degree)
    say("case: fp64 shape", dims, degree, n_steps, n_obs, batch, speed, per_axis)
    K = 15
    xb_o, lam_o, tr_o, _ = oracle.project(w, iters=K)
    # ellipsoid model always valid; sphere model when the semi-axes are equal
    for sphere in ([False, True] if not per_axis else [False]):
        for kernel in (0, 1):
            xb_g, lam_g, tr_g, _ = run_gpu(w, K, sphere=sphere, static=(speed == 0.0),
                                           kernel=kernel)
            assert np.abs(tr_g - tr_o).max() <= 1e-9, (sphere, kernel)
            assert np.abs(xb_g - xb_o).max() <= 1e-9, (sphere, kernel)
            assert np.abs(lam_g - lam_o).max() <= 1e-9, (sphere, kernel)


def test_fp64_kinematic_blocks_off_and_no_obstacles():
    for vm, am, n_obs in [(0.0, 2.0, 3), (1.5, 0.0, 3), (0.0, 0.0, 2), (1.5, 2.0, 0)]:
        w = wl.tiny(dims=2, batch=4, n_obs=n_obs, n_steps=40, seed=9)
        w.v_max, w.a_max = vm, am
        say("case: fp64 blocks", vm, am, n_obs)
        xb_o, lam_o, tr_o, _ = oracle.project(w, iters=10)
        xb_g, lam_g, tr_g, _ = run_gpu(w, 10)
        assert np.abs(xb_g - xb_o).max() <= 1e-9
        assert np.abs(lam_g - lam_o).max() <= 1e-9
        assert np.abs(tr_g - tr_o).max() <= 1e-9


def test_fp64_centre_tie_and_warm_start():
    """A point exactly at an obstacle centre (pushed along +x), from a warm start."""
    w = wl.tiny(dims=2, batch=2, n_obs=1, degree=5, n_steps=11, seed=3)
    w.obs_centre = np.array([[2.0, 0.0]])
    w.obs_axes = np.array([[0.5, 0.5]])
    n = w.degree
    line = np.stack([np.linspace(0, 4, n + 1), np.zeros(n + 1)])
    w.xi = np.stack([line, line + 0.01])
    lam0 = np.random.default_rng(0).normal(size=w.xi.shape) * 0.1
    say("case: fp64 centre tie")
    xb_o, lam_o, tr_o, _ = oracle.project(w, iters=6, lam=lam0)
    xb_g, lam_g, tr_g, _ = run_gpu(w, 6, lam=lam0)
    assert np.abs(xb_g - xb_o).max() <= 1e-9
    assert np.abs(lam_g - lam_o).max() <= 1e-9


@pytest.mark.parametrize("dims,n_obs,speed,per_axis", [
    (3, 5, 0.4, True),      # moving ellipsoids: every obstacle tested
    (3, 5, 0.0, True),      # static ellipsoids: the culled loop
    (2, 100, 0.0, False),   # static circles in two chunks
])
def test_fp64_residuals_entry_point(dims, n_obs, speed, per_axis):
    tj = _tj()
    w = wl.tiny(dims=dims, batch=9, n_obs=n_obs, degree=8, n_steps=70, per_axis=per_axis,
                speed=speed, seed=21)
    say("case: residuals entry", dims, n_obs, speed, per_axis)
    xb = w.xi + np.random.default_rng(2).normal(size=w.xi.shape) * 0.3
    solver = tj.Solver.for_workload(w, sphere=False if per_axis else None)
    xi, obs = tj.device_workload(w, torch.float64)
    xbd = torch.as_tensor(xb, device="cuda").contiguous()
    r = torch.zeros(w.batch, dtype=torch.float64, device="cuda")
    m = torch.zeros_like(r)
    solver.residuals(xbd, obs, r, m)
    torch.cuda.synchronize()
    ro, mo = oracle.residuals(w, xb)
    np.testing.assert_allclose(r.cpu().numpy(), ro, atol=1e-10)
    np.testing.assert_allclose(m.cpu().numpy(), mo, atol=1e-10)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_residuals_independent_of_the_projection_launch_shape(precision):
    """The residual kernel keeps its own launch shape: with 100 time steps (128
    threads per sample) every projection shape, including 4 samples per workgroup of
    the wave kernel, gives the same residuals bit for bit (regression: the residual
    launch once took the projection's samples-per-workgroup count)."""
    tj = _tj()
    w = wl.tiny(dims=2, batch=37, n_obs=7, degree=10, n_steps=100, speed=0.5, seed=5)
    say("case: residual launch shapes", precision)
    solver = tj.Solver.for_workload(w, precision=precision)
    dt = solver.dtype
    xb = w.xi + np.random.default_rng(3).normal(size=w.xi.shape) * 0.3
    _, obs = tj.device_workload(w, dt)
    xbd = torch.as_tensor(xb, dtype=dt, device="cuda").contiguous()
    outs = []
    for kernel, spw in [(0, 1), (0, 2), (1, 1), (1, 2), (1, 3), (1, 4)]:
        solver.set_launch(kernel, spw)
        r = torch.zeros(w.batch, dtype=dt, device="cuda")
        solver.residuals(xbd, obs, r)
        torch.cuda.synchronize()
        outs.append(r.cpu().numpy())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    if precision == "fp64":
        np.testing.assert_allclose(outs[0], oracle.residuals(w, xb)[0], atol=1e-10)
    solver.close()


def test_fp64_resumable_tile_invariant_and_deterministic():
    w = wl.config1(batch=37)  # ragged for 2 and 4 samples per workgroup
    say("case: resumable / tile invariance")
    for kernel, tbs in ((0, (1, 2)), (1, (1, 2, 4))):
        runs = [run_gpu(w, 20, kernel=kernel, tb=tb) for tb in tbs]
        runs.append(run_gpu(w, 20, kernel=kernel, tb=tbs[0], split=[7, 13]))
        runs.append(run_gpu(w, 20, kernel=kernel, tb=tbs[0]))
        for r in runs[1:]:
            for x, y in zip(runs[0][:3], r[:3]):
                assert np.array_equal(x, y), kernel
    a = run_gpu(w, 20, kernel=0)
    b = run_gpu(w, 20, kernel=1)
    for x, y in zip(a[:3], b[:3]):
        assert np.abs(x - y).max() <= 1e-11


def test_zero_batch_zero_iters_and_capacity():
    tj = _tj()
    w = wl.config1(batch=4)
    solver = tj.Solver.for_workload(w, max_batch=4)
    xi, obs = tj.device_workload(w, torch.float64)
    xb = xi.clone()
    lm = torch.zeros_like(xi)
    solver.project(xi, w.boundary, obs, xb, lm, 0)
    solver.project(xi[:0], w.boundary, obs, xb[:0], lm[:0], 5)
    torch.cuda.synchronize()
    assert torch.equal(xb, xi)
    big = torch.zeros((5, 2, 11), dtype=torch.float64, device="cuda")
    with pytest.raises(tj.TrajamError) as e:
        solver.project(big, w.boundary, obs, big.clone(), big.clone(), 1)
    assert e.value.status == tj.TRAJAM_ERR_CAPACITY
    with pytest.raises(tj.TrajamError) as e:
        solver.project(xi, w.boundary, obs, xb, lm, -1)
    assert e.value.status == tj.TRAJAM_ERR_INVALID


# ------------------------------------------------------------------ FP32 --


def _fp32_check(w, iters, tol_wp=1e-3, tol_res=1e-4, kernel=None):
    w = w.rounded(np.float32)   # both sides see the float32 inputs the device gets
    xb_o, lam_o, tr_o, _ = oracle.project(w, iters=iters)
    xb_g, lam_g, tr_g, fl = run_gpu(w, iters, precision="fp32", kernel=kernel)
    wp = np.abs(waypoints(w, xb_g) - waypoints(w, xb_o)).max(axis=(1, 2))
    r_g = oracle.residuals(w, xb_g)[0]
    r_o = oracle.residuals(w, xb_o)[0]
    dr = np.abs(r_g - r_o)
    say(f"  waypoint err max {wp.max():.3e} p99 {np.percentile(wp, 99):.3e} median "
        f"{np.median(wp):.3e} m; residual err max {dr.max():.3e} p99 "
        f"{np.percentile(dr, 99):.3e} median {np.median(dr):.3e}")
    assert wp.max() <= tol_wp
    assert np.abs(r_g - r_o).max() <= tol_res
    # boundary rows
    n, T = w.degree, w.horizon
    for ax in range(w.dims):
        x0, v0, a0, xf = w.boundary[ax]
        assert np.abs(xb_g[:, ax, 0] - x0).max() <= 1e-10
        assert np.abs(xb_g[:, ax, n] - xf).max() <= 1e-10
    assert not np.any(fl & 1)
    return wp, r_g, r_o


@pytest.mark.parametrize("kernel", [0, 1])
def test_fp32_config4_moving_circles(kernel):
    """Config-4 geometry (100 circles moving at up to 1 m/s, 15 AM iterations) on 256
    samples: moving obstacles are culled against 16-lane row boxes with their own
    time ranges."""
    w = wl.config4_scene(7, batch=256)
    say("case: cfg4 fp32 moving circles, kernel", kernel)
    _fp32_check(w, 15, kernel=kernel)


@pytest.mark.parametrize("kernel", [0, 1])
def test_fp32_moving_ellipsoids_three_waves(kernel):
    """120 moving ellipsoids in 3D, 150 time steps (three waves / three steps a lane)."""
    w = wl.tiny(dims=3, batch=16, n_obs=120, degree=9, n_steps=150, speed=0.4, per_axis=True,
                seed=77)
    say("case: fp32 moving ellipsoids, kernel", kernel)
    _fp32_check(w, 20, kernel=kernel)


@pytest.mark.parametrize("kernel", [0, 1])
def test_fp32_config2_full_size(kernel):
    """Config 2 at full size (B = 1024, 50 circles, 50 iterations), the bench launch."""
    w = wl.config2()
    say("case: cfg2 fp32 full, kernel", kernel)
    _fp32_check(w, w.iters, kernel=kernel)


def test_fp32_config2_sampled_long_run():
    w = wl.config2(batch=96)
    say("case: cfg2 fp32 100 iterations")
    _fp32_check(w, 100)


# ------------------------------------------------------------------ BF16 --


def _sampled_check(w, precision, iters, idx, tol_wp=1e-3, tol_res=1e-4, sphere=None,
                   kernel=None):
    """GPU at the full batch (the benchmark's launch), oracle on sampled samples."""
    w = w.rounded(np.float32)
    xb_g, lam_g, tr_g, fl = run_gpu(w, iters, precision=precision, sphere=sphere,
                                    kernel=kernel)
    ws = dataclasses.replace(w, xi=np.ascontiguousarray(w.xi[idx]))
    xb_o, _, _, _ = oracle.project(ws, iters=iters)
    xg = xb_g[idx]
    wp = np.abs(waypoints(ws, xg) - waypoints(ws, xb_o)).max(axis=(1, 2))
    r_g = oracle.residuals(ws, xg)[0]
    r_o = oracle.residuals(ws, xb_o)[0]
    dr = np.abs(r_g - r_o)
    say(f"  {precision} vs FP64 oracle: waypoint err max {wp.max():.3e} median "
        f"{np.median(wp):.3e} m; residual err max {dr.max():.3e} median {np.median(dr):.3e}")
    assert wp.max() <= tol_wp
    assert dr.max() <= tol_res
    assert not np.any(fl & 1)
    n = w.degree
    for ax in range(w.dims):
        assert np.abs(xb_g[:, ax, 0] - w.boundary[ax, 0]).max() <= 1e-10
        assert np.abs(xb_g[:, ax, n] - w.boundary[ax, 3]).max() <= 1e-10
    return wp, dr


@pytest.mark.parametrize("kernel", [0, 1])
def test_bf16_config3_full_launch_sampled(kernel):
    """Config 3 (3D, degree 15, 150 steps, 200 ellipsoids, B = 4096, 50 iterations):
    QP product on bf16 matrix cores with hi/lo split and one refinement pass."""
    w = wl.config3()
    idx = np.arange(kernel, w.batch, 43)
    say("case: cfg3 bf16 full launch, sampled", len(idx), "kernel", kernel)
    _sampled_check(w, "bf16", w.iters, idx, sphere=False, kernel=kernel)


def test_fp32_config3_full_launch_sampled():
    w = wl.config3()
    idx = np.arange(7, w.batch, 97)
    say("case: cfg3 fp32 full launch, sampled", len(idx))
    _sampled_check(w, "fp32", w.iters, idx, sphere=False)


@pytest.mark.parametrize("kernel,tb", [(0, 1), (0, 2), (1, 1), (1, 3)])
def test_bf16_small_2d_tiles(kernel, tb):
    """bf16 matrix-core QP with several samples per workgroup (16-column tile holds
    tb x dims columns), including a ragged last workgroup."""
    w = wl.config2(batch=203)
    say("case: bf16 2D tiles", tb)
    w = w.rounded(np.float32)
    xb_o, _, _, _ = oracle.project(w, iters=30)
    xb_g, _, _, _ = run_gpu(w, 30, precision="bf16", tb=tb, kernel=kernel)
    wp = np.abs(waypoints(w, xb_g) - waypoints(w, xb_o)).max()
    say(f"  waypoint err {wp:.3e}")
    assert wp <= 1e-3
