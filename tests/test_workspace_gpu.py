"""Workspace bounds (Paper III, eq bound_con: rows G = [-P; P] through the slack step)
on the GPU against the FP64 oracle: every iterate in FP64 under both kernels, the
residuals entry point, a multi-agent problem, and FP32 at config-2 size."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2408_10731_amd import workloads as wl

torch = pytest.importorskip("torch")

from test_gpu_parity import run_gpu, waypoints  # noqa: E402


def box_scene(batch=16, n_obs=10, box=((-1.0, 14.6), (31.0, 15.4)), precision="fp64"):
    w = wl.config2(batch=batch, seed=11)
    return dataclasses.replace(w, obs_centre=w.obs_centre[:n_obs], obs_vel=w.obs_vel[:n_obs],
                               obs_axes=w.obs_axes[:n_obs], workspace=np.array(box, dtype=np.float64),
                               precision=precision)


@pytest.mark.gpu
@pytest.mark.parametrize("kernel", [0, 1])
def test_fp64_workspace_every_iterate(kernel):
    w = box_scene()
    print("case: workspace fp64 kernel", kernel, flush=True)
    K = 12
    for k in (1, 2, 5, K):
        xo, lo, tro, _ = oracle.project(w, iters=k)
        xg, lg, trg, _ = run_gpu(w, k, kernel=kernel)
        np.testing.assert_allclose(xg, xo, atol=1e-9)
        np.testing.assert_allclose(lg, lo, atol=1e-9)
        np.testing.assert_allclose(trg, tro, atol=1e-9)
    # the rows are active: without them the iterates differ
    xn, _, _, _ = run_gpu(dataclasses.replace(w, workspace=None), K, kernel=kernel)
    assert np.abs(xn - xg).max() > 1e-3


@pytest.mark.gpu
def test_fp64_workspace_residuals_entry_point():
    from paper_2408_10731_amd import trajam as tj
    w = box_scene(batch=9)
    s = tj.Solver.for_workload(w, precision="fp64")
    xi, obs = tj.device_workload(w, torch.float64)
    res = torch.zeros(w.batch, dtype=torch.float64, device="cuda")
    rmax = torch.zeros_like(res)
    s.residuals(xi, obs, res, res_max=rmax)
    torch.cuda.synchronize()
    ro, mo = oracle.residuals(w, w.xi)
    np.testing.assert_allclose(res.cpu().numpy(), ro, atol=1e-10)
    np.testing.assert_allclose(rmax.cpu().numpy(), mo, atol=1e-10)
    s.close()


@pytest.mark.gpu
def test_fp64_workspace_multi_agent():
    w = wl.tiny_agents(dims=2, n_agents=3, batch=2, n_obs=1)
    lo = w.boundary[..., 0].min(axis=0) - 0.3
    hi = w.boundary[..., 0].max(axis=0) + 0.3
    lo = np.minimum(lo, w.boundary[..., 3].min(axis=0) - 0.3)
    hi = np.maximum(hi, w.boundary[..., 3].max(axis=0) + 0.3)
    lo[1] += 0.6   # a tight band in y that the samples leave
    hi[1] -= 0.6
    w = dataclasses.replace(w, workspace=np.stack([lo, hi]), precision="fp64")
    from paper_2408_10731_amd import trajam as tj
    print("case: workspace agents", flush=True)
    K = 6
    xo, lo_, tro = oracle.project_agents(w, iters=K)[:3]
    s = tj.Solver.for_workload(w, precision="fp64")
    xi, obs = tj.device_workload(w, torch.float64)
    xb, lam = xi.clone(), torch.zeros_like(xi)
    tr = torch.zeros((K, w.batch), dtype=torch.float64, device="cuda")
    s.project(xi, w.boundary, obs, xb, lam, K, res_trace=tr)
    torch.cuda.synchronize()
    np.testing.assert_allclose(xb.cpu().numpy(), xo, atol=1e-9)
    np.testing.assert_allclose(tr.cpu().numpy(), tro, atol=1e-9)
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("kernel", [0, 1])
def test_fp32_workspace_config2_size(kernel):
    """Config 2 (1024 samples, 50 circles) inside the band |y - 15| <= 1.2 (which the
    samples leave): FP32 final waypoints within 1e-3 m of the FP64 oracle; the oracle's
    residual of the FP32 result within 2e-4 of its own (50 iterations that have not
    converged carry FP32 rounding: 1.2e-4 measured) and within twice what the same
    comparison gives without the band, plus 5e-5."""
    w = dataclasses.replace(wl.config2(batch=1024), workspace=np.array(((-1.0, 13.8), (31.0, 16.2))),
                            precision="fp32")
    print("case: workspace fp32 cfg2 kernel", kernel, flush=True)
    # the band is active: without obstacles the samples already leave it
    w0 = dataclasses.replace(w, obs_centre=w.obs_centre[:0], obs_vel=w.obs_vel[:0], obs_axes=w.obs_axes[:0])
    assert (oracle.residuals(w0, w.xi)[0] > 1e-3).mean() > 0.05
    K = 50
    xo, _, tro, _ = oracle.project(w, iters=K)
    xg, _, trg, _ = run_gpu(w, K, precision="fp32", kernel=kernel)
    assert np.abs(waypoints(w, xg) - waypoints(w, xo)).max() <= 1e-3
    dev = np.abs(oracle.residuals(w, xg)[0] - oracle.residuals(w, xo)[0]).max()
    # the same comparison without the band: the rows must not degrade FP32 accuracy
    wn = dataclasses.replace(w, workspace=None)
    xon = oracle.project(wn, iters=K)[0]
    xgn = run_gpu(wn, K, precision="fp32", kernel=kernel)[0]
    dev_n = np.abs(oracle.residuals(wn, xgn)[0] - oracle.residuals(wn, xon)[0]).max()
    print(f"  residual deviation fp32 vs fp64: {dev:.2e} with the band, {dev_n:.2e} without", flush=True)
    assert dev <= 2e-4 and dev <= 2.0 * dev_n + 5e-5
