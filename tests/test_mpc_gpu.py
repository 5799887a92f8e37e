"""The receding-horizon loop on the GPU (paper_2408_10731_amd/mpc.py, trajam_mpc_shift)
against the FP64 oracle (oracle/mpc.py)."""
import dataclasses

import numpy as np
import pytest

import oracle
from oracle import mpc as ompc
from paper_2408_10731_amd import workloads as wl

torch = pytest.importorskip("torch")


def test_host_state_matches_the_oracle_state():
    """The package's de Casteljau evaluation of the executed state against the
    oracle's basis sums (CPU)."""
    from paper_2408_10731_amd import mpc
    c = np.random.default_rng(4).normal(size=(3, 16))
    for t in (0.0, 1.3, 7.9, 20.0, 23.5):
        got = mpc.trajectory_state(c, 20.0, t)
        exp = ompc.state_at(c, 20.0, t)
        for g, e in zip(got, exp):
            np.testing.assert_allclose(g, e, rtol=1e-11, atol=1e-11)


@pytest.mark.gpu
@pytest.mark.parametrize("delta", [3.0, -1.25, 30.0, 41.0])
@pytest.mark.parametrize("keep", [1, 0])
def test_gpu_shift_matches_oracle_matrix(delta, keep):
    from paper_2408_10731_amd import trajam as tj
    w = wl.config4_scene(5, n_obs=4, batch=37)
    print("case: mpc shift", delta, keep, flush=True)
    s = tj.Solver.for_workload(w, precision="fp64")
    rng = np.random.default_rng(8)
    xb = torch.as_tensor(rng.normal(size=(37, 2, 11)) * 5, device="cuda")
    lam = torch.as_tensor(rng.normal(size=(37, 2, 11)), device="cuda")
    xn, xbn, ln = torch.zeros_like(xb), torch.zeros_like(xb), torch.full_like(xb, 7.0)
    st = torch.cuda.current_stream().cuda_stream
    tj.trajam_mpc_shift(s.handle, 37, delta, keep, xb.data_ptr(), lam.data_ptr(), xn.data_ptr(), xbn.data_ptr(),
                        ln.data_ptr(), st)
    torch.cuda.synchronize()
    S = ompc.shift_matrix(w.degree, w.horizon, delta)
    exp = np.einsum("jk,bdk->bdj", S, xb.cpu().numpy())
    scale = 1 + np.abs(exp).max()
    np.testing.assert_allclose(xn.cpu().numpy(), exp, atol=1e-10 * scale)
    assert torch.equal(xn, xbn)
    np.testing.assert_array_equal(ln.cpu().numpy(), lam.cpu().numpy() if keep else 0.0)
    # in place: every output aliasing its input
    tj.trajam_mpc_shift(s.handle, 37, delta, keep, xb.data_ptr(), lam.data_ptr(), xb.data_ptr(), xb.data_ptr(),
                        lam.data_ptr(), st)
    torch.cuda.synchronize()
    assert torch.equal(xb, xn)
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("keep", [True, False])
def test_gpu_mpc_loop_matches_oracle_per_cycle(keep):
    """FP64, a small moving-obstacle scene: every cycle's projected samples and
    multipliers within 1e-9 of the oracle's loop, the same executed sample and the same
    boundary rows."""
    from paper_2408_10731_amd import mpc, trajam as tj
    w = wl.config4_scene(77, n_obs=12, batch=6)
    n_cyc, delta, K = 4, 3.0, 8
    print("case: mpc loop fp64", keep, flush=True)
    ref = ompc.mpc(w, n_cyc, delta, K, keep_lambda=keep)
    s = tj.Solver.for_workload(w, precision="fp64")
    xi0 = torch.as_tensor(w.xi, dtype=torch.float64, device="cuda")
    m = mpc.MPC(s, xi0, w.boundary, (w.obs_centre, w.obs_vel, w.obs_axes), K, delta, keep_lambda=keep)
    for c in range(n_cyc):
        np.testing.assert_allclose(m.boundary, ref[c].boundary, atol=1e-9)
        np.testing.assert_allclose(m.xi.cpu().numpy(), ref[c].xi, atol=1e-9)
        out = m.cycle()
        torch.cuda.synchronize()
        assert out["executed"] == ref[c].executed, c
        # the state after the cycle's projection is what the shift consumed: compare
        # through the next cycle's samples, and the trace directly
        np.testing.assert_allclose(out["trace"].cpu().numpy(), ref[c].trace, atol=1e-9)
    s.close()


@pytest.mark.gpu
def test_gpu_mpc_fp32_config4_sizes_cycle_is_consistent():
    """FP32 at the MPC workload's size (1000 samples, 10 iterations a cycle, 100 moving
    circles): after each cycle the executed sample's shifted first coefficient is the
    next cycle's start position (the state the host evaluated at delta)."""
    from paper_2408_10731_amd import mpc, trajam as tj
    w = wl.config4_scene(90_001, batch=1000)
    K, delta = 10, 3.0
    print("case: mpc fp32 cfg4", flush=True)
    s = tj.Solver.for_workload(w, precision="fp32")
    xi0 = torch.as_tensor(w.xi, dtype=torch.float32, device="cuda")
    m = mpc.MPC(s, xi0, w.boundary, (w.obs_centre, w.obs_vel, w.obs_axes), K, delta)
    for c in range(3):
        out = m.cycle()
        torch.cuda.synchronize()
        i = out["executed"]
        np.testing.assert_allclose(m.xi[i, :, 0].double().cpu().numpy(), m.boundary[:, 0], atol=2e-4)
        assert m.xi.dtype == torch.float32
    s.close()
