"""GPU parity of the penalty continuation (trajam_project_continuation) against the
oracle's orc_project_cont.

* FP64: every iterate (xb^k, lam^k), every residual and every level within 1e-9 /
  exactly, over runs long enough to climb the ladder; the state split over calls.
* FP32 at config-2 size: final waypoints within 1e-3 m and the oracle's recomputed
  residual within 1e-4 on sampled samples, with the levels the device reached.
* The continuation with one level equals trajam_project bit for bit.
"""
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


def _gpu(w, precision, cont, iters_list, spw=1, sphere=None):
    tj = _tj()
    s = tj.Solver.for_workload(w, precision=precision, sphere=sphere)
    s.set_launch(1, spw)
    s.set_continuation(*cont)
    dt = s.dtype
    xi, obs = tj.device_workload(w, dt)
    xb, lam = xi.clone(), torch.zeros_like(xi)
    state = s.cont_state(w.batch)
    out = []
    for k in iters_list:
        tr = torch.zeros((k, w.batch), dtype=dt, device="cuda")
        s.project_continuation(xi, w.boundary, obs, xb, lam, state, k, res_trace=tr)
        torch.cuda.synchronize()
        out.append((xb.double().cpu().numpy(), lam.double().cpu().numpy(), tr.double().cpu().numpy(),
                    s.cont_levels(state)))
    s.close()
    return out


@pytest.mark.parametrize("dims,n_obs,speed,per_axis", [(2, 4, 0.0, False), (3, 5, 0.3, True), (2, 6, 0.4, False)])
def test_fp64_every_iterate_and_level(dims, n_obs, speed, per_axis):
    w = wl.tiny(dims=dims, batch=5, n_obs=n_obs, degree=7, n_steps=60, speed=speed, per_axis=per_axis,
                seed=61 + dims)
    cont = (6, 2.0, 2, 0.0, 1e-8)          # every check with a residual above 1e-8 climbs (a decision
    #                                        far from rounding: both sides agree on it)
    K = 16
    say("case: continuation fp64", dims, n_obs, speed, per_axis)
    g = _gpu(w, "fp64", cont, [1] * K, sphere=not per_axis)
    xb, lam, state = w.xi.copy(), np.zeros_like(w.xi), None
    top = 0
    for k in range(K):
        xb, lam, tr, lt, state = oracle.project_cont(w, *cont, iters=1, xi_bar=xb, lam=lam, state=state)
        gx, gl, gt, (glev, gcnt, gref) = g[k]
        assert np.abs(gx - xb).max() <= 1e-9, k
        assert np.abs(gl - lam).max() <= 1e-9, k
        assert np.abs(gt[0] - tr[0]).max() <= 1e-9, k
        assert np.array_equal(glev, state[0]) and np.array_equal(gcnt, state[1]), k
        np.testing.assert_allclose(gref, state[2], atol=1e-9)
        top = max(top, int(glev.max()))
    say(f"  {K} iterates within 1e-9, levels equal, highest level {top}")
    assert top >= 3


def test_fp64_one_call_equals_split_calls_and_the_oracle():
    w = wl.config1(batch=16)
    cont = (10, 2.0, 10, 0.9, 1e-3)
    say("case: continuation fp64 cfg1, 100 iterations")
    (xb1, lam1, tr1, st1), = _gpu(w, "fp64", cont, [100], spw=2)
    parts = _gpu(w, "fp64", cont, [37, 63], spw=2)
    np.testing.assert_array_equal(parts[-1][0], xb1)
    np.testing.assert_array_equal(parts[-1][1], lam1)
    xo, lo, to, lto, sto = oracle.project_cont(w, *cont, iters=100)
    assert np.abs(xb1 - xo).max() <= 1e-9 and np.abs(lam1 - lo).max() <= 1e-9
    assert np.abs(tr1 - to).max() <= 1e-9
    assert np.array_equal(st1[0], sto[0])
    say(f"  levels reached {np.bincount(st1[0])}")


def test_one_level_equals_plain_projection():
    tj = _tj()
    w = wl.config2(batch=256).rounded(np.float32)
    say("case: continuation with one level vs trajam_project, fp32")
    s = tj.Solver.for_workload(w, precision="fp32")
    s.set_launch(1, 1)
    xi, obs = tj.device_workload(w, torch.float32)
    xb, lam = xi.clone(), torch.zeros_like(xi)
    s.project(xi, w.boundary, obs, xb, lam, 30)
    s.set_continuation(1, 2.0, 5, 0.9, 1e-3)
    xb2, lam2 = xi.clone(), torch.zeros_like(xi)
    s.project_continuation(xi, w.boundary, obs, xb2, lam2, s.cont_state(w.batch), 30)
    torch.cuda.synchronize()
    assert torch.equal(xb, xb2) and torch.equal(lam, lam2)
    s.close()


def test_fp32_config2_sampled_against_the_oracle():
    """Config 2 at full size (1024 samples, 50 circles, 100 steps) with the ladder of
    the benchmark (10 levels, growth 2, window 10, stall 0.9, tol 1e-3), 150 iterations;
    16 sampled samples against the FP64 oracle from the same float inputs."""
    w = wl.config2().rounded(np.float32)
    cont = (10, 2.0, 10, 0.9, 1e-3)
    K = 150
    say("case: continuation fp32 cfg2, 150 iterations")
    (xb, lam, tr, (lev, cnt, ref)), = _gpu(w, "fp32", cont, [K])
    idx = np.arange(5, 1024, 64)
    ws = w.subset(1024)
    ws.xi = np.ascontiguousarray(w.xi[idx])
    xo, _, to, lto, sto = oracle.project_cont(ws, *cont, iters=K)
    P, _, _ = oracle.bernstein(w.degree, w.n_steps, w.horizon)
    wp = np.abs(np.einsum("tm,bdm->btd", P, xb[idx] - xo)).max()
    dr = np.abs(oracle.residuals(ws, xb[idx])[0] - oracle.residuals(ws, xo)[0]).max()
    say(f"  waypoint err {wp:.2e} m, residual err {dr:.2e}; device levels {np.bincount(lev, minlength=10)}, "
        f"sampled levels equal on {int(np.sum(lev[idx] == sto[0]))} of {idx.size}")
    assert wp <= 1e-3 and dr <= 1e-4
