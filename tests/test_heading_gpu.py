"""GPU parity of the heading / multi-circle variant (trajam_heading_*) against the FP64
oracle (oracle/heading.py), through the C ABI.

Bars: FP64 waypoints (x, c, y, s and psi at every time step), multipliers and both
residuals within 1e-9 (relative to max(1, |x|)) after 1, 4 and 12 iterations; the
coefficients themselves within k 16 eps kappa after k iterations, kappa the condition
number of the free block of Q + rho F'F (about 1e6: a right-hand side summed in another
order moves the coefficients along directions that F hardly sees, 7e-10 in a CPU replay
of the kernel's order against 2e-12 on the waypoints); FP32 (state in float, matrices from FP64): waypoints
within 1e-3 m, heading within 1e-3 rad and residuals within 1e-3 (max(1, r)) after 10
iterations, the FP32 rounding of the iterates growing through the multipliers
(observed below 1e-4).  Split calls equal one call bitwise.  Edge cases: no obstacles,
batch 1, an empty batch, iters = 0 (only the boundary coefficients set), 64 and 128
time steps, degrees 4 and 11, a ragged last workgroup; invalid calls fail on the host.
"""
import dataclasses

import numpy as np
import pytest

from oracle import heading as oh
from paper_2408_10731_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _tj():
    from paper_2408_10731_amd import trajam as tj
    return tj


def run(w, iters, precision, state=None, lam=None, trace=True):
    tj = _tj()
    dt = torch.float64 if precision == "fp64" else torch.float32
    s = tj.HeadingSolver(w, precision=precision)
    st = torch.as_tensor(w.xi0 if state is None else state, dtype=dt, device="cuda").contiguous()
    lm = (torch.zeros_like(st) if lam is None else torch.as_tensor(lam, dtype=dt, device="cuda").contiguous())
    tr = torch.zeros((iters, st.shape[0], 2), dtype=dt, device="cuda") if (trace and iters) else None
    s.project(st, lm, iters, tr)
    torch.cuda.synchronize()
    out = (st.double().cpu().numpy(), lm.double().cpu().numpy(),
           tr.double().cpu().numpy() if tr is not None else None)
    s.close()
    return out


def rel(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b)))) if a.size else 0.0


def coefficient_kappa(w):
    ops = oh.operators(w)
    nv = w.n_v
    Qbar = ops.Qg + w.rho * ops.F.T @ ops.F
    free = list(range(3, nv - 1)) + list(range(nv, 2 * nv))
    return float(np.linalg.cond(Qbar[np.ix_(free, free)]))


def waypoint_rel(w, a, b):
    P = oh.operators(w).P
    return rel(np.einsum("tk,brk->brt", P, a), np.einsum("tk,brk->brt", P, b))


def test_heading_fp64_matches_the_oracle_per_iterate():
    w = wl.heading_scene(11, n_obs=5, n_circles=3, batch=70, flow="opposite")
    say("case: heading FP64, n_o 5, n_c 3, B 70 (ragged last workgroup)")
    kappa = coefficient_kappa(w)
    for k in (1, 4, 12):
        g_st, g_lm, g_tr = run(w, k, "fp64")
        o_st, o_lm, o_tr = oh.iterate(w, k)
        e = (waypoint_rel(w, g_st, o_st), rel(g_lm, o_lm), rel(g_tr, o_tr), rel(g_st, o_st))
        bound = k * 16 * np.finfo(np.float64).eps * kappa
        say(f"  {k} iterations: waypoints {e[0]:.1e}, multipliers {e[1]:.1e}, residuals {e[2]:.1e}, "
            f"coefficients {e[3]:.1e} (bound {bound:.1e})")
        assert max(e[:3]) <= 1e-9 and e[3] <= bound


def test_heading_fp32_within_the_bar():
    w = wl.heading_scene(12, n_obs=30, n_circles=4, batch=257, flow="same")
    say("case: heading FP32, n_o 30, n_c 4, B 257, 10 iterations")
    g_st, g_lm, g_tr = run(w, 10, "fp32")
    idx = np.arange(0, 257, 16)
    ws = dataclasses.replace(w, xi0=w.xi0[idx])
    o_st, _, o_tr = oh.iterate(ws, 10)
    ops = oh.operators(w)
    wp = max(np.abs(np.einsum("tk,bk->bt", ops.P, g_st[idx, r] - o_st[:, r])).max() for r in (0, 2))
    hd = np.abs(np.einsum("tk,bk->bt", ops.P, g_st[idx, 4] - o_st[:, 4])).max()
    rr = rel(g_tr[:, idx], o_tr)
    say(f"  {idx.size} samples: waypoints {wp:.2e} m, heading {hd:.2e} rad, residuals {rr:.2e}")
    assert wp <= 1e-3 and hd <= 1e-3 and rr <= 1e-3


def test_heading_paper_size_sampled():
    """Paper II's setting: 1000 samples, a crowd of 30, 4 circles, 10 iterations (one
    control cycle); sampled samples of the full launch against the oracle (FP32 bar),
    the boundary rows exact to FP32 rounding."""
    w = wl.heading_scene(13, n_obs=30, n_circles=4, batch=1000, flow="static")
    say("case: heading FP32 paper size B 1000, n_o 30, n_c 4")
    g_st, _, g_tr = run(w, 10, "fp32")
    idx = np.arange(7, 1000, 111)
    ws = dataclasses.replace(w, xi0=w.xi0[idx])
    o_st, _, o_tr = oh.iterate(ws, 10)
    ops = oh.operators(w)
    wp = max(np.abs(np.einsum("tk,bk->bt", ops.P, g_st[idx, r] - o_st[:, r])).max() for r in (0, 2))
    rr = rel(g_tr[:, idx], o_tr)
    say(f"  waypoints {wp:.2e} m, residuals {rr:.2e}")
    assert wp <= 1e-3 and rr <= 1e-3
    for grp in range(2):
        got = np.einsum("rk,bk->br", ops.A[:, :w.n_v], g_st[:, 2 * grp])
        assert np.abs(got - w.boundary[grp][None]).max() <= 1e-4


def test_heading_split_calls_equal_one_call():
    w = wl.heading_scene(14, n_obs=8, n_circles=2, batch=33)
    say("case: heading split calls, FP32 and FP64")
    for prec in ("fp32", "fp64"):
        a_st, a_lm, a_tr = run(w, 9, prec)
        s1, l1, t1 = run(w, 4, prec)
        s2, l2, t2 = run(w, 5, prec, state=s1, lam=l1)
        assert np.array_equal(a_st, s2) and np.array_equal(a_lm, l2)
        assert np.array_equal(a_tr, np.concatenate([t1, t2]))


@pytest.mark.parametrize("case", ["no_obstacles", "batch1", "steps64", "steps128_deg11", "deg4"])
def test_heading_edge_cases(case):
    kw = dict(no_obstacles=dict(n_obs=0, n_circles=1, batch=9),
              batch1=dict(n_obs=4, n_circles=2, batch=1),
              steps64=dict(n_obs=3, n_circles=2, batch=5, n_steps=64),
              steps128_deg11=dict(n_obs=3, n_circles=3, batch=6, n_steps=128, degree=11),
              deg4=dict(n_obs=2, n_circles=2, batch=4, degree=4, n_steps=20))[case]
    w = wl.heading_scene(15, **kw)
    say("case: heading edge", case)
    g_st, g_lm, g_tr = run(w, 6, "fp64")
    o_st, o_lm, o_tr = oh.iterate(w, 6)
    e = (waypoint_rel(w, g_st, o_st), rel(g_lm, o_lm), rel(g_tr, o_tr), rel(g_st, o_st))
    say(f"  waypoints {e[0]:.1e}, multipliers {e[1]:.1e}, residuals {e[2]:.1e}, coefficients {e[3]:.1e}")
    assert max(e[:3]) <= 1e-9 and e[3] <= 6 * 16 * np.finfo(np.float64).eps * coefficient_kappa(w)


def test_heading_iters0_empty_batch_and_errors():
    tj = _tj()
    w = wl.heading_scene(16, n_obs=3, n_circles=2, batch=5)
    say("case: heading iters 0, empty batch, invalid calls")
    g_st, g_lm, _ = run(w, 0, "fp64", trace=False)
    ops = oh.operators(w)
    ref = np.stack([oh.meet_boundary(w, ops, x) for x in w.xi0])
    assert rel(g_st, ref) <= 1e-12 and not np.any(g_lm)
    s = tj.HeadingSolver(w, precision="fp64")
    empty = torch.zeros((0, 5, w.n_v), dtype=torch.float64, device="cuda")
    s.project(empty, empty.clone(), 3)
    big = torch.zeros((6, 5, w.n_v), dtype=torch.float64, device="cuda")
    with pytest.raises(tj.TrajamError) as e:
        tj.trajam_heading_project(s.handle, 6, big.data_ptr(), big.data_ptr(), 2, None, None)
    assert e.value.status == tj.TRAJAM_ERR_CAPACITY
    s.close()
    for bad in (dict(degree=12), dict(n_steps=129), dict(radii=np.zeros(9)), dict(rho=0.0)):
        args = dict(degree=10, n_steps=100, horizon=20.0, v_max=2.0, a_max=2.0, rho=1.0, radii=[0.0],
                    n_obstacles=1, max_batch=4)
        args.update(bad)
        with pytest.raises((tj.TrajamError, ValueError)):
            tj.trajam_heading_create(tj.make_heading_problem(**args))
    h = tj.trajam_heading_create(tj.make_heading_problem(10, 100, 20.0, 2.0, 2.0, 1.0, [0.0], 1, 4))
    with pytest.raises(tj.TrajamError) as e:   # no scene yet
        tj.trajam_heading_project(h, 1, big.data_ptr(), big.data_ptr(), 1, None, None)
    assert e.value.status == tj.TRAJAM_ERR_INVALID
    tj.trajam_heading_destroy(h)


def test_heading_receding_horizon_matches_the_oracle():
    """Paper II's MPC on the heading variant (FP64): each cycle's executed sample, its
    result, multipliers and next start rows against the oracle's loop, cycle by cycle,
    carrying the multipliers over and clearing them, with the next samples moved on or
    drawn afresh."""
    from paper_2408_10731_amd import mpc as mp
    w = wl.heading_scene(17, n_obs=6, n_circles=3, batch=12, flow="opposite")
    kappa = coefficient_kappa(w)
    for keep, redraw in ((True, None), (False, None), (True, 77)):
        say("case: heading receding horizon FP64, 3 cycles, keep_lambda", keep, "redraw", redraw)
        ref = oh.mpc(w, 3, 0.5, 6, keep_lambda=keep, redraw_seed=redraw)
        m = mp.HeadingMPC(w, 6, 0.5, keep_lambda=keep, precision="fp64", redraw_seed=redraw)
        for k, c in enumerate(ref):
            g_state = m.state.cpu().numpy()
            out = m.cycle()
            assert out["executed"] == c.executed, k
            assert waypoint_rel(w, g_state, c.state) <= 1e-9
            np.testing.assert_allclose(out["boundary"], c.boundary, atol=1e-9)
            np.testing.assert_allclose(out["boundary_psi"], c.boundary_psi, atol=1e-9)
            res_g = torch.as_tensor(out["coefficients"])
            assert waypoint_rel(w, res_g.numpy()[None], c.result[c.executed][None]) <= 1e-9
            assert rel(out["trace"].cpu().numpy(), c.trace) <= 1e-9
        m.close()
