"""Pins of the oracle's penalty continuation (thesis ch. 4, Alg 1: the penalties are
raised while the residuals stay above a threshold; ch. 7: the QP inverse cached for ten
increasing penalties, used in later iterations).  The ladder, the per-trajectory level
and the stall check are readings listed in the design notes; these tests check the
oracle against what those readings and the mathematics fix, each by a route of its
own."""
import numpy as np
import pytest

import oracle
from paper_2408_10731_amd import workloads as wl

from test_oracle_pins import _algebraic_residual_products, stacked_F

PARAMS = dict(n_levels=10, growth=2.0, window=3, stall=0.9, tol=1e-3)


def _scene(seed=21, batch=3, n_obs=4, n_steps=30):
    return wl.tiny(dims=2, batch=batch, n_obs=n_obs, seed=seed, n_steps=n_steps)


def test_one_level_or_unit_growth_is_the_plain_iteration():
    w = _scene()
    xb0, lam0, tr0, _ = oracle.project(w, iters=40)
    for kw in (dict(PARAMS, n_levels=1), dict(PARAMS, growth=1.0, window=1, stall=2.0)):
        xb, lam, tr, lt, _ = oracle.project_cont(w, iters=40, **kw)
        np.testing.assert_array_equal(xb, xb0)
        np.testing.assert_array_equal(lam, lam0)
        np.testing.assert_array_equal(tr, tr0)


def _run_steps(w, K, **kw):
    """One iteration a call (the state carried), recording every iterate."""
    xb, lam, state = w.xi.copy(), np.zeros_like(w.xi), None
    hist = [(xb, lam, None)]
    for _ in range(K):
        xb, lam, tr, lt, state = oracle.project_cont(w, iters=1, xi_bar=xb, lam=lam, state=state, **kw)
        hist.append((xb, lam, (tr[0], lt[0])))
    return hist, state


def test_levels_rise_and_the_split_run_equals_one_call():
    w = _scene(seed=23, batch=4, n_obs=5)
    kw = dict(PARAMS, window=2, stall=0.0, tol=0.0)   # every check with a residual raises the level
    hist, state = _run_steps(w, 25, **kw)
    xb, lam, tr, lt, st = oracle.project_cont(w, iters=25, **kw)
    np.testing.assert_array_equal(hist[-1][0], xb)
    np.testing.assert_array_equal(hist[-1][1], lam)
    for a, b in zip(state, st):
        np.testing.assert_array_equal(a, b)
    assert lt.max() >= 3                          # the ladder is used


def test_qp_and_multiplier_use_the_level_penalty():
    """Per iteration k with level l(k): lambda^{k+1} = lambda^k - rho_l F^T r^k and the QP
    stationarity on the free coefficients lambda^{k+1}_f = (xb^{k+1} - xi)_f
    + rho_l [F^T F xb^{k+1} - F^T e^{k+1}]_f (eqs lag, affine_trans / matrix_vec with the
    level's penalty), F stacked explicitly, F^T e^{k+1} = F^T F xb^k - F^T r^k from the
    projections' characterization."""
    w = _scene(seed=25, batch=2, n_obs=3, n_steps=25)
    kw = dict(PARAMS, window=2, stall=0.0, tol=0.0)
    hist, _ = _run_steps(w, 14, **kw)
    P, Pd, Pdd = oracle.bernstein(w.degree, w.n_steps, w.horizon)
    FtF = stacked_F(P, Pd, Pdd, w.n_obs).T @ stacked_F(P, Pd, Pdd, w.n_obs)
    free = list(range(3, w.degree))
    used = set()
    for k in range(1, len(hist)):
        xb0, lam0, _ = hist[k - 1]
        xb1, lam1, (res, lev) = hist[k]
        for i in range(w.batch):
            rho = w.rho * kw["growth"] ** lev[i]
            used.add(int(lev[i]))
            ftr = _algebraic_residual_products(w, xb0[i])
            np.testing.assert_allclose(lam1[i], lam0[i] - rho * ftr, atol=1e-9)
            for ax in range(w.dims):
                fte = FtF @ xb0[i, ax] - ftr[ax]
                stat = (xb1[i, ax] - w.xi[i, ax]) + rho * (FtF @ xb1[i, ax] - fte)
                np.testing.assert_allclose(lam1[i, ax, free], stat[free], atol=1e-9)
    assert len(used) >= 3


def test_level_trace_follows_the_stall_check():
    """The levels follow the stated check, replayed from the oracle's own residual trace:
    non-decreasing, changed only at check iterations, by one, never past the ladder, and
    raised exactly when the residual is above tol and above stall times the reference
    (0 before the first check)."""
    w = _scene(seed=27, batch=6, n_obs=6, n_steps=40)
    kw = dict(PARAMS, window=3, stall=0.9, n_levels=5)
    K = 60
    _, _, tr, lt, (lev, cnt, ref) = oracle.project_cont(w, iters=K, **kw)
    for i in range(w.batch):
        level, count, r0 = 0, 0, 0.0
        for k in range(K):
            assert lt[k, i] == level, (i, k)
            count += 1
            if count == kw["window"]:
                up = tr[k, i] > kw["tol"] and tr[k, i] > kw["stall"] * r0
                level = min(level + (1 if up else 0), kw["n_levels"] - 1)
                r0, count = tr[k, i], 0
        assert lev[i] == level and cnt[i] == count and ref[i] == r0
    assert np.all(np.diff(lt, axis=0) >= 0) and np.all(np.diff(lt, axis=0) <= 1)
    assert lt.max() <= kw["n_levels"] - 1 and lt.max() > 0


def test_converged_samples_keep_their_penalty():
    """A feasible, boundary-consistent sample has residual 0 at every check: its level
    never rises (the check requires res > tol)."""
    from test_oracle_pins import feasible_workload
    w = feasible_workload()
    _, _, tr, lt, (lev, _, _) = oracle.project_cont(w, iters=30, **dict(PARAMS, window=1, stall=0.0))
    assert tr.max() < 1e-10 and lt.max() == 0 and lev.max() == 0


def test_planted_inverted_stall_check_is_caught():
    oracle.set_fault(9)
    try:
        with pytest.raises(AssertionError):
            test_level_trace_follows_the_stall_check()
    finally:
        oracle.set_fault(0)
