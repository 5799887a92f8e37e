"""Pins of the receding-horizon oracle (oracle/mpc.py): the window shift against
direct evaluation of the Bernstein sums, its group property and endpoints, the
executed state against the basis's closed-form endpoint derivatives, and the loop
against plain projections."""
import dataclasses
from math import comb

import numpy as np
import pytest

import oracle
from oracle import mpc as ompc
from paper_2408_10731_amd import workloads as wl


def bern_eval(xi, T, t):
    """p(t) of one axis by the definition (any t, also outside [0, T])."""
    n = len(xi) - 1
    u = t / T
    return sum(xi[k] * comb(n, k) * u ** k * (1 - u) ** (n - k) for k in range(n + 1))


@pytest.mark.parametrize("n,T,delta", [(10, 30.0, 3.0), (15, 20.0, 2.0), (5, 4.0, 0.7), (10, 10.0, 10.0)])
def test_shift_is_the_same_polynomial_moved_in_time(n, T, delta):
    rng = np.random.default_rng(n)
    S = ompc.shift_matrix(n, T, delta)
    for _ in range(5):
        xi = rng.normal(size=n + 1)
        xs = S @ xi
        for s in np.linspace(0.0, T, 13):
            assert abs(bern_eval(xs, T, s) - bern_eval(xi, T, s + delta)) <= 1e-9 * (1 + np.abs(xi).max())


def test_shift_group_property_and_special_cases():
    n, T = 10, 30.0
    np.testing.assert_allclose(ompc.shift_matrix(n, T, 0.0), np.eye(n + 1), atol=1e-10)
    a, b = 1.5, 2.25
    np.testing.assert_allclose(ompc.shift_matrix(n, T, a) @ ompc.shift_matrix(n, T, b),
                               ompc.shift_matrix(n, T, a + b), atol=1e-9)
    # a constant stays constant; a line moves by its slope times delta
    S = ompc.shift_matrix(n, T, 3.0)
    np.testing.assert_allclose(S @ np.full(n + 1, 2.5), np.full(n + 1, 2.5), atol=1e-12)
    lin = np.arange(n + 1) / n * T            # p(t) = t (linear precision)
    np.testing.assert_allclose(S @ lin, lin + 3.0, atol=1e-10)
    # shifting by the whole horizon: the first coefficient is the old end point
    xi = np.random.default_rng(2).normal(size=n + 1)
    assert abs((ompc.shift_matrix(n, T, T) @ xi)[0] - xi[-1]) <= 1e-9


def test_state_at_matches_the_endpoint_closed_forms():
    n, T = 10, 30.0
    xi = np.random.default_rng(3).normal(size=(2, n + 1))
    p, v, a = ompc.state_at(xi, T, 0.0)
    np.testing.assert_allclose(p, xi[:, 0], atol=1e-14)
    np.testing.assert_allclose(v, n / T * (xi[:, 1] - xi[:, 0]), atol=1e-13)
    np.testing.assert_allclose(a, n * (n - 1) / T ** 2 * (xi[:, 2] - 2 * xi[:, 1] + xi[:, 0]), atol=1e-13)
    p, v, a = ompc.state_at(xi, T, T)
    np.testing.assert_allclose(p, xi[:, -1], atol=1e-12)
    np.testing.assert_allclose(v, n / T * (xi[:, -1] - xi[:, -2]), atol=1e-12)
    # against central differences of the position at an interior time
    t, h = 7.3, 1e-4
    pm = ompc.state_at(xi, T, t - h)[0]
    pp = ompc.state_at(xi, T, t + h)[0]
    p0, v0, a0 = ompc.state_at(xi, T, t)
    np.testing.assert_allclose(v0, (pp - pm) / (2 * h), rtol=1e-6, atol=1e-8)
    np.testing.assert_allclose(a0, (pp - 2 * p0 + pm) / h ** 2, rtol=1e-4, atol=1e-4)


def _scene():
    return wl.config4_scene(77, n_obs=12, batch=6)


def test_first_cycle_is_a_plain_projection_and_the_next_starts_where_the_robot_is():
    w = _scene()
    cyc = ompc.mpc(w, 3, 3.0, 8)
    xb, lam, tr, _ = oracle.project(w, iters=8)
    np.testing.assert_array_equal(cyc[0].xi_bar, xb)
    np.testing.assert_array_equal(cyc[0].lam, lam)
    for c in range(1, 3):
        prev, cur = cyc[c - 1], cyc[c]
        p, v, a = ompc.state_at(prev.xi_bar[prev.executed], w.horizon, 3.0)
        np.testing.assert_allclose(cur.boundary[:, 0], p, atol=1e-12)
        np.testing.assert_allclose(cur.boundary[:, 1], v, atol=1e-12)
        np.testing.assert_allclose(cur.boundary[:, 2], a, atol=1e-12)
        np.testing.assert_array_equal(cur.boundary[:, 3], w.boundary[:, 3])
        # the executed sample's shifted coefficients start at the new start state
        S = ompc.shift_matrix(w.degree, w.horizon, 3.0)
        np.testing.assert_allclose(cur.xi[prev.executed][:, 0], p, atol=1e-9)
        np.testing.assert_allclose(cur.xi, np.einsum("jk,bdk->bdj", S, prev.xi_bar), atol=1e-12)
        # the cycle is the projection of the shifted samples from (shifted, reused lambda),
        # among obstacles moved on by the elapsed time
        wc = dataclasses.replace(w, xi=cur.xi, boundary=cur.boundary,
                                 obs_centre=w.obs_centre + w.obs_vel * 3.0 * c)
        xb2, lam2, _, _ = oracle.project(wc, xi_bar=cur.xi, lam=prev.lam, iters=8)
        np.testing.assert_allclose(cur.xi_bar, xb2, atol=1e-12)
        np.testing.assert_allclose(cur.lam, lam2, atol=1e-12)
        res = oracle.residuals(wc, cur.xi_bar)[0]
        assert cur.executed == ompc.executed_sample(res)


def test_executed_sample_rule():
    assert ompc.executed_sample([3e-7, 1e-9, 2e-3]) == 0        # both below the quantum: lowest index
    assert ompc.executed_sample([5e-3, 1.2e-6, 1.5e-6]) == 1    # keys 5000, 1, 1: the lower index
    assert ompc.executed_sample([5e-3, 2.5e-6, 1.5e-6]) == 2    # keys 5000, 2, 1


def test_reset_multipliers_arm_differs_only_by_lambda():
    w = _scene()
    a = ompc.mpc(w, 2, 3.0, 8, keep_lambda=True)
    b = ompc.mpc(w, 2, 3.0, 8, keep_lambda=False)
    np.testing.assert_array_equal(a[0].xi_bar, b[0].xi_bar)
    np.testing.assert_array_equal(a[1].xi, b[1].xi)
    wc = dataclasses.replace(w, xi=b[1].xi, boundary=b[1].boundary,
                             obs_centre=w.obs_centre + w.obs_vel * 3.0)
    xb2, _, _, _ = oracle.project(wc, xi_bar=b[1].xi, lam=np.zeros_like(b[1].xi), iters=8)
    np.testing.assert_allclose(b[1].xi_bar, xb2, atol=1e-12)
    assert not np.allclose(a[1].xi_bar, b[1].xi_bar)


def test_a_transposed_or_reversed_shift_is_caught_by_the_evaluation_pin():
    """Plausible mistakes in the shift (the transposed matrix, the window moved the
    wrong way) fail the pin that evaluates both polynomials."""
    n, T, delta = 10, 30.0, 3.0
    xi = np.random.default_rng(5).normal(size=n + 1)

    def ok(S):
        xs = S @ xi
        return all(abs(bern_eval(xs, T, s) - bern_eval(xi, T, s + delta)) <= 1e-9 * (1 + np.abs(xi).max())
                   for s in np.linspace(0.0, T, 13))
    assert ok(ompc.shift_matrix(n, T, delta))
    assert not ok(ompc.shift_matrix(n, T, delta).T)
    assert not ok(ompc.shift_matrix(n, T, -delta))
