"""Pins of the multi-agent oracle (joint projection of N agents with pairwise
avoidance, thesis ch. 7 (Paper IV) in the projection form of ch. 6), each independent of the
oracle's joint assembly:

* N = 1 is the single-robot oracle;
* the joint QP equals the closed form that splits every right-hand side into its
  agent mean and the deviations: with L = N I - 1 1^T the pair Gram, the mean solves
  the single-robot QP and each deviation the QP with H + N rho P^T P (both solved
  here with numpy from the pinned basis);
* F^T r is the gradient of 1/2 |r|^2 (every polar target here is the Euclidean
  projection onto a sphere's exterior or a ball, so 1/2 dist^2 has gradient r):
  central finite differences pin every block's sign and index, the pair rows' too;
* F^T e = F^T F xb - F^T r with F^T F written out per agent;
* relabelling agents permutes the result; a converged crossing keeps every pair at
  least the combined radius apart and meets the boundary rows; agents that never
  come close converge to their single-robot projections;
* planted mistakes (sign of a pair's row for its second agent, a wrong pair Gram)
  make a pin fail.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2408_10731_amd import workloads as wl


def _single(w, a):
    return dataclasses.replace(w, xi=np.ascontiguousarray(w.xi[:, a]), boundary=w.boundary[a],
                               n_agents=1)


def test_one_agent_is_the_single_robot_oracle():
    for dims in (2, 3):
        w = wl.tiny_agents(dims=dims, n_agents=1, batch=3, n_obs=2)
        xb, lm, tr, tm = oracle.project_agents(w, iters=12)
        xs, ls, ts, ms = oracle.project(_single(w, 0), iters=12)
        np.testing.assert_allclose(xb[:, 0], xs, atol=1e-12)
        np.testing.assert_allclose(lm[:, 0], ls, atol=1e-12)
        np.testing.assert_allclose(tr, ts, atol=1e-12)


def _kkt_solve(H, A, q, b):
    nv = H.shape[0]
    K = np.zeros((nv + 4, nv + 4))
    K[:nv, :nv] = H
    K[nv:, :nv] = A
    K[:nv, nv:] = A.T
    return np.linalg.solve(K, np.concatenate([q, b]))[:nv]


def _joint_qp_pin(N, dims=2, seed=0):
    w = wl.tiny_agents(dims=dims, n_agents=N, n_obs=2)
    pr = oracle.problem_of(w)
    A, H = oracle.constraint_matrices(pr)
    P, _, _ = oracle.bernstein(w.degree, w.n_steps, w.horizon)
    rng = np.random.default_rng(seed)
    q = rng.normal(size=(N, w.n_v))
    b = rng.normal(size=(N, 4))
    got = oracle.agents_qp(pr, q, b)
    qm, bm = q.mean(0), b.mean(0)
    mean = _kkt_solve(H, A, qm, bm)
    Hd = H + N * w.rho * P.T @ P
    want = np.stack([mean + _kkt_solve(Hd, A, q[a] - qm, b[a] - bm) for a in range(N)])
    return np.abs(got - want).max()


@pytest.mark.parametrize("N", [2, 3, 5])
def test_joint_qp_is_mean_plus_deviation_closed_form(N):
    assert _joint_qp_pin(N) <= 1e-10


def _grad_pin(dims=2, seed=1, h=1e-6):
    """max |F^T r - grad 1/2 |r|^2| over every coefficient, at a configuration with
    active pairs, obstacles and kinematic rows."""
    w = wl.tiny_agents(dims=dims, n_agents=3, n_obs=2, seed=5 + dims)
    rng = np.random.default_rng(seed)
    # squeeze the agents towards the centre so that pairs are active
    xb = w.xi[0] * 0.35 + rng.normal(scale=0.05, size=w.xi[0].shape)
    _, ftr, r2 = oracle.agents_polar_products(w, xb)
    assert r2 > 1e-3
    g = np.zeros_like(xb)
    for idx in np.ndindex(*xb.shape):
        e = np.zeros_like(xb)
        e[idx] = h
        rp = oracle.agents_polar_products(w, xb + e)[2]
        rm = oracle.agents_polar_products(w, xb - e)[2]
        g[idx] = 0.25 * (rp - rm) / h
    return np.abs(ftr - g).max() / max(1.0, np.abs(g).max())


@pytest.mark.parametrize("dims", [2, 3])
def test_joint_FtR_is_gradient_of_half_squared_residual(dims):
    assert _grad_pin(dims) <= 1e-6


@pytest.mark.parametrize("dims", [2, 3])
def test_joint_FtE_is_FtF_xb_minus_FtR(dims):
    w = wl.tiny_agents(dims=dims, n_agents=4, n_obs=2)
    xb = w.xi[1] * 0.4
    fte, ftr, _ = oracle.agents_polar_products(w, xb)
    P, Pd, Pdd = oracle.bernstein(w.degree, w.n_steps, w.horizon)
    N = w.n_agents
    single = w.n_obs * P.T @ P + Pd.T @ Pd + Pdd.T @ Pdd
    L = N * np.eye(N) - np.ones((N, N))
    ftf = np.einsum("mn,adn->adm", single, xb) + np.einsum("ab,mn,bdn->adm", L, P.T @ P, xb)
    np.testing.assert_allclose(fte, ftf - ftr, atol=1e-11)


def test_relabelling_agents_permutes_the_result():
    w = wl.tiny_agents(dims=3, n_agents=4, n_obs=1, batch=2)
    perm = np.array([2, 0, 3, 1])
    wp = dataclasses.replace(w, xi=np.ascontiguousarray(w.xi[:, perm]), boundary=w.boundary[perm])
    a = oracle.project_agents(w, iters=15)
    b = oracle.project_agents(wp, iters=15)
    np.testing.assert_allclose(b[0], a[0][:, perm], atol=1e-11)
    np.testing.assert_allclose(b[1], a[1][:, perm], atol=1e-11)
    np.testing.assert_allclose(b[2], a[2], atol=1e-11)


@pytest.mark.parametrize("dims", [2, 3])
def test_converged_crossing_keeps_pairs_apart(dims):
    w = wl.tiny_agents(dims=dims, n_agents=4, n_obs=1, batch=2)
    xb, _, tr, _ = oracle.project_agents(w, iters=400)
    assert tr[-1].max() <= 1e-8
    P, _, _ = oracle.bernstein(w.degree, w.n_steps, w.horizon)
    p = np.einsum("tm,badm->batd", P, xb)
    R = 2 * w.agent_radius
    for a in range(w.n_agents):
        for b in range(a + 1, w.n_agents):
            assert np.linalg.norm(p[:, a] - p[:, b], axis=-1).min() >= R - 1e-6
        np.testing.assert_allclose(xb[:, a, :, 0], np.broadcast_to(w.boundary[a, :, 0], (2, dims)),
                                   atol=1e-10)
        np.testing.assert_allclose(xb[:, a, :, -1], np.broadcast_to(w.boundary[a, :, 3], (2, dims)),
                                   atol=1e-10)
    # the straight lines all cross the centre at mid-horizon: the raw samples collide
    p0 = np.einsum("tm,badm->batd", P, w.xi)
    assert np.linalg.norm(p0[:, 0] - p0[:, 2], axis=-1).min() < R


def test_agents_that_never_meet_converge_to_single_robot_projections():
    w = wl.tiny_agents(dims=2, n_agents=2, n_obs=1, batch=2)
    xi = w.xi.copy()
    bnd = w.boundary.copy()
    # move agent 1's whole task 20 m away
    xi[:, 1, 1] += 20.0
    bnd[1, 1, 0] += 20.0
    bnd[1, 1, 3] += 20.0
    w = dataclasses.replace(w, xi=xi, boundary=bnd)
    xb, _, tr, _ = oracle.project_agents(w, iters=300)
    assert tr[-1].max() <= 1e-9
    for a in range(2):
        xs, _, ts, _ = oracle.project(_single(w, a), iters=300)
        assert ts[-1].max() <= 1e-9
        np.testing.assert_allclose(xb[:, a], xs, atol=1e-7)


def _agent_pins_pass():
    try:
        assert _joint_qp_pin(3) <= 1e-10
        assert _grad_pin(2) <= 1e-6
    except AssertionError:
        return False
    return True


@pytest.mark.parametrize("fault", [6, 7])
def test_planted_agent_mistakes_are_caught(fault):
    """A pair's row entering its second agent with the wrong sign (6), or a wrong
    pair Gram in the joint matrix (7), makes a pin fail."""
    assert _agent_pins_pass()
    oracle.set_fault(fault)
    try:
        assert not _agent_pins_pass()
    finally:
        oracle.set_fault(0)
