"""Materialised polar variables (trajam_polar) element by element against the
oracle's polar steps (thesis ch. 6, eqs comp_alpha, comp_beta, comp_d for the
obstacles; alpha_v, compute_dv / alpha_a, compute_da for the kinematic blocks).

Tolerances: FP64 d within 1e-12 (relative), angles within 1e-10 (wrapped), the
kinematic targets e = bound d dir(alpha, beta) within 1e-10 of the oracle's; FP32
inputs rounded to float first, d within 2e-6 relative, angles within 2e-4 wherever the
scaled offset is not tiny (|u_xy| > 1e-2; the angle of a near-zero vector is
ill-conditioned), kinematic targets within 1e-4 of the bound.
"""
import numpy as np
import pytest

import oracle
from paper_2408_10731_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _maps(w, xb):
    """p, v, a [B, n_p, D] of coefficients xb [B, D, n_v] (oracle basis)."""
    mats = oracle.bernstein(w.degree, w.n_steps, w.horizon)
    return tuple(np.einsum("tm,bdm->btd", M, xb) for M in mats)


def _wrapped(a, b):
    return np.abs((a - b + np.pi) % (2 * np.pi) - np.pi)


def _dir(al, be, D):
    if D == 3:
        return np.stack([np.cos(al) * np.sin(be), np.sin(al) * np.sin(be), np.cos(be)], -1)
    return np.stack([np.cos(al), np.sin(al)], -1)


def _check(w, xb, al, be, d, kin, precision, entries=None):
    D, n_p = w.dims, w.n_steps
    p, v, a = _maps(w, xb)
    t = np.arange(n_p) * (w.horizon / (n_p - 1))
    fp64 = precision == "fp64"
    if entries is None:
        entries = [(b, j, k) for b in range(xb.shape[0]) for j in range(w.n_obs) for k in range(n_p)]
    for b, j, k in entries:
        c = w.obs_centre[j] + w.obs_vel[j] * t[k]
        xt = p[b, k] - c
        ra, rb, rd, _ = oracle.polar_obstacle(xt, w.obs_axes[j])
        assert abs(d[b, j, k] - rd) <= (1e-12 if fp64 else 2e-6) * rd, (b, j, k, d[b, j, k], rd)
        u = xt / w.obs_axes[j]
        if fp64 or np.hypot(u[0], u[1]) > 1e-2:
            tol = 1e-10 if fp64 else 2e-4
            assert _wrapped(al[b, j, k], ra) <= tol, (b, j, k)
            assert _wrapped(be[b, j, k], rb) <= tol, (b, j, k)
    # kinematic blocks: rebuild e = bound d dir(alpha, beta) and compare with the oracle
    bs = sorted({e[0] for e in entries})
    for blk, (q, bound) in enumerate(((v, w.v_max), (a, w.a_max))):
        ka, kb, kd = kin[:, 3 * blk], kin[:, 3 * blk + 1], kin[:, 3 * blk + 2]
        for b in bs:
            e_g = bound * kd[b, :n_p, None] * _dir(ka[b, :n_p], kb[b, :n_p], D)
            e_o = np.array([oracle.polar_bound(q[b, k], bound) for k in range(n_p)])
            np.testing.assert_allclose(e_g, e_o, atol=1e-10 if fp64 else 1e-4 * bound)


def _run_case(w, precision, speed, per_axis):
    from paper_2408_10731_amd import trajam as tj
    if precision == "fp32":
        w = w.rounded(np.float32)   # the values the FP32 path receives
    rng = np.random.default_rng(5)
    xb = w.xi + rng.normal(size=w.xi.shape) * 0.4
    solver = tj.Solver.for_workload(w, precision=precision, sphere=False if per_axis else None)
    dt = solver.dtype
    if precision == "fp32":
        xb = xb.astype(np.float32).astype(np.float64)
    _, obs = tj.device_workload(w, dt, static=(speed == 0.0))
    xbd = torch.as_tensor(xb, dtype=dt, device="cuda").contiguous()
    al, be, d, kin = solver.polar(xbd, obs)
    torch.cuda.synchronize()
    B = w.xi.shape[0]
    kin = kin.double().cpu().numpy()
    assert kin.shape == (B, 6, w.n_steps)
    if w.n_obs == 0:
        assert al is None and be is None and d is None
        al = be = d = np.zeros((B, 0, w.n_steps))
    else:
        # beta not requested: alpha and d unchanged, bitwise
        al2, be2, d2, _ = solver.polar(xbd, None, beta=False)
        torch.cuda.synchronize()
        assert be2 is None and torch.equal(al, al2) and torch.equal(d, d2)
        al, be, d = (x.double().cpu().numpy() for x in (al, be, d))
        assert al.shape == (B, w.n_obs, w.n_steps)
    _check(w, xb, al, be, d, kin, precision)
    solver.close()


@pytest.mark.parametrize("dims,speed,per_axis,precision", [
    (2, 0.5, False, "fp64"),   # moving circles
    (3, 0.3, True, "fp64"),    # moving ellipsoids
    (2, 0.0, True, "fp64"),    # static ellipses
    (2, 0.5, False, "fp32"),
    (3, 0.3, True, "fp32"),
])
def test_polar_variables_match_the_oracle(dims, speed, per_axis, precision):
    w = wl.tiny(dims=dims, batch=5, n_obs=7, degree=7, n_steps=70, speed=speed, per_axis=per_axis,
                seed=31 + dims)
    print("case: polar", dims, speed, per_axis, precision, flush=True)
    _run_case(w, precision, speed, per_axis)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_polar_ragged_row_passes_and_long_horizon(precision):
    """150 steps and 19 moving ellipsoids (2,850 elements a sample: one workgroup's
    threads take about 11 each, crossing rows mid-wave), 3D, degree 9."""
    w = wl.tiny(dims=3, batch=4, n_obs=19, degree=9, n_steps=150, speed=0.3, per_axis=True, seed=41)
    print("case: polar ragged rows", precision, flush=True)
    _run_case(w, precision, 0.3, True)


@pytest.mark.parametrize("dims", [2, 3])
def test_polar_without_obstacles_writes_the_kinematic_blocks(dims):
    w = wl.tiny(dims=dims, batch=3, n_obs=0, degree=6, n_steps=40, seed=43)
    print("case: polar no obstacles", dims, flush=True)
    _run_case(w, "fp64", 0.0, False)


def test_polar_config2_sampled_and_packed_obstacle_reuse():
    """Config-2 sizes (1024 samples, 50 circles, 100 steps, FP32) on 300 sampled
    entries; a second call with the obstacles packed by the first (None) is bitwise
    identical."""
    from paper_2408_10731_amd import trajam as tj
    w = wl.config2().rounded(np.float32)
    print("case: polar config 2", flush=True)
    solver = tj.Solver.for_workload(w, precision="fp32")
    xi, obs = tj.device_workload(w, torch.float32)
    xb = xi + 0.3 * torch.randn(xi.shape, generator=torch.Generator(device="cuda").manual_seed(3),
                                device="cuda")
    out1 = solver.polar(xb, obs)
    out2 = solver.polar(xb, None)
    torch.cuda.synchronize()
    for x1, x2 in zip(out1, out2):
        assert torch.equal(x1, x2)
    al, be, d, kin = (x.double().cpu().numpy() for x in out1)
    rng = np.random.default_rng(8)
    entries = list(zip(rng.integers(0, w.batch, 300), rng.integers(0, w.n_obs, 300),
                       rng.integers(0, w.n_steps, 300)))
    _check(w, xb.double().cpu().numpy(), al, be, d, kin, "fp32", entries)
    solver.close()


@pytest.mark.parametrize("dims,other,precision", [(2, "zero", "fp64"), (3, "random", "fp64"),
                                                  (3, "zero", "fp32")])
def test_polar_sphere_model_ignores_other_semi_axes(dims, other, precision):
    """Sphere model: only obs_axes[j][0] (the radius) is read; the other entries may be
    zero or anything else and the polar variables are those of the sphere, the same as
    the projection uses.  Compared with the oracle on the true spheres, and bitwise
    with a call whose other entries equal the radius."""
    from paper_2408_10731_amd import trajam as tj
    w = wl.tiny(dims=dims, batch=4, n_obs=6, degree=7, n_steps=70, speed=0.4, seed=47 + dims)
    if precision == "fp32":
        w = w.rounded(np.float32)
    print("case: polar sphere model", dims, other, precision, flush=True)
    solver = tj.Solver.for_workload(w, precision=precision, sphere=True)
    dt = solver.dtype
    rng = np.random.default_rng(9)
    xb = w.xi + rng.normal(size=w.xi.shape) * 0.4
    if precision == "fp32":
        xb = xb.astype(np.float32).astype(np.float64)
    xbd = torch.as_tensor(xb, dtype=dt, device="cuda").contiguous()
    _, (c, v, a) = tj.device_workload(w, dt, static=False)
    a_odd = a.clone()
    a_odd[:, 1:] = 0.0 if other == "zero" else torch.as_tensor(
        rng.uniform(0.05, 3.0, size=(w.n_obs, dims - 1)), dtype=dt, device="cuda")
    ref = solver.polar(xbd, (c, v, a))
    ref = tuple(x.clone() for x in ref)
    got = solver.polar(xbd, (c, v, a_odd))
    torch.cuda.synchronize()
    for x1, x2 in zip(ref, got):
        assert torch.equal(x1, x2)
    al, be, d, kin = (x.double().cpu().numpy() for x in got)
    assert np.all(np.isfinite(al)) and np.all(np.isfinite(d))
    _check(w, xb, al, be, d, kin, precision)
    solver.close()


def test_polar_many_obstacles_unstaged_and_split_over_workgroups():
    """2,100 moving ellipsoids (their fields exceed the LDS stage, so they are read from
    the packed records) and 2 samples (each sample's 84,000 elements split over many
    workgroups), 3D, FP64: 500 sampled entries against the oracle."""
    w = wl.tiny(dims=3, batch=2, n_obs=2100, degree=6, n_steps=40, speed=0.3, per_axis=True, seed=53)
    print("case: polar 2100 obstacles", flush=True)
    from paper_2408_10731_amd import trajam as tj
    solver = tj.Solver.for_workload(w, precision="fp64", sphere=False)
    rng = np.random.default_rng(6)
    xb = w.xi + rng.normal(size=w.xi.shape) * 0.4
    _, obs = tj.device_workload(w, torch.float64, static=False)
    al, be, d, kin = (x.cpu().numpy() for x in solver.polar(torch.as_tensor(xb, device="cuda").contiguous(), obs))
    entries = list(zip(rng.integers(0, w.batch, 500), rng.integers(0, w.n_obs, 500),
                       rng.integers(0, w.n_steps, 500)))
    entries += [(1, w.n_obs - 1, w.n_steps - 1), (0, 0, 0), (1, 0, 0), (0, w.n_obs - 1, w.n_steps - 1)]
    _check(w, xb, al, be, d, kin, "fp64", entries)
    solver.close()
