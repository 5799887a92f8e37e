"""Learned warm start: pins of the FP64 network oracle (CPU), GPU parity of the
forward pass, every parameter gradient, the loss and the Adam step, the warm-start
fallback, and what the trained network gains over the cold start."""
import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from paper_2408_10731_amd import workloads as wl

# ------------------------------------------------------------------ oracle pins


def _net(widths, seed=0):
    rng = np.random.default_rng(seed)
    return rng.normal(size=omlp.n_params(widths)) * 0.5


def test_backprop_matches_central_differences():
    widths = [5, 7, 6, 3]
    p = _net(widths, 1)
    rng = np.random.default_rng(2)
    x = rng.normal(size=(4, 5))
    t = rng.normal(size=(4, 3))

    def loss(q):
        y, _ = omlp.forward(q, widths, x)
        return omlp.mse(y, t)[0]

    y, acts = omlp.forward(p, widths, x)
    _, dy = omlp.mse(y, t)
    g = omlp.backward(p, widths, acts, dy)
    h = 1e-6
    fd = np.array([(loss(p + h * e) - loss(p - h * e)) / (2 * h) for e in np.eye(p.size)])
    np.testing.assert_allclose(g, fd, atol=1e-7, rtol=1e-6)


def test_single_layer_is_affine_and_relu_blocks_gradient():
    widths = [4, 2]
    p = _net(widths, 3)
    x = np.random.default_rng(4).normal(size=(6, 4))
    y, _ = omlp.forward(p, widths, x)
    W = p[:8].reshape(2, 4)
    np.testing.assert_allclose(y, x @ W.T + p[8:], atol=1e-14)
    # all hidden pre-activations negative: nothing flows to the first layer
    widths = [3, 4, 2]
    p = np.zeros(omlp.n_params(widths))
    p[12:16] = -1.0                    # hidden bias -1, zero hidden weights -> z = -1 < 0
    p[16:24] = 1.0
    y, acts = omlp.forward(p, widths, np.ones((2, 3)))
    g = omlp.backward(p, widths, acts, np.ones((2, 2)))
    assert np.all(g[:16] == 0.0)


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([0.3, -2.0, 1e-3, -4e-2])
    p1, m, v = omlp.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=1e-12)
    np.testing.assert_allclose(p1, -0.01 * np.sign(g), rtol=1e-9)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


# -------------------------------------------------------------------- GPU parity

torch = pytest.importorskip("torch")


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


@pytest.mark.gpu
@pytest.mark.parametrize("widths,batch", [([526, 256, 256, 22], 300), ([5, 7, 3], 1),
                                          ([33, 65, 17], 129)])
@pytest.mark.parametrize("precision,tol", [(0, 1e-4), (1, 1e-3)])
def test_gpu_forward_and_gradients_match_oracle(widths, batch, precision, tol):
    """Forward output, loss and every parameter gradient against the FP64 oracle on
    the same float32 weights and inputs.  In bf16 mode the oracle rounds each
    product's operands to bf16 like the kernel (so the ReLU decisions agree) and the
    only difference left is fp32 accumulation; the error of the bf16 mode against
    the unrounded FP64 network is checked separately below (<= 2e-2)."""
    from paper_2408_10731_amd import trajam as tj
    from paper_2408_10731_amd.warmstart import init_params
    print("case: mlp", widths, batch, precision, flush=True)
    rng = np.random.default_rng(7)
    p32 = init_params(widths, 3)
    x = rng.normal(size=(batch, widths[0])).astype(np.float32)
    t = rng.normal(size=(batch, widths[-1])).astype(np.float32)
    bf = precision == 1
    # keep only samples with no hidden pre-activation within fp32 rounding of zero:
    # a ReLU decision there is not fixed by the mathematics at this precision
    _, acts = omlp.forward(p32.astype(np.float64), widths, x.astype(np.float64), bf16=bf)
    layers = omlp.unpack(p32.astype(np.float64), widths)
    keep = np.ones(batch, dtype=bool)
    for l in range(1, len(widths) - 1):
        W, b = layers[l - 1]
        z = omlp._mm(acts[l - 1], W.T, bf) + b
        keep &= ~np.any(np.abs(z) < 1e-5 * (1 + np.abs(z).max()), axis=1)
    assert keep.mean() >= 0.75
    x, t = np.ascontiguousarray(x[keep]), np.ascontiguousarray(t[keep])
    batch = int(keep.sum())
    y_o, acts = omlp.forward(p32.astype(np.float64), widths, x.astype(np.float64), bf16=bf)
    loss_o, dy_o = omlp.mse(y_o, t.astype(np.float64))
    g_o = omlp.backward(p32.astype(np.float64), widths, acts, dy_o, bf16=bf)

    shape = tj.mlp_shape(widths)
    st = torch.cuda.current_stream().cuda_stream
    P = torch.as_tensor(p32, device="cuda")
    X = torch.as_tensor(x, device="cuda")
    T = torch.as_tensor(t, device="cuda")
    hid = sum(widths[1:-1])
    acts_d = torch.zeros(max(hid, 1) * batch, device="cuda")
    Y = torch.zeros((batch, widths[-1]), device="cuda")
    dY = torch.zeros_like(Y)
    L = torch.zeros(1, device="cuda")
    G = torch.zeros_like(P)
    scr = torch.zeros(2 * batch * max(widths[1:-1] + [1]), device="cuda")
    tj.trajam_mlp_forward(shape, batch, precision, P.data_ptr(), X.data_ptr(), acts_d.data_ptr(),
                          Y.data_ptr(), st)
    tj.trajam_mlp_mse(batch * widths[-1], Y.data_ptr(), T.data_ptr(), dY.data_ptr(), L.data_ptr(), st)
    tj.trajam_mlp_backward(shape, batch, precision, P.data_ptr(), X.data_ptr(), acts_d.data_ptr(),
                           dY.data_ptr(), G.data_ptr(), scr.data_ptr(), st)
    torch.cuda.synchronize()
    assert _rel(Y.cpu().numpy(), y_o) <= tol
    assert abs(L.item() - loss_o) <= tol * abs(loss_o)
    g = G.cpu().numpy()
    off = 0
    for l in range(len(widths) - 1):
        n = widths[l + 1] * widths[l]
        for sl in (slice(off, off + n), slice(off + n, off + n + widths[l + 1])):
            assert _rel(g[sl], g_o[sl]) <= tol, (l, sl)
        off += n + widths[l + 1]


@pytest.mark.gpu
def test_gpu_bf16_mode_error_against_fp64_network():
    """The bf16 mode against the unrounded FP64 network: forward and gradients within
    2e-2 (norm-wise relative)."""
    from paper_2408_10731_amd import trajam as tj
    from paper_2408_10731_amd.warmstart import init_params
    widths, batch = [526, 256, 256, 22], 512
    rng = np.random.default_rng(11)
    p32 = init_params(widths, 5)
    x = rng.normal(size=(batch, widths[0])).astype(np.float32)
    t = rng.normal(size=(batch, widths[-1])).astype(np.float32)
    y_o, acts = omlp.forward(p32.astype(np.float64), widths, x.astype(np.float64))
    _, dy_o = omlp.mse(y_o, t.astype(np.float64))
    g_o = omlp.backward(p32.astype(np.float64), widths, acts, dy_o)
    shape = tj.mlp_shape(widths)
    st = torch.cuda.current_stream().cuda_stream
    P, X, T = (torch.as_tensor(a, device="cuda") for a in (p32, x, t))
    acts_d = torch.zeros(512 * batch, device="cuda")
    Y = torch.zeros((batch, 22), device="cuda")
    dY, L, G = torch.zeros_like(Y), torch.zeros(1, device="cuda"), torch.zeros_like(P)
    scr = torch.zeros(2 * batch * 256, device="cuda")
    tj.trajam_mlp_forward(shape, batch, 1, P.data_ptr(), X.data_ptr(), acts_d.data_ptr(), Y.data_ptr(), st)
    tj.trajam_mlp_mse(batch * 22, Y.data_ptr(), T.data_ptr(), dY.data_ptr(), L.data_ptr(), st)
    tj.trajam_mlp_backward(shape, batch, 1, P.data_ptr(), X.data_ptr(), acts_d.data_ptr(),
                           dY.data_ptr(), G.data_ptr(), scr.data_ptr(), st)
    torch.cuda.synchronize()
    ey, eg = _rel(Y.cpu().numpy(), y_o), _rel(G.cpu().numpy(), g_o)
    print(f"  bf16 vs FP64 network: forward {ey:.2e}, gradient {eg:.2e}", flush=True)
    assert ey <= 2e-2 and eg <= 2e-2


@pytest.mark.gpu
def test_gpu_adam_matches_oracle():
    from paper_2408_10731_amd import trajam as tj
    rng = np.random.default_rng(8)
    n = 1000
    p, g, m, v = (rng.normal(size=n).astype(np.float32) for _ in range(4))
    v = np.abs(v)
    P, G, M, V = (torch.as_tensor(a, device="cuda") for a in (p, g, m, v))
    for step in (1, 7):
        tj.trajam_mlp_adam(n, P.data_ptr(), G.data_ptr(), M.data_ptr(), V.data_ptr(), step, 1e-3,
                           0.9, 0.999, 1e-8, torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        p, m, v = omlp.adam(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                            v.astype(np.float64), step)
        np.testing.assert_allclose(P.cpu().numpy(), p, rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(M.cpu().numpy(), m, rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(V.cpu().numpy(), v, rtol=1e-5, atol=1e-7)
        p, m, v = p.astype(np.float32), m.astype(np.float32), v.astype(np.float32)


@pytest.mark.gpu
def test_gpu_warm_apply_nan_and_fallback():
    from paper_2408_10731_amd import trajam as tj
    st = torch.cuda.current_stream().cuda_stream
    B, D, nv = 5, 2, 11
    xi = torch.randn((B, D, nv), device="cuda")
    y = torch.randn((B, D * nv), device="cuda")
    y[2, 5] = float("nan")
    xb0 = torch.empty_like(xi)
    lam0 = torch.empty_like(xi)
    fl = torch.zeros(B, dtype=torch.int32, device="cuda")
    tj.trajam_warm_apply(B, D, nv, y.data_ptr(), xi.data_ptr(), 0.5, None, xb0.data_ptr(),
                         lam0.data_ptr(), fl.data_ptr(), st)
    torch.cuda.synchronize()
    d = (y * 0.5).reshape(B, D, nv)
    assert fl.cpu().tolist() == [0, 0, 4, 0, 0]
    assert torch.equal(xb0[2], xi[2]) and torch.all(lam0[2] == 0)
    for b in (0, 1, 3, 4):
        torch.testing.assert_close(xb0[b], xi[b] + d[b])
        assert torch.all(lam0[b][:, [0, 1, 2, nv - 1]] == 0)
        torch.testing.assert_close(lam0[b][:, 3:nv - 1], d[b][:, 3:nv - 1])
    # with boundary coefficients: those are written exactly, the free ones as before
    bc = np.array([[1.0, 1.25, 1.5, 7.0], [-2.0, -2.0, -2.0, 3.5]])
    xb1 = torch.empty_like(xi)
    lam1 = torch.empty_like(xi)
    fl1 = torch.zeros(B, dtype=torch.int32, device="cuda")
    tj.trajam_warm_apply(B, D, nv, y.data_ptr(), xi.data_ptr(), 0.5, bc, xb1.data_ptr(),
                         lam1.data_ptr(), fl1.data_ptr(), st)
    torch.cuda.synchronize()
    assert torch.equal(xb1[2], xi[2]) and fl1.cpu().tolist() == [0, 0, 4, 0, 0]
    for b in (0, 1, 3, 4):
        got = xb1[b].cpu().numpy()
        np.testing.assert_array_equal(got[:, [0, 1, 2, nv - 1]], bc.astype(np.float32))
        torch.testing.assert_close(xb1[b][:, 3:nv - 1], xi[b][:, 3:nv - 1] + d[b][:, 3:nv - 1])
        assert torch.equal(lam1[b], lam0[b])
    rw = torch.tensor([0.1, 0.5, 0.0, float("nan"), 0.2], device="cuda")
    rc = torch.tensor([0.2, 0.4, 0.0, 0.3, 0.2], device="cuda")
    before = xb0.clone()
    tj.trajam_warm_fallback(B, D, nv, rw.data_ptr(), rc.data_ptr(), xi.data_ptr(), xb0.data_ptr(),
                            lam0.data_ptr(), fl.data_ptr(), st)
    torch.cuda.synchronize()
    assert fl.cpu().tolist() == [0, 4, 4, 4, 0]
    assert torch.equal(xb0[0], before[0]) and torch.equal(xb0[4], before[4])
    for b in (1, 3):
        assert torch.equal(xb0[b], xi[b]) and torch.all(lam0[b] == 0)


def _iters_to(trace, tol=1e-3):
    med = np.median(trace, axis=1)
    hit = np.nonzero(med <= tol)[0]
    return int(hit[0]) + 1 if hit.size else None


@pytest.mark.gpu
def test_gpu_trained_warm_start_gains_over_cold_start():
    """Trained on solver-generated scenes of the 2D 50-circle family (seeds disjoint
    from the held-out ones), the warm start reaches the batch-median residual 1e-3
    in fewer AM iterations than the cold start on held-out scenes; the final
    residual is judged by the oracle."""
    from paper_2408_10731_amd import trajam as tj, warmstart as ws
    fam = ws.family_scene("cfg2")
    k_obs = 50
    train_seeds = np.arange(10_000, 10_512)
    data = ws.generate(fam, train_seeds, 256, k_obs, iters=300)
    print(f"case: warm-start gain, {data.x.shape[0]} training pairs", flush=True)
    w0 = fam(int(train_seeds[0]), 4)
    net = ws.Net(ws.widths_for(w0, k_obs), seed=0, precision=0, max_batch=1024)
    curve = ws.train(net, data, epochs=30, batch=512, lr=1e-3)
    print("  loss", [round(c, 5) for c in curve[::5]], flush=True)
    assert curve[-1] < curve[0]
    gains = []
    for seed in (90_001, 90_002):
        w = fam(seed, 1024)
        solver = tj.Solver.for_workload(w, precision="fp32")
        xi, obs = tj.device_workload(w, torch.float32)
        K = 200
        trc = torch.zeros((K, w.batch), device="cuda")
        xb, lam = xi.clone(), torch.zeros_like(xi)
        solver.project(xi, w.boundary, obs, xb, lam, K, res_trace=trc)
        xb0, lam0, fl = ws.warm_start(solver, net, w, xi, obs, k_obs)
        trw = torch.zeros_like(trc)
        solver.project(xi, w.boundary, obs, xb0, lam0, K, res_trace=trw)
        torch.cuda.synchronize()
        ic, iw = _iters_to(trc.cpu().numpy()), _iters_to(trw.cpu().numpy())
        fb = int((fl.cpu().numpy() & 4).astype(bool).sum())
        print(f"  scene {seed}: cold {ic} iterations, warm {iw}, fallbacks {fb}", flush=True)
        gains.append((ic, iw))
        r_final = oracle.residuals(w.rounded(np.float32), xb0.double().cpu().numpy())[0]
        assert np.median(r_final) <= 1e-3
    assert all(iw is not None and (ic is None or iw < ic) for ic, iw in gains)
