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
                                          ([33, 65, 17], 129), ([44, 256, 256, 22], 8192),
                                          ([30, 17], 2000)])
@pytest.mark.parametrize("precision,tol", [(0, 1e-4), (1, 1e-3)])
def test_gpu_forward_and_gradients_match_oracle(widths, batch, precision, tol):
    """Forward output, loss and every parameter gradient against the FP64 oracle on
    the same float32 weights and inputs.  Batch 8192 splits each weight gradient over
    the batch (partial products added by a second kernel); the single-layer network
    runs without a workspace.  In bf16 mode the oracle rounds each
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
    L = torch.zeros(tj.MLP_MSE_LOSS_FLOATS, device="cuda")
    G = torch.zeros_like(P)
    scr = torch.zeros(2 * batch * max(widths[1:-1] + [1]), device="cuda")
    tj.trajam_mlp_forward(shape, batch, precision, P.data_ptr(), X.data_ptr(), acts_d.data_ptr(),
                          Y.data_ptr(), st)
    tj.trajam_mlp_mse(batch * widths[-1], Y.data_ptr(), T.data_ptr(), dY.data_ptr(), L.data_ptr(), st)
    tj.trajam_mlp_backward(shape, batch, precision, P.data_ptr(), X.data_ptr(), acts_d.data_ptr(),
                           dY.data_ptr(), G.data_ptr(), scr.data_ptr(), st)
    torch.cuda.synchronize()
    assert _rel(Y.cpu().numpy(), y_o) <= tol
    assert abs(L[0].item() - loss_o) <= tol * abs(loss_o)
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
    dY, L, G = torch.zeros_like(Y), torch.zeros(tj.MLP_MSE_LOSS_FLOATS, device="cuda"), torch.zeros_like(P)
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
@pytest.mark.parametrize("widths,batch", [([44, 256, 256, 22], 1024), ([44, 256, 256, 22], 1037),
                                          ([5, 7, 3], 1), ([33, 65, 17], 129),
                                          ([512, 300, 4, 9], 21)])
def test_gpu_fused_inference_matches_oracle(widths, batch):
    """trajam_mlp_infer (one launch, activations on chip, thin layers split over lane
    groups) against the FP64 oracle network: same fp32 products as the layer-by-layer
    forward, so the same tolerance (1e-4 relative to the output scale)."""
    from paper_2408_10731_amd import trajam as tj
    rng = np.random.default_rng(len(widths) * 1000 + batch)
    params = (rng.normal(size=omlp.n_params(widths)) * 0.3).astype(np.float32)
    x = rng.normal(size=(batch, widths[0])).astype(np.float32)
    print("case: mlp infer", widths, batch, flush=True)
    want, _ = omlp.forward(params.astype(np.float64), widths, x.astype(np.float64))
    pd = torch.as_tensor(params, device="cuda")
    xd = torch.as_tensor(x, device="cuda")
    y = torch.full((batch, widths[-1]), float("nan"), device="cuda")
    packed = torch.full_like(pd, float("nan"))
    st = torch.cuda.current_stream().cuda_stream
    tj.trajam_mlp_pack_infer(tj.mlp_shape(widths), pd.data_ptr(), packed.data_ptr(), st)
    tj.trajam_mlp_infer(tj.mlp_shape(widths), batch, packed.data_ptr(), xd.data_ptr(), y.data_ptr(),
                        st)
    torch.cuda.synchronize()
    got = y.double().cpu().numpy()
    err = np.abs(got - want).max() / max(1.0, np.abs(want).max())
    print(f"  max rel err {err:.2e}", flush=True)
    assert err <= 1e-4


@pytest.mark.gpu
def test_gpu_warm_features_apply_and_fallback():
    """Probe features [(xb - xi), lam] * s; the jump moves the free coefficients of xb,
    sets their multipliers to xb_out - xi and leaves the boundary coefficients and
    their multipliers; the fallback keeps the probe state of samples whose jump does
    not lower the residual, is NaN, or is not finite, and flags them."""
    from paper_2408_10731_amd import trajam as tj
    st = torch.cuda.current_stream().cuda_stream
    B, D, nv = 5, 2, 11
    dim = D * nv
    g = torch.Generator(device="cuda").manual_seed(3)
    xi = torch.randn((B, D, nv), device="cuda", generator=g)
    xb = torch.randn((B, D, nv), device="cuda", generator=g)
    lam = torch.randn((B, D, nv), device="cuda", generator=g)
    x = torch.empty((B, 2 * dim), device="cuda")
    tj.trajam_warm_features(B, D, nv, xi.data_ptr(), xb.data_ptr(), lam.data_ptr(), 0.5,
                            x.data_ptr(), st)
    torch.cuda.synchronize()
    assert torch.equal(x[:, :dim], ((xb - xi) * 0.5).reshape(B, dim))
    assert torch.equal(x[:, dim:], (lam * 0.5).reshape(B, dim))
    y = torch.randn((B, dim), device="cuda", generator=g)
    y[3, 4] = float("nan")
    xw = torch.empty_like(xb)
    lw = torch.empty_like(lam)
    tj.trajam_warm_apply(B, D, nv, y.data_ptr(), 2.0, xi.data_ptr(), xb.data_ptr(), lam.data_ptr(),
                         xw.data_ptr(), lw.data_ptr(), st)
    torch.cuda.synchronize()
    dx = (2.0 * y).reshape(B, D, nv)
    bnd = [0, 1, 2, nv - 1]
    free = list(range(3, nv - 1))
    assert torch.equal(xw[:, :, bnd], xb[:, :, bnd])
    assert torch.equal(lw[:, :, bnd], lam[:, :, bnd])
    ok = torch.ones(B, dtype=torch.bool)
    ok[3] = False
    torch.testing.assert_close(xw[ok][:, :, free], (xb + dx)[ok][:, :, free])
    # the fixed-point multiplier of every free coefficient (sample 3 holds a NaN)
    assert torch.equal(lw[ok][:, :, free], (xw - xi)[ok][:, :, free])
    rw = torch.tensor([0.1, 0.5, 0.2, 0.1, float("nan")], device="cuda")
    rc = torch.tensor([0.2, 0.4, 0.2, 0.3, 0.3], device="cuda")
    fl = torch.full((B,), 7, dtype=torch.int32, device="cuda")
    before_x, before_l = xw.clone(), lw.clone()
    tj.trajam_warm_fallback(B, D, nv, rw.data_ptr(), rc.data_ptr(), xb.data_ptr(), lam.data_ptr(),
                            xw.data_ptr(), lw.data_ptr(), fl.data_ptr(), st)
    torch.cuda.synchronize()
    # 0: lower residual -> jump kept; 1: higher; 2: equal -> kept (not above);
    # 3: non-finite state; 4: NaN residual
    assert fl.cpu().tolist() == [0, 4, 0, 4, 4]
    for b in (0, 2):
        assert torch.equal(xw[b], before_x[b]) and torch.equal(lw[b], before_l[b])
    for b in (1, 3, 4):
        assert torch.equal(xw[b], xb[b]) and torch.equal(lw[b], lam[b])


@pytest.mark.gpu
@pytest.mark.parametrize("widths,batch,D,nv", [([44, 256, 256, 22], 1024, 2, 11), ([44, 256, 256, 22], 37, 2, 11),
                                               ([96, 160, 48], 21, 3, 16), ([32, 40, 16], 5, 2, 8)])
def test_gpu_fused_warm_jump_matches_oracle(widths, batch, D, nv):
    """The matrix-core warm jump (features, bf16 network, jump in one launch) against the
    FP64 oracle of the same steps with both operands of every product rounded to bf16
    (oracle.mlp.forward(bf16=True), the decision of ReLU in the kernel's precision):
    the jumped free coefficients within 2e-3 relative to the largest step, boundary
    coefficients and their multipliers unchanged, free multipliers xb_out - xi."""
    from paper_2408_10731_amd import trajam as tj
    rng = np.random.default_rng(batch + nv)
    dim = D * nv
    params = (rng.normal(size=omlp.n_params(widths)) * 0.15).astype(np.float32)
    xi = rng.normal(size=(batch, D, nv)).astype(np.float32)
    xb = (xi + 0.3 * rng.normal(size=xi.shape)).astype(np.float32)
    lam = (0.2 * rng.normal(size=xi.shape)).astype(np.float32)
    in_s, out_s = 0.7, 1.3
    shape = tj.mlp_shape(widths)
    st = torch.cuda.current_stream().cuda_stream
    print("case: warm jump", widths, batch, flush=True)
    dp = torch.as_tensor(params, device="cuda")
    n = tj.trajam_warm_pack_mfma(shape, None, None, st)
    packed = torch.zeros(n, dtype=torch.uint8, device="cuda")
    tj.trajam_warm_pack_mfma(shape, dp.data_ptr(), packed.data_ptr(), st)
    dxi, dxb, dl = (torch.as_tensor(a, device="cuda") for a in (xi, xb, lam))
    xo, lo = torch.empty_like(dxb), torch.empty_like(dl)
    tj.trajam_warm_jump(shape, batch, D, nv, packed.data_ptr(), in_s, out_s, dxi.data_ptr(), dxb.data_ptr(),
                        dl.data_ptr(), xo.data_ptr(), lo.data_ptr(), st)
    torch.cuda.synchronize()
    x = np.concatenate([(xb - xi).reshape(batch, dim), lam.reshape(batch, dim)], 1).astype(np.float64) * in_s
    y, _ = omlp.forward(params.astype(np.float64), widths, x, bf16=True)
    want = xb.astype(np.float64) + out_s * y.reshape(batch, D, nv)
    got_x, got_l = xo.double().cpu().numpy(), lo.double().cpu().numpy()
    bnd = [0, 1, 2, nv - 1]
    free = list(range(3, nv - 1))
    assert np.array_equal(got_x[:, :, bnd], xb[:, :, bnd]) and np.array_equal(got_l[:, :, bnd], lam[:, :, bnd])
    scale = max(1.0, np.abs(out_s * y).max())
    err = np.abs(got_x[:, :, free] - want[:, :, free]).max() / scale
    assert err <= 2e-3, err
    np.testing.assert_allclose(got_l[:, :, free], got_x[:, :, free] - xi[:, :, free], atol=1e-6)


@pytest.mark.gpu
def test_gpu_trained_warm_start_gains_over_cold_start():
    """Trained on solver-generated pairs of the 2D 50-circle family (scene seeds
    10,000+, disjoint from the held-out ones), the probe-and-jump warm start against the
    cold start on a held-out set fixed in advance: the first 16 scene seeds from 90,001,
    none skipped.  Per scene, each arm's iterations to a batch-median residual <= 1e-3
    (probe included) and its wall time for exactly those iterations (probe, features,
    network, jump and check included) are measured; an arm that never reaches the
    tolerance within K = 200 iterations is charged K iterations and the time of K.
    The warm start must need fewer iterations and less wall time in total and fewer
    iterations on most scenes; every scene, including losses, is printed.  The
    oracle recomputes the warm arm's final residuals from the device result."""
    from paper_2408_10731_amd import trajam as tj, warmstart as ws
    fam = ws.family_scene("cfg2")
    data = ws.generate(fam, np.arange(10_000, 11_024), 64, k0=ws.K0, cap=150)
    print(f"case: warm-start gain, {data.x.shape[0]} training pairs", flush=True)
    w0 = fam(10_000, 4)
    net = ws.Net(ws.widths_for(w0), seed=0, precision=0, max_batch=1024)
    curve = ws.train(net, data, epochs=20, batch=512, lr=1e-3)
    print("  loss", [round(c, 5) for c in curve[::4]], flush=True)
    assert curve[-1] < 0.5 * curve[0]
    K = 200
    seeds = list(range(90_001, 90_017))
    it_c = it_w = 0
    t_c = t_w = 0.0
    wins = 0

    def timed(fn):
        fn()   # untimed pass (first-launch effects)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    for seed in seeds:
        w = fam(seed, 1024)
        solver = tj.Solver.for_workload(w, precision="fp32")
        xi, obs = tj.device_workload(w, torch.float32)
        trc = torch.zeros((K, w.batch), device="cuda")
        xb, lam = xi.clone(), torch.zeros_like(xi)
        solver.project(xi, w.boundary, obs, xb, lam, K, res_trace=trc)
        ctx = ws.WarmContext(solver, net, w.batch)
        xw, lw, fl, trp = ctx.run(xi, w.boundary, obs)
        trw = torch.zeros((K - ws.K0, w.batch), device="cuda")
        solver.project(xi, w.boundary, obs, xw, lw, K - ws.K0, res_trace=trw)
        torch.cuda.synchronize()
        ic = ws.iterations_to(trc.cpu().numpy())
        iw = ws.iterations_to(np.concatenate([trp.cpu().numpy(), trw.cpu().numpy()]))
        r_final = oracle.residuals(w.rounded(np.float32), xw.double().cpu().numpy())[0]
        ic = K if ic is None else ic
        iw = K if iw is None else iw
        fb = int((fl.cpu().numpy() & 4).astype(bool).sum())

        def cold():
            xb.copy_(xi)
            lam.zero_()
            solver.project(xi, w.boundary, obs, xb, lam, ic)

        def warm():
            x2, l2, _, _ = ctx.run(xi, w.boundary, obs)
            if iw > ws.K0:
                solver.project(xi, w.boundary, obs, x2, l2, iw - ws.K0)

        tc, tw = timed(cold), timed(warm)
        print(f"  scene {seed}: cold {ic} it {tc:.3f} ms, warm {iw} it {tw:.3f} ms, "
              f"fallbacks {fb}, oracle final median residual (warm) {np.median(r_final):.1e}"
              + ("" if iw < ic else "  <- warm not fewer"), flush=True)
        it_c += ic
        it_w += iw
        t_c += tc
        t_w += tw
        wins += iw < ic
        solver.close()
    print(f"  total over {len(seeds)} scenes: cold {it_c} it {t_c:.3f} ms, warm {it_w} it "
          f"{t_w:.3f} ms; warm fewer iterations on {wins}", flush=True)
    assert it_w < it_c and t_w < t_c and wins > len(seeds) // 2


def test_oracle_bf16_rounding_matches_torch():
    """Pins oracle.mlp.to_bf16 against torch's float32 -> bfloat16 conversion on the CPU
    (round to nearest even) over 2e6 random bit patterns -- every exponent, subnormals,
    negatives, infinities and NaNs -- plus exact ties of both parities, the largest
    finite float32 (rounds to infinity) and signed zeros."""
    import torch
    rng = np.random.default_rng(20240810)
    bits = rng.integers(0, 2 ** 32, size=2_000_000, dtype=np.uint64).astype(np.uint32)
    ties = (rng.integers(0, 2 ** 16, size=200_000, dtype=np.uint64).astype(np.uint32) << 16) | 0x8000
    special = np.array([0x00000000, 0x80000000, 0x7F800000, 0xFF800000, 0x7F7FFFFF, 0xFF7FFFFF,
                        0x00000001, 0x80008000, 0x00018000, 0x7FC00000, 0x7FFFFFFF, 0xFFFFFFFF,
                        0x3F808000, 0x3F818000, 0x3F807FFF, 0x3F808001], dtype=np.uint32)
    f = np.concatenate([bits, ties, special]).view(np.float32)
    want = torch.from_numpy(f.copy()).to(torch.bfloat16).to(torch.float32).numpy()
    got = omlp.to_bf16(f).astype(np.float32)
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan].view(np.uint32), want[~nan].view(np.uint32))
    assert ties.size == 200_000 and np.isinf(omlp.to_bf16(np.float32(3.4028235e38)))
