"""Learned velocity surrogate on the GPU: MFMA GEMM and training kernels
against the FP64 reference (oracle/mlp.py), features against the oracle's
power spectrum, and two closed-form pins of learned mode (a network that is
never confident reduces to the unsmoothed search; a confident constant
network reduces to the fixed-velocity filter)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import mlp  # noqa: E402
from paper_1408_3526_amd import scenes  # noqa: E402


def _b():
    from paper_1408_3526_amd import binding
    binding.lib()
    return binding


def _bf(a):
    return torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).cuda()


@pytest.mark.parametrize("M,N,K", [(100, 70, 48), (64, 64, 32), (4096, 128, 1152), (37, 130, 200),
                                   (65600, 128, 256), (66001, 192, 64)])
@pytest.mark.parametrize("epi", [0, 1, 2])
def test_gemm_nt_matches_reference(M, N, K, epi):
    b = _b()
    rng = np.random.default_rng(M * 7 + N + K + epi)
    A = mlp.bf16_round(rng.normal(size=(M, K)))
    B = mlp.bf16_round(rng.normal(size=(N, K)))
    bias = rng.normal(size=N).astype(np.float32)
    aux = mlp.bf16_round(rng.normal(size=(M, N)))
    C = torch.empty(M, N, device="cuda")
    Cb = torch.empty(M, N, dtype=torch.bfloat16, device="cuda")
    b.mlp_gemm_nt(_bf(A), _bf(B), bias=torch.from_numpy(bias).cuda(), epi=epi, aux=_bf(aux), out_f32=C, out_bf16=Cb)
    torch.cuda.synchronize()
    ref = A @ B.T + bias
    if epi == 1:
        ref = np.maximum(ref, 0)
    elif epi == 2:
        ref = np.where(aux > 0, ref, 0)
    got = C.cpu().numpy().astype(np.float64)
    scale = np.abs(A).max() * np.abs(B).max() * K
    assert np.abs(got - ref).max() <= 1e-6 * scale
    assert np.array_equal(Cb.cpu().float().numpy(), mlp.bf16_round(got.astype(np.float32)).astype(np.float32))


def test_transpose():
    b = _b()
    x = torch.randn(77, 130, device="cuda").to(torch.bfloat16)
    out = torch.empty(130, 77, dtype=torch.bfloat16, device="cuda")
    b.mlp_transpose(x, out)
    torch.cuda.synchronize()
    assert torch.equal(out, x.t().contiguous())


def _trainer_with(params, n):
    """A Trainer whose FP32 master weights (and their BF16 copies) are params."""
    from paper_1408_3526_amd import learned
    b = _b()
    tr = learned.Trainer(seed=1, batch=n)
    for k, a in zip(("W1", "b1", "W2", "b2", "W3", "b3"), params):
        tr.p[k].copy_(torch.from_numpy(np.asarray(a, np.float32)))
    b.mlp_to_bf16(tr.p["W1"], tr.bf["W1"])
    b.mlp_to_bf16(tr.p["W2"], tr.bf["W2"])
    return tr


@pytest.mark.parametrize("n,seed", [(512, 3), (1000, 4)])
def test_training_gradients_within_elementwise_bounds(n, seed):
    """Every element of dW1, db1, dW2, db2, dW3, db3 and the loss of one
    training batch lies inside the interval oracle/mlp.grads_iv derives around
    the FP64 reference: FP32 accumulation error in any order, and one BF16 ulp
    (or either ReLU mask) wherever the rounding of H1, H2, dH2 or dH1 can go
    either way.  Labels sit near the network's output so that both
    confidence targets occur, each clear of the threshold.""" 
    from mlp_cases import random_params
    rng = np.random.default_rng(seed)
    X = mlp.bf16_round(rng.normal(size=(n, mlp.N_IN)))
    params = random_params(rng)
    O = mlp.forward(X, params)[-1]
    # half the samples within 0.2 of the output in both components (target
    # 1), the others 0.3-0.6 away in one (target 0): both targets, each at
    # least 0.05 from the 0.25 threshold
    near = rng.uniform(-0.2, 0.2, size=(n, 2))
    far = near.copy()
    far[np.arange(n), rng.integers(0, 2, n)] = rng.choice([-1, 1], n) * rng.uniform(0.3, 0.6, n)
    lab = np.float32(O[:, :2] + np.where(rng.uniform(size=(n, 1)) < 0.5, near, far))
    tr = _trainer_with(params, n)
    loss = tr.grads(_bf(X), torch.from_numpy(lab).cuda())
    torch.cuda.synchronize()
    (lm, lr), g = mlp.grads_iv(X, lab, params, wv=tr.wv, half_step=tr.half_step)
    assert mlp.within(float(loss.item()), lm, lr), (float(loss.item()), lm, lr)
    for k, (mid, rad) in g.items():
        got = tr.g[k].cpu().numpy().astype(np.float64)
        ok = mlp.within(got, mid, rad)
        excess = (np.abs(got - mid) - rad)[~ok]
        assert ok.all(), (k, int((~ok).sum()), float(excess.max()) if excess.size else 0.0)
        print("%s: %d elements, median bound %.2e x max|G|, %.1f%% of bounds above 1e-3 x max|G|"
              % (k, got.size, np.median(rad) / np.abs(mid).max(), 100 * np.mean(rad > 1e-3 * np.abs(mid).max())))


def test_training_gradients_exact_on_integer_data():
    """Integer inputs and weights whose every FP32 sum is exactly
    representable (checked): the GPU's loss gradients equal the FP64
    reference bit for bit, element by element."""
    from mlp_cases import exactness_premise, integer_case
    X, lab, params = integer_case()
    n = X.shape[0]
    assert exactness_premise(X, lab, params, n) < 1.0
    tr = _trainer_with(params, n)
    tr.grads(_bf(X), torch.from_numpy(np.asarray(lab, np.float32)).cuda())
    torch.cuda.synchronize()
    _, rg = mlp.loss_and_grads(X, lab, params, wv=tr.wv, half_step=tr.half_step, bf16=True)
    for k, G in zip(("W1", "b1", "W2", "b2", "W3", "b3"), rg):
        got = tr.g[k].cpu().numpy().astype(np.float64)
        assert np.array_equal(got, G), (k, int(np.sum(got != G)))


def test_adam_step():
    b = _b()
    rng = np.random.default_rng(4)
    p = rng.normal(size=1000).astype(np.float32)
    g = rng.normal(size=1000).astype(np.float32)
    m = rng.normal(size=1000).astype(np.float32) * 0.1
    v = np.abs(rng.normal(size=1000)).astype(np.float32) * 0.1
    tp, tg, tm, tv = (torch.from_numpy(a.copy()).cuda() for a in (p, g, m, v))
    pb = torch.empty(1000, dtype=torch.bfloat16, device="cuda")
    b.mlp_adam(tp, tg, tm, tv, pb, lr=1e-2, step=3)
    torch.cuda.synchronize()
    m2 = 0.9 * m + 0.1 * g
    v2 = 0.999 * v + 0.001 * g * g
    ref = p - 1e-2 * (m2 / (1 - 0.9 ** 3)) / (np.sqrt(v2 / (1 - 0.999 ** 3)) + 1e-8)
    assert np.abs(tp.cpu().numpy() - ref).max() <= 1e-5
    assert torch.equal(pb, tp.to(torch.bfloat16))


def _check_features(orc, cfg, frames, pts, F, S_gpu):
    """Element-wise: the GPU's local spectrum at each anchor within
    TAU_S * max|S| of the oracle's (direct window DFT), and every one of its
    1152 BF16 features inside mlp.features_iv's bound around the oracle's.
    Returns the oracle's features and bounds."""
    xs, rads = [], []
    for i, (x, y) in enumerate(pts):
        S = orc.pixel_series(cfg, frames, x, y)["S"][-1]
        scale = np.abs(S).max()
        assert np.abs(S_gpu[i] - S).max() <= mlp.TAU_S * scale, (x, y, np.abs(S_gpu[i] - S).max() / scale)
        _, P = orc.flow_R(cfg, S, want_P=True)
        xr, rad = mlp.features_iv(P, scale)
        err = np.abs(F[i].astype(np.float64) - xr)
        assert np.all(err <= rad), (x, y, int(np.sum(err > rad)), float(np.max(err / rad)))
        xs.append(xr)
        rads.append(rad)
    return np.array(xs), np.array(rads)


def test_features_match_oracle(orc):
    """Search mode with feature output: at sampled anchors (corners, borders,
    interior) every feature is within its derived bound of the oracle's
    log power spectrum, and the spectrum itself within TAU_S of the largest
    bin."""
    b = _b()
    sc = scenes.flow_scene(5, H=36, W=40, T=10, n_targets=2, band_width=(6, 9))
    g = scenes.grid(-4, 4, 0.5)
    f = b.Filter(36, 40, 16, 16, 8, g, g, write_features=True)
    dev = torch.from_numpy(sc.frames).cuda()
    for t in range(10):
        f.push_frame(dev[t])
    pts = [(39, 35), (20, 20), (15, 30), (0, 0), (5, 33), (39, 0), (0, 35)]
    F = f.features().float().cpu().numpy()
    F = np.array([F[y, x] for (x, y) in pts])
    S_gpu = f.spectrum([p[0] for p in pts], [p[1] for p in pts]).cpu().numpy()
    torch.cuda.synchronize()
    f.close()
    del dev
    torch.cuda.empty_cache()
    cfg = orc.Cfg(H=36, W=40, Mx=16, My=16, Mz=8, gx=g, gy=g)
    _check_features(orc, cfg, sc.frames, pts, F, S_gpu)


def test_inference_kernels_within_bounds():
    """The network's inference kernels on realistic inputs, called directly
    (two MFMA GEMM layers and the head) and through a learned-mode context
    (rmdf_learned_network, the launch sequence a push uses): every output
    (vx, vy, confidence) lies inside the interval oracle/mlp.forward_iv
    derives around the FP64 forward pass of the shipped network."""
    import os

    from paper_1408_3526_amd import learned
    if not os.path.exists(learned.DEFAULT_WEIGHTS):
        pytest.skip("no trained weights shipped")
    b = _b()
    w = np.load(learned.DEFAULT_WEIGHTS)
    params = mlp.unpack(w)
    rng = np.random.default_rng(21)
    n = 3000
    # log-spectrum-like inputs: a smooth decay over the bins plus noise
    X = mlp.bf16_round(rng.normal(size=(n, mlp.N_IN)) * 1.5 - np.linspace(0, 6, mlp.N_IN)[None, :] + 3.0)
    W1b = _bf(params[0])
    W2b = _bf(params[2])
    h1 = torch.empty(n, mlp.N_H1, dtype=torch.bfloat16, device="cuda")
    h2 = torch.empty(n, mlp.N_H2, dtype=torch.bfloat16, device="cuda")
    vc = torch.empty(n, 3, device="cuda")
    f32 = lambda a: torch.from_numpy(np.asarray(a, np.float32)).cuda()  # noqa: E731
    b.mlp_gemm_nt(_bf(X), W1b, bias=f32(params[1]), epi=1, out_bf16=h1)
    b.mlp_gemm_nt(h1, W2b, bias=f32(params[3]), epi=1, out_bf16=h2)
    b.mlp_infer_head(h2, f32(params[4]), f32(params[5]), vc)
    got = vc.cpu().numpy().astype(np.float64)
    # the same network through the context (rmdf_learned_network: the
    # kernels and launch sequence of a learned-mode push), on the same inputs
    g = scenes.grid(-4, 4, 0.5)
    f = b.Filter(20, 20, 16, 16, 8, g, g, velocity_mode=b.VEL_LEARNED)
    f.set_weights(w)
    fused = f.learned_network(_bf(X)).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    f.close()
    fw = mlp.forward_iv(X, 0, params)
    Om, Or = fw["O"]
    clo, chi = mlp.sigmoid_iv(Om[:, 2], Or[:, 2])
    for name, out in (("GEMM kernels", got), ("learned-mode network", fused)):
        assert mlp.within(out[:, :2], Om[:, :2], Or[:, :2]).all(), name
        assert np.all((out[:, 2] >= clo) & (out[:, 2] <= chi)), name
    print("output bound: median %.2e, max %.2e (px/frame)" % (np.median(Or[:, :2]), Or[:, :2].max()))
    # one kernel against the three: the same bits
    assert np.array_equal(got, fused)


def _network_blob(kind, rng):
    from paper_1408_3526_amd import learned
    if kind == "shipped":
        import os
        if not os.path.exists(learned.DEFAULT_WEIGHTS):
            pytest.skip("no trained weights shipped")
        return np.load(learned.DEFAULT_WEIGHTS).astype(np.float32)
    parts = [rng.normal(size=(mlp.N_H1, mlp.N_IN)) / np.sqrt(mlp.N_IN), rng.normal(size=mlp.N_H1) * 0.1,
             rng.normal(size=(mlp.N_H2, mlp.N_H1)) / np.sqrt(mlp.N_H1), rng.normal(size=mlp.N_H2) * 0.1,
             rng.normal(size=(3, mlp.N_H2)) / np.sqrt(mlp.N_H2), rng.normal(size=3) * 0.1]
    return np.concatenate([np.ravel(p) for p in parts]).astype(np.float32)


@pytest.mark.parametrize("n", [1, 127, 128, 129, 3000, 41000])
@pytest.mark.parametrize("kind", ["shipped", "random"])
def test_network_kernel_equals_layer_kernels(n, kind):
    """The learned-mode network (rmdf_learned_network: one kernel, the
    features streamed through LDS by direct loads and the hidden layers kept
    on chip) gives bit for bit what the two GEMM layers with BF16 outputs and
    the head give when launched one after the other: the same rounding
    points and the same accumulation order.  Row counts around the 128-row
    workgroup tile, and a ragged many-tile case longer than the context's
    frame."""
    b = _b()
    rng = np.random.default_rng(1000 + n)
    w = _network_blob(kind, rng)
    params = mlp.unpack(w)
    X = mlp.bf16_round(rng.normal(size=(n, mlp.N_IN)) * 1.5 - np.linspace(0, 6, mlp.N_IN)[None, :] + 3.0)
    Xd = _bf(X)
    f32 = lambda a: torch.from_numpy(np.asarray(a, np.float32)).cuda()  # noqa: E731
    h1 = torch.empty(n, mlp.N_H1, dtype=torch.bfloat16, device="cuda")
    h2 = torch.empty(n, mlp.N_H2, dtype=torch.bfloat16, device="cuda")
    vc = torch.empty(n, 3, device="cuda")
    b.mlp_gemm_nt(Xd, _bf(params[0]), bias=f32(params[1]), epi=1, out_bf16=h1)
    b.mlp_gemm_nt(h1, _bf(params[2]), bias=f32(params[3]), epi=1, out_bf16=h2)
    b.mlp_infer_head(h2, f32(params[4]), f32(params[5]), vc)
    g = scenes.grid(-4, 4, 0.5)
    f = b.Filter(20, 20, 16, 16, 8, g, g, velocity_mode=b.VEL_LEARNED)
    try:
        f.set_weights(w)
        one = f.learned_network(Xd)
        torch.cuda.synchronize()
    finally:
        f.close()
    got, ref = one.cpu().numpy(), vc.cpu().numpy()
    assert np.array_equal(got.view(np.int32), ref.view(np.int32)), \
        "%d of %d rows differ" % (int(np.any(got != ref, axis=1).sum()), n)
    # the case is not degenerate: both ReLU sides and a spread of outputs occur
    assert 0.01 < float((h1.float() > 0).float().mean()) < 0.99
    if n > 1:
        assert np.ptp(ref[:, 0]) > 0 and np.ptp(ref[:, 2]) > 0


def _blob(b3):
    w = np.zeros(mlp.N_H1 * mlp.N_IN + mlp.N_H1 + mlp.N_H2 * mlp.N_H1 + mlp.N_H2 + 3 * mlp.N_H2 + 3, np.float32)
    w[-3:] = b3
    return w


def test_learned_never_confident_is_unsmoothed_search(orc):
    b = _b()
    sc = scenes.flow_scene(6, H=34, W=37, T=11, n_targets=2, band_width=(6, 9))
    g = scenes.grid(-4, 4, 0.5)
    f = b.Filter(34, 37, 16, 16, 8, g, g, velocity_mode=b.VEL_LEARNED, conf_threshold=0.9)
    f.set_weights(_blob([0.0, 0.0, -20.0]))
    dev = torch.from_numpy(sc.frames).cuda()
    for t in range(11):
        f.push_frame(dev[t])
    out = f.output().cpu().numpy()
    _, idx = f.velocity()
    idx = idx.cpu().numpy()
    vc = f.learned_output().cpu().numpy()
    torch.cuda.synchronize()
    f.close()
    assert np.all(vc[..., 2] < 1e-6) and np.all(idx >= 0)
    r = orc.run(orc.Cfg(H=34, W=37, Mx=16, My=16, Mz=8, gx=g, gy=g, alpha=0.0), sc.frames, want_rs=True)
    rs = r["rs_all"][-1]
    srt = np.sort(rs, -1)
    scale = np.maximum(np.maximum(np.abs(rs).max(-1), 1e-3 * r["en_all"][-1]), 1e-30)
    tied = srt[..., -1] - srt[..., -2] <= 1e-4 * scale
    agree = idx == r["idx"][-1]
    assert agree[~tied].mean() >= 0.999
    rms = float(np.sqrt(np.mean(sc.frames[-1].astype(np.float64) ** 2)))
    assert np.abs(out - r["out"][-1])[agree].max() <= 1e-3 * rms


def test_learned_confident_constant_is_fixed_velocity(orc):
    b = _b()
    sc = scenes.flow_scene(7, H=34, W=37, T=11, n_targets=2, band_width=(6, 9))
    g = scenes.grid(-4, 4, 0.5)
    v = (1.3, -0.7)
    f = b.Filter(34, 37, 16, 16, 8, g, g, velocity_mode=b.VEL_LEARNED, conf_threshold=0.9)
    f.set_weights(_blob([v[0], v[1], 20.0]))
    dev = torch.from_numpy(sc.frames).cuda()
    outs = []
    for t in range(11):
        f.push_frame(dev[t])
        outs.append(f.output().cpu().numpy())
    vxy, idx = f.velocity()
    vxy, idx = vxy.cpu().numpy(), idx.cpu().numpy()
    torch.cuda.synchronize()
    f.close()
    assert np.all(idx == -2)
    assert np.allclose(vxy[..., 0], v[0]) and np.allclose(vxy[..., 1], v[1])
    r = orc.run(orc.Cfg(H=34, W=37, Mx=16, My=16, Mz=8, gx=g, gy=g, vmode=2, fvx=v[0], fvy=v[1]), sc.frames)
    for t in range(11):
        rms = float(np.sqrt(np.mean(sc.frames[t].astype(np.float64) ** 2)))
        assert np.abs(outs[t] - r["out"][t]).max() <= 1e-3 * rms, t


def test_short_training_reduces_loss():
    from paper_1408_3526_amd import learned
    X, lab, true = learned.harvest([11, 12], H=64, W=80, T=14, per_seq=2500)
    assert X.shape == (5000, 1152) and lab.shape == (5000, 2)
    tr, losses = learned.train(X, lab, steps=300, batch=1024)
    assert losses[-1][1] < 0.7 * losses[0][1], losses


def test_trained_network_against_search():
    """The shipped network (trained by paper_1408_3526_amd.learned on seeds
    1000-1049) on a held-out seed: the learned mode's PEF residual is within
    5% of the plain search's (its acceptance bar), it is confident on part of
    the frame, and the gain is printed (residual, velocity RMSE)."""
    import os

    from paper_1408_3526_amd import learned
    if not os.path.exists(learned.DEFAULT_WEIGHTS):
        pytest.skip("no trained weights shipped")
    w = np.load(learned.DEFAULT_WEIGHTS)
    r = learned.evaluate(w, [2100], H=256, W=320, T=30)
    s, l = r["search"], r["learned"]
    print("search", s, "learned", l)
    assert l["residual_rms"] <= 1.05 * s["residual_rms"]
    assert l["fallback_rate"] < 1.0


def test_sampled_learned_640x512_against_oracle(orc):
    """Learned mode on 640x512 frames with the shipped network, the
    configuration the benchmark times (16x16x8, 17x17 grid at 0.5 px/frame,
    confidence threshold 0.9).  At sampled anchors of the last frame, element
    by element: the spectrum and the 1152 features within their derived
    bounds of the oracle's; the network's outputs inside the interval that
    those feature bounds give through the FP64 forward pass (mlp.forward_iv);
    the anchor takes the network's velocity (index -2) exactly where its
    confidence reaches 0.9 (and where the oracle's confidence interval lies on
    one side of 0.9, that side), otherwise the instantaneous search's grid
    maximum; the output equals the oracle's filter (eq. 4 with eq. 8) at the
    velocity taken."""
    _sampled_learned(orc, 512, 640, 12, 2203, 17, 34)


def test_sampled_learned_2560x2048_against_oracle(orc):
    """As the 640x512 case on a frame whose features (2560x2048 x 1152 BF16,
    6.0e9 elements) and observer state pass 2^32 elements: the 64-bit address
    paths of the first pass, the network kernel, the confident-anchor list
    and the finish pass, at sampled anchors including the last row and
    column."""
    _sampled_learned(orc, 2048, 2560, 9, 2207, 23, 14)


def _sampled_learned(orc, H, W, T, seed, pseed, nrand):
    import os

    from paper_1408_3526_amd import learned
    if not os.path.exists(learned.DEFAULT_WEIGHTS):
        pytest.skip("no trained weights shipped")
    w = np.load(learned.DEFAULT_WEIGHTS)
    b = _b()
    sc = scenes.flow_scene(seed, H=H, W=W, T=T)
    g = scenes.grid(-4, 4, 0.5)
    f = b.Filter(H, W, 16, 16, 8, g, g, velocity_mode=b.VEL_LEARNED, conf_threshold=0.9, write_features=True)
    f.set_weights(w)
    dev = torch.from_numpy(sc.frames).cuda()
    for t in range(T):
        f.push_frame(dev[t])
    rng = np.random.default_rng(pseed)
    pts = [(0, 0), (W - 1, H - 1), (W - 1, 0), (0, H - 1), (15, 15), (W // 2, H // 2), (W - 3, H - 2)]
    pts += [(int(rng.integers(0, W)), int(rng.integers(0, H))) for _ in range(nrand)]
    xs = torch.tensor([p[0] for p in pts], device="cuda")
    ys = torch.tensor([p[1] for p in pts], device="cuda")
    F = f.features()[ys, xs].float().cpu().numpy().astype(np.float64)
    vc = f.learned_output()[ys, xs].cpu().numpy()
    vxy, idx = f.velocity()
    vxy, idx = vxy[ys, xs].cpu().numpy(), idx[ys, xs].cpu().numpy()
    out = f.output()[ys, xs].cpu().numpy()
    S_gpu = f.spectrum([p[0] for p in pts], [p[1] for p in pts]).cpu().numpy()
    torch.cuda.synchronize()
    f.close()
    del dev
    torch.cuda.empty_cache()

    cfg = orc.Cfg(H=H, W=W, Mx=16, My=16, Mz=8, gx=g, gy=g, alpha=0.0)
    Xr, Xrad = _check_features(orc, cfg, sc.frames, pts, F, S_gpu)
    # network outputs inside the interval propagated from the feature bounds
    params = mlp.unpack(w)
    fw = mlp.forward_iv(Xr, Xrad, params)
    Om, Or = fw["O"]
    assert mlp.within(vc[:, :2], Om[:, :2], Or[:, :2]).all()
    clo, chi = mlp.sigmoid_iv(Om[:, 2], Or[:, 2])
    assert np.all((vc[:, 2] >= clo) & (vc[:, 2] <= chi))
    confident = vc[:, 2] >= 0.9
    assert np.array_equal(idx == -2, confident)
    assert np.array_equal(vxy[confident], vc[confident, :2])
    assert not np.any(confident & (chi < 0.9)) and np.all(confident | (clo < 0.9))

    rms = float(np.sqrt(np.mean(sc.frames[T - 1].astype(np.float64) ** 2)))
    for i, (x, y) in enumerate(pts):
        p = orc.pixel_series(cfg, sc.frames, x, y)
        S = p["S"][-1]
        R, P = orc.flow_R(cfg, S, want_P=True)
        if not confident[i]:
            # fallback: first maximum of the instantaneous R (ties: any near-maximal pick)
            scale = max(np.abs(R).max(), 1e-3 * P.sum(), 1e-30)
            assert 0 <= idx[i] < len(R)
            assert R[idx[i]] >= R.max() - 1e-4 * scale, (x, y)
            srt = np.sort(R)
            if srt[-1] - srt[-2] > 1e-4 * scale:
                assert idx[i] == int(np.argmax(R)), (x, y)
            assert vxy[i, 0] == np.float32(g[idx[i] % len(g)]) and vxy[i, 1] == np.float32(g[idx[i] // len(g)])
        ihat = orc.background(cfg, orc.coeffs(cfg, float(vxy[i, 0]), float(vxy[i, 1])), S)
        ts, xd, yd = T - 1 - cfg.dt, x - cfg.dx, y - cfg.dy
        delayed = float(sc.frames[ts, yd, xd]) if (xd >= 0 and yd >= 0) else 0.0
        assert abs(out[i] - (delayed - ihat)) <= 1e-3 * rms, (x, y, out[i], delayed - ihat)
    print("sampled anchors: %d, confident: %d, output bound median %.3g px/frame"
          % (len(pts), int(confident.sum()), float(np.median(Or[:, :2]))))


@pytest.mark.parametrize("H,W", [(45, 70), (29, 37)])
def test_learned_mode_ragged_tiles_against_oracle(orc, H, W):
    """Learned mode with work tiles of 7, 16 and 32 rows and frame widths
    that leave idle columns in the last workgroup, a threshold (0.6) that
    lets the network decide about half the anchors: each anchor's network
    output equals, bit for bit, what the network gives on the features the
    push wrote (rmdf_learned_network); and against the oracle at every
    anchor, the network's velocity is taken exactly where its confidence
    reaches the threshold, the fallback is the instantaneous search's first
    maximum, and the output is the oracle's filter (eq. 4 with eq. 8) at the
    velocity taken."""
    import os

    from paper_1408_3526_amd import learned
    if not os.path.exists(learned.DEFAULT_WEIGHTS):
        pytest.skip("no trained weights shipped")
    w = np.load(learned.DEFAULT_WEIGHTS)
    b = _b()
    T, thr = 12, 0.6
    sc = scenes.flow_scene(2301 + H, H=H, W=W, T=T, n_targets=2, band_width=(6, 10))
    g = scenes.grid(-4, 4, 0.5)
    dev = torch.from_numpy(sc.frames).cuda()
    cfg = orc.Cfg(H=H, W=W, Mx=16, My=16, Mz=8, gx=g, gy=g, alpha=0.0)
    r = orc.run(cfg, sc.frames, want_rs=True, want_spec=True)
    rs = r["rs_all"][-1]
    srt = np.sort(rs, -1)
    scale = np.maximum(np.maximum(np.abs(rs).max(-1), 1e-3 * r["en_all"][-1]), 1e-30)
    tied = srt[..., -1] - srt[..., -2] <= 1e-4 * scale
    rms = float(np.sqrt(np.mean(sc.frames[-1].astype(np.float64) ** 2)))
    for tr in (7, 16, 32):
        f = b.Filter(H, W, 16, 16, 8, g, g, velocity_mode=b.VEL_LEARNED, conf_threshold=thr, tile_rows=tr,
                     write_features=True)
        f.set_weights(w)
        for t in range(T):
            f.push_frame(dev[t])
        vxy, idx = f.velocity()
        feats = f.features()
        alone = f.learned_network(feats.reshape(H * W, -1)).cpu().numpy().reshape(H, W, 3)
        out, vxy, idx, vc = f.output().cpu().numpy(), vxy.cpu().numpy(), idx.cpu().numpy(), f.learned_output().cpu().numpy()
        torch.cuda.synchronize()
        f.close()
        assert np.array_equal(vc, alone), tr
        confident = vc[..., 2] >= thr
        assert np.array_equal(idx == -2, confident), tr
        assert 0 < confident.sum() < H * W, (tr, int(confident.sum()))
        assert np.array_equal(vxy[confident], vc[confident][:, :2]), tr
        fb = ~confident
        assert np.all((idx == r["idx"][-1])[fb & ~tied]), tr
        agree = fb & (idx == r["idx"][-1])
        assert np.abs(out - r["out"][-1])[agree].max() <= 1e-3 * rms, tr
        ys, xs = np.nonzero(confident)
        for y, x in zip(ys, xs):
            ihat = orc.background(cfg, orc.coeffs(cfg, float(vxy[y, x, 0]), float(vxy[y, x, 1])), r["spec"][y, x])
            yd, xd = y - cfg.dy, x - cfg.dx
            delayed = float(sc.frames[T - 1 - cfg.dt, yd, xd]) if (xd >= 0 and yd >= 0) else 0.0
            assert abs(out[y, x] - (delayed - ihat)) <= 1e-3 * rms, (tr, x, y)
        print("%dx%d, %d-row tiles: %d of %d anchors took the network's velocity"
              % (W, H, tr, int(confident.sum()), H * W))


def test_refused_push_changes_nothing():
    """A push refused for missing learned weights (RMDF_E_STATE) is checked
    before any launch: the frame count, the non-finite counter and the delay
    ring are as before, so the pushes that follow give the same outputs as a
    context that never saw the refused frame."""
    b = _b()
    sc = scenes.flow_scene(8, H=34, W=37, T=9, n_targets=2, band_width=(6, 9))
    g = scenes.grid(-4, 4, 0.5)
    dev = torch.from_numpy(sc.frames).cuda()
    bad = dev[0].clone()
    bad[3, 5] = float("nan")
    bad[10, 1] = float("inf")
    w = _blob([0.4, -0.3, -20.0])
    f = b.Filter(34, 37, 16, 16, 8, g, g, velocity_mode=b.VEL_LEARNED, conf_threshold=0.9)
    with pytest.raises(b.RmdfError) as ei:
        f.push_frame(bad)
    assert ei.value.status == b.RMDF_E_STATE
    assert f.frames_pushed() == 0 and f.nonfinite_count() == 0
    f.set_weights(w)
    ref = b.Filter(34, 37, 16, 16, 8, g, g, velocity_mode=b.VEL_LEARNED, conf_threshold=0.9)
    ref.set_weights(w)
    for t in range(9):
        f.push_frame(dev[t])
        ref.push_frame(dev[t])
    out, out_ref = f.output(), ref.output()
    (vxy, idx), (vxy_r, idx_r) = f.velocity(), ref.velocity()
    torch.cuda.synchronize()
    assert f.frames_pushed() == 9 and f.nonfinite_count() == 0
    assert torch.equal(out, out_ref) and torch.equal(vxy, vxy_r) and torch.equal(idx, idx_r)
    f.close()
    ref.close()


def test_learned_network_arguments():
    """rmdf_learned_network refuses a context that is not in learned mode or
    has no weights, and an empty, missing or misaligned input, before any
    launch."""
    b = _b()
    g = scenes.grid(-4, 4, 0.5)
    feat = torch.zeros(16, 1152, dtype=torch.bfloat16, device="cuda")
    vc = torch.zeros(16, 3, device="cuda")
    plain = b.Filter(20, 20, 16, 16, 8, g, g)
    assert b.lib().rmdf_learned_network(plain.ctx, feat.data_ptr(), 16, vc.data_ptr()) == b.RMDF_E_STATE
    plain.close()
    f = b.Filter(20, 20, 16, 16, 8, g, g, velocity_mode=b.VEL_LEARNED)
    assert b.lib().rmdf_learned_network(f.ctx, feat.data_ptr(), 16, vc.data_ptr()) == b.RMDF_E_STATE
    f.set_weights(_blob([0.5, -0.25, 3.0]))
    assert b.lib().rmdf_learned_network(f.ctx, feat.data_ptr(), 0, vc.data_ptr()) == b.RMDF_E_INVAL
    assert b.lib().rmdf_learned_network(f.ctx, None, 16, vc.data_ptr()) == b.RMDF_E_INVAL
    # the network kernel loads 16-byte pieces: a misaligned feature pointer is refused
    assert b.lib().rmdf_learned_network(f.ctx, feat.data_ptr() + 2, 15, vc.data_ptr()) == b.RMDF_E_INVAL
    out = f.learned_network(feat).cpu().numpy()
    torch.cuda.synchronize()
    f.close()
    # zero weights but the biases: every row gives (0.5, -0.25, sigmoid(3))
    assert np.allclose(out[:, 0], 0.5) and np.allclose(out[:, 1], -0.25)
    assert np.allclose(out[:, 2], 1.0 / (1.0 + np.exp(-3.0)), rtol=1e-6)
