"""Pins of the certified element-wise bounds in oracle/mlp.py (CPU).

The GPU's network and its gradients are checked element by element against
intervals that contain every result FP32 accumulation in any order, BF16
round-to-nearest-even at the stored activations and gradient rows, and ReLU
masks taken from them can give.  Here those intervals are pinned without a
GPU:
  * exact arithmetic collapses them: on integer data whose dot products are
    exactly representable in FP32, an FP32 emulation equals the FP64 values
    bit for bit, and both lie inside;
  * an FP32 emulation of the library's arithmetic, with its sums taken in
    several different orders, lies inside every interval on realistic data;
  * plausible mistakes in that emulation (a dropped ReLU mask, a skipped BF16
    rounding, a wrong sign of the confidence gradient, a transposed weight
    block) fall outside, so the element-wise check has teeth."""
import numpy as np
import pytest

from oracle import mlp

from mlp_cases import exactness_premise, integer_case, random_params


def _bf(a):
    return mlp.bf16_round(np.asarray(a, np.float32)).astype(np.float32)


def _dot(A, B, order):
    """FP32 matrix product with the K sum taken in one of several orders."""
    A = np.asarray(A, np.float32)
    B = np.asarray(B, np.float32)
    if order == 0:
        return A @ B
    if order == 1:
        return A[:, ::-1] @ B[::-1, :]
    # blocked: partial products of 16-term blocks, then the block sums in reverse
    K = A.shape[1]
    acc = np.zeros((A.shape[0], B.shape[1]), np.float32)
    for k0 in reversed(range(0, K, 16)):
        acc = acc + (A[:, k0:k0 + 16] @ B[k0:k0 + 16, :]).astype(np.float32)
    return acc


def emulate(X, lab, params, wv, hs, order=0, mistake=None):
    """FP32 emulation of the library's training kernels (forward, head, the
    three backward GEMMs and the column sums)."""
    W1, b1, W2, b2, W3, b3 = [np.float32(a) for a in params]
    W1b, W2b = _bf(W1), _bf(W2)
    X = _bf(X)
    n = X.shape[0]
    Z1 = _dot(X, W1b.T, order) + b1
    H1 = np.maximum(Z1, 0).astype(np.float32)
    if mistake != "no_h1_rounding":
        H1 = _bf(H1)
    H2 = _bf(np.maximum(_dot(H1, W2b.T, order) + b2, 0))
    O = _dot(H2, W3.T, order) + b3
    e = (O[:, :2] - np.float32(lab)).astype(np.float32)
    t = (np.max(np.abs(e), axis=1) <= hs).astype(np.float32)
    sp = (1.0 / (1.0 + np.exp(-O[:, 2]))).astype(np.float32)
    inv = np.float32(1.0 / n)
    dO = np.empty((n, 3), np.float32)
    dO[:, :2] = np.float32(2 * wv) * e * inv
    dO[:, 2] = ((t - sp) if mistake == "conf_sign" else (sp - t)) * inv
    dW3 = _dot(dO.T, H2, order)
    db3 = dO.sum(0, dtype=np.float32)
    dH2 = _bf(np.where(H2 > 0, _dot(dO, W3, order), 0))
    dW2 = _dot(dH2.T, H1, order)
    db2 = dH2.sum(0, dtype=np.float32)
    W2u = W2b
    if mistake == "transposed_block":
        W2u = W2b.copy()
        W2u[:8, :8] = W2b[:8, :8].T
    G1 = _dot(dH2, W2u, order)
    dH1 = _bf(G1 if mistake == "no_mask" else np.where(H1 > 0, G1, 0))
    dW1 = _dot(dH1.T, X, order)
    db1 = dH1.sum(0, dtype=np.float32)
    return {"W1": dW1, "b1": db1, "W2": dW2, "b2": db2, "W3": dW3, "b3": db3}, O


@pytest.fixture(scope="module")
def realistic():
    rng = np.random.default_rng(11)
    n = 384
    X = mlp.bf16_round(rng.normal(size=(n, mlp.N_IN)))
    lab = np.float32(rng.uniform(-3, 3, size=(n, 2)))
    params = random_params(rng)
    loss, g = mlp.grads_iv(X, lab, params, wv=1.0, half_step=0.25)
    return X, lab, params, loss, g


@pytest.mark.parametrize("order", [0, 1, 2])
def test_fp32_emulation_lies_inside_every_interval(realistic, order):
    X, lab, params, _, g = realistic
    got, _ = emulate(X, lab, params, 1.0, 0.25, order=order)
    for k, (mid, rad) in g.items():
        ok = mlp.within(got[k], mid, rad)
        assert ok.all(), (k, order, int((~ok).sum()))
        # the intervals are tight: a small fraction of one BF16 ulp of the
        # tensor's scale on average
        assert np.median(rad) <= 2.0 ** -6 * np.abs(mid).max(), k


def test_intervals_agree_with_point_reference(realistic):
    X, lab, params, loss, g = realistic
    rl, rg = mlp.loss_and_grads(X, lab.astype(np.float64), params, bf16=True)
    assert abs(rl - loss[0]) <= loss[1] + 1e-12 * abs(rl)
    for k, G in zip(("W1", "b1", "W2", "b2", "W3", "b3"), rg):
        assert mlp.within(G, *g[k]).all(), k


@pytest.mark.parametrize("mistake,where", [("no_mask", "W1"), ("no_h1_rounding", "W2"), ("conf_sign", "W3"),
                                           ("transposed_block", "W1")])
def test_planted_mistakes_fall_outside(realistic, mistake, where):
    X, lab, params, _, g = realistic
    got, _ = emulate(X, lab, params, 1.0, 0.25, mistake=mistake)
    ok = mlp.within(got[where], *g[where])
    assert not ok.all(), mistake


def test_integer_case_is_exact_in_fp32():
    X, lab, params = integer_case()
    n = X.shape[0]
    assert exactness_premise(X, lab, params, n) < 1.0
    got, O = emulate(X, lab, params, 1.0, 0.25, order=2)
    _, rg = mlp.loss_and_grads(X, lab, params, bf16=True)
    for k, G in zip(("W1", "b1", "W2", "b2", "W3", "b3"), rg):
        assert np.array_equal(got[k].astype(np.float64), G), k
    # the case exercises both confidence targets, both ReLU states and
    # gradients of both signs
    _, _, _, H1, H2, O64 = mlp.forward(X, params, bf16=True)
    t = np.max(np.abs(O64[:, :2] - lab), axis=1) <= 0.25
    assert 0 < t.sum() < n
    assert 0.1 < (H1 > 0).mean() < 0.9 and 0.1 < (H2 > 0).mean() < 0.9
    assert (rg[0] > 0).any() and (rg[0] < 0).any()


@pytest.fixture(scope="module")
def anchor_spectrum(orc):
    """The oracle's local spectrum at two anchors of a small flow scene (one
    at the frame corner, one inside)."""
    from paper_1408_3526_amd import scenes
    sc = scenes.flow_scene(5, H=36, W=40, T=10, n_targets=2, band_width=(6, 9))
    g = scenes.grid(-4, 4, 0.5)
    cfg = orc.Cfg(H=36, W=40, Mx=16, My=16, Mz=8, gx=g, gy=g, alpha=0.0)
    return cfg, [orc.pixel_series(cfg, sc.frames, x, y)["S"][-1] for (x, y) in ((0, 0), (25, 30))]


def _hermitian_noise(rng, shape, eta):
    """Complex noise of modulus <= eta in every bin with N(-k) = conj N(k)."""
    z = rng.uniform(0, eta, size=shape) * np.exp(2j * np.pi * rng.uniform(size=shape))
    neg = np.conj(z[(-np.arange(shape[0])) % shape[0]][:, (-np.arange(shape[1])) % shape[1]][:, :, (-np.arange(shape[2])) % shape[2]])
    return 0.5 * (z + neg)


def _fp32_features(P, mean_removed=True, eps_rel=1e-6, planes=None):
    """FP32 emulation of the kernel's feature step from a power spectrum."""
    P = np.asarray(P, np.float32)
    eps = np.float32(max(eps_rel * float(P.max()), 1e-30))
    L = np.log(P + eps).astype(np.float32)
    mean = np.float32(L.astype(np.float32).sum(dtype=np.float32) / np.float32(L.size))
    x = L[:9] if planes is None else L[planes]
    if mean_removed:
        x = x - mean
    return mlp.bf16_round(x.reshape(-1))


def test_feature_bound_contains_spectrum_errors(orc, anchor_spectrum):
    cfg, spectra = anchor_spectrum
    rng = np.random.default_rng(3)
    for S in spectra:
        eta = mlp.TAU_S * np.abs(S).max()
        _, P = orc.flow_R(cfg, S, want_P=True)
        x, rad = mlp.features_iv(P, np.abs(S).max())
        for _ in range(5):
            Sp = S + _hermitian_noise(rng, S.shape, eta)
            _, Pp = orc.flow_R(cfg, Sp, want_P=True)
            got = _fp32_features(Pp)
            assert np.all(np.abs(got - x) <= rad), float(np.max(np.abs(got - x) / rad))
        # where the power is well above the floor the bound is a few
        # hundredths (the BF16 step plus the shift of the mean, which the
        # bins near the floor dominate)
        strong = P[:9].reshape(-1) > 1e-3 * P.max()
        assert np.median(rad[strong]) <= 0.05


@pytest.mark.parametrize("mistake", ["no_mean", "eps_1e-5", "planes_swapped"])
def test_feature_bound_rejects_mistakes(orc, anchor_spectrum, mistake):
    cfg, spectra = anchor_spectrum
    S = spectra[1]
    _, P = orc.flow_R(cfg, S, want_P=True)
    x, rad = mlp.features_iv(P, np.abs(S).max())
    kw = {"no_mean": dict(mean_removed=False), "eps_1e-5": dict(eps_rel=1e-5),
          "planes_swapped": dict(planes=[0, 2, 1, 3, 4, 5, 6, 7, 8])}[mistake]
    got = _fp32_features(P, **kw)
    assert not np.all(np.abs(got - x) <= rad), mistake
