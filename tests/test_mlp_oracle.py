"""Pins of the FP64 learned-model reference: its gradients equal central
finite differences of its own loss (no BF16 rounding, so the loss is smooth
except at the ReLU kinks, which random inputs avoid), and its feature map
matches the definition on a hand-built spectrum."""
import numpy as np

from oracle import mlp


def _params(rng, scale=0.1):
    return [rng.normal(scale=scale, size=s) for s in
            [(mlp.N_H1, mlp.N_IN), (mlp.N_H1,), (mlp.N_H2, mlp.N_H1), (mlp.N_H2,), (mlp.N_OUT, mlp.N_H2), (mlp.N_OUT,)]]


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(7, mlp.N_IN))
    lab = rng.normal(size=(7, 2))
    params = _params(rng, 0.05)
    loss, grads = mlp.loss_and_grads(X, lab, params, wv=0.7, half_step=10.0, bf16=False)
    h = 1e-6
    for pi, (P, G) in enumerate(zip(params, grads)):
        flat = P.reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = mlp.loss_and_grads(X, lab, params, 0.7, 10.0, bf16=False)
            flat[idx] = old - h
            lm, _ = mlp.loss_and_grads(X, lab, params, 0.7, 10.0, bf16=False)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            g = G.reshape(-1)[idx]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)), (pi, idx, fd, g)


def test_bf16_round_is_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.0e38], np.float32)
    r = mlp.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -6 and r[3] == -2.5


def test_features_definition():
    rng = np.random.default_rng(1)
    P = rng.uniform(0.5, 2.0, size=(16, 16, 8))
    P[0, 0, :] = 0.0
    F = mlp.features_from_P(P)
    L = np.log(P + 1e-6 * P.max())
    assert F.shape == (1152,)
    assert np.allclose(F.reshape(9, 16, 8), L[:9] - L.mean())


def test_forward_on_selection_weights():
    """Weights that copy inputs through make the network a known function:
    with W1 = [I_128 | 0], W2 = [I_64 | 0], W3 selecting units 0..2, the
    output is relu(x[0..2] + b1[0..2]) shifted by b2 and b3 -- which fixes the
    [out][in] orientation, the bias additions and the ReLU placement (none
    on the output layer: negative b3 gives negative outputs)."""
    X = np.array([[0.75, -0.5, 2.0] + [0.25] * (mlp.N_IN - 3),
                  [-1.0, 3.0, 0.5] + [-0.25] * (mlp.N_IN - 3)])
    W1 = np.zeros((mlp.N_H1, mlp.N_IN))
    W1[np.arange(mlp.N_H1), np.arange(mlp.N_H1)] = 1.0
    b1 = np.zeros(mlp.N_H1)
    b1[:3] = [0.5, 0.25, -1.0]
    W2 = np.zeros((mlp.N_H2, mlp.N_H1))
    W2[np.arange(mlp.N_H2), np.arange(mlp.N_H2)] = 1.0
    b2 = np.zeros(mlp.N_H2)
    b2[:3] = [0.0, 1.0, 0.5]
    W3 = np.zeros((mlp.N_OUT, mlp.N_H2))
    W3[0, 0] = W3[1, 1] = W3[2, 2] = 1.0
    b3 = np.array([-2.0, 0.0, -0.125])
    O = mlp.forward(X, [W1, b1, W2, b2, W3, b3], bf16=False)[-1]
    relu = lambda v: np.maximum(v, 0.0)  # noqa: E731
    want = relu(relu(X[:, :3] + b1[:3]) + b2[:3]) + b3
    assert np.allclose(O, want, rtol=0, atol=1e-15)
    assert O[1, 0] == -2.0 + 0.0          # relu(-1 + 0.5) = 0, then b2 = 0: the output keeps b3 < 0


def test_features_are_scale_invariant():
    """The input map ln(P + 1e-6 max P) minus its mean does not change when
    the power spectrum is scaled (the floor scales with max P): a missing mean
    removal or an absolute floor fails this."""
    rng = np.random.default_rng(2)
    b = rng.normal(size=(16, 16, 8))
    P = np.abs(np.fft.fftn(b)) ** 2
    F = mlp.features_from_P(P)
    assert np.allclose(mlp.features_from_P(37.5 * P), F, atol=1e-12)
    assert np.allclose(mlp.features_from_P(1e-20 * P), F, atol=1e-12)
