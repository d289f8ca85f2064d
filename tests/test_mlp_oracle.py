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
