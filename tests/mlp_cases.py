"""Network test cases shared by the CPU pins of the element-wise bounds and
the GPU gradient tests (inputs only; all arithmetic is in oracle/mlp.py)."""
import numpy as np

from oracle import mlp


def random_params(rng, scale=1.0):
    """He-scaled weights and small random biases, FP32 values."""
    W1 = rng.normal(size=(mlp.N_H1, mlp.N_IN)) * np.sqrt(2.0 / mlp.N_IN) * scale
    W2 = rng.normal(size=(mlp.N_H2, mlp.N_H1)) * np.sqrt(2.0 / mlp.N_H1)
    W3 = rng.normal(size=(mlp.N_OUT, mlp.N_H2)) * np.sqrt(1.0 / mlp.N_H2)
    b1 = rng.normal(scale=0.1, size=mlp.N_H1)
    b2 = rng.normal(scale=0.1, size=mlp.N_H2)
    b3 = rng.normal(scale=0.1, size=mlp.N_OUT)
    return [np.float32(a).astype(np.float64) for a in (W1, b1, W2, b2, W3, b3)]


def integer_case(seed=0, n=512):
    """Integer-valued inputs and weights (dyadic labels and output bias)
    for which every FP32 operation of the forward and backward pass is exact;
    the confidence logit is 0 (W3's last row and b3's last entry are 0), so
    the sigmoid is exactly 1/2."""
    rng = np.random.default_rng(seed)
    X = rng.integers(-2, 3, size=(n, mlp.N_IN)).astype(np.float64)
    W1 = rng.choice([-1.0, 0.0, 1.0], p=[0.03, 0.94, 0.03], size=(mlp.N_H1, mlp.N_IN))
    b1 = rng.integers(-3, 4, size=mlp.N_H1).astype(np.float64)
    W2 = rng.choice([-1.0, 0.0, 1.0], p=[0.06, 0.88, 0.06], size=(mlp.N_H2, mlp.N_H1))
    b2 = rng.integers(-3, 4, size=mlp.N_H2).astype(np.float64)
    W3 = np.zeros((mlp.N_OUT, mlp.N_H2))
    W3[:2] = rng.choice([-1.0, 0.0, 1.0], p=[0.2, 0.6, 0.2], size=(2, mlp.N_H2))
    b3 = np.array([0.25, -0.5, 0.0])
    params = [W1, b1, W2, b2, W3, b3]
    # labels a few quarter steps from the network's (integer-valued) output,
    # so that both confidence targets occur
    O = mlp.forward(X, params, bf16=True)[-1]
    lab = O[:, :2] + rng.integers(-3, 4, size=(n, 2)) * 0.25
    return X, lab, params


def exactness_premise(X, lab, params, n):
    """Every dot product of the pass has terms on a common dyadic grid q with
    sum |terms| < 2^24 q, so any FP32 summation order is exact; returns the
    largest such ratio (must be < 1)."""
    W1, b1, W2, b2, W3, b3 = params
    Xr, W1r, W2r, H1, H2, O = mlp.forward(X, params, bf16=True)
    worst = 0.0

    def chk(absA, absB, q, extra=0.0):
        nonlocal worst
        worst = max(worst, float(((absA @ absB) + extra).max()) / (2.0 ** 24 * q))

    def on_grid(a, q):
        return np.all(np.abs(a / q - np.round(a / q)) == 0)

    assert on_grid(H1, 1.0) and on_grid(H2, 1.0)
    chk(np.abs(X), np.abs(W1).T, 1.0, np.abs(b1).max())
    chk(np.abs(H1), np.abs(W2).T, 1.0, np.abs(b2).max())
    chk(np.abs(H2), np.abs(W3).T, 0.25, 0.5)
    e = O[:, :2] - lab
    dO = np.zeros((n, 3))
    dO[:, :2] = 2.0 * e / n
    t = (np.max(np.abs(e), axis=1) <= 0.25).astype(np.float64)
    dO[:, 2] = (0.5 - t) / n
    q = 0.25 * 2.0 / n
    assert on_grid(dO, q / 2)
    chk(np.abs(dO).T, np.abs(H2), q / 2)
    dH2 = mlp.bf16_round(np.where(H2 > 0, dO @ W3, 0.0))
    assert on_grid(dH2, q / 2)
    chk(np.abs(dH2).T, np.abs(H1), q / 2)
    dH1 = mlp.bf16_round(np.where(H1 > 0, dH2 @ W2, 0.0))
    assert on_grid(dH1, q / 2)
    chk(np.abs(dH1).T, np.abs(X), q / 2)
    return worst


