"""FP32 behaviour of the two temporal recursions the paper weighs (Sec. 1):
the classic sliding DFT (comb x(t) - x(t - M) into resonators with poles on
the unit circle) against the deadbeat observer, and of the row sliding DFT
with and without the periodic direct-DFT restart the GPU row kernel uses.

These are emulations in numpy float32 (64 sequences of one bin set, one row), to show
why the library uses the observer in time and restarts in space; the GPU
kernels themselves are checked over 2^20 frames in test_gpu_drift.py and at
the end of 1280-pixel rows by the sampled 1280x1024 parity test.
"""
import numpy as np


def test_observer_does_not_drift_where_the_fp32_sliding_dft_does():
    """64 independent sequences of 2^18 samples (offset 1000, noise 10).
    The sliding DFT's rounding errors are never removed (its poles sit on the
    unit circle), so their RMS over the sequences grows like a random walk;
    the observer's stay at the level of one window."""
    rng = np.random.default_rng(0)
    Mz, T, n = 8, 1 << 18, 64
    x = (rng.normal(size=(T, n)) * 10 + 1000).astype(np.float32)
    w = np.exp(2j * np.pi * np.arange(Mz) / Mz).astype(np.complex64)[None, :]
    inv = np.float32(1.0 / Mz)
    S = np.zeros((n, Mz), np.complex64)      # classic sliding DFT
    X = np.zeros((n, Mz), np.complex64)      # deadbeat observer (rotated-posterior form)
    zero = np.zeros(n, np.float32)
    m = np.arange(Mz)
    F = np.exp(2j * np.pi * np.outer(m, np.arange(Mz)) / Mz)     # [m, k]
    res = {}
    for t in range(T):
        xt = x[t]
        old = x[t - Mz] if t >= Mz else zero
        S = w * S + (xt - old).astype(np.complex64)[:, None]
        X = w * X
        X = X + ((xt.astype(np.complex64) - X.sum(axis=1)) * inv)[:, None]
        if t + 1 in (1 << 8, 1 << 12, 1 << 15, T):
            ref = x[t - Mz + 1:t + 1][::-1].astype(np.float64).T @ F        # [n, k]
            scale = np.abs(ref).max(axis=1, keepdims=True)
            es = np.sqrt(np.mean((np.abs(S - ref) / scale).max(axis=1) ** 2))
            eo = np.sqrt(np.mean((np.abs(Mz * X - ref) / scale).max(axis=1) ** 2))
            res[t + 1] = (es, eo)
    sdft = [v[0] for v in res.values()]
    obs = [v[1] for v in res.values()]
    assert max(obs) <= 1e-7, res
    assert sdft[-1] >= 10 * sdft[0], res


def test_row_recursion_restart_bounds_the_error():
    """Row sliding DFT (Mx = 16) along 64 rows of 1280 pixels in float32:
    without restarts the RMS error at the rows' end grows with the row
    length; with a direct-DFT restart every 16 columns (as the GPU row kernel
    does) it stays at the level of one segment."""
    rng = np.random.default_rng(1)
    W, Mx, n = 1280, 16, 64
    rows = (rng.normal(size=(W, n)) * 10 + 1000).astype(np.float32)
    w = np.exp(2j * np.pi * np.arange(Mx) / Mx).astype(np.complex64)[None, :]
    F = np.exp(2j * np.pi * np.outer(np.arange(Mx), np.arange(Mx)) / Mx)     # [m, k]
    F32 = F.astype(np.complex64)
    zero = np.zeros(n, np.float32)

    def rel_rms(A, xe):
        ref = rows[xe - Mx + 1:xe + 1][::-1].astype(np.float64).T @ F
        return np.sqrt(np.mean((np.abs(A - ref).max(axis=1) / np.abs(ref).max(axis=1)) ** 2))

    A = np.zeros((n, Mx), np.complex64)
    B = np.zeros((n, Mx), np.complex64)
    err = {}
    for x in range(W):
        old = rows[x - Mx] if x >= Mx else zero
        if x % 16 == 0 and x >= Mx:
            # restart: the direct DFT (float32) of the window ending at x - 1
            B = rows[x - Mx:x][::-1].T.astype(np.complex64) @ F32
        d = (rows[x] - old).astype(np.complex64)[:, None]
        A = w * A + d
        B = w * B + d
        if x + 1 in (64, W):
            err[x + 1] = (rel_rms(A, x), rel_rms(B, x))
    assert err[W][1] <= 2 * err[64][1] + 1e-8, err       # restarted: no growth
    assert err[W][0] >= 3 * err[64][0], err              # plain recursion: grows
