"""Plain definitions, evaluated directly on one analysis window at a time.

TEST INFRASTRUCTURE ONLY (part of the oracle).  These are the formulas of
Sec. 2 of the paper written out with NumPy: no recursion, no Hermitian
halving, no reordering.  They pin the recursive oracle in ``rmdf_oracle.c``.

Indexing: an analysis window anchored at n = (x, y, t) holds
``block[mx, my, mz] = I(t - mz, y - my, x - mx)`` (eq. 1: the window origin
m = 0 is the newest sample at n); samples outside the frame or before t = 0
are zero.
"""
from __future__ import annotations

import numpy as np


def block(frames: np.ndarray, x: int, y: int, t: int, M) -> np.ndarray:
    """The windowed block I(n - m), m in [0, M) per dimension (eq. 1, 6)."""
    Mx, My, Mz = M
    T, H, W = frames.shape
    b = np.zeros((Mx, My, Mz), np.float64)
    for mz in range(Mz):
        tt = t - mz
        if tt < 0 or tt >= T:
            continue
        for my in range(My):
            yy = y - my
            if yy < 0 or yy >= H:
                continue
            for mx in range(Mx):
                xx = x - mx
                if 0 <= xx < W:
                    b[mx, my, mz] = frames[tt, yy, xx]
    return b


def dft_matrix(M: int) -> np.ndarray:
    """F_1(m; k) = exp(+j 2 pi k m / M), rows m, columns k (eq. 7 per axis)."""
    m = np.arange(M)
    return np.exp(2j * np.pi * np.outer(m, m) / M)


def spectrum_of_block(b: np.ndarray) -> np.ndarray:
    """Eq. (6)-(7): S(k) = sum_m F(m; k) b(m), F = exp(+j2pi k.m/M)/sqrt(MxMyMz)."""
    Mx, My, Mz = b.shape
    Fx, Fy, Fz = dft_matrix(Mx), dft_matrix(My), dft_matrix(Mz)
    # the triple sum, one axis at a time (same terms, separable order)
    S = np.einsum("abc,ai,bj,ck->ijk", b.astype(np.complex128), Fx, Fy, Fz, optimize=True)
    return S / np.sqrt(Mx * My * Mz)


def spectrum(frames: np.ndarray, x: int, y: int, t: int, M) -> np.ndarray:
    return spectrum_of_block(block(frames, x, y, t, M))


def dirichlet(W: int, w) -> np.ndarray:
    """Eq. (3) with its limit at integer w."""
    w = np.asarray(w, np.float64)
    s = np.sin(np.pi * w)
    r = np.round(w)
    at_int = np.abs(w - r) < 1e-12
    safe = np.where(at_int, 1.0, s)
    val = np.sin(np.pi * W * w) / (W * safe)
    lim = np.where(((W - 1) * r.astype(np.int64)) % 2 == 0, 1.0, -1.0)
    return np.where(at_int, lim, val)


def fir_eq2(M, B, mp, v) -> np.ndarray:
    """Eq. (2): H(m; m', v) over the window, array [Mx, My, Mz] (real)."""
    Mx, My, Mz = M
    Bx, By = B
    Wx, Wy = 2 * Bx + 1, 2 * By + 1
    mx, my, mz = np.meshgrid(np.arange(Mx), np.arange(My), np.arange(Mz), indexing="ij")
    ax = (mx - mp[0] - v[0] * (mz - mp[2])) / Mx
    ay = (my - mp[1] - v[1] * (mz - mp[2])) / My
    return Wx * Wy / (Mx * My * Mz) * dirichlet(Wx, ax) * dirichlet(Wy, ay)


def coeffs_eq5(M, B, mp, v) -> np.ndarray:
    """Eq. (5): DFT of eq. (2), H(k) = sum_m F*(m; k) H(m)."""
    Hm = fir_eq2(M, B, mp, v).astype(np.complex128)
    Fx, Fy, Fz = (np.conj(dft_matrix(n)) for n in M)
    return np.einsum("abc,ai,bj,ck->ijk", Hm, Fx, Fy, Fz, optimize=True) / np.sqrt(np.prod(M))


def background_eq1(frames, x, y, t, M, B, mp, v) -> float:
    """Eq. (1): Ihat(n - m') = sum_m H(m; m', v) I(n - m) (direct convolution)."""
    return float(np.sum(fir_eq2(M, B, mp, v) * block(frames, x, y, t, M)))


def hann_window(M: int) -> np.ndarray:
    """Periodic Hann window w(m) = 1/2 - 1/2 cos(2 pi m / M); multiplying the
    block by it is the same operation as the 3-tap convolution of the spectrum
    with (-1/4, 1/2, -1/4) (Sec. 2, the convolution-theorem dual)."""
    m = np.arange(M)
    return 0.5 - 0.5 * np.cos(2 * np.pi * m / M)


def flow_block(b: np.ndarray) -> np.ndarray:
    """The sample-domain block whose spectrum is the high-passed, Hann-windowed
    spectrum: remove each time slice's spatial mean (drops kx = ky = 0 for every
    kz), then multiply by the separable periodic Hann window."""
    Mx, My, Mz = b.shape
    hp = b - b.mean(axis=(0, 1), keepdims=True)
    w = hann_window(Mx)[:, None, None] * hann_window(My)[None, :, None] * hann_window(Mz)[None, None, :]
    return hp * w


def autocorr_cyclic(s: np.ndarray, l) -> float:
    """sum_m s(m) s(m - l), cyclic in every axis, integer l (eq. 10 via the
    Wiener-Khinchin relation)."""
    sh = np.roll(s, shift=tuple(int(v) for v in l), axis=(0, 1, 2))   # sh[m] = s[m - l]
    return float(np.sum(s * sh))
