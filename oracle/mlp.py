"""FP64 reference of the learned velocity surrogate (TEST INFRASTRUCTURE ONLY).

Network (the library's learned mode): input x = the log power spectrum of a
pixel's window, 1152 values (kx = 0..8 of the 16x16x8 bins; the even
spectrum repeats them), layers 1152 -> 128 (ReLU) -> 64 (ReLU) -> 3.  Weights
are row-major [out][in].  Loss for a batch of n samples with labels (lx, ly):
  wv * ((o0 - lx)^2 + (o1 - ly)^2) / n  +  BCE(o2, t) / n,
  t = [max(|o0 - lx|, |o1 - ly|) <= half_step]  (t is a constant).
``bf16=True`` rounds, as the GPU does, the inputs, the first two weight
matrices and the stored activations/gradient rows to BF16 before use.

The paper has no learned part.  The input map (log scaling, the 1e-6 max P
floor, the mean removal) and the confidence target are choices made for this
library: parity unpinned beyond the properties the tests check (scale
invariance of the features, the forward pass on selection weights, gradients
against finite differences).
"""
from __future__ import annotations

import numpy as np

N_IN, N_H1, N_H2, N_OUT = 1152, 128, 64, 3


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a = np.asarray(x, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(blob):
    blob = np.asarray(blob, np.float64)
    o = 0
    out = []
    for shape in [(N_H1, N_IN), (N_H1,), (N_H2, N_H1), (N_H2,), (N_OUT, N_H2), (N_OUT,)]:
        n = int(np.prod(shape))
        out.append(blob[o:o + n].reshape(shape))
        o += n
    return out


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([np.ravel(a) for a in (W1, b1, W2, b2, W3, b3)]).astype(np.float32)


def forward(X, params, bf16=True):
    W1, b1, W2, b2, W3, b3 = params
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    Xr, W1r, W2r = r(X), r(W1), r(W2)
    H1 = r(np.maximum(Xr @ W1r.T + b1, 0.0))
    H2 = r(np.maximum(H1 @ W2r.T + b2, 0.0))
    O = H2 @ np.asarray(W3, np.float64).T + b3
    return Xr, W1r, W2r, H1, H2, O


def loss_and_grads(X, labels, params, wv=1.0, half_step=0.25, bf16=True):
    W1, b1, W2, b2, W3, b3 = params
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    Xr, W1r, W2r, H1, H2, O = forward(X, params, bf16)
    n = X.shape[0]
    e = O[:, :2] - labels
    t = (np.max(np.abs(e), axis=1) <= half_step).astype(np.float64)
    z = O[:, 2]
    bce = np.maximum(z, 0) - z * t + np.log1p(np.exp(-np.abs(z)))
    loss = np.sum(wv * np.sum(e * e, axis=1) + bce) / n
    dO = np.empty_like(O)
    dO[:, :2] = 2.0 * wv * e / n
    dO[:, 2] = (1.0 / (1.0 + np.exp(-z)) - t) / n
    dW3 = dO.T @ H2
    db3 = dO.sum(0)
    dH2 = r(np.where(H2 > 0, dO @ np.asarray(W3, np.float64), 0.0))
    dW2 = dH2.T @ H1
    db2 = dH2.sum(0)
    dH1 = r(np.where(H1 > 0, dH2 @ W2r, 0.0))
    dW1 = dH1.T @ Xr
    db1 = dH1.sum(0)
    return loss, (dW1, db1, dW2, db2, dW3, db3)


def features_from_P(P):
    """Learned-model input from the full power spectrum P[..., 16, 16, 8]
    (eq. 9): ln(P + 1e-6 max P) minus its mean over all 2048 bins, kept for
    kx = 0..8, flattened as [kx][ky][kz]."""
    P = np.asarray(P, np.float64)
    lead = P.shape[:-3]
    flat = P.reshape(lead + (-1,))
    eps = np.maximum(1e-6 * flat.max(axis=-1), 1e-30)
    L = np.log(P + eps[..., None, None, None])
    mean = L.reshape(lead + (-1,)).mean(axis=-1)
    F = L[..., :9, :, :] - mean[..., None, None, None]
    return F.reshape(lead + (9 * 16 * 8,))


# ---------------------------------------------------------------------------
# Element-wise bounds for the GPU's arithmetic.
#
# The library computes the network with FP32 accumulation in an order the
# hardware picks (MFMA tiles, shuffles, atomics), BF16 round-to-nearest-even
# at the stored activations (H1, H2) and gradient rows (dH2, dH1), and ReLU
# masks taken from them.  These functions carry every value as an interval
# [mid - rad, mid + rad] meant to contain the result of any such computation:
#   * a length-n FP32 dot product sum_i a_i b_i differs from the exact value
#     by a sum of n rounding errors, each at most u times a partial sum.  For
#     data of random sign the partial sums are random walks, so the error is
#     of the order of u sqrt(n sum_i (a_i b_i)^2); the bound used is LAMBDA = 10
#     times that with u = 2^-23 (one FP32 ulp per operation instead of the
#     half ulp of round-to-nearest, which also covers a truncating adder
#     inside the matrix cores).  The worst-case bound gamma_n sum |a_i b_i|
#     (gamma_n = n u / (1 - n u)) is kept for the exact-arithmetic pins; for
#     a 1152-term product it is about 40 times wider, wide enough to put half
#     of the first layer's BF16 outputs on a rounding boundary;
#   * ReLU and BF16 rounding are monotone, so an interval maps to the interval
#     between the images of its end points; where it straddles a rounding
#     boundary the image spans the two neighbouring BF16 values (one ulp), and
#     where it straddles 0 a ReLU mask may go either way (both are allowed);
#   * the confidence target t = [max|o - label| <= half_step] may take both
#     values where the interval of o straddles the threshold.
# A GPU value outside its interval is an error of the implementation, not of
# rounding.  The mid points are the FP64 values of the reference above.

U32 = 2.0 ** -23
LAMBDA = 10.0


def gamma(n):
    """Bound of the relative accumulation error of an n-term FP32 dot product."""
    return n * U32 / (1.0 - n * U32)


def _f64(a):
    return np.asarray(a, np.float64)


def fp32_dot_error(absA, absB, n):
    """Bound of the FP32 accumulation error of the products absA @ absB
    (element-wise magnitudes), n terms each: LAMBDA u sqrt(n sum (a b)^2)."""
    return LAMBDA * U32 * np.sqrt(n * ((absA * absA) @ (absB * absB)))


def iv_affine(Am, Ar, B, bias=None, Br=None):
    """[Am +- Ar] @ [B +- Br] (+ bias) in FP32, any summation order.  Returns
    (mid, rad).  Ar / Br may be 0 (exact operand)."""
    Am, B = _f64(Am), _f64(B)
    Ar = np.zeros_like(Am) if np.isscalar(Ar) and Ar == 0 else _f64(Ar)
    Br = np.zeros_like(B) if Br is None else _f64(Br)
    n = Am.shape[-1] + (0 if bias is None else 1)
    mid = Am @ B
    absA, absB = np.abs(Am) + Ar, np.abs(B) + Br
    rad = Ar @ np.abs(B) + np.abs(Am) @ Br + Ar @ Br
    if bias is not None:
        b = _f64(bias)
        mid = mid + b
        # the bias is one more term of the sum
        rad = rad + LAMBDA * U32 * np.sqrt(n * ((absA * absA) @ (absB * absB) + b * b))
    else:
        rad = rad + fp32_dot_error(absA, absB, n)
    return mid, rad


def _sum_iv(m, r):
    """Column sums of [m +- r] in FP32 (same error model as a dot product)."""
    n = m.shape[0]
    a = np.abs(m) + r
    return m.sum(0), r.sum(0) + LAMBDA * U32 * np.sqrt(n * (a * a).sum(0))


def iv_relu_bf16(mid, rad):
    """BF16(ReLU(v)) for every v in [mid - rad, mid + rad]: (lo, hi)."""
    return bf16_round(np.maximum(mid - rad, 0.0)), bf16_round(np.maximum(mid + rad, 0.0))


def iv_bf16(lo, hi):
    return bf16_round(lo), bf16_round(hi)


def _mr(lo, hi):
    return 0.5 * (lo + hi), 0.5 * (hi - lo)


def forward_iv(Xm, Xr, params):
    """Intervals of the forward pass for inputs in [Xm - Xr, Xm + Xr] (BF16
    values on the GPU side).  Returns a dict with (lo, hi) of H1 and H2 and
    (mid, rad) of the output O (vx, vy, logit)."""
    W1, b1, W2, b2, W3, b3 = params
    W1r, W2r = bf16_round(W1), bf16_round(W2)
    Z1 = iv_affine(Xm, Xr, W1r.T, b1)
    H1 = iv_relu_bf16(*Z1)
    H1m, H1r = _mr(*H1)
    Z2 = iv_affine(H1m, H1r, W2r.T, b2)
    H2 = iv_relu_bf16(*Z2)
    H2m, H2r = _mr(*H2)
    O = iv_affine(H2m, H2r, _f64(np.float32(W3)).T, np.float32(b3))
    return {"H1": H1, "H2": H2, "O": O, "W2r": W2r}


def sigmoid_iv(zm, zr, rel=8 * U32):
    """Interval of the FP32 sigmoid 1 / (1 + exp(-z)) for z in [zm - zr, zm + zr]
    (monotone; widened by `rel` for the FP32 exp, add and divide)."""
    lo = 1.0 / (1.0 + np.exp(-(zm - zr)))
    hi = 1.0 / (1.0 + np.exp(-(zm + zr)))
    return lo * (1 - rel), hi * (1 + rel)


def _mask_iv(Hlo, Hhi, gm, gr):
    """(H > 0) * g where H in [Hlo, Hhi] (H >= 0) and g in [gm - gr, gm + gr]:
    (lo, hi); an uncertain mask gives the hull of 0 and g's interval."""
    glo, ghi = gm - gr, gm + gr
    on = Hlo > 0
    off = Hhi == 0
    lo = np.where(on, glo, np.where(off, 0.0, np.minimum(glo, 0.0)))
    hi = np.where(on, ghi, np.where(off, 0.0, np.maximum(ghi, 0.0)))
    return lo, hi


def grads_iv(X, labels, params, wv=1.0, half_step=0.25):
    """Intervals of the loss and of every gradient of loss_and_grads(bf16=True)
    as the library computes them (X: the BF16 input values, exact).  Returns
    (loss_mid, loss_rad), {name: (mid, rad)} for W1, b1, W2, b2, W3, b3."""
    W1, b1, W2, b2, W3, b3 = params
    X = bf16_round(X)
    lab = _f64(np.float32(labels))
    n = X.shape[0]
    fw = forward_iv(X, 0, params)
    H1lo, H1hi = fw["H1"]
    H2lo, H2hi = fw["H2"]
    H1m, H1r = _mr(H1lo, H1hi)
    H2m, H2r = _mr(H2lo, H2hi)
    Om, Or = fw["O"]
    W3f = _f64(np.float32(W3))
    # e = o - label (one FP32 rounding)
    em = Om[:, :2] - lab
    er = Or[:, :2] + U32 * (np.abs(em) + Or[:, :2])
    # confidence target, possibly either value
    alo = np.max(np.maximum(np.abs(em) - er, 0.0), axis=1)
    ahi = np.max(np.abs(em) + er, axis=1)
    tlo = (ahi <= half_step).astype(np.float64)
    thi = (alo <= half_step).astype(np.float64)
    # dO = (2 wv e / n, (sigmoid(z) - t) / n), a few FP32 roundings each
    inv = 1.0 / n
    dOm = np.empty((n, 3))
    dOr = np.empty((n, 3))
    dOm[:, :2] = 2.0 * wv * em * inv
    dOr[:, :2] = 2.0 * wv * er * inv + gamma(3) * np.abs(2.0 * wv * inv) * (np.abs(em) + er)
    slo, shi = sigmoid_iv(Om[:, 2], Or[:, 2])
    dlo, dhi = (slo - thi) * inv, (shi - tlo) * inv
    dOm[:, 2] = 0.5 * (dlo + dhi)
    dOr[:, 2] = 0.5 * (dhi - dlo) + gamma(3) * np.maximum(np.abs(dlo), np.abs(dhi))
    g = {}
    g["W3"] = iv_affine(dOm.T, dOr.T, H2m, Br=H2r)
    g["b3"] = _sum_iv(dOm, dOr)
    # dH2 = BF16((H2 > 0) * dO W3)
    G2 = iv_affine(dOm, dOr, W3f)
    dH2lo, dH2hi = iv_bf16(*_mask_iv(H2lo, H2hi, *G2))
    dH2m, dH2r = _mr(dH2lo, dH2hi)
    g["W2"] = iv_affine(dH2m.T, dH2r.T, H1m, Br=H1r)
    g["b2"] = _sum_iv(dH2m, dH2r)
    # dH1 = BF16((H1 > 0) * dH2 W2)
    G1 = iv_affine(dH2m, dH2r, fw["W2r"])
    dH1lo, dH1hi = iv_bf16(*_mask_iv(H1lo, H1hi, *G1))
    dH1m, dH1r = _mr(dH1lo, dH1hi)
    g["W1"] = iv_affine(dH1m.T, dH1r.T, X)
    g["b1"] = _sum_iv(dH1m, dH1r)
    # loss: first-order bound from the intervals of o (and both targets where t
    # is uncertain), plus FP32 rounding of the per-sample terms and their sum
    z, zr = Om[:, 2], Or[:, 2]
    bce = lambda tt: np.maximum(z, 0) - z * tt + np.log1p(np.exp(-np.abs(z)))  # noqa: E731
    lm = np.sum(wv * np.sum(em * em, axis=1) + bce(tlo)) * inv
    lr = np.sum(wv * np.sum(2 * np.abs(em) * er + er * er, axis=1) + zr + np.abs(z) * (thi - tlo)) * inv
    lr += gamma(n + 8) * np.sum(wv * np.sum(em * em, axis=1) + np.abs(bce(tlo)) + np.abs(z)) * inv
    return (lm, lr), g


def within(got, mid, rad, slack=2.0 ** -40):
    """Boolean array: got lies in [mid - rad, mid + rad] (plus a relative slack
    for the FP64 rounding of mid and rad themselves)."""
    got, mid, rad = _f64(got), _f64(mid), _f64(rad)
    return np.abs(got - mid) <= rad + slack * (np.abs(mid) + rad)


# Spectrum error allowed for the GPU's local spectrum, relative to its largest
# bin: a bin comes out of about L = 128 sequential FP32 operations (row and
# column sliding DFTs with their restarts, the observer update) at magnitudes
# up to that of the largest bin; with random-walk accumulation of their
# rounding errors that is about sqrt(L) u = 6.7e-7, taken with a 1.5x margin.
TAU_S = 1.0e-6


def features_iv(P, max_abs_S, tau=TAU_S):
    """Element-wise bound of the GPU's BF16 features given that its local
    spectrum S is within eta = tau * max|S| of the reference in every bin.

    P is the reference power spectrum of the windowed, high-passed spectrum
    S' ([16, 16, 8]).  The Hann window and the high-pass do not amplify an
    error (absolute weights summing to 1 per axis), so |dS'| <= eta in every
    bin and |dP| <= 2 sqrt(P) eta + eta^2 (+ 4u P for the FP32 square); the
    floor eps = 1e-6 max P moves by at most 1e-6 max|dP|.  Then
      ln(P + eps) lies in [ln(P + eps - d), ln(P + eps + d)], d = dP + d_eps,
    which is tight where P >> eta^2 and, at the floor (P << eps), of the form
      |d ln| <= ln(1 + (2 sqrt(P) eta + eta^2 + d_eps) / eps),
    i.e. up to about 2 eta / sqrt(eps) there.  The mean over all 2048 bins
    moves by at most the mean of those bounds.  A fast FP32 logarithm adds
    4e-6 max(1, |ln|), and the BF16 rounding of x at most 2^-8 |x|.
    Returns (x_ref, rad) for the 1152 stored features."""
    P = np.asarray(P, np.float64)
    eta = tau * float(max_abs_S)
    eps = 1e-6 * P.max()
    dP = 2.0 * np.sqrt(P) * eta + eta * eta + 4.0 * 2.0 ** -24 * P
    d = dP + 1e-6 * dP.max()
    L = np.log(P + eps)
    lo = np.log(np.maximum(P + eps - d, 0.5 * eps))
    hi = np.log(P + eps + d)
    dL = np.maximum(L - lo, hi - L) + 4e-6 * np.maximum(1.0, np.abs(L))
    delta = dL[:9].reshape(-1) + dL.mean()
    x = features_from_P(P)
    return x, 2.0 ** -8 * (np.abs(x) + delta) + delta
