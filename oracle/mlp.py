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
