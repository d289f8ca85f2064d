"""Cell-averaging CFAR detector on the prediction-error output, in FP64.

TEST INFRASTRUCTURE ONLY (same rules as the rest of ``oracle/``).

The paper hands its prediction-error output to a detector (a threshold,
then a tracker: Sec. 1) without fixing one.  The detection stage built here
is the textbook two-sided cell-averaging CFAR on the output image x:

* training cells of pixel p: every in-frame q with
  max(|qx - px|, |qy - py|) <= guard + train, minus those with
  max(|qx - px|, |qy - py|) <= guard (the guard square holds p itself);
* mu = mean of x over the training cells, sigma^2 = mean of x^2 minus mu^2;
* detection: n > 0 and |x(p) - mu| > k * sigma, with n the number of
  training cells.

``cfar`` adds the shifted windows one offset at a time (the definition as
written); ``cfar_loops`` evaluates the same definition pixel by pixel with
plain Python loops and serves as its brute-force check.
"""
from __future__ import annotations

import numpy as np


def _window_sum(a: np.ndarray, r: int) -> np.ndarray:
    """out[y, x] = sum of a[y + dy, x + dx] over |dy|, |dx| <= r, in-frame only."""
    H, W = a.shape
    out = np.zeros_like(a)
    for dy in range(-r, r + 1):
        y0, y1 = max(0, -dy), min(H, H - dy)
        if y0 >= y1:
            continue
        for dx in range(-r, r + 1):
            x0, x1 = max(0, -dx), min(W, W - dx)
            if x0 >= x1:
                continue
            out[y0:y1, x0:x1] += a[y0 + dy:y1 + dy, x0 + dx:x1 + dx]
    return out


def cfar(x: np.ndarray, guard: int, train: int, k: float):
    """Returns (detections bool [H, W], mu, sigma, n)."""
    x = np.asarray(x, np.float64)
    R = guard + train
    one = np.ones_like(x)
    n = _window_sum(one, R) - _window_sum(one, guard)
    s1 = _window_sum(x, R) - _window_sum(x, guard)
    s2 = _window_sum(x * x, R) - _window_sum(x * x, guard)
    with np.errstate(invalid="ignore", divide="ignore"):
        mu = np.where(n > 0, s1 / np.maximum(n, 1), 0.0)
        var = np.where(n > 0, s2 / np.maximum(n, 1) - mu * mu, 0.0)
    sigma = np.sqrt(np.maximum(var, 0.0))
    det = (n > 0) & (np.abs(x - mu) > k * sigma)
    return det, mu, sigma, n


def cfar_loops(x, guard: int, train: int, k: float):
    """The same definition, one pixel and one training cell at a time."""
    x = np.asarray(x, np.float64)
    H, W = x.shape
    R = guard + train
    det = np.zeros((H, W), bool)
    sig = np.zeros((H, W))
    for py in range(H):
        for px in range(W):
            vals = []
            for qy in range(py - R, py + R + 1):
                for qx in range(px - R, px + R + 1):
                    if not (0 <= qy < H and 0 <= qx < W):
                        continue
                    if max(abs(qx - px), abs(qy - py)) <= guard:
                        continue
                    vals.append(x[qy, qx])
            if not vals:
                continue
            v = np.array(vals)
            mu = v.mean()
            s = np.sqrt(max((v * v).mean() - mu * mu, 0.0))
            sig[py, px] = s
            det[py, px] = abs(x[py, px] - mu) > k * s
    return det, sig
