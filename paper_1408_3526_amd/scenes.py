"""Seeded synthetic infrared-like scenes (inputs only).

This module holds none of the filter's arithmetic: it only draws frames and
their ground truth.  Both the GPU path's tests and the oracle's tests take
their inputs from here.  Everything is NumPy with PCG64 generators; every
random draw comes from a named sub-stream of ``SeedSequence(seed)`` so that
adding a draw to one part does not shift the others.

Scene families
--------------
* ``translate_scene``  - 1/f^2 Gaussian random-field clutter translated by an
  integer velocity (exact ``roll`` on a periodic canvas), a few additive
  Gaussian point targets, white noise.  (64x64, window 8x8x4 workload.)
* ``flow_scene``       - the same clutter advected by a smooth non-uniform
  velocity field (sum of four low-frequency sinusoids, max |v| = 3), an
  occluding straight band with its own texture and velocity (motion
  discontinuities at its edges), additive targets of random SNR, white or
  spatially varying noise.  (640x512 and 1280x1024, window 16x16x8
  workloads; also the training data of the learned velocity model.)
* ``paper_scene``      - the simulation of the paper's Sec. "Simulation":
  25 random sinusoids with a DC offset translating at (1.625, 0.625), one
  occluding point target at (-0.625, -0.375), white noise.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

try:  # SciPy is only needed by flow_scene
    from scipy import ndimage as _ndi
except Exception:  # pragma: no cover
    _ndi = None


def _streams(seed: int, names):
    ss = np.random.SeedSequence(int(seed))
    kids = ss.spawn(len(names))
    return {n: np.random.Generator(np.random.PCG64(k)) for n, k in zip(names, kids)}


def gaussian_field(rng: np.random.Generator, h: int, w: int, sigma: float = 1.0,
                   slope: float = 1.0) -> np.ndarray:
    """Periodic Gaussian random field whose power falls as 1/|f|^(2*slope)
    (slope 1: the 1/f^2 clutter spectrum), zero mean, standard deviation sigma."""
    fy = np.fft.fftfreq(h)[:, None]
    fx = np.fft.fftfreq(w)[None, :]
    f = np.sqrt(fx * fx + fy * fy)
    amp = np.zeros_like(f)
    amp[f > 0] = 1.0 / f[f > 0] ** slope
    noise = rng.normal(size=(h, w)) + 1j * rng.normal(size=(h, w))
    field = np.real(np.fft.ifft2(noise * amp))
    field -= field.mean()
    sd = field.std()
    return field * (sigma / sd if sd > 0 else 0.0)


def _psf_stamp(img: np.ndarray, cx: float, cy: float, amp: float, sigma: float,
               trunc: float = 4.0) -> None:
    """Add a Gaussian point spread function sampled at pixel centres,
    truncated at trunc*sigma."""
    h, w = img.shape
    r = int(np.ceil(trunc * sigma))
    x0, x1 = int(np.floor(cx)) - r, int(np.floor(cx)) + r + 1
    y0, y1 = int(np.floor(cy)) - r, int(np.floor(cy)) + r + 1
    xs = np.arange(max(x0, 0), min(x1, w))
    ys = np.arange(max(y0, 0), min(y1, h))
    if xs.size == 0 or ys.size == 0:
        return
    dx = xs[None, :] - cx
    dy = ys[:, None] - cy
    d2 = dx * dx + dy * dy
    g = amp * np.exp(-0.5 * d2 / (sigma * sigma))
    g[d2 > (trunc * sigma) ** 2] = 0.0
    img[ys[0]:ys[-1] + 1, xs[0]:xs[-1] + 1] += g


@dataclass
class Scene:
    frames: np.ndarray          # [T, H, W] float32
    velocity: np.ndarray        # [H, W, 2] true background velocity (vx, vy), px/frame
    targets: np.ndarray         # [n, T, 2] target centres (x, y) per frame
    band_mask: np.ndarray | None = None   # [T, H, W] bool, pixels covered by the band
    target_snr: np.ndarray | None = None  # [n] target amplitude / noise sigma, where defined


def translate_scene(seed: int, H: int = 64, W: int = 64, T: int = 32,
                    v=(1, -2), n_targets: int = 3, clutter_sigma: float = 10.0,
                    dc: float = 100.0, noise_sigma: float = 1.0, target_snr: float = 5.0,
                    psf_sigma: float = 0.7, max_target_speed: float = 3.0) -> Scene:
    """Clutter translated by an integer velocity v = (vx, vy) px/frame."""
    vx, vy = int(v[0]), int(v[1])
    st = _streams(seed, ["texture", "targets", "noise"])
    ch, cw = 2 * H, 2 * W
    canvas = gaussian_field(st["texture"], ch, cw, clutter_sigma) + dc
    frames = np.zeros((T, H, W), np.float64)
    for t in range(T):
        # I_t(x, y) = G(x - vx t, y - vy t) on the periodic canvas
        frames[t] = np.roll(canvas, shift=(vy * t, vx * t), axis=(0, 1))[:H, :W]
    tg = _targets(st["targets"], n_targets, H, W, T, max_target_speed)
    amp = target_snr * noise_sigma
    for t in range(T):
        for i in range(n_targets):
            _psf_stamp(frames[t], tg[i, t, 0], tg[i, t, 1], amp, psf_sigma)
    frames += st["noise"].normal(scale=noise_sigma, size=frames.shape)
    vel = np.zeros((H, W, 2))
    vel[..., 0], vel[..., 1] = vx, vy
    return Scene(frames.astype(np.float32), vel, tg)


def _targets(rng, n, H, W, T, vmax):
    pos0 = np.stack([rng.uniform(0.15 * W, 0.85 * W, n), rng.uniform(0.15 * H, 0.85 * H, n)], 1)
    ang = rng.uniform(0, 2 * np.pi, n)
    spd = rng.uniform(0, vmax, n)
    vel = np.stack([spd * np.cos(ang), spd * np.sin(ang)], 1)
    t = np.arange(T)[None, :, None]
    return pos0[:, None, :] + vel[:, None, :] * t


def smooth_velocity_field(rng, H: int, W: int, n_terms: int = 4, vmax: float = 3.0) -> np.ndarray:
    """v_c(x, y) = sum_i a_i sin(2 pi (p_i x / W + q_i y / H) + phi_i) per
    component c, p_i, q_i in {-2..2} not both zero, rescaled to max |v| = vmax."""
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    v = np.zeros((H, W, 2))
    for c in range(2):
        for _ in range(n_terms):
            while True:
                p, q = rng.integers(-2, 3, size=2)
                if p != 0 or q != 0:
                    break
            a = rng.uniform(-1, 1)
            ph = rng.uniform(0, 2 * np.pi)
            v[..., c] += a * np.sin(2 * np.pi * (p * xs / W + q * ys / H) + ph)
    mag = np.sqrt((v ** 2).sum(-1)).max()
    return v * (vmax / mag if mag > 0 else 0.0)


def flow_scene(seed: int, H: int = 512, W: int = 640, T: int = 200, n_targets: int = 20,
               clutter_sigma: float = 10.0, dc: float = 100.0, noise_sigma: float = 1.0,
               varying_noise: bool = False, snr=(2.0, 8.0), psf_sigma: float = 0.7,
               vmax: float = 3.0, band: bool = True, band_width=(40.0, 80.0),
               max_target_speed: float = 3.0) -> Scene:
    """Clutter advected by a smooth steady velocity field, an occluding band
    and additive targets.  I_t(x) = G(x + D_t(x)) with the displacement map
    D_t(x) = -v(x) + D_{t-1}(x - v(x)) (so I_t(x) = I_{t-1}(x - v(x)))."""
    if _ndi is None:
        raise RuntimeError("flow_scene needs scipy")
    st = _streams(seed, ["texture", "velocity", "band", "targets", "noise", "noise_map"])
    ch, cw = 2 * H, 2 * W
    G = gaussian_field(st["texture"], ch, cw, clutter_sigma) + dc
    v = smooth_velocity_field(st["velocity"], H, W, 4, vmax)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)

    # band: random orientation, width, own texture and velocity
    brng = st["band"]
    theta = brng.uniform(0, np.pi)
    bw = brng.uniform(*band_width)
    bc = np.array([brng.uniform(0.3 * W, 0.7 * W), brng.uniform(0.3 * H, 0.7 * H)])
    bsp = brng.uniform(0.5, vmax)
    bang = brng.uniform(0, 2 * np.pi)
    bv = np.array([bsp * np.cos(bang), bsp * np.sin(bang)])
    Gb = gaussian_field(brng, ch, cw, clutter_sigma) + dc + brng.uniform(-2, 2) * clutter_sigma
    nrm = np.array([np.cos(theta), np.sin(theta)])

    if varying_noise:
        s = gaussian_field(st["noise_map"], H, W, 1.0, slope=2.0)
        s = (s - s.min()) / max(s.max() - s.min(), 1e-12)
        sig = 0.5 + 1.5 * s
    else:
        sig = np.full((H, W), noise_sigma)

    tg = _targets(st["targets"], n_targets, H, W, T, max_target_speed)
    amps = st["targets"].uniform(snr[0], snr[1], n_targets) * noise_sigma

    # cubic-spline coefficients of the periodic canvases, computed once
    Gc = _ndi.spline_filter(G, order=3, mode="grid-wrap")
    Gbc = _ndi.spline_filter(Gb, order=3, mode="grid-wrap")
    frames = np.zeros((T, H, W), np.float32)
    mask_all = np.zeros((T, H, W), bool)
    Dx = np.zeros((H, W))
    Dy = np.zeros((H, W))
    label = v.copy()
    for t in range(T):
        if t > 0:
            # D_t(x) = -v(x) + D_{t-1}(x - v(x)), bilinear on the smooth map
            cy, cx = ys - v[..., 1], xs - v[..., 0]
            Dx_prev = _ndi.map_coordinates(Dx, [cy, cx], order=1, mode="nearest")
            Dy_prev = _ndi.map_coordinates(Dy, [cy, cx], order=1, mode="nearest")
            Dx = -v[..., 0] + Dx_prev
            Dy = -v[..., 1] + Dy_prev
        img = _ndi.map_coordinates(Gc, [ys + Dy, xs + Dx], order=3, mode="grid-wrap", prefilter=False)
        if band:
            c_t = bc + bv * t
            dist = (xs - c_t[0]) * nrm[0] + (ys - c_t[1]) * nrm[1]
            m = np.abs(dist) < 0.5 * bw
            if m.any():
                bimg = _ndi.map_coordinates(Gbc, [ys[m] - bv[1] * t, xs[m] - bv[0] * t],
                                            order=3, mode="grid-wrap", prefilter=False)
                img[m] = bimg
            mask_all[t] = m
        for i in range(n_targets):
            _psf_stamp(img, tg[i, t, 0], tg[i, t, 1], amps[i], psf_sigma)
        img += st["noise"].normal(size=(H, W)) * sig
        frames[t] = img.astype(np.float32)
    if band:
        label[mask_all[-1]] = bv
    return Scene(frames, label, tg, mask_all, amps / noise_sigma)


def paper_scene(seed: int = 7, H: int = 64, W: int = 64, T: int = 64,
                n_comp: int = 25, v_clutter=(1.625, 0.625), v_target=(-0.625, -0.375),
                noise_sigma: float = 0.1) -> Scene:
    """The synthetic scene of the paper's simulation section: 25 sinusoids,
    frequencies uniform on [-2/9, 2/9] cycles/pixel per axis, random phase,
    magnitude 0.1, DC 10, translating at v_clutter; one occluding target of
    peak 1.0 with a Gaussian PSF (sigma 1 px) truncated below 0.1, centred in
    the final frame; white noise sigma 0.1."""
    st = _streams(seed, ["texture", "noise"])
    rng = st["texture"]
    f = rng.uniform(-2.0 / 9.0, 2.0 / 9.0, size=(n_comp, 2))
    ph = rng.uniform(0, 2 * np.pi, n_comp)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    frames = np.zeros((T, H, W))
    cx_end, cy_end = (W - 1) / 2.0, (H - 1) / 2.0
    tg = np.zeros((1, T, 2))
    for t in range(T):
        xx = xs - v_clutter[0] * t
        yy = ys - v_clutter[1] * t
        img = 10.0 + 0.1 * np.cos(2 * np.pi * (f[:, 0, None, None] * xx + f[:, 1, None, None] * yy)
                                  + ph[:, None, None]).sum(0)
        px = cx_end + v_target[0] * (t - (T - 1))
        py = cy_end + v_target[1] * (t - (T - 1))
        tg[0, t] = (px, py)
        g = np.exp(-0.5 * ((xs - px) ** 2 + (ys - py) ** 2))
        m = g >= 0.1
        img[m] = g[m]
        frames[t] = img
    frames += st["noise"].normal(scale=noise_sigma, size=frames.shape)
    vel = np.zeros((H, W, 2))
    vel[..., 0], vel[..., 1] = v_clutter
    return Scene(frames.astype(np.float32), vel, tg)


def grid(lo: float, hi: float, step: float) -> np.ndarray:
    """Uniform candidate grid lo, lo+step, ..., hi (inclusive)."""
    n = int(round((hi - lo) / step)) + 1
    return lo + step * np.arange(n)
