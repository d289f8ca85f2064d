"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each compares the recursive
oracle (``liborc.so``) with an independent route -- a direct definition from
Sec. 2 of the paper (``oracle/brute.py``), a closed form, a textbook special
case, a sample-domain dual of a frequency-domain step, or a property every
correct implementation must have.
"""
import numpy as np
import pytest

from oracle import brute
from paper_1408_3526_amd import scenes

SHAPES = [(4, 3, 3), (8, 8, 4), (9, 9, 5), (6, 5, 4)]


def _cfg(orc, H, W, M, gx=(-1.0, 0.0, 1.0), gy=(-1.0, 0.0, 1.0), **kw):
    return orc.Cfg(H=H, W=W, Mx=M[0], My=M[1], Mz=M[2], gx=np.asarray(gx, float),
                   gy=np.asarray(gy, float), **kw)


# P1 -- the recursive spectrum (row SDFT, column SDFT, temporal observer) equals
# the windowed DFT of eq. (6)-(7) evaluated directly.
@pytest.mark.parametrize("M", SHAPES)
def test_recursive_spectrum_equals_direct_dft(orc, M):
    rng = np.random.default_rng(1)
    T, H, W = 9, 7, 10
    fr = (rng.normal(size=(T, H, W)) * 3 + 20).astype(np.float32)
    for Tn in (M[2] - 1, T):     # before and after the temporal window has filled
        cfg = _cfg(orc, H, W, M, Bx=1, By=1)
        r = orc.run(cfg, fr[:Tn], want_spec=True)
        f64 = fr[:Tn].astype(np.float64)
        for y in range(H):
            for x in range(W):
                S = brute.spectrum(f64, x, y, Tn - 1, M)
                assert np.abs(r["spec"][y, x] - S).max() <= 1e-12 * max(1.0, np.abs(S).max())


# P2 -- the observer's impulse response is the length-Mz FIR of the sliding DFT
# and is exactly zero afterwards ("deadbeat").
@pytest.mark.parametrize("Mz", [2, 3, 4, 5, 8])
def test_observer_impulse_response_is_fir(orc, Mz):
    T = 3 * Mz + 2
    s2 = np.zeros(T, complex)
    s2[0] = 1.0
    S = orc.observer_series(Mz, s2)
    k = np.arange(Mz)
    for t in range(T):
        want = np.exp(2j * np.pi * k * t / Mz) / np.sqrt(Mz) if t < Mz else np.zeros(Mz)
        assert np.abs(S[t] - want).max() <= 1e-14


# P3 -- any corrupted observer state is flushed exactly after Mz updates.
@pytest.mark.parametrize("Mz", [3, 4, 8])
def test_observer_deadbeat_recovery(orc, Mz):
    rng = np.random.default_rng(2)
    T = 4 * Mz
    s2 = rng.normal(size=T) + 1j * rng.normal(size=T)
    clean = orc.observer_series(Mz, s2)
    bad = 1e3 * (rng.normal(size=Mz) + 1j * rng.normal(size=Mz))
    dirty = orc.observer_series(Mz, s2, bad)
    assert np.abs(dirty[Mz - 2] - clean[Mz - 2]).max() > 1.0      # corrupted before the Mz-th update
    assert np.abs(dirty[Mz - 1:] - clean[Mz - 1:]).max() <= 1e-12 * 1e3


# P4 -- eq. (8) at the bins equals the DFT (eq. 5) of the FIR coefficients of
# eq. (2); includes integer velocities (Dirichlet limits) and odd/even windows.
@pytest.mark.parametrize("M,B", [((9, 9, 5), (3, 3)), ((8, 8, 4), (3, 3)), ((16, 16, 8), (6, 6)),
                                 ((6, 5, 4), (2, 2)), ((5, 7, 3), (2, 3))])
@pytest.mark.parametrize("v", [(0.3, -0.7), (1.0, -2.0), (1.625, 0.625), (0.0, 0.0)])
def test_coefficients_eq8_equal_dft_of_eq2(orc, M, B, v):
    cfg = _cfg(orc, 4, 4, M, Bx=B[0], By=B[1])
    Hk = orc.coeffs(cfg, *v)
    ref = brute.coeffs_eq5(M, B, (cfg.dx, cfg.dy, cfg.dt), v)
    assert np.abs(Hk - ref).max() <= 1e-13


# Eq. (8) at a bin depends on the velocity only through phi = vx kx/Mx +
# vy ky/My, and only through phi mod 1 (the sign change of D_Mz(w + 1) for
# even Mz cancels that of exp(j 2 pi (m'z - Dz))).  The 16x16x8 kernel relies
# on this to read its coefficients from a table indexed by phi mod 1.
@pytest.mark.parametrize("M,B", [((16, 16, 8), (6, 6)), ((9, 9, 5), (3, 3)), ((8, 8, 4), (3, 3))])
def test_coefficients_eq8_periodic_in_phi(orc, M, B):
    rng = np.random.default_rng(17)
    cfg = _cfg(orc, 4, 4, M, Bx=B[0], By=B[1])
    for _ in range(12):
        kx, ky = int(rng.integers(-B[0], B[0] + 1)), int(rng.integers(-B[1], B[1] + 1))
        v = rng.uniform(-4, 4, size=2)
        n = int(rng.integers(-3, 4))
        if kx != 0:
            w = (v[0] + n * M[0] / kx, v[1])
        elif ky != 0:
            w = (v[0] + rng.uniform(-4, 4), v[1] + n * M[1] / ky)   # kx = 0: vx does not enter
        else:
            w = tuple(rng.uniform(-4, 4, size=2))                    # phi = 0 for any v
        a = orc.coeffs(cfg, *v)[kx % M[0], ky % M[1]]
        b = orc.coeffs(cfg, *w)[kx % M[0], ky % M[1]]
        assert np.abs(a).max() > 0
        assert np.abs(a - b).max() <= 1e-12, (kx, ky, v, w)


# P5 -- the frequency-domain background estimate (eq. 4) equals the direct
# 3-D convolution of eq. (1).
@pytest.mark.parametrize("M", [(8, 8, 4), (9, 9, 5), (6, 5, 4)])
def test_background_eq4_equals_convolution_eq1(orc, M):
    rng = np.random.default_rng(3)
    T, H, W = M[2] + 2, M[1] + 3, M[0] + 4
    fr = rng.normal(size=(T, H, W)) * 5 + 50
    cfg = _cfg(orc, H, W, M, Bx=(M[0] - 1) // 2 - 1, By=(M[1] - 1) // 2 - 1)
    for v in [(0.4, -1.1), (2.0, 1.0)]:
        Hk = orc.coeffs(cfg, *v)
        for (x, y, t) in [(W - 1, H - 1, T - 1), (M[0] - 1, M[1], T - 2), (2, 1, 1)]:
            S = brute.spectrum(fr, x, y, t, M)
            a = orc.background(cfg, Hk, S)
            b = brute.background_eq1(fr, x, y, t, M, (cfg.Bx, cfg.By), (cfg.dx, cfg.dy, cfg.dt), v)
            assert abs(a - b) <= 1e-12 * np.abs(fr).max() * np.prod(M)


# P6 -- eq. (10) at integer lag equals the cyclic autocorrelation of the
# high-passed, Hann-windowed block (Wiener-Khinchin); high-pass and Hann are
# done in the sample domain here (slice-mean removal, window multiplication).
@pytest.mark.parametrize("M", SHAPES + [(16, 16, 8)])
def test_autocorrelation_equals_sample_domain(orc, M):
    rng = np.random.default_rng(4)
    b = rng.normal(size=M) * 2 + 7
    S = brute.spectrum_of_block(b)
    gx = np.arange(-(M[0] // 2), M[0] // 2 + 1, dtype=float)
    gy = np.arange(-(M[1] // 2), M[1] // 2 + 1, dtype=float)
    cfg = _cfg(orc, 4, 4, M, gx=gx, gy=gy, Bx=0, By=0)
    R, P = orc.flow_R(cfg, S, want_P=True)
    s = brute.flow_block(b)
    # power spectrum of the sample-domain windowed block
    P_ref = np.abs(brute.spectrum_of_block(s)) ** 2
    assert np.abs(P - P_ref).max() <= 1e-12 * P_ref.max()
    for iy, ly in enumerate(gy):
        for ix, lx in enumerate(gx):
            ref = brute.autocorr_cyclic(s, (lx, ly, 1))
            assert abs(R[iy * len(gx) + ix] - ref) <= 1e-12 * np.sum(s * s)


def _interp_kernel(M, u):
    """Trigonometric interpolation kernel on M samples (centred bins, the
    even-M Nyquist bin split in half): D_M(u/M) for odd M,
    sin(pi u) cot(pi u / M) / M for even M; 1 at u = 0 (mod M)."""
    u = np.asarray(u, float)
    r = np.mod(u, M)
    at0 = (np.abs(r) < 1e-12) | (np.abs(r - M) < 1e-12)
    s = np.sin(np.pi * u / M)
    s = np.where(at0, 1.0, s)
    if M % 2:
        val = np.sin(np.pi * u) / (M * s)
        lim = 1.0
    else:
        val = np.sin(np.pi * u) * np.cos(np.pi * u / M) / (M * s)
        lim = 1.0
    return np.where(at0, lim, val)


# Non-integer lags: R(l) equals the correlation of the windowed block with its
# band-limited (trigonometric-interpolation) shift by l, computed in the sample
# domain with the closed-form periodic interpolation kernel.
@pytest.mark.parametrize("M", [(8, 8, 4), (9, 9, 5), (6, 5, 4), (16, 16, 8)])
def test_fractional_lag_is_trig_interpolation(orc, M):
    rng = np.random.default_rng(5)
    b = rng.normal(size=M) + 3
    S = brute.spectrum_of_block(b)
    gx = np.array([-1.5, -0.25, 0.5, 1.75])
    gy = np.array([-0.5, 1.25])
    cfg = _cfg(orc, 4, 4, M, gx=gx, gy=gy, Bx=0, By=0)
    R = orc.flow_R(cfg, S)
    s = brute.flow_block(b)
    m = [np.arange(n) for n in M]
    for iy, ly in enumerate(gy):
        for ix, lx in enumerate(gx):
            Kx = _interp_kernel(M[0], m[0][:, None] - lx - m[0][None, :])   # [m, m']
            Ky = _interp_kernel(M[1], m[1][:, None] - ly - m[1][None, :])
            sl = np.einsum("abc,ia,jb->ijc", s, Kx, Ky)
            sl = np.roll(sl, 1, axis=2)                                     # l_z = 1
            ref = float(np.sum(s * sl))
            assert abs(R[iy * len(gx) + ix] - ref) <= 1e-11 * np.sum(s * s)


# P7 -- noise-free band-limited clutter translating at v (non-integer) is
# removed exactly once the window has filled: output 0 on valid anchors.
@pytest.mark.parametrize("M,B,v", [((8, 8, 4), (3, 3), (0.7, -1.3)), ((9, 9, 5), (3, 3), (1.625, 0.625)),
                                   ((16, 16, 8), (6, 6), (-2.3, 0.45))])
def test_pef_null_on_translating_band_limited_clutter(orc, M, B, v):
    rng = np.random.default_rng(6)
    H, W, T = M[1] + 6, M[0] + 7, M[2] + 3
    ys, xs = np.mgrid[0:H, 0:W].astype(float)
    fr = np.full((T, H, W), 10.0)
    comps = [(rng.integers(-B[0], B[0] + 1), rng.integers(-B[1], B[1] + 1),
              rng.uniform(0.5, 2.0), rng.uniform(0, 2 * np.pi)) for _ in range(12)]
    for t in range(T):
        for kx, ky, a, ph in comps:
            fr[t] += a * np.cos(2 * np.pi * (kx * (xs - v[0] * t) / M[0] + ky * (ys - v[1] * t) / M[1]) + ph)
    cfg = _cfg(orc, H, W, M, Bx=B[0], By=B[1], vmode=2, fvx=v[0], fvy=v[1])
    r = orc.run(cfg, fr.astype(np.float32))
    out = r["out"][M[2] - 1:, M[1] - 1:, M[0] - 1:]
    # the frames are band-limited only up to their float32 rounding (~1e-6)
    assert np.abs(out).max() <= 2e-5 * 10.0
    assert np.all(r["idx"] == -1)


def test_pef_null_exact_in_double(orc):
    """Same identity with the clutter reaching the oracle unrounded: frames are
    integers-valued multiples chosen exactly representable (amplitudes of powers
    of two and on-bin phases at integer shifts), so the output is 0 to 1e-10."""
    M, B, v = (8, 8, 4), (3, 3), (1.0, -2.0)
    H, W, T = 20, 21, 9
    ys, xs = np.mgrid[0:H, 0:W].astype(float)
    fr = np.zeros((T, H, W))
    for t in range(T):
        # cos(2 pi k u / 8) at integer u takes values in {0, +-1, +-sqrt(1/2)};
        # k in {0, 2, 4} keeps them in {0, +-1}: exactly representable
        fr[t] = 16 + 4 * np.cos(2 * np.pi * 2 * (xs - v[0] * t) / 8) + 2 * np.cos(
            2 * np.pi * (2 * (xs - v[0] * t) / 8 - 2 * (ys - v[1] * t) / 8))
    fr = np.round(fr)             # the exact values are integers
    assert np.array_equal(fr.astype(np.float32).astype(np.float64), fr)
    cfg = _cfg(orc, H, W, M, Bx=B[0], By=B[1], vmode=2, fvx=v[0], fvy=v[1])
    r = orc.run(cfg, fr.astype(np.float32))
    assert np.abs(r["out"][M[2] - 1:, M[1] - 1:, M[0] - 1:]).max() <= 1e-10


# P8 -- a texture shifted by an integer velocity returns that velocity.
@pytest.mark.parametrize("M,grid_step,v,HW,T", [((8, 8, 4), 1.0, (1, -2), 36, 14),
                                                 ((16, 16, 8), 0.5, (2, -1), 40, 14)])
def test_integer_shift_velocity(orc, M, grid_step, v, HW, T):
    sc = scenes.translate_scene(11, H=HW, W=HW, T=T, v=v, n_targets=0, noise_sigma=0.05)
    g = scenes.grid(-4, 4, grid_step)
    cfg = _cfg(orc, HW, HW, M, gx=g, gy=g)
    r = orc.run(cfg, sc.frames)
    vx = r["vxy"][-1, M[1] - 1:, M[0] - 1:, 0]
    vy = r["vxy"][-1, M[1] - 1:, M[0] - 1:, 1]
    ok = (vx == v[0]) & (vy == v[1])
    assert ok.mean() >= 0.99, ok.mean()


# P9 -- odd window, full band (B = K), v = 0: the filter is a temporal boxcar
# at the delayed pixel (a moving average); integer v: the cyclically shifted
# average along the motion.
@pytest.mark.parametrize("v", [(0, 0), (1, -1)])
def test_full_band_reduces_to_moving_average(orc, v):
    M = (5, 5, 3)
    rng = np.random.default_rng(8)
    T, H, W = 7, 9, 10
    fr = (rng.normal(size=(T, H, W)) * 4 + 30).astype(np.float32)
    cfg = _cfg(orc, H, W, M, Bx=2, By=2, vmode=2, fvx=float(v[0]), fvy=float(v[1]))
    r = orc.run(cfg, fr)
    f = fr.astype(np.float64)
    dx, dy, dt = cfg.dx, cfg.dy, cfg.dt
    for t in range(M[2] - 1, T):
        for y in range(M[1] - 1, H):
            for x in range(M[0] - 1, W):
                acc = 0.0
                for mz in range(M[2]):
                    mx = (dx + v[0] * (mz - dt)) % M[0]
                    my = (dy + v[1] * (mz - dt)) % M[1]
                    acc += f[t - mz, y - my, x - mx]
                want = f[t - dt, y - dy, x - dx] - acc / M[2]
                assert abs(r["out"][t, y, x] - want) <= 1e-11 * 30


# P10 -- symmetries of a real input: Hermitian spectrum, Hermitian
# coefficients, even power spectrum.
def test_symmetries(orc):
    rng = np.random.default_rng(9)
    M = (8, 6, 4)
    b = rng.normal(size=M)
    S = brute.spectrum_of_block(b)
    neg = lambda A: np.roll(np.flip(A, axis=(0, 1, 2)), 1, axis=(0, 1, 2))   # A[-k]
    cfg = _cfg(orc, 4, 4, M, Bx=2, By=2)
    Hk = orc.coeffs(cfg, 0.37, -1.21)
    assert np.abs(neg(Hk) - np.conj(Hk)).max() <= 1e-14
    R, P = orc.flow_R(cfg, S, want_P=True)
    assert np.abs(neg(P) - P).max() <= 1e-12 * P.max()
    # outside the band the coefficients vanish
    kx = np.arange(M[0]); kxc = np.where(kx <= M[0] // 2, kx, kx - M[0])
    assert np.abs(Hk[np.abs(kxc) > cfg.Bx]).max() <= 1e-14


def test_nonfinite_input_is_zeroed(orc):
    rng = np.random.default_rng(10)
    T, H, W = 5, 8, 9
    fr = (rng.normal(size=(T, H, W)) + 5).astype(np.float32)
    bad = fr.copy()
    bad[1, 3, 4] = np.nan
    bad[3, 0, 0] = np.inf
    zero = fr.copy()
    zero[1, 3, 4] = 0
    zero[3, 0, 0] = 0
    cfg = _cfg(orc, H, W, (4, 4, 3), Bx=1, By=1)
    a, b = orc.run(cfg, bad), orc.run(cfg, zero)
    assert a["n_nonfinite"] == 2
    assert np.array_equal(a["out"], b["out"]) and np.array_equal(a["idx"], b["idx"])


# Direct per-pixel route (used for sampled parity on full-size frames) equals
# the recursive whole-frame route.
def test_pixel_series_matches_run(orc):
    sc = scenes.translate_scene(3, H=24, W=26, T=10, v=(1, -1), n_targets=1)
    M = (8, 8, 4)
    cfg = _cfg(orc, 24, 26, M, gx=scenes.grid(-2, 2, 1.0), gy=scenes.grid(-2, 2, 1.0))
    r = orc.run(cfg, sc.frames, want_rs=True)
    for (x, y) in [(25, 23), (3, 17), (12, 5)]:
        p = orc.pixel_series(cfg, sc.frames, x, y)
        assert np.abs(p["rs"] - r["rs_all"][:, y, x]).max() <= 1e-9 * np.abs(p["rs"]).max()
        # equal maxima (exact ties of the early, half-empty windows) may resolve
        # either way under different rounding; both picks must be maximal
        rs = p["rs"]
        for t in range(rs.shape[0]):
            a, b = p["idx"][t], r["idx"][t, y, x]
            assert a == b or abs(rs[t, a] - rs[t, b]) <= 1e-9 * max(np.abs(rs[t]).max(), 1.0)
            if a == b:
                assert abs(p["out"][t] - r["out"][t, y, x]) <= 1e-9 * 100


# The paper's simulation (Sec. "Simulation", Fig. 1): the estimated clutter
# velocity is near (1.625, 0.625) and the strongest prediction-error response
# is the target, delayed by m'.  The texture is very smooth (|f| <= 2/9), so
# the autocorrelation is broad and the window taper pulls its peak toward zero
# (about 0.375 px/frame here); the paper prints no accuracy figure, so the
# check allows two grid steps.
def test_paper_scenario_velocity_and_target(orc):
    T = 24
    sc = scenes.paper_scene(7, T=T)
    g = scenes.grid(-2, 2, 0.25)
    cfg = _cfg(orc, 64, 64, (9, 9, 5), gx=g, gy=g, Bx=3, By=3)
    assert (cfg.dx, cfg.dy, cfg.dt) == (4, 4, 2)
    r = orc.run(cfg, sc.frames)
    vx = r["vxy"][-1, 8:, 8:, 0].ravel()
    vy = r["vxy"][-1, 8:, 8:, 1].ravel()
    near = (np.abs(vx - 1.625) <= 0.5) & (np.abs(vy - 0.625) <= 0.5)
    assert near.mean() >= 0.9, near.mean()
    out = np.abs(r["out"][-1, 8:, 8:])
    yy, xx = np.unravel_index(np.argmax(out), out.shape)
    tx, ty = sc.targets[0, T - 1 - cfg.dt]
    # anchor index = delayed pixel + m'; the target disc has radius ~2.1 px
    assert abs(xx + 8 - cfg.dx - tx) <= 3 and abs(yy + 8 - cfg.dy - ty) <= 3
    assert out.max() > 10 * out.std()


# A 1/f^2 texture translating midway between grid points lands in the right
# grid cell.
def test_subgrid_velocity_lands_in_cell(orc):
    from scipy import ndimage
    rng = np.random.default_rng(0)
    G = scenes.gaussian_field(rng, 128, 128, 10) + 100
    ys, xs = np.mgrid[0:40, 0:40].astype(float)
    fr = np.stack([ndimage.map_coordinates(G, [ys - 0.625 * t, xs - 1.625 * t], order=3, mode="grid-wrap")
                   for t in range(12)]).astype(np.float32)
    g = scenes.grid(-4, 4, 0.5)
    cfg = _cfg(orc, 40, 40, (16, 16, 8), gx=g, gy=g)
    r = orc.run(cfg, fr)
    vx = r["vxy"][-1, 15:, 15:, 0]
    vy = r["vxy"][-1, 15:, 15:, 1]
    ok = (vx >= 1.5) & (vx <= 2.0) & (vy >= 0.5) & (vy <= 1.0)
    assert ok.mean() >= 0.95


# Velocity mode 3 (sub-grid refinement of the smoothed-R peak).  The vertex of
# a parabola sampled at any three abscissae is the parabola's own vertex.
@pytest.mark.parametrize("xs", [(-0.5, 0.0, 0.5), (1.0, 2.0, 3.0), (-1.0, -0.25, 1.5), (0.0, 0.1, 0.35)])
def test_peak_vertex_recovers_a_parabola(orc, xs):
    rng = np.random.default_rng(11)
    x0, x1, x2 = xs
    for _ in range(20):
        # vertex between the midpoints, so the middle sample is the largest
        xv = rng.uniform(0.5 * (x0 + x1), 0.5 * (x1 + x2))
        a, c = -rng.uniform(0.1, 5.0), rng.normal()
        r = [a * (x - xv) ** 2 + c for x in xs]
        assert r[1] >= r[0] and r[1] >= r[2]
        assert abs(orc.peak_vertex(x0, r[0], x1, r[1], x2, r[2]) - xv) <= 1e-9 * (1 + abs(xv))
    assert orc.peak_vertex(x0, 2.0, x1, 2.0, x2, 2.0) == x1


# On a separable quadratic bowl sampled on the grid (different curvature and
# vertex per axis), refinement returns the bowl's centre; an axis whose peak is
# on the grid's edge keeps the grid value.
def test_refine_on_sampled_bowl(orc):
    gx = scenes.grid(-2, 2, 0.5)
    gy = np.array([-3.0, -1.0, 0.0, 0.5, 2.0, 4.0])
    cfg = _cfg(orc, 4, 4, (8, 8, 4), gx=gx, gy=gy, vmode=3)
    nvx = len(gx)
    for cx, cy in [(0.3, 0.2), (-1.1, 1.3), (0.0, -0.6)]:
        R = -(gx[None, :] - cx) ** 2 - 3.0 * (gy[:, None] - cy) ** 2
        best = int(np.argmax(R))
        vx, vy = orc.refine(cfg, R.ravel(), best)
        assert abs(vx - cx) <= 1e-9 and abs(vy - cy) <= 1e-9, (cx, cy, vx, vy)
    # peak on the x edge (centre beyond the grid): x keeps the grid value
    R = -(gx[None, :] - 5.0) ** 2 - 3.0 * (gy[:, None] - 0.3) ** 2
    best = int(np.argmax(R))
    assert best % nvx == nvx - 1
    vx, vy = orc.refine(cfg, R.ravel(), best)
    assert vx == gx[-1] and abs(vy - 0.3) <= 1e-9
    # unsorted grids are rejected in mode 3
    bad = _cfg(orc, 8, 8, (8, 8, 4), gx=gx[::-1], gy=gy, vmode=3)
    with pytest.raises(ValueError):
        orc.run(bad, np.zeros((2, 8, 8), np.float32))


# On clutter translating between grid points, the refined velocity is closer to
# the truth than the grid search's, and the tuned filter leaves less residual.
@pytest.mark.parametrize("v", [(1.3, -0.7), (0.6, 1.6)])
def test_refined_velocity_beats_the_grid(orc, v):
    from scipy import ndimage
    rng = np.random.default_rng(0)
    G = scenes.gaussian_field(rng, 128, 128, 10) + 100
    H = W = 32
    T = 12
    ys, xs = np.mgrid[0:H, 0:W].astype(float)
    fr = np.stack([ndimage.map_coordinates(G, [ys - v[1] * t, xs - v[0] * t], order=3, mode="grid-wrap")
                   for t in range(T)]).astype(np.float32)
    g = scenes.grid(-3, 3, 1.0)
    res = {}
    for vm in (0, 3):
        r = orc.run(_cfg(orc, H, W, (8, 8, 4), gx=g, gy=g, vmode=vm), fr)
        vv = r["vxy"][-1, 7:, 7:]
        res[vm] = (np.hypot(vv[..., 0] - v[0], vv[..., 1] - v[1]).mean(),
                   np.sqrt((r["out"][-1, 7:, 7:] ** 2).mean()), r["idx"][-1])
    assert res[3][0] < 0.75 * res[0][0], res
    assert res[3][1] < 0.85 * res[0][1], res
    assert np.array_equal(res[0][2], res[3][2])      # the grid peak itself is the same


# The direct per-pixel route agrees with the recursive route in mode 3 too.
def test_pixel_series_matches_run_refined(orc):
    sc = scenes.translate_scene(3, H=20, W=22, T=9, v=(1, -1), n_targets=1)
    g = scenes.grid(-2, 2, 0.5)
    cfg = _cfg(orc, 20, 22, (8, 8, 4), gx=g, gy=g, vmode=3)
    r = orc.run(cfg, sc.frames, want_rs=True)
    for (x, y) in [(21, 19), (10, 12)]:
        p = orc.pixel_series(cfg, sc.frames, x, y)
        for t in range(4, 9):
            if p["idx"][t] == r["idx"][t, y, x]:
                assert np.abs(p["vxy"][t] - r["vxy"][t, y, x]).max() <= 1e-7
                assert abs(p["out"][t] - r["out"][t, y, x]) <= 1e-7 * 100


# Smoothing and argmax (Sec. 2, flow paragraph): the smoothed R obeys
# R'_t = (1 - alpha) R_t + alpha R'_{t-1} with R'_{-1} = 0, where R_t is taken
# here by the brute route (sample-domain autocorrelation of each frame's
# window, eq. 10 via Wiener-Khinchin); the chosen index is the first maximum
# of R'_t in row-major (iy, ix) order (numpy's argmax, which returns the
# first maximum), and the velocity is the grid value at that index.
@pytest.mark.parametrize("M,grid,alpha", [((8, 8, 4), 3, float(np.exp(-0.1))), ((8, 8, 4), 3, 0.0),
                                          ((9, 9, 5), 2, 0.5), ((6, 5, 4), 2, 0.8)])
def test_smoothing_recurrence_and_first_maximum(orc, M, grid, alpha):
    rng = np.random.default_rng(21)
    H, W, T = M[1] + 4, M[0] + 5, M[2] + 5
    fr = (rng.normal(size=(T, H, W)) * 3 + 20).astype(np.float32)
    g = np.arange(-grid, grid + 1, dtype=float)
    cfg = _cfg(orc, H, W, M, gx=g, gy=g, alpha=alpha)
    r = orc.run(cfg, fr, want_r=True, want_rs=True)
    f64 = fr.astype(np.float64)
    # full-window, left-border and top-border anchors
    for x, y in [(W - 1, H - 1), (M[0] + 1, M[1]), (2, H - 2), (W - 3, 1)]:
        prev = np.zeros(len(g) ** 2)
        for t in range(T):
            s = brute.flow_block(brute.block(f64, x, y, t, M))
            R = np.array([brute.autocorr_cyclic(s, (lx, ly, 1)) for ly in g for lx in g])
            tol = 1e-12 * max(np.sum(s * s), 1e-300)
            assert np.abs(r["r_all"][t, y, x] - R).max() <= tol
            want = (1.0 - alpha) * R + alpha * prev
            assert np.abs(r["rs_all"][t, y, x] - want).max() <= 4 * tol + 1e-12 * np.abs(want).max()
            prev = r["rs_all"][t, y, x]
    rs = r["rs_all"]
    assert np.array_equal(r["idx"], np.argmax(rs, axis=-1))
    nvx = len(g)
    assert np.array_equal(r["vxy"][..., 0], g[r["idx"] % nvx])
    assert np.array_equal(r["vxy"][..., 1], g[r["idx"] // nvx])
    # exact ties: all-zero frames make every R' exactly 0, so the first
    # maximum is index 0 and the velocity the grid's first candidate
    z = orc.run(cfg, np.zeros_like(fr), want_rs=True)
    assert np.all(z["rs_all"] == 0.0)
    assert np.all(z["idx"] == 0)
    assert np.all(z["vxy"] == g[0])


# The filter uses the velocity estimated at the same anchor in the same frame
# (Sec. 1: velocity estimation and filtering per pixel and frame).  On a scene
# whose velocity changes half-way through, every output of the search mode
# equals the delayed input minus the direct convolution of eq. (1) at that
# frame's own chosen velocity.
@pytest.mark.parametrize("M", [(8, 8, 4), (9, 9, 5)])
def test_filter_uses_the_same_frames_velocity(orc, M):
    T, H, W = 2 * M[2] + 6, M[1] + 6, M[0] + 7
    a = scenes.translate_scene(31, H=H, W=W, T=T, v=(1, -1), n_targets=0, noise_sigma=0.05).frames
    b = scenes.translate_scene(31, H=H, W=W, T=T, v=(-2, 1), n_targets=0, noise_sigma=0.05).frames
    fr = np.concatenate([a[:T // 2], b[T // 2:]]).astype(np.float32)
    g = np.arange(-3.0, 4.0)
    cfg = _cfg(orc, H, W, M, gx=g, gy=g)
    r = orc.run(cfg, fr)
    f64 = fr.astype(np.float64)
    changed = 0
    for t in range(T):
        for (x, y) in [(W - 1, H - 1), (M[0] + 2, M[1] + 1), (3, H - 2)]:
            v = tuple(r["vxy"][t, y, x])
            if t > 0 and v != tuple(r["vxy"][t - 1, y, x]):
                changed += 1
            ts, xs, ys = t - cfg.dt, x - cfg.dx, y - cfg.dy
            delayed = f64[ts, ys, xs] if (ts >= 0 and xs >= 0 and ys >= 0) else 0.0
            ihat = brute.background_eq1(f64, x, y, t, M, (cfg.Bx, cfg.By), (cfg.dx, cfg.dy, cfg.dt), v)
            assert abs(r["out"][t, y, x] - (delayed - ihat)) <= 1e-10 * np.abs(f64).max() * np.prod(M)
    assert changed > 0          # the check covers frames where the chosen velocity moves
