"""GPU parity of velocity mode 3 (the smoothed-R peak refined between grid
points, eq. (8) evaluated at the refined velocity) against the FP64 oracle.

Bars, on top of the plain-search bars of test_gpu_parity.py:
  * grid peak index: identical on >= 99.9% of non-tied anchors (same tie rule);
  * refined velocity: within 2e-3 grid steps of the oracle's wherever the
    indices agree and each refined axis is well conditioned, i.e. the peak
    stands above its two neighbours on that axis by >= 1e-2 of the R scale in
    total (the vertex moves by about h dR / curvature for a change dR of the
    three values, and FP32 evaluation changes them by ~1e-6 of the scale);
    an axis whose peak is on the grid's edge keeps the grid value exactly;
  * prediction-error output: <= 1e-3 x frame RMS on those anchors.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1408_3526_amd import scenes  # noqa: E402


def _binding():
    from paper_1408_3526_amd import binding
    binding.lib()
    return binding


def _cfg(orc, H, W, M, g, **kw):
    return orc.Cfg(H=H, W=W, Mx=M[0], My=M[1], Mz=M[2], gx=g, gy=g, vmode=3, **kw)


def run_gpu(frames, M, g, **kw):
    b = _binding()
    T, H, W = frames.shape
    f = b.Filter(H, W, *M, g, g, velocity_mode=b.VEL_REFINED, **kw)
    dev = torch.from_numpy(np.ascontiguousarray(frames)).cuda()
    out, idx, vxy = [], [], []
    for t in range(T):
        f.push_frame(dev[t])
        out.append(f.output().cpu().numpy())
        v, i = f.velocity()
        vxy.append(v.cpu().numpy())
        idx.append(i.cpu().numpy())
    res = {"out": np.stack(out), "idx": np.stack(idx), "vxy": np.stack(vxy), "lattice": f.coeff_lattice()}
    torch.cuda.synchronize()
    f.close()
    return res


def _take(a, i):
    return np.take_along_axis(a, i[..., None], -1)[..., 0]


def check_refined(gres, rs_all, en_all, oidx, ovxy, oout, frames, g):
    nvx = nvy = len(g)
    h = float(np.min(np.diff(g))) if len(g) > 1 else 1.0
    n_well = 0
    for t in range(frames.shape[0]):
        rs = rs_all[t]
        srt = np.sort(rs, axis=-1)
        scale = np.maximum(np.maximum(np.abs(rs).max(axis=-1), 1e-3 * en_all[t]), 1e-30)
        tied = (srt[..., -1] - srt[..., -2]) <= 1e-4 * scale
        gi, oi = gres["idx"][t], oidx[t]
        agree = gi == oi
        frac = agree[~tied].mean() if (~tied).any() else 1.0
        assert frac >= 0.999, (t, frac)
        ix, iy = oi % nvx, oi // nvx
        r1 = _take(rs, oi)
        well = agree & ~tied
        for axis, inner, step in ((0, (ix > 0) & (ix < nvx - 1), 1), (1, (iy > 0) & (iy < nvy - 1), nvx)):
            lo = _take(rs, np.clip(oi - step, 0, rs.shape[-1] - 1)) - r1
            hi = _take(rs, np.clip(oi + step, 0, rs.shape[-1] - 1)) - r1
            curv = -(lo + hi) / scale
            well &= ~inner | (curv >= 1e-2)
            # an edge peak keeps the grid value exactly
            edge = agree & ~inner
            grid = (g[ix] if axis == 0 else g[iy]).astype(np.float32)
            assert np.array_equal(gres["vxy"][t][..., axis][edge], grid[edge])
        dv = np.abs(gres["vxy"][t].astype(np.float64) - ovxy[t]).max(axis=-1)
        if well.any():
            assert dv[well].max() <= 2e-3 * h, (t, dv[well].max())
            rms = float(np.sqrt(np.mean(frames[t].astype(np.float64) ** 2)))
            err = np.abs(gres["out"][t] - oout[t])[well]
            assert err.max() <= 1e-3 * rms, (t, err.max(), rms)
        # every refined velocity lies within half a grid step of its grid peak
        # (uniform grids; the vertex lies between the midpoints)
        ok = agree
        assert np.all(np.abs(gres["vxy"][t][..., 0][ok] - g[gi[ok] % nvx]) <= 0.5 * h + 1e-5)
        assert np.all(np.abs(gres["vxy"][t][..., 1][ok] - g[gi[ok] // nvx]) <= 0.5 * h + 1e-5)
        n_well += int(well.sum())
    return n_well


_ORC_CACHE = {}


def _oracle_run(orc, key, cfg, frames):
    if key not in _ORC_CACHE:
        _ORC_CACHE[key] = orc.run(cfg, frames, want_rs=True)
    return _ORC_CACHE[key]


@pytest.mark.parametrize("variant", [2, 1])
def test_refined_16x16x8(orc, variant):
    """16x16x8 window, 17x17 grid at 0.5 px/frame, non-uniform flow with an
    occluding band; both per-pixel kernels (wave per anchor, generic)."""
    T, H, W = 10, 24, 22
    sc = scenes.flow_scene(5, H=H, W=W, T=T, n_targets=2)
    g = scenes.grid(-4, 4, 0.5)
    M = (16, 16, 8)
    gres = run_gpu(sc.frames, M, g, kernel_variant=variant)
    assert gres["lattice"] == 0
    r = _oracle_run(orc, "16", _cfg(orc, H, W, M, g), sc.frames)
    n = check_refined(gres, r["rs_all"], r["en_all"], r["idx"], r["vxy"], r["out"], sc.frames, g)
    assert n > 0.5 * T * H * W, n


def test_refined_paper_configuration(orc):
    """The paper's 9x9x5 window, B = 3, 0.25 px/frame grid, on its scene."""
    T = 16
    sc = scenes.paper_scene(7, T=T)
    g = scenes.grid(-2, 2, 0.25)
    M = (9, 9, 5)
    gres = run_gpu(sc.frames, M, g)
    r = orc.run(_cfg(orc, 64, 64, M, g), sc.frames, want_rs=True)
    n = check_refined(gres, r["rs_all"], r["en_all"], r["idx"], r["vxy"], r["out"], sc.frames, g)
    assert n > 0.5 * T * 64 * 64, n


@pytest.mark.parametrize("H,W,tile", [(33, 70, 8), (5, 6, 0), (1, 13, 4)])
def test_refined_ragged_8x8x4(orc, H, W, tile):
    rng = np.random.default_rng(H * 100 + W)
    T = 9
    fr = (scenes.gaussian_field(rng, 2 * H + 8, 2 * W + 8, 10.0)[:H, :W] + 100.0)
    fr = np.stack([np.roll(fr, (t, -t), (0, 1)) + rng.normal(size=(H, W)) for t in range(T)]).astype(np.float32)
    g = scenes.grid(-2, 2, 1.0)
    M = (8, 8, 4)
    gres = run_gpu(fr, M, g, tile_rows=tile)
    r = orc.run(_cfg(orc, H, W, M, g), fr, want_rs=True)
    check_refined(gres, r["rs_all"], r["en_all"], r["idx"], r["vxy"], r["out"], fr, g)


@pytest.mark.parametrize("variant", [2, 1])
def test_refined_nonuniform_grid(orc, variant):
    """A strictly increasing but non-uniform grid: the vertex through three
    unequally spaced points (both kernels)."""
    T, H, W = 9, 20, 23
    sc = scenes.flow_scene(11, H=H, W=W, T=T, n_targets=1, band_width=(4, 6))
    g = np.array([-3.5, -2.0, -1.2, -0.5, 0.0, 0.3, 0.9, 1.6, 2.5, 3.6])
    M = (16, 16, 8)
    gres = run_gpu(sc.frames, M, g, kernel_variant=variant)
    r = _oracle_run(orc, "nonuniform", _cfg(orc, H, W, M, g), sc.frames)
    nvx = len(g)
    n_well = 0
    for t in range(T):
        rs = r["rs_all"][t]
        srt = np.sort(rs, axis=-1)
        scale = np.maximum(np.maximum(np.abs(rs).max(axis=-1), 1e-3 * r["en_all"][t]), 1e-30)
        tied = (srt[..., -1] - srt[..., -2]) <= 1e-4 * scale
        agree = gres["idx"][t] == r["idx"][t]
        if (~tied).any():
            assert agree[~tied].mean() >= 0.999
        oi = r["idx"][t]
        ix, iy = oi % nvx, oi // nvx
        r1 = _take(rs, oi)
        well = agree & ~tied
        for inner, step in (((ix > 0) & (ix < nvx - 1), 1), ((iy > 0) & (iy < nvx - 1), nvx)):
            lo = _take(rs, np.clip(oi - step, 0, rs.shape[-1] - 1)) - r1
            hi = _take(rs, np.clip(oi + step, 0, rs.shape[-1] - 1)) - r1
            well &= ~inner | (-(lo + hi) / scale >= 1e-2)
        dv = np.abs(gres["vxy"][t].astype(np.float64) - r["vxy"][t]).max(axis=-1)
        if well.any():
            assert dv[well].max() <= 2e-3 * 0.3, (t, dv[well].max())
        n_well += int(well.sum())
    assert n_well > 0.4 * T * H * W, n_well


def test_refined_sampled_640x512(orc):
    """The benchmark workload's shape and launch configuration in mode 3;
    the oracle computes sampled anchors from their direct window spectra."""
    T = 12
    sc = scenes.flow_scene(1, H=512, W=640, T=T, n_targets=20)
    g = scenes.grid(-4, 4, 0.5)
    M = (16, 16, 8)
    gres = run_gpu(sc.frames[:T], M, g)
    cfg = _cfg(orc, 512, 640, M, g)
    rng = np.random.default_rng(4)
    pts = [(0, 0), (639, 511), (320, 256)] + [(int(rng.integers(0, 640)), int(rng.integers(0, 512))) for _ in range(12)]
    n_well = 0
    for (x, y) in pts:
        p = orc.pixel_series(cfg, sc.frames, x, y, T=T)
        sub = {k: gres[k][:, y:y + 1, x:x + 1] for k in ("out", "idx", "vxy")}
        n_well += check_refined(sub, p["rs"][:, None, None, :], p["en"][:, None, None], p["idx"][:, None, None],
                                p["vxy"][:, None, None, :], p["out"][:, None, None], sc.frames[:T], g)
    assert n_well > 0.5 * T * len(pts), n_well


def test_refined_lowers_the_residual():
    """On clutter moving between grid points the refined mode's prediction
    error is smaller than the grid search's (GPU only, 192x160 frames)."""
    b = _binding()
    T, H, W = 30, 160, 192
    sc = scenes.flow_scene(9, H=H, W=W, T=T, n_targets=0)
    g = scenes.grid(-4, 4, 0.5)
    dev = torch.from_numpy(sc.frames).cuda()
    res = {}
    for mode in (b.VEL_SEARCH, b.VEL_REFINED):
        f = b.Filter(H, W, 16, 16, 8, g, g, velocity_mode=mode)
        for t in range(T):
            f.push_frame(dev[t])
        res[mode] = f.output().cpu().numpy()[16:, 16:]
        f.close()
    rp = float(np.sqrt(np.mean(res[b.VEL_SEARCH] ** 2)))
    rr = float(np.sqrt(np.mean(res[b.VEL_REFINED] ** 2)))
    assert rr < 0.95 * rp, (rr, rp)


def test_refined_mode_arguments():
    b = _binding()
    g = scenes.grid(-2, 2, 0.5)
    with pytest.raises(b.RmdfError) as e:
        b.Filter(20, 20, 8, 8, 4, g[::-1], g, velocity_mode=b.VEL_REFINED)
    assert e.value.status == b.RMDF_E_INVAL
    with pytest.raises(b.RmdfError) as e:
        b.Filter(20, 20, 16, 16, 8, g, g, velocity_mode=b.VEL_REFINED, write_features=True)
    assert e.value.status == b.RMDF_E_UNSUPPORTED
    spec = [dict(H=20, W=20, M=(8, 8, 4), gx=g, gy=g)]
    with pytest.raises(b.RmdfError) as e:
        b.Batch(spec, velocity_mode=b.VEL_REFINED)
    assert e.value.status == b.RMDF_E_UNSUPPORTED
