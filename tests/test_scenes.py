"""The seeded input generators (paper_1408_3526_amd/scenes.py): reproducible
per seed, independent sub-streams, and ground truth consistent with the
frames they draw (the motion model each family states)."""
import numpy as np
import pytest

from paper_1408_3526_amd import scenes


def test_same_seed_same_frames_other_seed_other_frames():
    for make in (lambda s: scenes.translate_scene(s, H=20, W=24, T=4),
                 lambda s: scenes.flow_scene(s, H=24, W=28, T=4, n_targets=2, band_width=(4, 6)),
                 lambda s: scenes.paper_scene(s, H=16, W=16, T=4)):
        a, b, c = make(5), make(5), make(6)
        assert a.frames.dtype == np.float32
        assert np.array_equal(a.frames, b.frames) and np.array_equal(a.velocity, b.velocity)
        assert not np.array_equal(a.frames, c.frames)


def test_named_sub_streams_are_independent():
    # the texture and the noise do not depend on how many targets are drawn:
    # the frames differ only near the one target
    a = scenes.translate_scene(3, H=32, W=32, T=2, n_targets=0)
    b = scenes.translate_scene(3, H=32, W=32, T=2, n_targets=1)
    d = np.abs(a.frames - b.frames) > 1e-6
    assert 0 < d.sum() < 0.1 * d.size


@pytest.mark.parametrize("v", [(1, -2), (0, 3), (-2, 0)])
def test_translate_scene_is_an_exact_integer_translation(v):
    sc = scenes.translate_scene(1, H=24, W=30, T=5, v=v, n_targets=0, noise_sigma=0.0)
    vx, vy = v
    for t in range(4):
        a, b = sc.frames[t].astype(np.float64), sc.frames[t + 1].astype(np.float64)
        # I_{t+1}(x, y) = I_t(x - vx, y - vy) wherever both are inside the frame
        ys = slice(max(vy, 0), 24 + min(vy, 0))
        xs = slice(max(vx, 0), 30 + min(vx, 0))
        ys0 = slice(max(vy, 0) - vy, 24 + min(vy, 0) - vy)
        xs0 = slice(max(vx, 0) - vx, 30 + min(vx, 0) - vx)
        assert np.array_equal(b[ys, xs], a[ys0, xs0])
    assert np.all(sc.velocity[..., 0] == vx) and np.all(sc.velocity[..., 1] == vy)


def test_flow_scene_advects_along_its_labels():
    # without band, targets and noise, I_t(x) = I_{t-1}(x - v(x)): sampling the
    # previous frame at x - v(x) predicts the next one far better than the
    # previous frame itself does
    from scipy import ndimage
    H, W = 48, 56
    sc = scenes.flow_scene(2, H=H, W=W, T=3, n_targets=0, noise_sigma=0.0, band=False)
    v = sc.velocity
    assert v.shape == (H, W, 2)
    assert abs(np.sqrt((v ** 2).sum(-1)).max() - 3.0) < 1e-9       # rescaled to max |v| = 3
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    prev, nxt = sc.frames[1].astype(np.float64), sc.frames[2].astype(np.float64)
    warped = ndimage.map_coordinates(prev, [ys - v[..., 1], xs - v[..., 0]], order=3, mode="nearest")
    inner = (slice(6, H - 6), slice(6, W - 6))
    err_warp = np.sqrt(np.mean((warped - nxt)[inner] ** 2))
    err_still = np.sqrt(np.mean((prev - nxt)[inner] ** 2))
    assert err_warp < 0.3 * err_still, (err_warp, err_still)


def test_flow_scene_band_and_targets_ground_truth():
    sc = scenes.flow_scene(4, H=40, W=48, T=6, n_targets=3, band_width=(8, 12))
    assert sc.band_mask.shape == (6, 40, 48) and sc.band_mask[-1].any()
    # labels inside the band at the last frame are the band's single velocity
    inside = sc.velocity[sc.band_mask[-1]]
    assert np.allclose(inside, inside[0])
    # targets move at constant velocity
    d = np.diff(sc.targets, axis=1)
    assert np.allclose(d, d[:, :1, :])
    assert sc.target_snr.shape == (3,) and np.all((sc.target_snr >= 2) & (sc.target_snr <= 8))


def test_grid_is_inclusive_and_uniform():
    g = scenes.grid(-4, 4, 0.5)
    assert len(g) == 17 and g[0] == -4 and g[-1] == 4 and np.allclose(np.diff(g), 0.5)
    assert list(scenes.grid(-2, 2, 1.0)) == [-2, -1, 0, 1, 2]


def test_gaussian_field_moments_and_spectrum_slope():
    rng = np.random.default_rng(0)
    f = scenes.gaussian_field(rng, 128, 128, 3.0)
    assert abs(f.mean()) < 1e-9 and abs(f.std() - 3.0) < 1e-9
    # radially averaged power falls as 1/f^2: a factor of about 4 per octave
    P = np.abs(np.fft.fft2(f)) ** 2
    fy, fx = np.meshgrid(np.fft.fftfreq(128), np.fft.fftfreq(128), indexing="ij")
    r = np.sqrt(fx ** 2 + fy ** 2)
    lo = P[(r > 0.05) & (r < 0.07)].mean()
    hi = P[(r > 0.10) & (r < 0.14)].mean()
    assert 2.5 < lo / hi < 6.5, lo / hi
