"""The paper's own configuration and simulated scene, checked against the
values it prints (tests/golden/paper_configuration.json, Sec. 3
'Parameterization' and 'Simulation', Sec. 5 'Implementation')."""
import inspect
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import oracle  # noqa: E402
from paper_1408_3526_amd import scenes  # noqa: E402

GOLD = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_configuration.json")))


def test_default_parameters_reproduce_the_paper_set():
    p = GOLD["parameterization"]
    M = [2 * k + 1 for k in p["K"]]
    assert M == p["window_lengths_2K_plus_1"]
    g = scenes.grid(-2.0, 2.0, p["lag_grid_step"])
    lo, hi = p["lag_grid_quarters"]
    assert np.allclose(g, np.arange(lo, hi + 1) / 4.0)
    cfg = oracle.Cfg(H=p["N"][1], W=p["N"][0], Mx=M[0], My=M[1], Mz=M[2], gx=g, gy=g)
    assert (cfg.Bx, cfg.By) == tuple(p["B"])
    assert (cfg.dx, cfg.dy, cfg.dt) == tuple(p["m_prime"])
    assert cfg.alpha == float(np.exp(-1.0 / 10.0))
    wl = bench.WORKLOADS["paper64"]
    assert (wl["W"], wl["H"]) == tuple(p["N"]) and list(wl["M"]) == M
    assert np.allclose(scenes.grid(*wl["grid"]), g)


def test_paper_scene_follows_the_simulation_recipe():
    s = GOLD["simulation"]
    sig = inspect.signature(scenes.paper_scene).parameters
    assert tuple(sig["v_clutter"].default) == tuple(s["v_clutter"])
    assert tuple(sig["v_target"].default) == tuple(s["v_target"])
    assert sig["n_comp"].default == s["n_components"]
    assert sig["noise_sigma"].default == s["noise_sigma"]
    T = 24
    sc = scenes.paper_scene(7, T=T, noise_sigma=0.0)
    fr = sc.frames.astype(np.float64)
    H, W = fr.shape[1:]
    # the target sits at the centre of the final frame and occludes the clutter
    # wherever its PSF is at least the truncation level
    tx, ty = sc.targets[0, T - 1]
    assert (tx, ty) == ((W - 1) / 2.0, (H - 1) / 2.0)
    ys, xs = np.mgrid[0:H, 0:W]
    g = np.exp(-((xs - tx) ** 2 + (ys - ty) ** 2) / (2 * s["target_psf_sigma"] ** 2)) * s["target_peak"]
    disc = g >= s["target_truncation"]
    assert np.allclose(fr[-1][disc], g[disc], atol=1e-6)
    # clutter: DC 10 plus 25 components of magnitude 0.1
    bound = s["n_components"] * s["component_magnitude"]
    assert np.all(np.abs(fr[-1][~disc] - s["dc_offset"]) <= bound + 1e-5)
    # translation at v_clutter: 8 frames move it by exactly (13, 5) pixels
    dxy = (8 * np.array(s["v_clutter"])).astype(int)
    a, b = fr[0], fr[8]
    far = np.ones((H, W), bool)
    for t in (0, 8):
        px, py = sc.targets[0, t]
        far &= np.hypot(xs - px, ys - py) > 4
        far &= np.hypot(xs - dxy[0] - px, ys - dxy[1] - py) > 4
    shifted = b[dxy[1]:, dxy[0]:]
    orig = a[:H - dxy[1], :W - dxy[0]]
    m = far[dxy[1]:, dxy[0]:] & far[:H - dxy[1], :W - dxy[0]]
    assert m.sum() > 1000
    assert np.abs(shifted[m] - orig[m]).max() <= 1e-5


def test_paper_rate_quoted_by_the_benchmark():
    r = GOLD["implementation_rates_hz"]["cpp_parallel_rows_8_threads"]
    assert bench.PAPER_RATE["paper64"]["value"] == r * 64 * 64
