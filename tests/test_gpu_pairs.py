"""Frame pairs (rmdf_push_frames): two frames through one pass of the
16x16x8 per-pixel kernel give the results of two single pushes, bit for bit;
contexts the pair kernel does not serve fall back to single pushes."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1408_3526_amd import scenes  # noqa: E402


def _b():
    from paper_1408_3526_amd import binding
    binding.lib()
    return binding


def _run_pair(frames, chunks, M=(16, 16, 8), grid=None, with_outs=True, **kw):
    """The same frames through single pushes (context A) and through
    rmdf_push_frames in the given chunk sizes (context B); every frame's
    output, and the final state readouts, of both."""
    b = _b()
    T, H, W = frames.shape
    g = grid if grid is not None else scenes.grid(-4, 4, 0.5)
    dev = torch.from_numpy(np.ascontiguousarray(frames)).cuda()
    fa = b.Filter(H, W, *M, g, g, **kw)
    fb = b.Filter(H, W, *M, g, g, **kw)
    outs_a, outs_b = [], []
    for t in range(T):
        fa.push_frame(dev[t])
        outs_a.append(fa.output())
    t = 0
    for c in chunks:
        if with_outs:
            o = [torch.full((H, W), float("nan"), device="cuda") for _ in range(c)]
            fb.push_frames([dev[t + i] for i in range(c)], o)
            outs_b += o
        else:
            fb.push_frames([dev[t + i] for i in range(c)])
            outs_b += [None] * (c - 1) + [fb.output()]
        t += c
    assert t == T
    xs = [0, W - 1, W // 2, min(3, W - 1)]
    ys = [0, H - 1, H // 2, min(5, H - 1)]
    res = []
    for f in (fa, fb):
        v, i = f.velocity()
        res.append(dict(out=f.output(), vxy=v, idx=i, rs=f.smoothed_r(), spec=f.spectrum(xs, ys),
                        n=f.frames_pushed(), bad=f.nonfinite_count()))
    torch.cuda.synchronize()
    fa.close()
    fb.close()
    return outs_a, outs_b, res[0], res[1]


def _assert_equal(outs_a, outs_b, ra, rb):
    for t, (oa, ob) in enumerate(zip(outs_a, outs_b)):
        if ob is not None:
            assert torch.equal(oa, ob), t
    for k in ("out", "vxy", "idx", "rs", "spec"):
        assert torch.equal(ra[k], rb[k]), k
    assert ra["n"] == rb["n"] and ra["bad"] == rb["bad"]


@pytest.mark.parametrize("case", ["flow", "ragged_odd", "tiny", "nonfinite"])
def test_pairs_equal_single_pushes(case):
    """Ragged tiles, an odd frame count (the last frame alone), frames
    smaller than the window and non-finite samples: pairs equal single
    pushes frame by frame."""
    if case == "flow":
        fr = scenes.flow_scene(3, H=40, W=47, T=12, n_targets=3, band_width=(8, 12)).frames
        chunks, kw = [2] * 6, dict(tile_rows=16)
    elif case == "ragged_odd":
        fr = scenes.flow_scene(4, H=33, W=70, T=11, n_targets=2, band_width=(6, 9)).frames
        chunks, kw = [3, 2, 1, 5], dict(tile_rows=8)
    elif case == "tiny":
        rng = np.random.default_rng(5)
        fr = (rng.normal(size=(9, 3, 5)) * 5 + 20).astype(np.float32)
        chunks, kw = [2, 2, 2, 3], dict(tile_rows=32)
    else:
        fr = scenes.flow_scene(6, H=24, W=30, T=10, n_targets=2, band_width=(4, 6)).frames.copy()
        fr[3, 5, 7] = np.nan
        fr[4, 0, 0] = np.inf
        fr[7, 23, 29] = -np.inf
        chunks, kw = [4, 4, 2], dict(tile_rows=8)
    _assert_equal(*_run_pair(fr, chunks, **kw))


@pytest.mark.parametrize("dt", [0, 1, 7])
def test_pairs_every_output_delay(dt):
    """Output delays m'_t = 0 (a pair's second frame is its own delayed
    sample), 1 (the first frame is) and Mz - 1: the delay ring keeps every
    sample a pair reads."""
    fr = scenes.flow_scene(7, H=30, W=29, T=12, n_targets=2, band_width=(6, 9)).frames
    _assert_equal(*_run_pair(fr, [2] * 6, delay=(-1, -1, dt), tile_rows=8))


def test_pairs_without_output_buffers():
    """No caller buffers: the pair's first output goes to the context's own
    scratch, and the state, smoothed R and the last frame's results still
    equal single pushes."""
    fr = scenes.flow_scene(10, H=26, W=31, T=10, n_targets=2).frames
    _assert_equal(*_run_pair(fr, [2, 2, 2, 2, 2], with_outs=False, tile_rows=8))


def test_pairs_fixed_velocity():
    fr = scenes.flow_scene(8, H=32, W=36, T=10, n_targets=2).frames
    b = _b()
    _assert_equal(*_run_pair(fr, [2] * 5, velocity_mode=b.VEL_FIXED, fixed_v=(1.25, -0.5)))


def test_pairs_full_size_frames():
    """The benchmark workload's shape and launch configuration (640x512,
    32-row tiles, 17x17 grid at 0.5)."""
    fr = scenes.flow_scene(1, H=512, W=640, T=8, n_targets=20).frames
    _assert_equal(*_run_pair(fr, [2, 2, 2, 2]))


@pytest.mark.parametrize("other", ["ring", "refined", "window_8x8x4"])
def test_contexts_without_pairs_fall_back(other):
    """Contexts the pair kernel does not serve push the frames one by one
    (the outputs still land in the caller's buffers)."""
    b = _b()
    if other == "window_8x8x4":
        fr = scenes.translate_scene(2, H=21, W=30, T=7, v=(1, -1)).frames
        g1 = scenes.grid(-3, 3, 1.0)
        _assert_equal(*_run_pair(fr, [2, 3, 2], M=(8, 8, 4), grid=g1))
        return
    fr = scenes.flow_scene(9, H=20, W=26, T=7, n_targets=1).frames
    kw = dict(temporal=b.TEMPORAL_RING) if other == "ring" else dict(velocity_mode=b.VEL_REFINED)
    _assert_equal(*_run_pair(fr, [2, 3, 2], **kw))


def test_push_frames_arguments():
    """Bad arguments are refused before any launch: the frame count does not move."""
    b = _b()
    g = scenes.grid(-4, 4, 0.5)
    f = b.Filter(20, 20, 16, 16, 8, g, g)
    fr = torch.zeros((20, 20), device="cuda")
    import ctypes
    L = b.lib()
    arr = (ctypes.c_void_p * 2)(fr.data_ptr(), None)
    assert L.rmdf_push_frames(f.ctx, 2, arr, None) == b.RMDF_E_INVAL
    assert L.rmdf_push_frames(f.ctx, 0, arr, None) == b.RMDF_E_INVAL
    assert L.rmdf_push_frames(f.ctx, 1, None, None) == b.RMDF_E_INVAL
    assert f.frames_pushed() == 0
    f.close()
    learned = b.Filter(20, 20, 16, 16, 8, g, g, velocity_mode=b.VEL_LEARNED)
    arr = (ctypes.c_void_p * 2)(fr.data_ptr(), fr.data_ptr())
    assert L.rmdf_push_frames(learned.ctx, 2, arr, None) == b.RMDF_E_STATE
    assert learned.frames_pushed() == 0
    learned.close()
