"""Batched streams (one hipGraph launch per step, persistent work-queue
kernel) against eager single-stream contexts and the oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1408_3526_amd import scenes  # noqa: E402


def _streams():
    g1 = scenes.grid(-3, 3, 1.0)
    g5 = scenes.grid(-4, 4, 0.5)
    g25 = scenes.grid(-2, 2, 0.25)
    return [
        dict(H=40, W=36, M=(8, 8, 4), gx=g1, gy=g1, frames=scenes.translate_scene(1, H=40, W=36, T=10, v=(1, -1)).frames),
        dict(H=33, W=41, M=(16, 16, 8), gx=g5, gy=g5,
             frames=scenes.flow_scene(2, H=33, W=41, T=10, n_targets=2, band_width=(6, 9)).frames),
        dict(H=30, W=29, M=(9, 9, 5), gx=g25, gy=g25, frames=scenes.paper_scene(3, H=30, W=29, T=10).frames),
        dict(H=21, W=70, M=(8, 8, 4), gx=g1, gy=g1, frames=scenes.translate_scene(4, H=21, W=70, T=10, v=(-2, 1)).frames),
    ]


@pytest.mark.parametrize("tile,schedule", [(8, 0), (32, 0), (8, 1), (32, 2), (16, 3)])
def test_batch_graph_replays_equal_eager(tile, schedule):
    """Every schedule of the tile families (one kernel per family, one mixed
    kernel, small families on a parallel graph branch, launched after or
    before the large ones) gives the eager single-stream results bit for bit."""
    from paper_1408_3526_amd import binding
    st = _streams()
    T = 10
    b = binding.Batch(st, tile_rows=tile)
    b.set_schedule(schedule)
    singles = [binding.Filter(s["H"], s["W"], *s["M"], s["gx"], s["gy"], tile_rows=tile) for s in st]
    dev = [torch.from_numpy(s["frames"]).cuda() for s in st]
    for t in range(T):
        # zero-copy input for even steps, copying push for odd steps
        if t % 2 == 0:
            for i, d in enumerate(dev):
                _copy_to(b.input(i), d[t])
            b.launch()
        else:
            b.push([d[t] for d in dev])
        torch.cuda.synchronize()
        for i, sgl in enumerate(singles):
            sgl.push_frame(dev[i][t])
        torch.cuda.synchronize()
        for i, sgl in enumerate(singles):
            o_b, v_b, i_b = b.output(i)
            torch.cuda.synchronize()
            o_s = sgl.output()
            v_s, i_s = sgl.velocity()
            torch.cuda.synchronize()
            assert torch.equal(o_b, o_s), (t, i)
            assert torch.equal(i_b, i_s), (t, i)
            assert torch.equal(v_b, v_s), (t, i)
    for sgl in singles:
        sgl.close()
    b.close()


def _copy_to(ptr, src):
    """Device-to-device copy of a torch tensor into a raw device address,
    complete on return (device-wide synchronisation before and after)."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    torch.cuda.synchronize()
    rc = hip.hipMemcpy(ctypes.c_void_p(ptr), ctypes.c_void_p(src.data_ptr()), src.numel() * 4, 3)
    assert rc == 0
    # a device-to-device hipMemcpy may return before the copy is done, and the
    # batch runs on a stream that does not wait for the null stream
    torch.cuda.synchronize()


@pytest.mark.parametrize("variant", [0, 1])
def test_batch_matches_oracle(orc, variant):
    """Every stream against the oracle; variant 1 puts the 16x16x8 stream on
    the generic tile kernel."""
    from paper_1408_3526_amd import binding
    st = _streams()
    b = binding.Batch(st, kernel_variant=variant)
    dev = [torch.from_numpy(s["frames"]).cuda() for s in st]
    T = 10
    for t in range(T):
        b.push([d[t] for d in dev])
    torch.cuda.synchronize()
    for i, s in enumerate(st):
        out, vxy, idx = (x.cpu().numpy() for x in b.output(i))
        cfg = orc.Cfg(H=s["H"], W=s["W"], Mx=s["M"][0], My=s["M"][1], Mz=s["M"][2], gx=s["gx"], gy=s["gy"])
        r = orc.run(cfg, s["frames"], want_rs=True)
        rs = r["rs_all"][-1]
        srt = np.sort(rs, axis=-1)
        scale = np.maximum(np.maximum(np.abs(rs).max(-1), 1e-3 * r["en_all"][-1]), 1e-30)
        tied = (srt[..., -1] - srt[..., -2]) <= 1e-4 * scale
        agree = idx == r["idx"][-1]
        assert agree[~tied].mean() >= 0.999
        rms = float(np.sqrt(np.mean(s["frames"][-1].astype(np.float64) ** 2)))
        assert np.abs(out - r["out"][-1])[agree].max() <= 1e-3 * rms
    b.close()


@pytest.mark.parametrize("schedule", [0, 1])
def test_batch_many_tiny_streams_equal_eager(schedule):
    """36 streams of all three window families at degenerate sizes (single
    pixels, single rows and columns, frames smaller than the window): the
    persistent queues hold many one-item streams, and every stream's output,
    velocity and index still equal its single-stream context's, bit for bit,
    frame after frame."""
    from paper_1408_3526_amd import binding
    rng = np.random.default_rng(36)
    g1, g5, g25 = scenes.grid(-3, 3, 1.0), scenes.grid(-4, 4, 0.5), scenes.grid(-2, 2, 0.25)
    shapes = [((8, 8, 4), g1), ((9, 9, 5), g25), ((16, 16, 8), g5)]
    sizes = [(1, 1), (1, 17), (19, 1), (3, 3), (2, 40), (7, 5)]
    T = 6
    st = []
    for k in range(36):
        M, g = shapes[k % 3]
        H, W = sizes[(k // 3) % len(sizes)]
        fr = (rng.normal(size=(T, H, W)) * 4 + 30).astype(np.float32)
        st.append(dict(H=H, W=W, M=M, gx=g, gy=g, frames=fr))
    b = binding.Batch(st, tile_rows=4)
    b.set_schedule(schedule)
    singles = [binding.Filter(s["H"], s["W"], *s["M"], s["gx"], s["gy"], tile_rows=4) for s in st]
    dev = [torch.from_numpy(s["frames"]).cuda() for s in st]
    for t in range(T):
        b.push([d[t] for d in dev])
        for i, sgl in enumerate(singles):
            sgl.push_frame(dev[i][t])
        torch.cuda.synchronize()
        for i, sgl in enumerate(singles):
            o_b, v_b, i_b = b.output(i)
            v_s, i_s = sgl.velocity()
            o_s = sgl.output()
            torch.cuda.synchronize()
            assert torch.equal(o_b, o_s), (t, i)
            assert torch.equal(v_b, v_s), (t, i)
            assert torch.equal(i_b, i_s), (t, i)
    for sgl in singles:
        sgl.close()
    b.close()


def test_batch_autotune_and_latency():
    from paper_1408_3526_amd import binding
    st = _streams()
    b = binding.Batch(st)
    dev = [torch.from_numpy(s["frames"]).cuda() for s in st]
    for t in range(3):
        b.push([d[t] for d in dev])
    rep = b.autotune(iters=3)
    assert "tile_rows" in rep and "median step" in rep
    b.set_timing(True)
    for t in range(5):
        b.push([d[t % 10] for d in dev])
    lat = b.latency()
    assert lat["steps"] == 5 and 0 < lat["p50_ms"] <= lat["p99_ms"]
    b.close()


def test_batch_rejects_bad_schedule_and_tiles():
    """Out-of-range schedules, stream indexes and tile heights are refused
    with RMDF_E_INVAL, and the batch stays usable."""
    from paper_1408_3526_amd import binding
    st = _streams()[:2]
    b = binding.Batch(st, tile_rows=8)
    for bad in (-1, 4):
        with pytest.raises(binding.RmdfError) as ei:
            b.set_schedule(bad)
        assert ei.value.status == binding.RMDF_E_INVAL
    for s, ty in ((2, 8), (-2, 8), (0, 0)):
        with pytest.raises(binding.RmdfError) as ei:
            b.set_tiles(s, ty)
        assert ei.value.status == binding.RMDF_E_INVAL
    b.set_schedule(3)
    b.push([torch.from_numpy(s["frames"][0]).cuda() for s in st])
    torch.cuda.synchronize()
    b.close()


def test_batch_full_size_streams_equal_eager():
    """One stream of each size class of the 24-stream workload, at full size
    (320x256 at 8x8x4, 640x512 and 1280x1024 at 16x16x8), with the tile heights
    and schedule the autotuner picks for it: every frame's outputs, velocities
    and indexes equal those of single-stream contexts with the same tile
    heights, bit for bit."""
    from paper_1408_3526_amd import binding
    g1, g5 = scenes.grid(-4, 4, 1.0), scenes.grid(-4, 4, 0.5)
    T = 10
    st = [dict(H=256, W=320, M=(8, 8, 4), gx=g1, gy=g1, tile=4,
               frames=scenes.flow_scene(101, H=256, W=320, T=T).frames),
          dict(H=512, W=640, M=(16, 16, 8), gx=g5, gy=g5, tile=32,
               frames=scenes.flow_scene(102, H=512, W=640, T=T).frames),
          dict(H=1024, W=1280, M=(16, 16, 8), gx=g5, gy=g5, tile=64,
               frames=scenes.flow_scene(103, H=1024, W=1280, T=T, n_targets=50).frames)]
    b = binding.Batch(st)
    for i, s in enumerate(st):
        b.set_tiles(i, s["tile"])
    b.set_schedule(0)
    singles = [binding.Filter(s["H"], s["W"], *s["M"], s["gx"], s["gy"], tile_rows=s["tile"]) for s in st]
    dev = [torch.from_numpy(s["frames"]).cuda() for s in st]
    for t in range(T):
        b.push([d[t] for d in dev])
        for i, sgl in enumerate(singles):
            sgl.push_frame(dev[i][t])
        torch.cuda.synchronize()
        for i, sgl in enumerate(singles):
            o_b, v_b, i_b = b.output(i)
            o_s = sgl.output()
            v_s, i_s = sgl.velocity()
            torch.cuda.synchronize()
            assert torch.equal(o_b, o_s), (t, i)
            assert torch.equal(v_b, v_s), (t, i)
            assert torch.equal(i_b, i_s), (t, i)
    for sgl in singles:
        sgl.close()
    b.close()
