"""Checkpoint and restore of a filter context (rmdf_save_state /
rmdf_load_state) on the GPU.

* A context restored from a state saved after frame t continues the stream
  bit for bit as the saved context does (outputs, velocities, indices,
  smoothed R, spectra, frame and non-finite counts), for every kernel form,
  with the state in device or in host memory.
* A state from another configuration, a short buffer or a damaged header is
  refused and leaves the context as it was; streams owned by a batch refuse
  loads and single pushes.
* Recovery: the observer is deadbeat (Sec. 1; pinned in FP64 by the oracle's
  recovery test), so a state whose spectrum part is damaged is flushed after
  Kt pushes -- the spectrum then equals the undamaged stream's up to FP32
  rounding, while after Kt - 1 pushes the damage is still visible.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1408_3526_amd import scenes  # noqa: E402


def _b():
    from paper_1408_3526_amd import binding
    binding.lib()
    return binding


CASES = {
    "16x16x8": dict(M=(16, 16, 8), grid=(-4, 4, 0.5), kw={}),
    "16x16x8-ring": dict(M=(16, 16, 8), grid=(-4, 4, 0.5), kw=dict(temporal=1)),
    "16x16x8-direct": dict(M=(16, 16, 8), grid=(-4, 4, 0.5), kw=dict(temporal=2)),
    "16x16x8-refined": dict(M=(16, 16, 8), grid=(-2, 2, 0.5), kw=dict(velocity_mode=3)),
    "16x16x8-generic": dict(M=(16, 16, 8), grid=(-2, 2, 0.5), kw=dict(kernel_variant=1)),
    "16x16x8-learned": dict(M=(16, 16, 8), grid=(-4, 4, 0.5), kw=dict(velocity_mode=1)),
    "8x8x4": dict(M=(8, 8, 4), grid=(-2, 2, 1.0), kw={}),
    "9x9x5": dict(M=(9, 9, 5), grid=(-2, 2, 0.25), kw={}),
}
H, W, T, T_SAVE = 37, 45, 18, 9
XS, YS = [0, 44, 20, 31], [0, 36, 18, 5]


def _frames(seed=3):
    sc = scenes.flow_scene(seed, H=H, W=W, T=T, n_targets=2, band_width=(6, 9))
    fr = sc.frames.copy()
    fr[3, 5, 7] = np.nan            # one non-finite sample before the save
    fr[11, 2, 3] = np.inf           # and one after it
    return torch.from_numpy(fr).cuda()


def _filter(case, **over):
    b = _b()
    c = CASES[case]
    g = scenes.grid(*c["grid"])
    kw = dict(c["kw"], **over)
    f = b.Filter(H, W, *c["M"], g, g, **kw)
    if kw.get("velocity_mode") == 1:
        from paper_1408_3526_amd import learned
        f.set_weights(np.load(learned.DEFAULT_WEIGHTS))
    return f


def _readouts(f):
    v, i = f.velocity()
    return dict(out=f.output().cpu().numpy(), vxy=v.cpu().numpy(), idx=i.cpu().numpy(),
                rs=f.smoothed_r().cpu().numpy(), spec=f.spectrum(XS, YS).cpu().numpy(),
                t=f.frames_pushed(), nonfinite=f.nonfinite_count())


def _equal(a, b, what):
    for k in a:
        if isinstance(a[k], np.ndarray):
            assert np.array_equal(a[k], b[k], equal_nan=True), (what, k)
        else:
            assert a[k] == b[k], (what, k, a[k], b[k])


@pytest.mark.parametrize("where", ["device", "host"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_restored_context_continues_bit_for_bit(case, where):
    dev = _frames()
    a = _filter(case)
    for t in range(T_SAVE):
        a.push_frame(dev[t])
    at_save = _readouts(a)
    buf = None if where == "device" else np.empty(a.state_bytes(), np.uint8)
    buf = a.save_state(buf)
    later = []
    for t in range(T_SAVE, T):
        a.push_frame(dev[t])
        later.append(_readouts(a))
    a.close()

    b = _filter(case)
    b.push_frame(dev[T - 1])          # some other history, replaced by the load
    b.load_state(buf)
    _equal(at_save, _readouts(b), "after load")
    for k, t in enumerate(range(T_SAVE, T)):
        b.push_frame(dev[t])
        _equal(later[k], _readouts(b), "frame %d" % t)
    assert later[-1]["nonfinite"] == 2
    b.close()


def test_state_layout_and_size():
    f = _filter("16x16x8")
    hw = H * W
    sections = [hw * 1024 * 8, hw * 289 * 4, hw * (4 + 2) * 4, hw * 4, hw * 8, hw * 4]
    n = 128
    for s in sections:
        n = -(-n // 256) * 256 + s
    assert f.state_bytes() == n
    f.close()


def test_refused_loads_change_nothing():
    b = _b()
    dev = _frames()
    a = _filter("16x16x8")
    for t in range(T_SAVE):
        a.push_frame(dev[t])
    buf = a.save_state()
    f = _filter("16x16x8")
    for t in range(4):
        f.push_frame(dev[t])
    before = _readouts(f)

    def refused(blob, status=b.RMDF_E_INVAL):
        with pytest.raises(b.RmdfError) as e:
            f.load_state(blob)
        assert e.value.status == status
        _equal(before, _readouts(f), "after a refused load")

    refused(buf[:-1])                                  # short buffer
    bad = buf.clone()
    bad[0] = 0                                         # not a saved state
    refused(bad)
    bad = buf.clone()
    bad[8:12] = torch.tensor([9, 0, 0, 0], dtype=torch.uint8)   # unknown version
    refused(bad)
    # another configuration: frame width, grid values (same size), delay, smoother
    g = scenes.grid(-4, 4, 0.5)
    for other in (b.Filter(H, W + 1, 16, 16, 8, g, g), b.Filter(H, W, 16, 16, 8, g + 0.25, g),
                  b.Filter(H, W, 16, 16, 8, g, g, delay=(8, 8, 3)), b.Filter(H, W, 16, 16, 8, g, g, alpha=0.5),
                  b.Filter(H, W, 16, 16, 8, g, g, temporal=1)):
        with pytest.raises(b.RmdfError) as e:
            other.load_state(buf)
        assert e.value.status == b.RMDF_E_INVAL
        other.close()
    f.load_state(buf)                                  # the right one still loads
    assert f.frames_pushed() == T_SAVE
    a.close()
    f.close()


def test_batch_streams_refuse_loads_and_single_pushes():
    b = _b()
    g = scenes.grid(-1, 1, 1.0)
    bt = b.Batch([dict(H=24, W=20, M=(8, 8, 4), gx=g, gy=g)])
    ctx = ctypes.c_void_p()
    assert b.lib().rmdf_batch_stream_ctx(bt.b, 0, ctypes.byref(ctx)) == 0
    n = ctypes.c_size_t()
    assert b.lib().rmdf_state_bytes(ctx, ctypes.byref(n)) == 0
    buf = torch.zeros(n.value, dtype=torch.uint8, device="cuda")
    assert b.lib().rmdf_save_state(ctx, buf.data_ptr(), n.value) == 0      # saving is allowed
    assert b.lib().rmdf_load_state(ctx, buf.data_ptr(), n.value) == b.RMDF_E_STATE
    frame = torch.zeros(24, 20, device="cuda")
    assert b.lib().rmdf_push_frame(ctx, frame.data_ptr()) == b.RMDF_E_STATE
    bt.close()


@pytest.mark.parametrize("case", ["16x16x8", "16x16x8-generic", "8x8x4", "9x9x5"])
def test_damaged_spectrum_state_is_flushed_after_kt_pushes(case):
    dev = _frames()
    Mz = CASES[case]["M"][2]
    a = _filter(case)
    for t in range(T_SAVE):
        a.push_frame(dev[t])
    scale = float(np.abs(a.spectrum(XS, YS).cpu().numpy()).max())
    blob = a.save_state(np.empty(a.state_bytes(), np.uint8))
    # the first section (observer state, at byte 256) filled with finite noise
    # of the spectrum's own scale
    nbytes = _observer_bytes(case)
    noise = np.random.default_rng(5).normal(scale=scale, size=nbytes // 4).astype(np.float32)
    blob[256:256 + nbytes] = noise.view(np.uint8)
    b = _filter(case)
    b.load_state(blob)
    for k in range(Mz):
        a.push_frame(dev[T_SAVE + k])
        b.push_frame(dev[T_SAVE + k])
        err = np.abs(a.spectrum(XS, YS).cpu().numpy() - b.spectrum(XS, YS).cpu().numpy()).max()
        if k == Mz - 2:
            assert err > 1e-3 * scale, (k, err, scale)     # still damaged one push before
        if k == Mz - 1:
            assert err <= 1e-5 * scale, (k, err, scale)    # flushed after Kt pushes
    a.close()
    b.close()


def _observer_bytes(case):
    Mx, My, Mz = CASES[case]["M"]
    planes = {8: 4, 9: 5, 16: 8}[Mx]
    return H * W * planes * My * Mz * 8


def test_restore_then_frame_pairs_equals_single_pushes():
    """A state saved after an odd number of frames, restored, and continued by
    frame pairs gives what the saved context gives by single pushes (the
    ring slot arithmetic and the pair kernel both resume from the saved frame
    count)."""
    dev = _frames()
    a = _filter("16x16x8")
    for t in range(5):
        a.push_frame(dev[t])
    blob = a.save_state()
    ref = []
    for t in range(5, T):
        a.push_frame(dev[t])
        ref.append(a.output().cpu().numpy())
    a.close()
    b = _filter("16x16x8")
    b.load_state(blob)
    outs = [torch.empty(H, W, device="cuda") for _ in range(5, T)]
    b.push_frames([dev[t] for t in range(5, T)], outs)
    for k, o in enumerate(outs):
        assert np.array_equal(o.cpu().numpy(), ref[k]), k
    assert b.frames_pushed() == T
    b.close()
