"""Allocation-free spectrum readout (rmdf_spectrum_noalloc) against the
allocating call (rmdf_spectrum) through the C ABI: the same kernel on the same
state, so the two must agree bit for bit; two calls in a row, the second with
fewer anchors (the shared device array keeps the first call's coordinates
beyond the second call's count, which must not matter); its size limit and
argument errors."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1408_3526_amd import scenes  # noqa: E402


def _b():
    from paper_1408_3526_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("M,grid,kw", [((16, 16, 8), (-4, 4, 0.5), {}),
                                       ((16, 16, 8), (-4, 4, 0.5), {"temporal": 1}),
                                       ((8, 8, 4), (-4, 4, 1.0), {}),
                                       ((9, 9, 5), (-2, 2, 0.25), {})])
def test_noalloc_spectrum_equals_allocating_call(M, grid, kw):
    b = _b()
    H, W, T = 40, 46, 10
    sc = scenes.flow_scene(31, H=H, W=W, T=T, n_targets=2, band_width=(6, 9))
    g = scenes.grid(*grid)
    f = b.Filter(H, W, *M, g, g, **kw)
    dev = torch.from_numpy(sc.frames).cuda()
    rng = np.random.default_rng(5)
    sizes = (700, 37)
    for t in range(T):
        f.push_frame(dev[t])
        if t < T - 2:
            continue
        for n in sizes:   # two calls in a row, the second smaller
            xs = rng.integers(0, W, n).astype(np.int32)
            ys = rng.integers(0, H, n).astype(np.int32)
            xs[:2], ys[:2] = (0, W - 1), (0, H - 1)
            ref = f.spectrum(xs, ys)
            got = f.spectrum_noalloc(xs, ys)
            torch.cuda.synchronize()
            print("window %s %s, frame %d, %d anchors" % (M, kw, t, n), flush=True)
            assert torch.equal(torch.view_as_real(got), torch.view_as_real(ref)), (M, kw, t, n)
    f.close()


def test_noalloc_spectrum_limits():
    b = _b()
    H, W = 20, 24
    sc = scenes.flow_scene(32, H=H, W=W, T=3, n_targets=1, band_width=(4, 6))
    g = scenes.grid(-4, 4, 0.5)
    f = b.Filter(H, W, 16, 16, 8, g, g)
    dev = torch.from_numpy(sc.frames).cuda()
    f.push_frame(dev[0])
    # the largest accepted count, with every anchor of the frame repeated
    n = b.SPECTRUM_NOALLOC_MAX
    idx = np.arange(n) % (H * W)
    xs, ys = (idx % W).astype(np.int32), (idx // W).astype(np.int32)
    ref = f.spectrum(xs[:H * W], ys[:H * W])
    got = f.spectrum_noalloc(xs, ys)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(got[:H * W]), torch.view_as_real(ref))
    assert torch.equal(torch.view_as_real(got[H * W:2 * H * W]), torch.view_as_real(ref))
    # one more is refused before anything is enqueued (the output pointer is
    # never used)
    xs1 = np.zeros(n + 1, np.int32)
    small = torch.zeros(16, device="cuda")
    st = b.lib().rmdf_spectrum_noalloc(f.ctx, n + 1, xs1.ctypes.data, xs1.ctypes.data, small.data_ptr())
    assert st == b.RMDF_E_INVAL
    assert b"RMDF_SPECTRUM_NOALLOC_MAX" in b.lib().rmdf_last_error(f.ctx)
    torch.cuda.synchronize()
    assert torch.count_nonzero(small).item() == 0
    # an anchor outside the frame is refused
    with pytest.raises(b.RmdfError) as ei:
        f.spectrum_noalloc(np.array([W], np.int32), np.array([0], np.int32))
    assert ei.value.status == b.RMDF_E_INVAL
    # zero anchors: nothing to do
    f.spectrum_noalloc(np.zeros(0, np.int32), np.zeros(0, np.int32))
    f.close()
