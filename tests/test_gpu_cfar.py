"""GPU parity of the CFAR detection stage (rmdf_cfar) against the FP64
oracle (oracle/cfar.py).

Bars: sigma within 1e-4 of the image's largest |x| per pixel; detections
identical wherever the oracle's margin ||x - mu| - k sigma| exceeds 1e-4 of
the image's largest |x| (closer to the threshold the FP32 sums may decide
either way, as with ties of the velocity argmax)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import cfar as C  # noqa: E402
from paper_1408_3526_amd import scenes  # noqa: E402


def _binding():
    from paper_1408_3526_amd import binding
    binding.lib()
    return binding


def check(x, guard, train, k):
    b = _binding()
    det, lev = b.cfar(torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda(), guard, train, k, want_level=True)
    det, lev = det.cpu().numpy().astype(bool), lev.cpu().numpy()
    x64 = x.astype(np.float32).astype(np.float64)
    odet, mu, sig, n = C.cfar(x64, guard, train, k)
    scale = np.abs(x64).max()
    assert np.abs(lev - sig).max() <= 1e-4 * scale, np.abs(lev - sig).max()
    margin = np.abs(np.abs(x64 - mu) - k * sig)
    clear = margin > 1e-4 * scale
    assert np.array_equal(det[clear], odet[clear])
    return int(odet.sum())


@pytest.mark.parametrize("H,W,guard,train,k", [(37, 131, 2, 4, 3.0), (1, 70, 0, 3, 2.0), (16, 64, 1, 1, 2.5),
                                               (200, 300, 3, 13, 4.0), (5, 3, 4, 2, 1.0), (130, 17, 0, 16, 3.5),
                                               (512, 640, 2, 4, 4.0), (512, 640, 3, 13, 3.0)])
def test_cfar_parity_random(H, W, guard, train, k):
    rng = np.random.default_rng(H * 7 + W)
    x = rng.normal(size=(H, W)) * 2.0 + 0.3
    for _ in range(max(1, H * W // 500)):
        x[rng.integers(0, H), rng.integers(0, W)] += rng.uniform(8, 20) * rng.choice([-1, 1])
    check(x, guard, train, k)


def test_cfar_parity_on_filter_output():
    """The detector on the prediction error of the 16x16x8 filter."""
    b = _binding()
    T, H, W = 14, 160, 200
    sc = scenes.flow_scene(3, H=H, W=W, T=T, n_targets=8)
    g = scenes.grid(-4, 4, 0.5)
    f = b.Filter(H, W, 16, 16, 8, g, g)
    dev = torch.from_numpy(sc.frames).cuda()
    for t in range(T):
        f.push_frame(dev[t])
    out = f.output().cpu().numpy()
    f.close()
    n = check(out, 2, 4, 4.0)
    assert n > 0


def test_cfar_arguments():
    b = _binding()
    x = torch.zeros((8, 8), device="cuda")
    for guard, train, k in [(0, 0, 3.0), (10, 7, 3.0), (-1, 2, 3.0), (1, 2, -1.0), (1, 2, float("nan"))]:
        with pytest.raises(b.RmdfError) as e:
            b.cfar(x, guard, train, k)
        assert e.value.status == b.RMDF_E_INVAL
