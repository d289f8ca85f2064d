"""Long-run numerical robustness of the FP32 GPU recursions.

The temporal observer is a deadbeat (finite-impulse-response) estimator: a
rounding error made at frame t has left the state after Mz more updates
(Sec. 1; pinned in FP64 by the oracle's deadbeat-recovery test), so its
error does not grow with the number of frames.  The spatial sliding DFTs
restart from a direct-DFT seed every 16 columns and every tile of rows.
Here 2^20 frames (about 1e6) go through the three forms of the spectrum
(observer state; ring of 2-D spectra; the direct form, which has no
recursion at all and shows the error level without one) and the local
spectrum at a few anchors is compared with the direct DFT of the current
window, in FP64, at checkpoints.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import brute  # noqa: E402

N_FRAMES = 1 << 20
CHECKS = (1 << 6, 1 << 10, 1 << 14, 1 << 17, N_FRAMES)
H, W, M = 18, 20, (16, 16, 8)
PTS = [(0, 0), (19, 17), (10, 9), (15, 4)]


def _run(temporal):
    from paper_1408_3526_amd import binding
    binding.lib()
    g = np.array([-1.0, 0.0, 1.0])
    f = binding.Filter(H, W, *M, g, g, temporal=temporal)
    gen = torch.Generator(device="cuda").manual_seed(1234)
    xs, ys = np.array([p[0] for p in PTS]), np.array([p[1] for p in PTS])
    errs = {}
    chunk = 4096
    done = 0
    while done < N_FRAMES:
        # white noise on a large offset: the comb subtracts nearly equal values
        fr = torch.randn((chunk, H, W), generator=gen, device="cuda") * 10.0 + 1000.0
        for i in range(chunk):
            f.push_frame(fr[i])
            done += 1
            if done in CHECKS:
                spec = f.spectrum(xs, ys).cpu().numpy().astype(np.complex128)
                win = fr[max(0, i - M[2] + 1):i + 1].cpu().numpy().astype(np.float64)
                if win.shape[0] < M[2]:
                    win = np.concatenate([np.zeros((M[2] - win.shape[0], H, W)), win])
                ref = np.stack([brute.spectrum(win, x, y, M[2] - 1, M) for x, y in PTS])
                errs[done] = float(np.abs(spec - ref).max() / np.abs(ref).max())
    torch.cuda.synchronize()
    f.close()
    return errs


@pytest.mark.parametrize("temporal", [0, 1, 2])
def test_no_drift_over_a_million_frames(temporal):
    errs = _run(temporal)
    print("temporal mode %d: relative spectrum error by frame %s" % (temporal, errs))
    assert max(errs.values()) <= 1e-5, errs
    # no growth: the last checkpoint is within a small factor of the first
    assert errs[N_FRAMES] <= 4 * max(errs[CHECKS[0]], 1e-7), errs
