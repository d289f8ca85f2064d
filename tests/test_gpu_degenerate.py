"""Degenerate inputs through every kernel form, checked against what the
method fixes in closed form (no oracle needed).

* All-zero frames: every spectrum, power spectrum and autocorrelation value
  is exactly 0, so the first maximum of the smoothed R is grid index 0 (the
  tie rule), the velocity is the grid's first candidate (on the grid's edge,
  so sub-grid refinement keeps it), and the output is exactly 0.
* Constant frames: the only non-zero bin is the spatial-temporal DC, where
  eq. (8) is (Mx My Mz)^(-1/2) for every velocity, so the background
  estimate (eq. 4) equals the constant and the prediction error (eq. 1) is 0
  on every anchor whose window lies inside the frames, whichever velocity
  the argmax picks.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1408_3526_amd import scenes  # noqa: E402

FORMS = [
    # (window, kernel_variant, temporal, velocity mode name, grid)
    ((16, 16, 8), 2, "observer", "search", (-4, 4, 0.5)),
    ((16, 16, 8), 1, "observer", "search", (-4, 4, 0.5)),
    ((16, 16, 8), 2, "ring", "search", (-4, 4, 0.5)),
    ((16, 16, 8), 2, "direct", "search", (-4, 4, 0.5)),
    ((16, 16, 8), 2, "observer", "refined", (-4, 4, 0.5)),
    ((8, 8, 4), 0, "observer", "search", (-4, 4, 1.0)),
    ((8, 8, 4), 0, "observer", "refined", (-4, 4, 1.0)),
    ((9, 9, 5), 0, "observer", "search", (-2, 2, 0.25)),
]


def _filter(b, H, W, M, variant, temporal, vmode, g):
    return b.Filter(H, W, *M, g, g, kernel_variant=variant,
                    temporal={"ring": b.TEMPORAL_RING, "direct": b.TEMPORAL_DIRECT}.get(temporal, b.TEMPORAL_OBSERVER),
                    velocity_mode=b.VEL_REFINED if vmode == "refined" else b.VEL_SEARCH)


def _run(f, frames):
    out, idx, vxy = [], [], []
    for t in range(frames.shape[0]):
        f.push_frame(frames[t])
        out.append(f.output().cpu().numpy())
        v, i = f.velocity()
        vxy.append(v.cpu().numpy())
        idx.append(i.cpu().numpy())
    torch.cuda.synchronize()
    return np.stack(out), np.stack(idx), np.stack(vxy)


@pytest.mark.parametrize("M,variant,temporal,vmode,grid", FORMS)
def test_zero_frames_give_exact_zeros_and_the_first_candidate(M, variant, temporal, vmode, grid):
    from paper_1408_3526_amd import binding as b
    b.lib()
    g = scenes.grid(*grid)
    H, W, T = 37, 53, M[2] + 3
    f = _filter(b, H, W, M, variant, temporal, vmode, g)
    fr = torch.zeros((T, H, W), dtype=torch.float32, device="cuda")
    out, idx, vxy = _run(f, fr)
    assert f.nonfinite_count() == 0
    f.close()
    assert np.all(out == 0.0)
    assert np.all(idx == 0)
    assert np.all(vxy[..., 0] == np.float32(g[0])) and np.all(vxy[..., 1] == np.float32(g[0]))


@pytest.mark.parametrize("M,variant,temporal,vmode,grid", FORMS)
def test_constant_frames_are_predicted_exactly(M, variant, temporal, vmode, grid):
    from paper_1408_3526_amd import binding as b
    b.lib()
    g = scenes.grid(*grid)
    c = 37.5
    H, W, T = 37, 53, M[2] + 3
    f = _filter(b, H, W, M, variant, temporal, vmode, g)
    fr = torch.full((T, H, W), c, dtype=torch.float32, device="cuda")
    out, _, _ = _run(f, fr)
    f.close()
    valid = out[M[2] - 1:, M[1] - 1:, M[0] - 1:]
    assert np.abs(valid).max() <= 1e-4 * c, np.abs(valid).max()


def test_constant_frames_640x512_bench_configuration():
    """The same closed form at the full 640x512 size, 16x16x8 window, 17x17
    grid, in the launch configuration the benchmark times (default kernel and
    tile height)."""
    from paper_1408_3526_amd import binding as b
    b.lib()
    g = scenes.grid(-4, 4, 0.5)
    M, H, W, c = (16, 16, 8), 512, 640, 123.25
    f = b.Filter(H, W, *M, g, g)
    fr = torch.full((H, W), c, dtype=torch.float32, device="cuda")
    for _ in range(M[2] + 2):
        f.push_frame(fr)
    out = f.output().cpu().numpy()
    torch.cuda.synchronize()
    f.close()
    valid = out[M[1] - 1:, M[0] - 1:]
    assert np.abs(valid).max() <= 1e-4 * c, np.abs(valid).max()
