"""Pins of the CFAR detector oracle (oracle/cfar.py): brute force on small
frames, the false-alarm rate on white Gaussian noise against its closed form,
and the invariances of the definition."""
import numpy as np
import pytest
from scipy import stats

from oracle import cfar as C


@pytest.mark.parametrize("H,W,guard,train", [(12, 10, 1, 2), (7, 15, 2, 3), (3, 4, 1, 1), (1, 9, 0, 2), (4, 4, 4, 1)])
def test_cfar_equals_brute_force(H, W, guard, train):
    rng = np.random.default_rng(H * 31 + W)
    x = rng.normal(size=(H, W)) * 3 + 1
    x[rng.integers(0, H), rng.integers(0, W)] += 25.0
    det, mu, sig, n = C.cfar(x, guard, train, 2.5)
    det2, sig2 = C.cfar_loops(x, guard, train, 2.5)
    assert np.allclose(sig, sig2, rtol=1e-12, atol=1e-12)
    assert np.array_equal(det, det2)
    # guard square covering the frame: no training cells, no detections
    if guard >= max(H, W):
        assert not det.any()


def test_false_alarm_rate_on_white_noise():
    """On i.i.d. N(0, s^2) noise the cell under test is independent of its
    training cells (the guard excludes it), so with n cells
    (x - mu) / sigma_hat = sqrt((1 + 1/n) n / (n - 1)) t_{n-1} exactly and
    P(false alarm) = 2 P(t_{n-1} > k / sqrt((1 + 1/n) n / (n - 1)))."""
    rng = np.random.default_rng(5)
    x = rng.normal(size=(1024, 1024)) * 7.0
    guard, train, k = 2, 4, 3.0
    det, _, _, n = C.cfar(x, guard, train, k)
    inner = n == n.max()
    nn = int(n.max())
    assert nn == (2 * (guard + train) + 1) ** 2 - (2 * guard + 1) ** 2
    pfa = 2 * stats.t.sf(k / np.sqrt((1 + 1 / nn) * nn / (nn - 1)), nn - 1)
    got = det[inner].mean()
    assert abs(got - pfa) <= 0.1 * pfa, (got, pfa)


def test_invariances():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(40, 50))
    x[10, 20] += 9
    x[30, 5] -= 8
    d0 = C.cfar(x, 1, 3, 3.5)[0]
    assert d0[10, 20] and d0[30, 5]
    assert np.array_equal(d0, C.cfar(4.0 * x, 1, 3, 3.5)[0])
    assert np.array_equal(d0, C.cfar(-x, 1, 3, 3.5)[0])          # two-sided
    assert np.array_equal(d0, C.cfar(x + 0.25, 1, 3, 3.5)[0])    # local mean removed
    # a constant image has sigma = 0 and no detections
    assert not C.cfar(np.full((9, 9), 3.0), 1, 2, 3.0)[0].any()
