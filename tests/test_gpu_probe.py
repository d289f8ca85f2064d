"""The HBM streaming probe behind bench.py's practical ceiling
(rmdf_hbm_probe): each kind does what it says on every element, cached and
non-temporal, with grids smaller and larger than the buffer."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nt", [False, True])
@pytest.mark.parametrize("blocks", [1, 7, 4096])
def test_probe_kinds(nt, blocks):
    from paper_1408_3526_amd import binding
    binding.lib()
    n = (1 << 20) + 48                       # floats: a whole number of 16-byte pieces, not of the grid
    src = torch.arange(n, dtype=torch.float32, device="cuda") % 1000
    dst = torch.zeros(n, dtype=torch.float32, device="cuda")
    binding.hbm_probe(2, src, dst, 4 * n, blocks, nt)          # copy
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    binding.hbm_probe(1, None, dst, 4 * n, blocks, nt)         # write
    torch.cuda.synchronize()
    ref = torch.tensor([1.0, 2.0, 3.0, 4.0], device="cuda").repeat(n // 4)
    assert torch.equal(dst, ref)
    sink = torch.zeros(blocks, dtype=torch.float32, device="cuda")
    binding.hbm_probe(0, src, sink, 4 * n, blocks, nt)         # read: partial sums per workgroup
    torch.cuda.synchronize()
    total = float(sink.double().sum())
    exact = float(src.double().sum())
    assert abs(total - exact) <= 1e-5 * exact
