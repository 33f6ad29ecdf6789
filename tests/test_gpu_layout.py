"""The layout study's kernels (storage block size B = 1 .. 128) against the
oracle: the mass apply and the structured DSS give the oracle's results for
every B and both tile shapes, on a mesh whose cell count is not a multiple
of the block size (a ragged last block)."""
import numpy as np
import pytest

from oracle import operators
from oracle.mesh import Mesh
from tests.gpu_util import check_err, note, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2607_02335_amd import fem
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    fem.lib()
    return fem


@pytest.mark.parametrize("p", [2, 3, 4, 5])
@pytest.mark.parametrize("B", [1, 2, 4, 8, 16, 32, 64, 128])
def test_layout_kernels_match_oracle(F, p, B):
    n = (5, 3, 7)
    note(f"layout p={p} B={B}")
    m = Mesh(p, n)
    L = F.LayoutStudy(p, n, B)
    rng = np.random.default_rng(300 + 10 * p + B)
    v = rng.uniform(-1, 1, (m.ncells, m.n1 ** 3))
    vd = L.pack(to_dev(v.ravel()))
    np.testing.assert_array_equal(to_np(L.unpack(vd)).reshape(v.shape), v)
    for tile in (16, 32):
        y = to_np(L.unpack(L.mass(vd, tile=tile))).reshape(v.shape)
        check_err(y, operators.mass_cells(m, v, dirichlet=False), 1e-13, f"layout mass p={p} B={B} tile={tile}")
    s = to_np(L.unpack(L.dss(vd))).reshape(v.shape)
    check_err(s, operators.dss(m, v), 1e-14, f"layout dss p={p} B={B}")
