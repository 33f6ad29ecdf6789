"""Multi-block DSS (Section 4.2, Algorithm "Unstructured Inter-Block
Summation") on the GPU against the oracle's geometric identification: the
k-star meshes (k = 3, 5 blocks around one macro-edge, with exchanged local
axes so shared faces meet in different orientations) and the unit cube cut
into 2^3 blocks with random rotations and reflections, in every precision;
every copy of a node ends with the same bits, and counting copies (DSS of
ones) is exact."""
import numpy as np
import pytest

from oracle import multiblock
from tests.gpu_util import check_err, note, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL = {0: 1e-14, 1: 1e-6, 2: 1e-2}


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2607_02335_amd import fem
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    fem.lib()
    return fem


def meshes():
    yield "3-star p=2 n=3", multiblock.star(2, 3, 3, twist=True)
    yield "5-star p=3 n=2", multiblock.star(3, 2, 5, twist=True)
    yield "3-star p=7 n=2", multiblock.star(7, 2, 3, twist=True)
    yield "3-star p=1 n=4", multiblock.star(1, 4, 3, twist=True)
    for seed in (1, 2):
        yield f"rotated split cube p=3 n=3 seed {seed}", multiblock.split_cube(3, 3, np.random.default_rng(seed))
    yield "rotated split cube p=2 n=5 seed 3", multiblock.split_cube(2, 5, np.random.default_rng(3))


@pytest.mark.parametrize("which", range(7))
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_multiblock_dss_matches_oracle(F, which, prec):
    name, mb = list(meshes())[which]
    note(f"multi-block dss {name} prec={prec}")
    D = F.MultiBlockDss(mb.p, mb.block_n, mb.corners)
    rng = np.random.default_rng(40 + which)
    v = rng.uniform(-1, 1, (mb.ncells(), mb.n1 ** 3))
    vd = D.pack(to_dev(v.ravel()), prec)
    vin = to_np(D.unpack(vd)).reshape(v.shape)            # after rounding to the precision
    D.dss(vd)
    s = to_np(D.unpack(vd)).reshape(v.shape)
    check_err(s, mb.dss(vin), TOL[prec], f"multi-block {name} prec={prec}")
    ids = mb.cell_node_ids()
    order = np.argsort(ids.ravel(), kind="stable")
    sv, iv = s.ravel()[order], ids.ravel()[order]
    first = np.r_[0, np.nonzero(np.diff(iv))[0] + 1]
    rep = np.repeat(sv[first], np.diff(np.r_[first, iv.size]))
    np.testing.assert_array_equal(sv, rep)                # copies of a node bitwise equal
    ones = D.pack(to_dev(np.ones(v.size)), prec)
    D.dss(ones)
    np.testing.assert_array_equal(to_np(D.unpack(ones)).reshape(v.shape), mb.dss(np.ones(v.shape)))
    st = D.stats()
    print(f"{name}: {st}", flush=True)
    D.close()
