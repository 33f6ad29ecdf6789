"""The matrix-core (MFMA) apply for p = 7 (the FP64 default) against the
oracle and against the plane-streamed VALU apply (FEM_OPT_APPLY_PLANES_P7):
Dirichlet and Neumann on ragged meshes (a partial last storage block,
partial 8-cell tiles, a single cell) with graded widths; FP32 and BF16 (the
plane-streamed kernel either way) on the same meshes; and the residual mode
through FP64 two-sweep smoother steps against the oracle's smoother."""
import numpy as np
import pytest

from oracle import operators, patches, solver
from oracle.mesh import Mesh
from tests.gpu_util import check_err, graded, note, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5, 2: 1e-2}


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2607_02335_amd import fem
    assert torch.cuda.is_available()
    return fem


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("n,bc", [((3, 2, 5), 0), ((5, 3, 2), 1), ((9, 4, 3), 0), ((1, 1, 1), 0), ((11, 7, 1), 1)])
def test_mfma_apply_matches_oracle_and_planes(F, prec, n, bc):
    note(f"p=7 mfma apply n={n} bc={bc} prec={prec}")
    m, w, rng = graded(7, n, 70 + prec)
    P = F.Problem(7, n, w, bc=bc)
    x = P.gather(to_dev(rng.uniform(-1, 1, m.nglob)), prec)
    y = P.apply(x)
    F.set_option(F.OPT_APPLY_PLANES_P7, 1)
    try:
        y2 = P.apply(x)
    finally:
        F.set_option(F.OPT_APPLY_PLANES_P7, 0)
    ref = operators.apply_cells(m, to_np(P.unpack(x)), dirichlet=(bc == 0))
    check_err(to_np(P.unpack(y)), ref, TOL[prec], f"mfma apply n={n} bc={bc} prec={prec}")
    check_err(to_np(P.unpack(y2)), ref, TOL[prec], f"planes apply n={n} bc={bc} prec={prec}")
    # padding cells of the last storage block are zero
    full = to_np(y).reshape(-1, 512, 64)
    pad = full[-1][:, m.ncells - 64 * (full.shape[0] - 1):]
    assert not np.any(pad)


@pytest.mark.parametrize("prec", [0])
def test_mfma_residual_in_smoother(F, prec):
    """Two sweeps use the residual apply rs - A z once."""
    note(f"p=7 smoother (mfma residual) prec={prec}")
    m, w, rng = graded(7, (3, 3, 4), 77)
    P = F.Problem(7, m.n, w)
    rc = rng.uniform(-1, 1, (m.ncells, m.n1 ** 3)) * ~operators.boundary_copies(m)
    rd = P.pack(to_dev(rc.ravel()), prec)
    z = to_np(P.unpack(P.smoother_step(rd, sweeps=2, omega=0.125)))
    ref = solver.smoother(m, operators.scatter(m, to_np(P.unpack(rd))), 2, 0.125,
                          schwarz=patches.SchwarzFactors(m))
    check_err(z, ref[m.dofs], TOL[prec], f"p=7 smoother 2 sweeps prec={prec}")
