"""CPU checks of the C-ABI library: it loads, exports every declared entry
point, and its host-side setup (1D reference element, fast-diagonalisation
data, sizes) agrees with the oracle.  No device call is made here."""
import numpy as np
import pytest

from oracle import basis
from paper_2607_02335_amd import fem


def test_library_exports_every_declared_symbol():
    L = fem.lib()
    names = fem.header_functions()
    assert len(names) >= 35
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert b"gfx950" in L.fem_version()


@pytest.mark.parametrize("p", range(1, 8))
def test_reference_matrices_match_oracle(p):
    M, K = fem.host_1d_matrices(p)
    np.testing.assert_allclose(M, basis.mass_1d(p), atol=1e-14)
    np.testing.assert_allclose(K, basis.stiffness_1d(p), atol=1e-12 * max(1, np.abs(K).max()))


def _patch_1d(p, h0, h1):
    """Oracle 1D matrices over two cells, restricted to interior nodes."""
    n1, nP = p + 1, 2 * p - 1
    M = np.zeros((2 * p + 1, 2 * p + 1))
    K = np.zeros_like(M)
    for c, h in enumerate((h0, h1)):
        sl = slice(c * p, c * p + n1)
        M[sl, sl] += basis.mass_1d(p, h)
        K[sl, sl] += basis.stiffness_1d(p, h)
    return M[1:-1, 1:-1], K[1:-1, 1:-1]


@pytest.mark.parametrize("p,h0,h1", [(1, 0.3, 0.7), (2, 0.05, 0.11), (3, 0.013, 0.02), (5, 0.2, 0.1),
                                     (7, 0.0417, 0.0623), (7, 1e-3, 2e-3)])
def test_fast_diagonalisation_identities(p, h0, h1):
    S, lam = fem.host_fd_1d(p, h0, h1)
    M, K = _patch_1d(p, h0, h1)
    nP = 2 * p - 1
    np.testing.assert_allclose(S.T @ M @ S, np.eye(nP), atol=1e-12)
    np.testing.assert_allclose(S.T @ K @ S, np.diag(lam), atol=1e-11 * lam.max())
    assert np.all(lam > 0) and np.all(np.diff(lam) >= 0)


def test_fd_inverse_of_kronecker_patch():
    """The 3D patch inverse assembled from the 1D FD data is the inverse of the
    oracle's plain-quadrature patch operator (brute force on one Q2 patch)."""
    from oracle import patches
    from oracle.mesh import Mesh
    p = 2
    rng = np.random.default_rng(0)
    w = [rng.uniform(0.5, 1.5, 3) for _ in range(3)]
    m = Mesh(p, (3, 3, 3), [v / v.sum() for v in w])
    v = (1, 2, 1)
    A = patches.patch_matrix(m, v)
    Sd, Ld = [], []
    for d in range(3):
        S, lam = fem.host_fd_1d(p, m.h[d][v[d] - 1], m.h[d][v[d]])
        Sd.append(S)
        Ld.append(lam)
    S3 = np.kron(np.kron(Sd[2], Sd[1]), Sd[0])
    lam3 = (Ld[2][:, None, None] + Ld[1][None, :, None] + Ld[0][None, None, :]).ravel()
    Ainv = S3 @ np.diag(1 / lam3) @ S3.T
    np.testing.assert_allclose(Ainv @ A, np.eye(A.shape[0]), atol=2e-13)


@pytest.mark.parametrize("p", range(1, 8))
def test_gll_nodes_match_oracle(p):
    np.testing.assert_allclose(fem.host_gll_nodes(p), basis.gll_nodes(p), atol=2e-16)


def test_host_entry_points_reject_bad_arguments():
    L = fem.lib()
    S = np.zeros(1)
    assert L.fem_host_fd_1d(0, 1.0, 1.0, S.ctypes.data, S.ctypes.data) == fem.FEM_EINVAL
    assert L.fem_host_fd_1d(2, -1.0, 1.0, S.ctypes.data, S.ctypes.data) == fem.FEM_EINVAL
    assert b"p in 1..7" in L.fem_last_error()


def test_footprint_arithmetic():
    # FP32 smoother: handle workspace + 3 FP64 + 2 FP32 solve vectors + b, u
    p, n = 3, 12
    cells = n ** 3
    cell_len = -(-cells // 64) * 64 * (p + 1) ** 3
    fp = fem.footprint_bytes(p, n, fem.F32)
    lower = cell_len * (8 * 5 + 4 * 2 + 8)          # vectors + smoother scratch
    assert lower < fp < lower * 3
    assert fem.footprint_bytes(7, 48, fem.F32) > fem.footprint_bytes(7, 24, fem.F32) * 7
    assert fem.lib().fem_prec_bytes(fem.BF16) == 2
