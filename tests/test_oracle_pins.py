"""Pins of the oracle against what the mathematics and the paper fix.

None of these re-derive the oracle's own formulas: they check textbook
closed forms, invariants of the continuous problem that the discrete one
inherits exactly, special cases that reduce to a direct solve, and the worked
example the paper prints for the DSS cascade.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import basis, element, multiblock, operators, patches, solver, twolevel
from oracle.mesh import Mesh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def graded_mesh(p, n, seed=11):
    rng = np.random.default_rng(seed)
    n3 = (n, n, n) if isinstance(n, int) else n
    w = []
    for nd in n3:
        v = rng.uniform(0.5, 1.5, nd)
        w.append(v / v.sum())
    return Mesh(p, n3, w)


# ---------------------------------------------------------------- 1D rules
def test_gll_nodes_textbook():
    np.testing.assert_allclose(basis.gll_nodes(1), [0, 1], atol=0)
    np.testing.assert_allclose(basis.gll_nodes(2), [0, 0.5, 1], atol=1e-15)
    s = 1 / math.sqrt(5)
    np.testing.assert_allclose(basis.gll_nodes(3), [0, (1 - s) / 2, (1 + s) / 2, 1], atol=1e-15)
    t = math.sqrt(3 / 7)
    np.testing.assert_allclose(basis.gll_nodes(4), [0, (1 - t) / 2, 0.5, (1 + t) / 2, 1], atol=1e-15)
    for p in range(2, 8):
        x = basis.gll_nodes(p)
        # GLL quadrature (weights from integrating the Lagrange basis) is
        # exact for polynomials of degree 2p-1.
        xq, wq = basis.gauss_rule(p + 1)
        wg = (basis.lagrange_values(x, xq).T * wq).sum(axis=1)
        for m in range(2 * p):
            assert abs(wg @ x ** m - 1 / (m + 1)) < 1e-14


def test_gauss_rule_exact_to_degree_2n_minus_1():
    for nq in range(1, 9):
        x, w = basis.gauss_rule(nq)
        for m in range(2 * nq):
            assert abs(w @ x ** m - 1 / (m + 1)) < 1e-14
        assert abs(w @ x ** (2 * nq) - 1 / (2 * nq + 1)) > 1e-12


def test_q2_1d_matrices_closed_form():
    # textbook P2 element on [0,1] with nodes 0, 1/2, 1
    M = np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) / 30
    K = np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / 3
    np.testing.assert_allclose(basis.mass_1d(2), M, atol=1e-15)
    np.testing.assert_allclose(basis.stiffness_1d(2), K, atol=1e-14)
    np.testing.assert_allclose(basis.mass_1d(2).sum(axis=1), [1 / 6, 2 / 3, 1 / 6], atol=1e-15)
    # the 3D plain-quadrature element on the unit cube is the Kronecker sum
    # of these textbook matrices (x fastest in the local numbering)
    A = element.element_stiffness(2, 1.0, 1.0, 1.0)
    ref = np.kron(np.kron(M, M), K) + np.kron(np.kron(M, K), M) + np.kron(np.kron(K, M), M)
    np.testing.assert_allclose(A, ref, atol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3, 5, 7])
def test_1d_invariants(p):
    h = 0.37
    K = basis.stiffness_1d(p, h)
    M = basis.mass_1d(p, h)
    np.testing.assert_allclose(K @ np.ones(p + 1), 0, atol=1e-12)
    assert abs(M.sum() - h) < 1e-14
    x = basis.gll_nodes(p) * h
    # stiffness on a linear function: only the end rows see the flux
    lin = K @ x
    np.testing.assert_allclose(lin[1:-1], 0, atol=1e-12)
    np.testing.assert_allclose([lin[0], lin[-1]], [-1, 1], atol=1e-12)


@pytest.mark.parametrize("p", [3, 7])
def test_element_factorisation_identity(p):
    hx, hy, hz = 0.31, 0.07, 0.55
    A = element.element_stiffness(p, hx, hy, hz)
    Kx, Ky, Kz = (basis.stiffness_1d(p, h) for h in (hx, hy, hz))
    Mx, My, Mz = (basis.mass_1d(p, h) for h in (hx, hy, hz))
    ref = np.kron(np.kron(Mz, My), Kx) + np.kron(np.kron(Mz, Ky), Mx) + np.kron(np.kron(Kz, My), Mx)
    np.testing.assert_allclose(A, ref, atol=1e-12 * np.abs(ref).max())
    # the regrouped form the oracle uses for large meshes
    Ax, Ay, Az, M3 = element.reference_directional(p)
    A2 = hy * hz / hx * Ax + hx * hz / hy * Ay + hx * hy / hz * Az
    np.testing.assert_allclose(A, A2, atol=1e-12 * np.abs(A).max())
    np.testing.assert_allclose(element.element_mass(p, hx, hy, hz),
                               np.kron(np.kron(Mz, My), Mx), atol=1e-15)
    assert np.allclose(A, A.T, atol=1e-13 * np.abs(A).max())


# ---------------------------------------------------------- global operator
@pytest.mark.parametrize("p", [2, 3])
def test_neumann_null_space(p):
    m = graded_mesh(p, 4)
    y = operators.apply_global(m, np.ones(m.nglob), dirichlet=False)
    A = operators.assemble(m)
    assert np.abs(y).max() <= 1e-13 * abs(A).max()


@pytest.mark.parametrize("p", [2, 3, 7])
def test_quadratics_exact(p):
    m = graded_mesh(p, 3 if p == 7 else 4)
    X, Y, Z = (m.coords_1d(d) for d in range(3))
    XX = np.tile(X, m.N[1] * m.N[2])
    YY = np.tile(np.repeat(Y, m.N[0]), m.N[2])
    interior = ~m.boundary_mask()
    # harmonic quadratic: every interior row of A u vanishes
    y = operators.apply_global(m, XX ** 2 - YY ** 2, dirichlet=False)
    assert np.abs(y[interior]).max() < 1e-12
    # -Laplace(x^2) = -2: interior rows equal -2 M 1
    y = operators.apply_global(m, XX ** 2, dirichlet=False)
    mass1 = operators.mass_global(m, np.ones(m.nglob), dirichlet=False)
    np.testing.assert_allclose(y[interior], -2 * mass1[interior], atol=1e-12)
    # energy of x^2 over the unit cube: int |grad x^2|^2 = 4/3
    u = XX ** 2
    assert abs(u @ operators.apply_global(m, u, dirichlet=False) - 4 / 3) < 1e-12


def bubble(m):
    X, Y, Z = (m.coords_1d(d) for d in range(3))
    bx, by, bz = X * (1 - X), Y * (1 - Y), Z * (1 - Z)
    return np.kron(np.kron(bz, by), bx), (bx, by, bz)


@pytest.mark.parametrize("p,n", [(2, 3), (3, 4), (7, 2)])
def test_bubble_energy(p, n):
    m = graded_mesh(p, n)
    u, _ = bubble(m)
    e = u @ operators.apply_global(m, u)
    assert abs(e - 1 / 900) < 1e-14


def test_dirichlet_operator_spd_and_symmetric():
    m = graded_mesh(2, 3)
    A = operators.assemble(m, dirichlet=True).toarray()
    assert np.abs(A - A.T).max() < 1e-14 * np.abs(A).max()
    inner = ~m.boundary_mask()
    ev = np.linalg.eigvalsh(A[np.ix_(inner, inner)])
    assert ev.min() > 0
    x = np.random.default_rng(5).uniform(-1, 1, m.nglob)
    np.testing.assert_allclose(A @ x, operators.apply_global(m, x), atol=1e-12)


# ------------------------------------------------------------------ DSS
def test_dss_multiplicity():
    m = graded_mesh(3, 3)
    s = operators.dss(m, np.ones((m.ncells, m.n1 ** 3)))
    # copies of interior vertex/edge/face/cell nodes
    counts = set(np.unique(s).astype(int))
    assert counts == {1, 2, 4, 8}
    mult = m.multiplicity()
    I = np.arange(m.nglob) % m.N[0]
    J = (np.arange(m.nglob) // m.N[0]) % m.N[1]
    K = np.arange(m.nglob) // (m.N[0] * m.N[1])

    def c(Ix, N):
        return np.where((Ix % m.p == 0) & (Ix > 0) & (Ix < N - 1), 2, 1)
    np.testing.assert_array_equal(mult, c(I, m.N[0]) * c(J, m.N[1]) * c(K, m.N[2]))


def test_dss_worked_example_2d():
    rows = {}
    with open(os.path.join(GOLDEN, "dss_vertex_2d.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                t = line.split()
                rows[t[0]] = [float(v) for v in t[1:]]
    m = Mesh(1, (2, 2, 1))
    v = np.zeros((m.ncells, 8))
    # the shared vertex (1,1,0): local corner of each cell
    g = m.gidx(1, 1, 0)
    names = {"nw": 2, "ne": 3, "sw": 0, "se": 1}
    for key, val in zip(["nw", "ne", "sw", "se"], rows["initial"]):
        e = names[key]
        l = int(np.nonzero(m.dofs[e] == g)[0][0])
        v[e, l] = val
    s = operators.dss(m, v)
    for key, val in zip(["nw", "ne", "sw", "se"], rows["after_y"]):
        e = names[key]
        l = int(np.nonzero(m.dofs[e] == g)[0][0])
        assert s[e, l] == val


def test_duality_pairing_lemma():
    m = graded_mesh(3, 3)
    rng = np.random.default_rng(9)
    f = rng.standard_normal((m.ncells, m.n1 ** 3))
    ug = rng.standard_normal(m.nglob)
    lhs = np.sum(f * operators.gather(m, ug))
    rhs = operators.scatter(m, f) @ ug
    assert abs(lhs - rhs) <= 1e-13 * abs(rhs)


# ------------------------------------------------------------- patches
@pytest.mark.parametrize("p", [2, 3])
def test_patch_matrix_is_restricted_global(p):
    m = graded_mesh(p, 3)
    A = operators.assemble(m).tocsr()
    for v in patches.interior_vertices(m):
        idx = patches.patch_nodes(m, v)
        ref = A[idx][:, idx].toarray()
        np.testing.assert_allclose(patches.patch_matrix(m, v), ref, atol=1e-12 * abs(ref).max())


@pytest.mark.parametrize("p", [2, 3])
def test_single_patch_is_exact_inverse(p):
    # n = 2: one interior vertex whose patch interior is the whole interior
    m = graded_mesh(p, 2)
    A = operators.assemble(m, dirichlet=True).tocsr()
    inner = np.nonzero(~m.boundary_mask())[0]
    r = np.zeros(m.nglob)
    r[inner] = np.random.default_rng(3).standard_normal(len(inner))
    z = patches.additive_schwarz(m, r)
    ref = np.zeros(m.nglob)
    ref[inner] = spla.spsolve(A[inner][:, inner].tocsc(), r[inner])
    np.testing.assert_allclose(z, ref, atol=1e-12 * np.abs(ref).max())
    # omega = 1, one sweep of the smoother is then an exact solve
    zs = solver.smoother(m, r, sweeps=1, omega=1.0)
    np.testing.assert_allclose(zs, ref, atol=1e-12 * np.abs(ref).max())


def test_schwarz_symmetric_positive_and_bounded():
    m = graded_mesh(2, 4)
    inner = np.nonzero(~m.boundary_mask())[0]
    nI = len(inner)
    f = patches.SchwarzFactors(m)
    P = np.zeros((nI, nI))
    for t in range(nI):
        e = np.zeros(m.nglob)
        e[inner[t]] = 1
        P[:, t] = f(e)[inner]
    assert np.abs(P - P.T).max() < 1e-12 * np.abs(P).max()
    A = operators.assemble(m, dirichlet=True).toarray()[np.ix_(inner, inner)]
    # eigenvalues of P A lie in (0, 8]: each node is covered by at most 8
    # patches and same-parity patches are disjoint
    L = np.linalg.cholesky(A)
    ev = np.linalg.eigvalsh(L.T @ P @ L)
    assert ev.min() > 0 and ev.max() <= 8 + 1e-10
    # multiplicity: P_AS applied to A_P-range vectors reproduces them
    v = patches.interior_vertices(m)[5]
    idx = patches.patch_nodes(m, v)
    assert set(idx) <= set(inner)


def test_at_cells_matches_full():
    m = graded_mesh(3, 4)
    r = np.random.default_rng(1).standard_normal(m.nglob) * (~m.boundary_mask())
    z = patches.SchwarzFactors(m)(r)
    cells = [0, 5, 21, 63]
    np.testing.assert_allclose(patches.additive_schwarz_at_cells(m, r, cells),
                               z[m.cell_dofs(cells)], atol=1e-13 * np.abs(z).max())


# --------------------------------------------------------------- solver
def test_cg_matches_textbook_cg_iterates():
    m = graded_mesh(2, 4)
    A = operators.assemble(m, dirichlet=True).tocsr()
    inner = np.nonzero(~m.boundary_mask())[0]
    Ai = A[inner][:, inner]
    b = np.random.default_rng(2).standard_normal(len(inner))
    ref = []
    spla.cg(Ai, b, rtol=1e-12, maxiter=8, callback=lambda xk: ref.append(xk.copy()))
    _, _, _, its = solver.fcg(lambda v: Ai @ v, lambda v: v, b, rtol=1e-30, maxit=8,
                              variant="pcg", record=True)
    for k in range(1, 8):
        np.testing.assert_allclose(its[k], ref[k - 1], rtol=0, atol=1e-10 * np.abs(ref[k - 1]).max())


def test_fcg_equals_pcg_for_static_preconditioner():
    m = graded_mesh(2, 4)
    b = operators.mass_global(m, np.random.default_rng(4).uniform(-1, 1, m.nglob))
    u1, k1, h1, it1 = solver.solve_poisson(m, b, rtol=1e-10, variant="pcg", record=True)
    u2, k2, h2, it2 = solver.solve_poisson(m, b, rtol=1e-10, variant="fcg", record=True)
    assert abs(k1 - k2) <= 1
    for k in range(min(k1, k2, 6)):
        np.testing.assert_allclose(it1[k], it2[k], atol=1e-8 * np.abs(u1).max())
    A = operators.assemble(m, dirichlet=True)
    assert np.linalg.norm(b - A @ u1) <= 1e-10 * np.linalg.norm(b) * 1.0001


@pytest.mark.parametrize("p,n", [(2, 4), (3, 3)])
def test_bubble_solve_is_galerkin_exact(p, n):
    m = graded_mesh(p, n)
    u, (bx, by, bz) = bubble(m)
    # f = -Laplace(u) = 2 (Y Z + X Z + X Y) in Q2 subset of Qp
    f = 2 * (np.kron(np.kron(bz, by), np.ones_like(bx)) + np.kron(np.kron(bz, np.ones_like(by)), bx)
             + np.kron(np.kron(np.ones_like(bz), by), bx))
    b = operators.mass_global(m, f)
    uh, k, hist, _ = solver.solve_poisson(m, b, rtol=1e-12)
    assert hist[-1] <= 1e-12
    assert np.abs(uh - u).max() < 1e-10


# ------------------------------------------------ storage ratio table
def test_storage_ratio_table():
    with open(os.path.join(GOLDEN, "storage_ratios.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for name, edge, stored, unique, sr, tr in rows:
        edge, stored, unique = int(edge), int(stored), int(unique)
        assert stored == edge ** 3
        assert unique == (edge - 1) ** 3
        assert abs(stored / unique - float(sr)) < 0.006
        # cell-wise apply moves read+write per stored DoF, the assembled one
        # read + read-accumulate-write per unique DoF: ratio 2/3 of storage
        assert abs(2 * stored / (3 * unique) - float(tr)) < 0.006


# ------------------------------------------------- smoother sweep algebra
@pytest.mark.parametrize("p", [2, 3])
def test_smoother_sweeps_on_a_single_patch(p):
    """n = 2: the one patch covers the whole interior, so P_AS = A_D^{-1} there
    and every damped sweep shrinks the error by (1 - omega):
    z_nu = (1 - (1 - omega)^nu) A_D^{-1} r.  With omega = 1/2 two sweeps give
    3/4 of the exact solve, with omega = 1 every sweep count gives the solve."""
    m = graded_mesh(p, 2)
    A = operators.assemble(m, dirichlet=True).tocsr()
    inner = np.nonzero(~m.boundary_mask())[0]
    r = np.zeros(m.nglob)
    r[inner] = np.random.default_rng(13).standard_normal(len(inner))
    exact = np.zeros(m.nglob)
    exact[inner] = spla.spsolve(A[inner][:, inner].tocsc(), r[inner])
    for omega, nu in ((0.5, 2), (1.0, 2), (1.0, 3), (0.5, 3), (0.3, 4)):
        z = solver.smoother(m, r, sweeps=nu, omega=omega)
        np.testing.assert_allclose(z, (1 - (1 - omega) ** nu) * exact, rtol=0,
                                   atol=1e-12 * np.abs(exact).max())
    assert abs(np.abs(solver.smoother(m, r, 2, 0.5)).max() / np.abs(exact).max() - 0.75) < 1e-12


def test_smoother_sweeps_closed_form():
    """nu sweeps of damped Richardson from zero are the polynomial
    (I - (I - omega B A)^nu) A^{-1} in the dense preconditioner B = P_AS and
    operator A = A_D on the interior of a mesh with 8 overlapping patches."""
    m = graded_mesh(2, 3)
    inner = np.nonzero(~m.boundary_mask())[0]
    nI = len(inner)
    A = operators.assemble(m, dirichlet=True).toarray()[np.ix_(inner, inner)]
    f = patches.SchwarzFactors(m)
    B = np.zeros((nI, nI))
    for t in range(nI):
        e = np.zeros(m.nglob)
        e[inner[t]] = 1
        B[:, t] = f(e)[inner]
    r = np.random.default_rng(17).standard_normal(nI)
    rg = np.zeros(m.nglob)
    rg[inner] = r
    Ainv_r = np.linalg.solve(A, r)
    for omega, nu in ((0.125, 2), (0.2, 3), (0.3, 2)):
        E = np.linalg.matrix_power(np.eye(nI) - omega * B @ A, nu)
        ref = Ainv_r - E @ Ainv_r
        z = solver.smoother(m, rg, sweeps=nu, omega=omega, schwarz=f)
        np.testing.assert_allclose(z[inner], ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        assert not np.any(z[m.boundary_mask()])


# ------------------------------------------- Section 3.3 preconditioners
def test_diagonal_closed_forms():
    """Diagonal of the assembled Laplacian on uniform cubes of side h, from
    the textbook 1D matrices: Q1 interior vertex 8 (h/3) = 8h/3; Q2 cell
    centre 3 h K11 M11^2 = 1024h/225, interior vertex 8 * 3 h K00 M00^2 =
    224h/225."""
    n = 4
    h = 1.0 / n
    m1 = Mesh(1, (n, n, n))
    d1 = operators.diagonal(m1)
    I = m1.gidx(2, 1, 3)
    assert abs(d1[I] - 8 * h / 3) < 1e-15
    m2 = Mesh(2, (n, n, n))
    d2 = operators.diagonal(m2)
    assert abs(d2[m2.gidx(3, 5, 1)] - 1024 * h / 225) < 1e-14        # (1,1,1) node of cell (1,2,0)
    assert abs(d2[m2.gidx(2, 4, 6)] - 224 * h / 225) < 1e-14         # interior vertex (1,2,3)
    # face-centre node shared by two cells: 2 h (K11 M11 M00 + M11 K11 M00 + M11 M11 K00)
    K, M = np.array([7, 16]) / 3, np.array([4, 16]) / 30
    face = 2 * h * (K[1] * M[1] * M[0] + M[1] * K[1] * M[0] + M[1] * M[1] * K[0])
    assert abs(d2[m2.gidx(3, 3, 2)] - face) < 1e-14
    # the element sum equals the diagonal of the assembled sparse matrix
    mg = graded_mesh(3, 3)
    np.testing.assert_allclose(operators.diagonal(mg), operators.assemble(mg).diagonal(), rtol=1e-13)


def test_jacobi_pcg_is_cg_on_the_scaled_system():
    """PCG with P = D^{-1} (Section 3.3, Jacobi) is textbook CG on
    D^{-1/2} A D^{-1/2} y = D^{-1/2} b with u = D^{-1/2} y: iterate by
    iterate."""
    m = graded_mesh(2, 4)
    inner = np.nonzero(~m.boundary_mask())[0]
    A = operators.assemble(m, dirichlet=True).tocsr()[inner][:, inner]
    d = operators.diagonal(m)
    b = np.zeros(m.nglob)
    b[inner] = np.random.default_rng(19).standard_normal(len(inner))
    s = 1 / np.sqrt(d[inner])
    As = (A.multiply(s[:, None]).multiply(s[None, :])).tocsr()
    ref = []
    spla.cg(As, s * b[inner], rtol=1e-14, maxiter=8, callback=lambda yk: ref.append(s * yk))
    _, _, _, its = solver.solve_poisson(m, b, rtol=1e-30, maxit=8, precond="jacobi", record=True)
    for k in range(1, 8):
        np.testing.assert_allclose(its[k][inner], ref[k - 1], rtol=0, atol=1e-10 * np.abs(ref[k - 1]).max())
    # P = S is the Riesz identity on the assembled interior: plain CG
    ref = []
    spla.cg(A, b[inner], rtol=1e-14, maxiter=6, callback=lambda yk: ref.append(yk.copy()))
    _, _, _, its = solver.solve_poisson(m, b, rtol=1e-30, maxit=6, precond="dss", record=True)
    for k in range(1, 6):
        np.testing.assert_allclose(its[k][inner], ref[k - 1], rtol=0, atol=1e-10 * np.abs(ref[k - 1]).max())


# --------------------------------------------------- two-level (Q1 coarse)
def test_hat_functions_partition_and_linear_reproduction():
    v = np.array([0.0, 0.2, 0.5, 0.55, 1.0])
    x = np.linspace(0, 1, 41)
    H = twolevel.hat_values(v, x)
    np.testing.assert_allclose(H.sum(axis=1), 1, atol=1e-15)
    np.testing.assert_allclose(H @ v, x, atol=1e-15)
    np.testing.assert_allclose(twolevel.hat_values(v, v), np.eye(len(v)), atol=0)


def test_prolongation_is_lagrange_at_vertices():
    m = graded_mesh(3, (4, 3, 5))
    P0 = twolevel.prolongation(m).toarray()
    i, j, k = twolevel.coarse_vertices(m)
    g = m.gidx(i * m.p, j * m.p, k * m.p)
    np.testing.assert_array_equal(P0[g], np.eye(len(g)))
    assert not np.any(P0[m.boundary_mask()])
    assert np.all(P0.sum(axis=1) <= 1 + 1e-14)


@pytest.mark.parametrize("p", [2, 3])
def test_galerkin_coarse_operator_is_the_q1_stiffness(p):
    """Q1 is a subspace of Qp and (p+1)-point Gauss integrates its gradients
    exactly, so P0^T A_D P0 equals the Q1 Laplacian of the same mesh."""
    m = graded_mesh(p, (4, 3, 5))
    T = twolevel.TwoLevel(m)
    m1 = Mesh(1, m.n, m.h)
    A1 = operators.assemble(m1, dirichlet=True).toarray()
    inner = ~m1.boundary_mask()
    np.testing.assert_allclose(T.A0.toarray(), A1[np.ix_(inner, inner)], atol=1e-13 * np.abs(A1).max())


def test_two_level_is_exact_for_linear_elements_and_symmetric():
    """p = 1: the coarse space is the whole space, so the coarse correction
    solves exactly and the post-smoother adds nothing: B = A^{-1}.  For p = 2
    with equal pre- and post-sweeps B is symmetric."""
    m = graded_mesh(1, (4, 5, 3))
    inner = np.nonzero(~m.boundary_mask())[0]
    A = operators.assemble(m, dirichlet=True).tocsr()[inner][:, inner]
    r = np.zeros(m.nglob)
    r[inner] = np.random.default_rng(23).standard_normal(len(inner))
    z = twolevel.TwoLevel(m, omega=0.2)(r)
    np.testing.assert_allclose(z[inner], spla.spsolve(A.tocsc(), r[inner]), atol=1e-12 * np.abs(z).max())
    m2 = graded_mesh(2, 3)
    inner = np.nonzero(~m2.boundary_mask())[0]
    T = twolevel.TwoLevel(m2, omega=0.2)
    B = np.zeros((len(inner), len(inner)))
    for t in range(len(inner)):
        e = np.zeros(m2.nglob)
        e[inner[t]] = 1
        B[:, t] = T(e)[inner]
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh((B + B.T) / 2).min() > 0


# ------------------------------------------------ multi-block DSS (Sec. 4.2)
def test_multiblock_cube_equals_the_single_mesh():
    """The cube cut into 2^3 blocks with aligned axes is the 2n^3 mesh: its
    DSS equals the single-block DSS cell by cell."""
    p, n = 2, 3
    mb = multiblock.split_cube(p, n)
    m = Mesh(p, (2 * n,) * 3)
    rng = np.random.default_rng(31)
    v = rng.standard_normal((mb.ncells(), m.n1 ** 3))
    # block (bx, by, bz), cell (i, j, k) -> big cell (bx n + i, ...)
    big = []
    for bz in range(2):
        for by in range(2):
            for bx in range(2):
                for k in range(n):
                    for j in range(n):
                        for i in range(n):
                            big.append((bx * n + i) + 2 * n * ((by * n + j) + 2 * n * (bz * n + k)))
    big = np.asarray(big)
    vb = np.zeros((m.ncells, m.n1 ** 3))
    vb[big] = v
    np.testing.assert_allclose(mb.dss(v), operators.dss(m, vb)[big], rtol=0, atol=1e-14)


def test_multiblock_node_counts_and_multiplicities():
    """3-star (three blocks around one macro-edge): by inclusion-exclusion
    3N^3 - 3N^2 + N nodes (N = np+1 per block edge: three shared faces, one
    line shared by all); a 5-star 5N^3 - 5N^2 + N.  Multiplicities: 3 on the
    interior of the shared line, 6 at its cell vertices; a randomly oriented
    split cube has the single mesh's node count and multiplicities of the
    product form 1, 2, 4, 8."""
    for k, p, n in ((3, 2, 3), (5, 3, 2)):
        mb = multiblock.star(p, n, k, twist=True)
        N = n * p + 1
        assert mb.nglob() == k * N ** 3 - k * N ** 2 + N
        mult = mb.dss(np.ones((mb.ncells(), mb.n1 ** 3)))
        assert set(np.unique(mult).astype(int)) == {1, 2, 4, 8, k, 2 * k}
    mb = multiblock.split_cube(3, 2, np.random.default_rng(3))
    assert mb.nglob() == (2 * 2 * 3 + 1) ** 3
    mult = mb.dss(np.ones((mb.ncells(), mb.n1 ** 3)))
    assert set(np.unique(mult).astype(int)) == {1, 2, 4, 8}
    # every copy of a node carries the same assembled value, and the
    # assembled sum is preserved: sum over nodes of DSS / multiplicity
    v = np.random.default_rng(4).standard_normal(mult.shape)
    s = mb.dss(v)
    ids = mb.cell_node_ids()
    for g in np.random.default_rng(5).choice(mb.nglob(), 50, replace=False):
        vals = s[ids == g]
        assert np.all(vals == vals[0])
    assert abs((s / mult).sum() - v.sum()) < 1e-10 * np.abs(v).sum()
