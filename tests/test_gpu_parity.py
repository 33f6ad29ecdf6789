"""Parity of the HIP path against the oracle on small meshes that span
several storage blocks and end in a ragged block.

Tolerances, for both the max-abs error relative to the largest oracle entry
and the l2-relative error (each printed): FP64 1e-12 (apply, patch inverse,
smoother); FP32 1e-5, the bound stated for the FP32 smoother step; BF16
storage with FP32 arithmetic 1e-2 (one BF16 rounding of input and output,
2^-9 relative each, amplified by the patch operators' conditioning; the
measured worst case is 4e-3).
"""
import numpy as np
import pytest

from oracle import operators, patches, solver
from oracle.mesh import Mesh
from tests.gpu_util import check_err, graded, l2_rel, note, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5, 2: 1e-2}


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2607_02335_amd import fem
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    fem.lib()
    return fem


def make(F, mesh, widths=None, bc=0):
    return F.Problem(mesh.p, mesh.n, widths if widths is not None else mesh.h, bc)


# ------------------------------------------------------------ apply
def test_apply_q2_8cubed_uniform(F):
    """Q2, 8^3 uniform cells, Dirichlet, x ~ U[-1,1] seed 0."""
    note("apply q2 8^3 uniform")
    m = Mesh(2, (8, 8, 8))
    x = np.random.default_rng(0).uniform(-1, 1, m.nglob)
    P = make(F, m)
    y = P.apply(P.gather(to_dev(x)))
    yc = to_np(P.unpack(y))
    ref = operators.apply_cells(m, operators.gather(m, x))
    assert rel_err(yc, ref) <= 1e-12
    yg = to_np(P.scatter(y))
    assert l2_rel(yg, operators.apply_global(m, x)) <= 1e-12


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_apply_all_degrees_ragged(F, p, prec):
    n = (5, 3, 4) if p < 6 else (3, 2, 3)
    note(f"apply p={p} prec={prec} n={n}")
    m, w, rng = graded(p, n, 100 + p)
    xc = rng.uniform(-1, 1, (m.ncells, m.n1 ** 3))      # broken (dual-like) input: every copy differs
    P = make(F, m)
    xd = P.pack(to_dev(xc.ravel()), prec)
    xin = to_np(P.unpack(xd))                            # what the device holds after rounding
    y = to_np(P.unpack(P.apply(xd)))
    ref = operators.apply_cells(m, xin)
    check_err(y, ref, TOL[prec], f"apply p={p} prec={prec}")


@pytest.mark.parametrize("p", [2, 3, 7])
def test_apply_neumann_and_mass(F, p):
    n = (4, 3, 5) if p < 7 else (3, 2, 2)
    note(f"neumann/mass p={p}")
    m, w, rng = graded(p, n, 7)
    x = rng.uniform(-1, 1, m.nglob)
    Pn = make(F, m, bc=1)
    y = to_np(Pn.scatter(Pn.apply(Pn.gather(to_dev(x)))))
    assert rel_err(y, operators.apply_global(m, x, dirichlet=False)) <= 1e-12
    ones = to_np(Pn.scatter(Pn.apply(Pn.gather(to_dev(np.ones(m.nglob))))))
    assert np.abs(ones).max() <= 1e-12 * np.abs(y).max()
    Pd = make(F, m)
    ym = to_np(Pd.scatter(Pd.mass_apply(Pd.gather(to_dev(x)))))
    assert rel_err(ym, operators.mass_global(m, x)) <= 1e-12


# ------------------------------------------------ converters, DSS, reductions
@pytest.mark.parametrize("p", [1, 3, 7])
def test_converters_and_dss(F, p):
    n = (6, 3, 4) if p < 7 else (3, 2, 3)
    note(f"converters/dss p={p}")
    m, w, rng = graded(p, n, 3)
    P = make(F, m)
    x = rng.standard_normal(m.nglob)
    xc = P.gather(to_dev(x))
    np.testing.assert_array_equal(to_np(P.unpack(xc)), operators.gather(m, x))
    np.testing.assert_array_equal(to_np(P.extract(xc)), x)
    v = rng.standard_normal((m.ncells, m.n1 ** 3))
    vd = P.pack(to_dev(v.ravel()))
    np.testing.assert_allclose(to_np(P.scatter(vd)), operators.scatter(m, v), rtol=0, atol=1e-12)
    s = to_np(P.unpack(P.dss(vd)))
    np.testing.assert_allclose(s, operators.dss(m, v), rtol=0, atol=1e-12)
    # every copy of a node holds the identical bits after the cascade
    sd = P.dss(vd)
    np.testing.assert_array_equal(to_np(P.unpack(P.gather(P.extract(sd)))), to_np(P.unpack(sd)))
    mult = to_np(P.unpack(P.dss(P.pack(to_dev(np.ones(v.size))))))
    np.testing.assert_array_equal(mult, m.multiplicity()[m.dofs])


def test_dss_cascade_worked_example(F):
    """The 2D four-cell example of Section 4.1, one axis pass at a time."""
    import os
    rows = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "dss_vertex_2d.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                t = line.split()
                rows[t[0]] = [float(q) for q in t[1:]]
    note("dss worked example")
    m = Mesh(1, (2, 2, 1))
    P = make(F, m)
    g = m.gidx(1, 1, 0)
    cells = {"nw": 2, "ne": 3, "sw": 0, "se": 1}
    v = np.zeros((4, 8))
    loc = {}
    for key, val in zip(["nw", "ne", "sw", "se"], rows["initial"]):
        e = cells[key]
        loc[key] = int(np.nonzero(m.dofs[e] == g)[0][0])
        v[e, loc[key]] = val
    vd = P.pack(to_dev(v.ravel()))
    for axis, stage in ((0, "after_x"), (1, "after_y")):
        P.dss_axis(vd, axis)
        got = to_np(P.unpack(vd))
        assert [got[cells[k], loc[k]] for k in ["nw", "ne", "sw", "se"]] == rows[stage]


def test_dot_and_assembled_norm(F):
    note("dot/norm")
    m, w, rng = graded(3, (7, 5, 3), 9)
    P = make(F, m)
    a = rng.standard_normal((m.ncells, m.n1 ** 3))
    u = rng.standard_normal(m.nglob)
    ad = P.pack(to_dev(a.ravel()))
    ud = P.gather(to_dev(u))
    ref = np.sum(a * operators.gather(m, u))
    assert abs(P.dot(ad, ud) - ref) <= 1e-12 * abs(ref) + 1e-12
    # pairing lemma on the device: <f, G u> = <G^T f, u>
    assert abs(P.dot(ad, ud) - operators.scatter(m, a) @ u) <= 1e-11 * np.abs(a).sum()
    nrm = np.linalg.norm(operators.scatter(m, a))
    assert abs(P.assembled_norm(ad) - nrm) <= 1e-12 * nrm
    assert P.dot(ad, P.convert(ud, 1)) == pytest.approx(ref, rel=1e-6)


# ---------------------------------------------------------- patch inverse
@pytest.mark.parametrize("p,n", [(1, (4, 3, 5)), (2, (5, 4, 3)), (3, (4, 5, 3)), (4, (3, 4, 3)),
                                 (5, (3, 2, 3)), (6, (2, 3, 2)), (7, (3, 3, 2)), (2, (2, 2, 2)),
                                 (3, (9, 2, 3))])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_patch_inverse_matches_lu(F, p, n, prec):
    note(f"patch_inverse p={p} n={n} prec={prec}")
    m, w, rng = graded(p, n, 20 + p)
    P = make(F, m)
    rc = rng.uniform(-1, 1, (m.ncells, m.n1 ** 3)) * ~operators.boundary_copies(m)
    rd = P.pack(to_dev(rc.ravel()), prec)
    rin = to_np(P.unpack(rd))
    z = P.patch_inverse(rd)
    zc = to_np(P.unpack(z))
    ref = patches.SchwarzFactors(m)(operators.scatter(m, rin))
    check_err(zc, ref[m.dofs], TOL[prec], f"patch_inverse p={p} n={n} prec={prec}")
    # exact continuity: every copy of a node holds the same bits
    zz = to_np(P.unpack(P.gather(P.extract(z), prec)))
    np.testing.assert_array_equal(zz, zc)


def test_patch_inverse_sees_only_the_assembly(F):
    """Two cell-wise residuals with the same assembly give the same output."""
    note("patch_inverse consistency")
    m, w, rng = graded(3, (4, 4, 3), 5)
    P = make(F, m)
    r = rng.standard_normal(m.nglob) * ~m.boundary_mask()
    split = rng.standard_normal((m.ncells, m.n1 ** 3))
    a = operators.gather(m, r) / m.multiplicity()[m.dofs]
    b = a + split - operators.gather(m, operators.scatter(m, split)) / m.multiplicity()[m.dofs]
    np.testing.assert_allclose(operators.scatter(m, b), operators.scatter(m, a), atol=1e-12)
    za = to_np(P.unpack(P.patch_inverse(P.pack(to_dev(a.ravel())))))
    zb = to_np(P.unpack(P.patch_inverse(P.pack(to_dev(b.ravel())))))
    assert rel_err(za, zb) <= 1e-12


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_smoother_matches_oracle(F, prec):
    note(f"smoother prec={prec}")
    m, w, rng = graded(2, (4, 5, 4), 31)
    P = make(F, m)
    rc = rng.uniform(-1, 1, (m.ncells, m.n1 ** 3)) * ~operators.boundary_copies(m)
    rd = P.pack(to_dev(rc.ravel()), prec)
    z = to_np(P.unpack(P.smoother_step(rd, sweeps=2, omega=0.125)))
    f = patches.SchwarzFactors(m)
    ref = solver.smoother(m, operators.scatter(m, to_np(P.unpack(rd))), 2, 0.125, schwarz=f)
    check_err(z, ref[m.dofs], TOL[prec], f"smoother 2 sweeps prec={prec}")
    z3 = to_np(P.unpack(P.smoother_step(rd, sweeps=3, omega=0.2)))
    ref3 = solver.smoother(m, operators.scatter(m, to_np(P.unpack(rd))), 3, 0.2, schwarz=f)
    check_err(z3, ref3[m.dofs], TOL[prec], f"smoother 3 sweeps prec={prec}")


# ---------------------------------------------------------------- solver
@pytest.mark.parametrize("variant,code", [("pcg", 1), ("fcg", 2)])
def test_pcg_iterates_equal_assembled_iterates(F, variant, code):
    """Equivalence theorem (Section 3.2): cell-wise iterates = G (assembled
    iterates), checked for the first iterations with the FP64 smoother, for
    the static (PCG) and the flexible (FCG) beta.  Stopping after k steps
    also checks the u update the direction pass carries one step late."""
    m, w, rng = graded(2, (4, 4, 5), 41)
    P = make(F, m)
    f = rng.uniform(-1, 1, m.nglob)
    b_glob = operators.mass_global(m, f)
    _, _, _, its = solver.solve_poisson(m, b_glob, rtol=1e-30, maxit=6, variant=variant, record=True)
    bd = P.mass_apply(P.gather(to_dev(f)))
    for k in range(1, 7):
        note(f"{variant} iterate k={k}")
        u, info = P.pcg_solve(bd, rtol=1e-30, maxit=k, smoother_prec=0, variant=code, raise_on_error=False)
        assert info["status"] == 4 and info["iters"] == k
        uk = to_np(P.extract(u))
        assert l2_rel(uk, its[k]) <= 1e-10
        np.testing.assert_array_equal(to_np(P.unpack(P.gather(P.extract(u)))), to_np(P.unpack(u)))


@pytest.mark.parametrize("p,n", [(2, (4, 3, 5)), (3, (3, 4, 3)), (7, (2, 3, 2))])
@pytest.mark.parametrize("sp", [0, 1, 2])
def test_bubble_solve(F, p, n, sp):
    """u = x(1-x)y(1-y)z(1-z) lies in Q_p: the discrete solution is its
    interpolant, whatever the smoother precision."""
    note(f"bubble p={p} n={n} sp={sp}")
    m, w, rng = graded(p, n, 50 + p)
    X, Y, Z = (m.coords_1d(d) for d in range(3))
    bx, by, bz = X * (1 - X), Y * (1 - Y), Z * (1 - Z)
    u_ex = np.kron(np.kron(bz, by), bx)
    one = np.ones_like
    f = 2 * (np.kron(np.kron(bz, by), one(bx)) + np.kron(np.kron(bz, one(by)), bx) + np.kron(np.kron(one(bz), by), bx))
    P = make(F, m)
    bd = P.mass_apply(P.gather(to_dev(f)))
    u, info = P.pcg_solve(bd, rtol=1e-10, maxit=500, smoother_prec=sp)
    assert info["status"] == 0 and info["relres"] <= 1e-10
    assert np.abs(to_np(P.extract(u)) - u_ex).max() <= 1e-9


@pytest.mark.parametrize("prec", [1, 2])
def test_distribute_assembled_before_demotion(F, prec):
    """A dual vector whose copies cancel under assembly (as a converging
    residual's do): demoting it copy by copy loses its assembly, assembling
    in FP64 first keeps it to the precision's relative accuracy."""
    note(f"distribute prec={prec}")
    m, w, rng = graded(3, (5, 4, 3), 77)
    P = make(F, m)
    small = rng.standard_normal(m.nglob) * ~m.boundary_mask() * 1e-8
    noise = rng.standard_normal((m.ncells, m.n1 ** 3)) * ~operators.boundary_copies(m)
    cancel = noise - operators.gather(m, operators.scatter(m, noise)) / m.multiplicity()[m.dofs]
    rc = operators.gather(m, small) / m.multiplicity()[m.dofs] + cancel     # G^T rc = small
    rd = P.pack(to_dev(rc.ravel()))
    exact = operators.scatter(m, rc)
    d = P.distribute_assembled(rd, prec)
    got = to_np(P.scatter(d))
    tol = {1: 1e-6, 2: 1e-2}[prec]
    assert l2_rel(got, exact) <= tol
    naive = to_np(P.scatter(P.convert(rd, prec)))
    assert l2_rel(naive, exact) > 10 * tol          # the floor the FP64 assembly avoids
    # every copy of a node holds the same value
    np.testing.assert_array_equal(to_np(P.unpack(P.gather(P.extract(d), prec))), to_np(P.unpack(d)))


@pytest.mark.parametrize("p,n", [(2, (17, 5, 9)), (3, (10, 3, 7)), (1, (33, 6, 5)), (3, (19, 9, 13)),
                                 (3, (40, 4, 3)), (2, (70, 3, 3))])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("mode", [1, 2])
def test_fused_sweep_matches_two_phase(F, p, n, prec, mode):
    """The fused patch sweeps (mode 1: restriction from the cell copies,
    mode 2: from the assembled residual) and the patch-buffer path solve the
    same patches and combine them in the same order; the sweep's output is
    continuous bit for bit and matches the oracle's additive Schwarz."""
    note(f"sweep mode {mode} vs two-phase p={p} n={n} prec={prec}")
    m, w, rng = graded(p, n, 90 + p)
    P = make(F, m)
    rd = P.pack(to_dev(rng.uniform(-1, 1, m.ncells * m.n1 ** 3)), prec)
    try:
        F.set_option(F.OPT_PI_FUSED, 0)
        z1 = to_np(P.unpack(P.smoother_step(rd, sweeps=2, omega=0.3)))
        F.set_option(F.OPT_PI_FUSED, mode)
        z2 = to_np(P.unpack(P.smoother_step(rd, sweeps=2, omega=0.3)))
        zc = P.patch_inverse(rd)
    finally:
        F.set_option(F.OPT_PI_FUSED, -1)
    assert rel_err(z1, z2) <= {0: 1e-14, 1: 1e-6}[prec]
    np.testing.assert_array_equal(to_np(P.unpack(P.gather(P.extract(zc), prec))), to_np(P.unpack(zc)))
    zref = patches.SchwarzFactors(m)(operators.scatter(m, to_np(P.unpack(rd)).astype(np.float64)))
    check_err(to_np(P.unpack(zc)), zref[m.dofs], TOL[prec], f"sweep mode {mode} p={p} n={n} prec={prec}")


@pytest.mark.parametrize("p,n", [(2, (9, 5, 4)), (3, (7, 4, 5)), (7, (3, 4, 2))])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("opt,val", [("PI_FUSED", 0), ("PI_FUSED", 1), ("PI_FUSED", 2), ("PI_FUSED", 3), ("PI_FUSED", 4),
                                     ("COMBINE_PER_CELL", 1), ("RESTRICT_FROM_CELLS", 1)])
def test_patch_inverse_variants_agree(F, p, n, prec, opt, val):
    """Every kernel-variant switch gives the default path's patch inverse up
    to summation-order rounding, continuous bit for bit."""
    if p > 3 and (opt != "PI_FUSED" or val >= 3):
        pytest.skip("switch only affects p <= 3")
    note(f"variant {opt}={val} p={p} n={n} prec={prec}")
    m, w, rng = graded(p, n, 50 + p)
    P = make(F, m)
    rd = P.pack(to_dev(rng.uniform(-1, 1, m.ncells * m.n1 ** 3)), prec)
    z0 = to_np(P.unpack(P.patch_inverse(rd)))
    code = getattr(F, "OPT_" + opt)
    F.set_option(code, val)
    try:
        zc = P.patch_inverse(rd)
    finally:
        F.set_option(code, -1 if opt == "PI_FUSED" else 0)
    z1 = to_np(P.unpack(zc))
    assert rel_err(z1, z0) <= {0: 1e-13, 1: 1e-6}[prec]
    np.testing.assert_array_equal(to_np(P.unpack(P.gather(P.extract(zc), prec))), z1)


@pytest.mark.parametrize("p,n,prec", [(3, (12, 10, 20), 0), (3, (9, 11, 30), 1), (2, (20, 9, 17), 0),
                                      (3, (50, 3, 8), 0), (2, (70, 4, 9), 1)])
def test_patch_inverse_slabs_identical(F, p, n, prec):
    """The z-slab schedule runs the same solve kernel on the same data:
    results are identical to one solve and one combine launch, for the plain
    and the accumulating (smoother) form.  In FP64 on rows of at least 48
    cells the single launch combines by global node rows while the slabs
    combine per (block, plane), so that case also shows the two combines
    agree bit for bit."""
    note(f"slabs p={p} n={n} prec={prec}")
    m, w, rng = graded(p, n, 70 + p)
    P = make(F, m)
    rd = P.pack(to_dev(rng.uniform(-1, 1, m.ncells * m.n1 ** 3)), prec)
    F.set_option(F.OPT_PI_FUSED, 0)
    try:
        z0 = to_np(P.unpack(P.patch_inverse(rd)))
        s0 = to_np(P.unpack(P.smoother_step(rd, sweeps=2, omega=0.3)))
        F.set_option(F.OPT_PI_SLAB_MB, 1)
        z1 = to_np(P.unpack(P.patch_inverse(rd)))
        s1 = to_np(P.unpack(P.smoother_step(rd, sweeps=2, omega=0.3)))
    finally:
        F.set_option(F.OPT_PI_SLAB_MB, 0)
        F.set_option(F.OPT_PI_FUSED, -1)
    np.testing.assert_array_equal(z1, z0)
    np.testing.assert_array_equal(s1, s0)


@pytest.mark.parametrize("p,n", [(3, (1, 4, 3)), (2, (5, 1, 1)), (7, (2, 1, 2)), (1, (1, 1, 1))])
@pytest.mark.parametrize("prec", [0, 1])
def test_degenerate_meshes(F, p, n, prec):
    """Meshes with one cell along a direction have no interior vertex: the
    patch inverse (and so the smoother) returns exactly zero, the apply still
    matches the oracle, and a solve converges at once on the zero system."""
    note(f"degenerate p={p} n={n} prec={prec}")
    m, w, rng = graded(p, n, 11)
    P = make(F, m)
    xc = rng.uniform(-1, 1, (m.ncells, m.n1 ** 3))
    xd = P.pack(to_dev(xc.ravel()), prec)
    z = to_np(P.unpack(P.patch_inverse(xd)))
    assert not np.any(z)
    assert not np.any(to_np(P.unpack(P.smoother_step(xd, sweeps=2, omega=0.3))))
    y = to_np(P.unpack(P.apply(xd)))
    assert rel_err(y, operators.apply_cells(m, to_np(P.unpack(xd)))) <= TOL[prec]


@pytest.mark.parametrize("p,n", [(3, (48, 2, 3)), (3, (65, 3, 2)), (2, (129, 2, 3)), (1, (80, 3, 2)), (7, (48, 2, 2)),
                                 (7, (64, 2, 2))])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_patch_inverse_long_rows(F, p, n, prec):
    """Rows of at least 48 cells take the assembly with lanes over cells (64
    cells per pass, the first lane of a later pass reading its left
    neighbour directly): at the threshold, one past a full pass, and two
    passes with a ragged tail, the patch inverse matches the oracle's
    additive Schwarz (all cells for p <= 3; for p = 7 the cells at both ends
    and the middle of every row, whose corner patches the oracle factors
    densely) and stays continuous bit for bit."""
    note(f"long rows p={p} n={n} prec={prec}")
    m, w, rng = graded(p, n, 60 + p)
    P = make(F, m)
    rd = P.pack(to_dev(rng.uniform(-1, 1, m.ncells * m.n1 ** 3)), prec)
    zc = P.patch_inverse(rd)
    z = to_np(P.unpack(zc))
    np.testing.assert_array_equal(to_np(P.unpack(P.gather(P.extract(zc), prec))), z)
    r_glob = operators.scatter(m, to_np(P.unpack(rd)).astype(np.float64))
    tol = TOL[prec]
    if p <= 3:
        zref = patches.SchwarzFactors(m)(r_glob)
        check_err(z, zref[m.dofs], tol, f"long rows p={p} n={n} prec={prec}")
    else:
        rows = np.arange(m.n[1] * m.n[2]) * m.n[0]
        cells = np.unique(np.concatenate([rows, rows + m.n[0] // 2, rows + m.n[0] - 1]))
        zref = patches.additive_schwarz_at_cells(m, r_glob, cells)
        check_err(z[cells], zref, tol, f"long rows p={p} n={n} prec={prec}")
