"""The simple preconditioners of Section 3.3 on the GPU against the oracle.

* fem_precond_apply: z = S r and z = D_cell^{-1} S r element by element
  against the oracle's assembled-space definitions (the Riesz identity, and
  division by the diagonal of the assembled operator) gathered to the
  cells, continuous bit for bit, zero on the Dirichlet boundary.
* pcg_solve_pc: the cell-wise iterates equal the oracle's assembled PCG
  iterates with the same preconditioner (the equivalence theorem of Section
  3.2), and full solves reach 1e-8 on the oracle's true residual.
"""
import numpy as np
import pytest

from oracle import operators, solver
from tests.gpu_util import check_err, graded, l2_rel, note, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2607_02335_amd import fem
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    fem.lib()
    return fem


@pytest.mark.parametrize("p,n", [(1, (5, 3, 4)), (2, (4, 5, 3)), (3, (6, 3, 5)), (7, (3, 2, 3))])
@pytest.mark.parametrize("kind", ["dss", "jacobi"])
@pytest.mark.parametrize("prec", [0, 1])
def test_precond_apply_matches_oracle(F, p, n, kind, prec):
    note(f"precond {kind} p={p} n={n} prec={prec}")
    m, w, rng = graded(p, n, 130 + p)
    P = F.Problem(p, n, w)
    rc = rng.uniform(-1, 1, (m.ncells, m.n1 ** 3))          # unassembled: every copy differs
    rd = P.pack(to_dev(rc.ravel()))
    code = F.PC_DSS if kind == "dss" else F.PC_JACOBI
    zd = P.precond_apply(rd, code, prec)
    z = to_np(P.unpack(zd))
    rg = operators.scatter(m, rc)
    ref = solver.dss_preconditioner(m, rg) if kind == "dss" else solver.jacobi(m, rg)
    check_err(z, ref[m.dofs], {0: 1e-12, 1: 1e-6}[prec], f"precond {kind} p={p} prec={prec}")
    np.testing.assert_array_equal(to_np(P.unpack(P.gather(P.extract(zd), prec))), z)
    assert not np.any(z[operators.boundary_copies(m)])


@pytest.mark.parametrize("kind", ["dss", "jacobi"])
def test_pcg_simple_preconditioner_iterates(F, kind):
    """Equivalence theorem (Section 3.2) with P = S and P = D_cell^{-1} S:
    the first iterates equal the oracle's assembled PCG iterates."""
    m, w, rng = graded(3, (4, 5, 4), 141)
    P = F.Problem(3, m.n, w)
    f = rng.uniform(-1, 1, m.nglob)
    b_glob = operators.mass_global(m, f)
    _, _, _, its = solver.solve_poisson(m, b_glob, rtol=1e-30, maxit=6, precond=kind, record=True)
    bd = P.mass_apply(P.gather(to_dev(f)))
    code = F.PC_DSS if kind == "dss" else F.PC_JACOBI
    for k in range(1, 7):
        note(f"{kind} iterate k={k}")
        u, info = P.pcg_solve(bd, rtol=1e-30, maxit=k, precond=code, raise_on_error=False)
        assert info["status"] == 4 and info["iters"] == k
        assert l2_rel(to_np(P.extract(u)), its[k]) <= 1e-10
        np.testing.assert_array_equal(to_np(P.unpack(P.gather(P.extract(u)))), to_np(P.unpack(u)))


@pytest.mark.parametrize("p,n", [(2, (6, 5, 7)), (3, (5, 6, 4)), (7, (3, 3, 4))])
@pytest.mark.parametrize("kind", ["dss", "jacobi"])
def test_pcg_simple_preconditioner_solves(F, p, n, kind):
    m, w, rng = graded(p, n, 150 + p)
    P = F.Problem(p, n, w)
    f = rng.uniform(-1, 1, m.nglob)
    b_glob = operators.mass_global(m, f)
    bd = P.mass_apply(P.gather(to_dev(f)))
    note(f"solve {kind} p={p} n={n}")
    code = F.PC_DSS if kind == "dss" else F.PC_JACOBI
    u, info = P.pcg_solve(bd, rtol=1e-8, maxit=5000, precond=code)
    assert info["status"] == 0 and info["relres"] <= 1e-8, info
    true = np.linalg.norm(b_glob - operators.apply_global(m, to_np(P.extract(u)))) / np.linalg.norm(b_glob)
    print(f"{kind} p={p} n={n}: {info['iters']} iterations, oracle residual {true:.2e}", flush=True)
    assert true <= 2e-8
    # the oracle's own solve with the same preconditioner agrees
    u_ref, k_ref, _, _ = solver.solve_poisson(m, b_glob, rtol=1e-8, maxit=5000, precond=kind)
    assert abs(k_ref - info["iters"]) <= max(2, k_ref // 50)
    assert l2_rel(to_np(P.extract(u)), u_ref) <= 1e-6
