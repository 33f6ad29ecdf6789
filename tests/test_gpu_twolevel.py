"""The two-level preconditioner on the GPU against the oracle.

* fem_two_level: one application (smoothing sweeps, exact Q1 coarse
  correction, sweeps) element by element against the oracle's
  oracle.twolevel.TwoLevel (prolongation by interpolation, Galerkin coarse
  operator, sparse LU), continuous bit for bit, zero on the boundary.
* pcg_solve_pc(FEM_PC_TWO_LEVEL): the first iterates equal the oracle's
  assembled PCG iterates with the same preconditioner (equivalence theorem,
  Section 3.2); solves reach 1e-8 on the oracle's true residual with FP64,
  FP32, BF16 and FP16 smoothers, and the iteration count does not grow with the
  mesh (the coarse level carries the low frequencies).
"""
import numpy as np
import pytest

import synth
from oracle import operators, solver, twolevel
from oracle.mesh import Mesh
from tests.gpu_util import check_err, graded, l2_rel, note, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5, 2: 1e-2}


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2607_02335_amd import fem
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    fem.lib()
    return fem


@pytest.mark.parametrize("p,n", [(1, (5, 4, 6)), (2, (4, 5, 3)), (3, (6, 3, 5)), (7, (3, 2, 3)), (3, (1, 4, 3))])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_two_level_apply_matches_oracle(F, p, n, prec):
    note(f"two-level p={p} n={n} prec={prec}")
    m, w, rng = graded(p, n, 170 + p)
    P = F.Problem(p, n, w)
    rc = rng.uniform(-1, 1, (m.ncells, m.n1 ** 3)) * ~operators.boundary_copies(m)
    rd = P.pack(to_dev(rc.ravel()), prec)
    for sweeps, omega in ((1, 0.2), (2, 0.125)):
        zd = P.two_level(rd, sweeps=sweeps, omega=omega)
        z = to_np(P.unpack(zd))
        ref = twolevel.TwoLevel(m, omega, sweeps, sweeps)(operators.scatter(m, to_np(P.unpack(rd))))
        check_err(z, ref[m.dofs], TOL[prec], f"two-level p={p} n={n} prec={prec} sweeps={sweeps}")
        np.testing.assert_array_equal(to_np(P.unpack(P.gather(P.extract(zd), prec))), z)
        assert not np.any(z[operators.boundary_copies(m)])


def test_two_level_pcg_iterates(F):
    m, w, rng = graded(2, (5, 4, 6), 181)
    P = F.Problem(2, m.n, w)
    f = rng.uniform(-1, 1, m.nglob)
    b_glob = operators.mass_global(m, f)
    T = twolevel.TwoLevel(m, 0.2, 1, 1)
    _, _, _, its = solver.fcg(lambda v: operators.apply_global(m, v), T, b_glob, rtol=1e-30, maxit=6,
                              variant="pcg", record=True)
    bd = P.mass_apply(P.gather(to_dev(f)))
    for k in range(1, 7):
        note(f"two-level iterate k={k}")
        u, info = P.pcg_solve(bd, rtol=1e-30, maxit=k, precond=F.PC_TWO_LEVEL, sweeps=1, omega=0.2,
                              raise_on_error=False)
        assert info["status"] == 4 and info["iters"] == k
        assert l2_rel(to_np(P.extract(u)), its[k]) <= 1e-10
        np.testing.assert_array_equal(to_np(P.unpack(P.gather(P.extract(u)))), to_np(P.unpack(u)))


@pytest.mark.parametrize("p", [2, 3, 7])
def test_two_level_iterations_do_not_grow_with_the_mesh(F, p):
    counts = {}
    for n in ((4, 8, 16) if p < 7 else (3, 6, 12)):
        m, w, rng = graded(p, n, 190 + p)
        P = F.Problem(p, n, w)
        f = rng.uniform(-1, 1, m.nglob)
        bd = P.mass_apply(P.gather(to_dev(f)))
        note(f"two-level solve p={p} n={n}")
        u, info = P.pcg_solve(bd, rtol=1e-8, maxit=500, precond=F.PC_TWO_LEVEL, smoother_prec=F.F32,
                              sweeps=1, omega=0.2)
        assert info["status"] == 0 and info["relres"] <= 1e-8
        b_glob = operators.mass_global(m, f)
        true = np.linalg.norm(b_glob - operators.apply_global(m, to_np(P.extract(u)))) / np.linalg.norm(b_glob)
        _, k1, _, _ = solver.solve_poisson(m, b_glob, rtol=1e-8, maxit=2000) if n <= 8 else (0, -1, 0, 0)
        print(f"p={p} n={n}: two-level {info['iters']} iterations (Schwarz alone {k1}), oracle residual {true:.2e}",
              flush=True)
        assert true <= 2e-8
        counts[n] = info["iters"]
    ns = sorted(counts)
    assert counts[ns[-1]] <= counts[ns[0]] + 6, counts


def test_q7_24_two_level_solves(F):
    wl = synth.workload_q7_graded()
    m = Mesh(7, wl.n, wl.widths)
    P = F.Problem(7, wl.n, wl.widths)
    X = [F.node_coords(7, wl.widths[d]) for d in range(3)]
    f = np.kron(np.kron(np.sin(np.pi * X[2]), np.sin(np.pi * X[1])), np.sin(np.pi * X[0])) + 0.01 * wl.noise
    bd = P.mass_apply(P.gather(to_dev(f)))
    b_glob = operators.mass_global(m, f)
    sol = {}
    for name, sp in (("fp64", 0), ("fp32", 1), ("bf16", 2), ("fp16", 3)):
        note(f"q7 24^3 two-level solve smoother={name}")
        u, info = P.pcg_solve(bd, rtol=1e-8, maxit=1000, smoother_prec=sp, precond=F.PC_TWO_LEVEL, sweeps=1,
                              omega=0.2)
        assert info["status"] == 0 and info["relres"] <= 1e-8, info
        ug = to_np(P.extract(u))
        true = np.linalg.norm(b_glob - operators.apply_global(m, ug)) / np.linalg.norm(b_glob)
        print(f"{name}: {info['iters']} iterations, true {true:.2e}, {info['seconds']:.3f} s", flush=True)
        assert true <= 2e-8, (name, true)
        sol[name] = ug
    for name in ("fp32", "bf16", "fp16"):
        assert l2_rel(sol[name], sol["fp64"]) <= 1e-5
