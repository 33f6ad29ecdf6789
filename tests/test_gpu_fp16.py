"""FP16 (IEEE binary16 storage, FP32 arithmetic) as the reduced precision of
the smoother, beside BF16.

* apply, patch inverse and two-sweep smoother for p = 2, 3, 7 against the
  FP64 oracle at 2e-3 (FP16 keeps 11 significant bits: unit roundoff 4.9e-4
  on every stored input and output), the patch inverse bitwise continuous;
* solves to 1e-8 with the FP16 Schwarz smoother, the two-level method and
  the Jacobi preconditioner: the solver stores its FP16 residual copies
  scaled by a power of two (late residuals lie far below FP16's normal
  range), and the oracle's true residual confirms the result;
* the server with an FP16 smoother equals standalone solves bit for bit, and
  mixed-degree FP16 batches equal single-problem calls bit for bit.
"""
import numpy as np
import pytest

import synth
from oracle import operators, patches, solver
from oracle.mesh import Mesh
from tests.gpu_util import check_err, graded, note, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL16 = 2e-3


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2607_02335_amd import fem
    assert torch.cuda.is_available()
    return fem


@pytest.mark.parametrize("p,n", [(2, (5, 4, 3)), (3, (4, 3, 5)), (7, (2, 3, 3))])
def test_fp16_apply_patch_inverse_smoother(F, p, n):
    note(f"fp16 p={p} n={n}")
    m, w, rng = graded(p, n, 60 + p)
    P = F.Problem(p, n, w)
    x = P.gather(to_dev(rng.uniform(-1, 1, m.nglob)), F.F16)
    y = P.apply(x)
    check_err(to_np(P.unpack(y)), operators.apply_cells(m, to_np(P.unpack(x))), TOL16, f"fp16 apply p={p}")
    rc = rng.uniform(-1, 1, (m.ncells, m.n1 ** 3)) * ~operators.boundary_copies(m)
    rd = P.pack(to_dev(rc.ravel()), F.F16)
    z = P.patch_inverse(rd)
    f = patches.SchwarzFactors(m)
    r_glob = operators.scatter(m, to_np(P.unpack(rd)))
    check_err(to_np(P.unpack(z)), f(r_glob)[m.dofs], TOL16, f"fp16 patch inverse p={p}")
    zz = P.unpack(P.gather(P.extract(z), F.F16))
    assert bool((zz == P.unpack(z)).all())
    zs = P.smoother_step(rd, sweeps=2, omega=0.125)
    ref = solver.smoother(m, r_glob, 2, 0.125, schwarz=f)
    check_err(to_np(P.unpack(zs)), ref[m.dofs], TOL16, f"fp16 smoother p={p}")


@pytest.mark.parametrize("precond,sweeps,omega", [(0, 2, 0.125), (3, 1, 0.2), (2, 2, 0.125)])
def test_fp16_solves_reach_1e8(F, precond, sweeps, omega):
    note(f"fp16 solve precond={precond}")
    m, w, rng = graded(3, 10, 91)
    P = F.Problem(3, 10, w)
    f = rng.uniform(-1, 1, m.nglob)
    b = P.mass_apply(P.gather(to_dev(f)))
    u, info = P.pcg_solve(b, rtol=1e-8, maxit=3000, smoother_prec=F.F16, precond=precond, sweeps=sweeps,
                          omega=omega)
    assert info["status"] == 0 and info["relres"] <= 1e-8, info
    u32, i32 = P.pcg_solve(b, rtol=1e-8, maxit=3000, smoother_prec=F.F32, precond=precond, sweeps=sweeps,
                           omega=omega)
    b_glob = operators.mass_global(m, f)
    ug = to_np(P.extract(u))
    true = np.linalg.norm(b_glob - operators.apply_global(m, ug)) / np.linalg.norm(b_glob)
    print(f"fp16 precond={precond}: {info['iters']} iterations (fp32 {i32['iters']}), oracle residual {true:.2e}",
          flush=True)
    assert true <= 2e-8
    assert info["iters"] <= 2 * i32["iters"] + 5


def test_fp16_server_equals_standalone(F):
    rng = np.random.default_rng(17)
    reqs = [(p, n, synth.request_rhs_nodal(p, (n, n, n), int(rng.integers(0, 2**31 - 1))))
            for p, n in [(7, 3), (3, 6), (2, 7), (3, 4)]]
    note("fp16 server")
    S = F.Server(hbm_budget=4 << 30, max_active=4, smoother_prec=F.F16, precond=F.PC_TWO_LEVEL, sweeps=1, omega=0.2)
    tickets = [S.submit(p, n, f, rtol=1e-8, maxit=800) for p, n, f in reqs]
    results = {}
    for _ in range(100000):
        S.step()
        for t in tickets:
            if t not in results:
                r = S.poll(t)
                if r is not None:
                    results[t] = r
        if len(results) == len(tickets):
            break
    S.close()
    for t, (p, n, f) in zip(tickets, reqs):
        u_srv, info = results[t]
        assert info["status"] == 0 and info["relres"] <= 1e-8, info
        P = F.Problem(p, n)
        b = P.mass_apply(P.gather(to_dev(f)))
        u, inf1 = P.pcg_solve(b, rtol=1e-8, maxit=800, smoother_prec=F.F16, precond=F.PC_TWO_LEVEL, sweeps=1,
                              omega=0.2)
        assert inf1["iters"] == info["iters"]
        np.testing.assert_array_equal(u_srv, to_np(P.extract(u)))
        m = Mesh(p, (n, n, n))
        bg = operators.mass_global(m, f)
        assert np.linalg.norm(bg - operators.apply_global(m, u_srv)) / np.linalg.norm(bg) <= 2e-8


def test_fp16_mixed_batch_equals_single(F):
    probs = [(7, (2, 2, 3)), (3, (5, 3, 4)), (2, (7, 4, 3))]
    note("fp16 mixed batch")
    B = F.Batch([(p, n, None) for p, n in probs])
    assert B.mixed
    rng = np.random.default_rng(23)
    meshes = [Mesh(p, n) for p, n in probs]
    xs = [P.gather(to_dev(rng.uniform(-1, 1, m.nglob)), F.F16) for P, m in zip(B.problems, meshes)]
    ys = [P.cell_vector(F.F16) for P in B.problems]
    zs = [P.cell_vector(F.F16) for P in B.problems]
    B.apply(xs, ys)
    B.patch_inverse(ys, zs)
    for P, x, y, z in zip(B.problems, xs, ys, zs):
        assert bool((P.apply(x) == y).all())
        assert bool((P.patch_inverse(y) == z).all())
    B.close()
