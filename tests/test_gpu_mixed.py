"""Mixed-degree launches: one launch per kernel phase over problems of the
degrees 2, 3 and 7 together (degree-uniform workgroups running each
degree's own kernel body).

* Batched apply and patch inverse, FP64 / FP32 / BF16, Dirichlet and Neumann,
  on meshes that reach the special cases of each body (a single cell
  layer without patches, ragged last storage blocks, long x rows): the mixed
  launches give every problem the same bits as one launch per degree and as
  its own single-problem call, and the oracle's values.
* A batch holding another degree (p = 4) falls back to one launch per degree.
* The solve server with mixed launches equals the server with one launch per
  degree, solve by solve (iterations and solution bits), for the Schwarz and
  the two-level preconditioner with FP32 and FP64 smoothers.
"""
import numpy as np
import pytest

import synth
from oracle import operators, patches
from oracle.mesh import Mesh
from tests.gpu_util import check_err, note, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5, 2: 1e-2}


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2607_02335_amd import fem
    assert torch.cuda.is_available()
    return fem


# degree, cells, Neumann; (2, (1, 3, 2)) has no interior vertex, (2, (50, 2, 2))
# has long x rows, (3, (13, 5, 2)) ends in a ragged storage block
MIXED = [(7, (3, 2, 2), False), (3, (5, 4, 3), False), (2, (9, 3, 2), True), (3, (2, 2, 2), True),
         (2, (1, 3, 2), False), (7, (2, 3, 3), True), (2, (50, 2, 2), False), (3, (13, 5, 2), False)]


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_mixed_batch_equals_per_degree_and_single(F, prec):
    note(f"mixed batch prec={prec}: " + " ".join(f"q{p}n{'x'.join(map(str, n))}{'N' if nm else ''}"
                                               for p, n, nm in MIXED))
    B = F.Batch([(p, n, None, F.NEUMANN if nm else F.DIRICHLET) for p, n, nm in MIXED])
    assert B.mixed
    rng = np.random.default_rng(31 + prec)
    meshes = [Mesh(p, n) for p, n, _ in MIXED]
    xs = [P.gather(to_dev(rng.uniform(-1, 1, m.nglob)), prec) for P, m in zip(B.problems, meshes)]
    ys = [P.cell_vector(prec) for P in B.problems]
    zs = [P.cell_vector(prec) for P in B.problems]
    B.apply(xs, ys)
    B.patch_inverse(ys, zs)
    B.set_mixed(False)
    assert not B.mixed
    ys2 = [P.cell_vector(prec) for P in B.problems]
    zs2 = [P.cell_vector(prec) for P in B.problems]
    B.apply(xs, ys2)
    B.patch_inverse(ys, zs2)
    for P, m, (p, n, nm), x, y, z, y2, z2 in zip(B.problems, meshes, MIXED, xs, ys, zs, ys2, zs2):
        tag = f"q{p} n{n} neumann={nm} prec={prec}"
        assert bool((y == y2).all()), "apply mixed vs per degree " + tag
        assert bool((z == z2).all()), "patch inverse mixed vs per degree " + tag
        assert bool((P.apply(x) == y).all()), "apply mixed vs single " + tag
        assert bool((P.patch_inverse(y) == z).all()), "patch inverse mixed vs single " + tag
        yref = operators.apply_cells(m, to_np(P.unpack(x)), dirichlet=not nm)
        check_err(to_np(P.unpack(y)), yref, TOL[prec], "mixed apply " + tag)
        if not nm:
            zref = patches.SchwarzFactors(m)(operators.scatter(m, to_np(P.unpack(y))))
            check_err(to_np(P.unpack(z)), zref[m.dofs], TOL[prec], "mixed patch inverse " + tag)
    B.close()


def test_batch_with_other_degree_falls_back(F):
    probs = [(4, (3, 3, 2)), (2, (4, 3, 3)), (7, (2, 2, 3))]
    note("batch with p = 4: per-degree launches")
    B = F.Batch([(p, n, None) for p, n in probs])
    assert not B.mixed
    rng = np.random.default_rng(9)
    meshes = [Mesh(p, n) for p, n in probs]
    xs = [P.gather(to_dev(rng.uniform(-1, 1, m.nglob)), 1) for P, m in zip(B.problems, meshes)]
    ys = [P.cell_vector(1) for P in B.problems]
    zs = [P.cell_vector(1) for P in B.problems]
    B.apply(xs, ys)
    B.patch_inverse(ys, zs)
    for P, x, y, z in zip(B.problems, xs, ys, zs):
        assert bool((P.apply(x) == y).all())
        assert bool((P.patch_inverse(y) == z).all())
    B.close()


def _serve(F, reqs, sp, pc, mixed):
    sweeps, omega = (2, 0.125) if pc == 0 else (1, 0.2)
    S = F.Server(hbm_budget=8 << 30, max_active=6, smoother_prec=sp, precond=pc, sweeps=sweeps, omega=omega)
    S.set_mixed(mixed)
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
    assert len(results) == len(tickets)
    return [results[t] for t in tickets]


@pytest.mark.parametrize("sp,pc", [(1, 0), (1, 3), (0, 3)])
def test_mixed_server_equals_per_degree(F, sp, pc):
    rng = np.random.default_rng(40 + sp + pc)
    reqs = []
    for p, n in [(7, 3), (3, 6), (2, 8), (3, 4), (2, 5), (7, 4), (2, 2), (3, 7)]:
        reqs.append((p, n, synth.request_rhs_nodal(p, (n, n, n), int(rng.integers(0, 2**31 - 1)))))
    note(f"server mixed vs per degree sp={sp} pc={pc}")
    a = _serve(F, reqs, sp, pc, True)
    b = _serve(F, reqs, sp, pc, False)
    for (p, n, f), (ua, ia), (ub, ib) in zip(reqs, a, b):
        assert ia["status"] == 0 and ia["relres"] <= 1e-8, (p, n, ia)
        assert ia["iters"] == ib["iters"], (p, n)
        np.testing.assert_array_equal(ua, ub)
    # and the oracle's residual of one solve per degree
    for (p, n, f), (u, info) in list(zip(reqs, a))[:3]:
        m = Mesh(p, (n, n, n))
        bg = operators.mass_global(m, f)
        true = np.linalg.norm(bg - operators.apply_global(m, u)) / np.linalg.norm(bg)
        assert true <= 2e-8, (p, n, true)
