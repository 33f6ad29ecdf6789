"""pcg_solve_noalloc (solver vectors in the library's fixed device scratch)
against pcg_solve on the same inputs: bit for bit, on two calls in a row
whose second is smaller (the scratch keeps the first call's contents), for
the Schwarz smoother in FP64 and FP32 and for the Jacobi preconditioner;
and a clear FEM_EINVAL for a problem whose vectors exceed the scratch."""
import numpy as np
import pytest

from oracle import operators
from tests.gpu_util import graded, note, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2607_02335_amd import fem
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    fem.lib()
    return fem


def _rhs(F, p, n, seed):
    m, w, rng = graded(p, n, seed)
    P = F.Problem(p, n, w)
    f = rng.uniform(-1, 1, m.nglob)
    return m, P, f, P.mass_apply(P.gather(to_dev(f)))


@pytest.mark.parametrize("sp,pc", [(0, 0), (1, 0), (0, 2)])
def test_noalloc_equals_pcg_solve_twice(F, sp, pc):
    cases = [(3, (9, 7, 8), 311), (2, (4, 3, 5), 312)]          # second call smaller
    for p, n, seed in cases:
        note(f"noalloc p={p} n={n} sp={sp} pc={pc}")
        m, P, f, b = _rhs(F, p, n, seed)
        u_ref, i_ref = P.pcg_solve(b, rtol=1e-8, maxit=2000, smoother_prec=sp, precond=pc)
        u = P.cell_vector()
        u, info = P.pcg_solve_noalloc(b, u, rtol=1e-8, maxit=2000, smoother_prec=sp, precond=pc)
        assert info["status"] == 0 and info["iters"] == i_ref["iters"] and info["relres"] == i_ref["relres"]
        np.testing.assert_array_equal(to_np(u), to_np(u_ref))
        b_glob = operators.mass_global(m, f)
        true = np.linalg.norm(b_glob - operators.apply_global(m, to_np(P.extract(u)))) / np.linalg.norm(b_glob)
        print(f"noalloc p={p} n={n} sp={sp} pc={pc}: {info['iters']} iterations, oracle residual {true:.2e}",
              flush=True)
        assert true <= 2e-8


def test_noalloc_rejects_problems_beyond_the_scratch(F):
    cap = F.lib().fem_noalloc_scratch_bytes()
    assert cap == 64 << 20
    note("noalloc too large")
    P = F.Problem(3, (32, 32, 32))                 # 2.1M entries: five FP64 vectors exceed 64 MiB
    assert 40 * P.cell_len > cap
    b = P.cell_vector()
    with pytest.raises(F.FemError) as e:
        P.pcg_solve_noalloc(b, P.cell_vector(), smoother_prec=F.F64)
    assert e.value.status == F.FEM_EINVAL and "scratch" in str(e.value)
