"""Error paths of the device calls, forced from the host with ordinary
inputs (every kernel runs to its normal end):

* a non-finite right-hand side makes pcg_solve report FEM_EBREAKDOWN after
  the first check instead of iterating on NaNs, for both preconditioner
  families and both (F)PCG variants; the server retires such a request with
  the same status and keeps serving the others;
* a maxit too small to converge returns FEM_ENOTCONV with the reached
  relative residual;
* aliased input and output pointers are rejected with FEM_EINVAL before any
  launch, and the output is left untouched.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import note, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2607_02335_amd import fem
    assert torch.cuda.is_available()
    return fem


@pytest.mark.parametrize("precond,variant", [(0, 1), (0, 2), (3, 2), (2, 1)])
def test_nonfinite_rhs_is_breakdown(F, precond, variant):
    note(f"NaN right-hand side precond={precond} variant={variant}")
    P = F.Problem(3, (4, 3, 5))
    f = np.ones(P.global_len)
    f[len(f) // 2] = np.nan
    b = P.mass_apply(P.gather(to_dev(f)))
    u, info = P.pcg_solve(b, rtol=1e-8, maxit=50, smoother_prec=F.F32, variant=variant, precond=precond,
                          raise_on_error=False)
    assert info["status"] == F.FEM_EBREAKDOWN, info
    assert info["iters"] == 0


def test_maxit_reports_not_converged(F):
    note("maxit too small")
    P = F.Problem(2, 6)
    f = synth.request_rhs_nodal(2, (6, 6, 6), 3)
    b = P.mass_apply(P.gather(to_dev(f)))
    u, info = P.pcg_solve(b, rtol=1e-12, maxit=3, raise_on_error=False)
    assert info["status"] == F.FEM_ENOTCONV and info["iters"] == 3
    assert 1e-12 < info["relres"] < 1.0
    with pytest.raises(F.FemError) as e:
        P.pcg_solve(b, rtol=1e-12, maxit=3)
    assert e.value.status == F.FEM_ENOTCONV


def test_server_retires_breakdown_and_serves_the_rest(F):
    note("server with a NaN request")
    S = F.Server(hbm_budget=2 << 30, max_active=4, smoother_prec=F.F32)
    good = [synth.request_rhs_nodal(2, (5, 5, 5), s) for s in (1, 2)]
    bad = np.ones((5 * 2 + 1) ** 3)
    bad[7] = np.inf
    tickets = [S.submit(2, 5, good[0]), S.submit(2, 5, bad), S.submit(2, 5, good[1])]
    results = {}
    for _ in range(10000):
        S.step()
        for t in tickets:
            if t not in results:
                r = S.poll(t)
                if r is not None:
                    results[t] = r
        if len(results) == 3:
            break
    S.close()
    assert results[tickets[1]][1]["status"] == F.FEM_EBREAKDOWN
    for t in (tickets[0], tickets[2]):
        assert results[t][1]["status"] == F.FEM_OK and results[t][1]["relres"] <= 1e-8


def test_aliased_pointers_rejected(F):
    import torch
    from paper_2607_02335_amd import fem
    note("aliasing")
    P = F.Problem(2, (3, 4, 2))
    x = P.gather(to_dev(np.linspace(0.0, 1.0, P.global_len)))
    keep = x.clone()
    calls = [
        ("fe_apply", lambda: fem.lib().fe_apply(P.h, x.data_ptr(), x.data_ptr(), F.F64)),
        ("fe_mass_apply", lambda: fem.lib().fe_mass_apply(P.h, x.data_ptr(), x.data_ptr(), F.F64)),
        ("patch_inverse", lambda: fem.lib().patch_inverse(P.h, x.data_ptr(), x.data_ptr(), F.F64)),
        ("smoother_step", lambda: fem.lib().smoother_step(P.h, x.data_ptr(), x.data_ptr(), F.F64, 2, 0.125)),
        ("fem_distribute_assembled", lambda: fem.lib().fem_distribute_assembled(P.h, x.data_ptr(), x.data_ptr(), F.F64)),
    ]
    for name, call in calls:
        st = call()
        assert st == F.FEM_EINVAL, (name, st)
        assert b"alias" in fem.lib().fem_last_error(), name
    torch.cuda.synchronize()
    assert bool((x == keep).all())
