"""Batched launches and the continuous-batching solve server.

* A batch of independent problems of mixed degree and size (drawn like the
  256-problem workload, smaller) runs FP32 apply and patch inverse in one
  launch per degree; each problem's result must equal its own single-problem
  launch bit for bit and match the FP64 oracle within the FP32 tolerance.
* The server's solves must equal standalone pcg_solve runs of the same
  problems: every per-problem reduction has a fixed order independent of
  what else is in flight, so a result is the same alone and in the mix.
"""
import numpy as np
import pytest

import synth
from oracle import operators, patches
from oracle.mesh import Mesh
from tests.gpu_util import check_err, note, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2607_02335_amd import fem
    assert torch.cuda.is_available()
    return fem


def small_batch(count=12, seed=3, nmax=7):
    return synth.batch_problems(count=count, seed=seed, nmin=2, nmax=nmax)


def test_batch_equals_single_and_oracle(F):
    wls = small_batch()
    note(f"batch of {len(wls)}: " + " ".join(f"q{w.p}n{w.n[0]}" for w in wls))
    B = F.Batch([(w.p, w.n, None) for w in wls])
    xs = [P.gather(to_dev(w.x), F.F32) for P, w in zip(B.problems, wls)]
    ys = [P.cell_vector(F.F32) for P in B.problems]
    zs = [P.cell_vector(F.F32) for P in B.problems]
    B.apply(xs, ys)
    B.patch_inverse(ys, zs)
    for P, w, x, y, z in zip(B.problems, wls, xs, ys, zs):
        m = Mesh(w.p, w.n, w.widths)
        ys1 = P.apply(x)
        assert bool((ys1 == y).all()), f"apply q{w.p} n{w.n}"
        zs1 = P.patch_inverse(y)
        assert bool((zs1 == z).all()), f"patch inverse q{w.p} n{w.n}"
        yref = operators.apply_cells(m, to_np(P.unpack(x)))
        check_err(to_np(P.unpack(y)), yref, 1e-5, f"batch apply q{w.p} n{w.n[0]}")
        zref = patches.SchwarzFactors(m)(operators.scatter(m, to_np(P.unpack(y))))
        check_err(to_np(P.unpack(z)), zref[m.dofs], 1e-5, f"batch patch inverse q{w.p} n{w.n[0]}")


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_long_rows_equals_single(F, prec):
    """Every mesh of a launch has at least 48 cells along x, so the batched
    launches take the assembly with lanes over cells and (FP64, p <= 3) the
    combine by global node rows: each problem's patch inverse equals its own
    single-problem launch bit for bit and matches the oracle."""
    probs = [(3, (50, 2, 3)), (3, (64, 3, 2)), (2, (70, 2, 2)), (2, (49, 3, 2))]
    note(f"long-row batch prec={prec}")
    B = F.Batch([(p, n, None) for p, n in probs])
    rng = np.random.default_rng(8)
    meshes = [Mesh(p, n) for p, n in probs]
    rs = [P.pack(to_dev(rng.uniform(-1, 1, m.ncells * m.n1 ** 3)), prec) for P, m in zip(B.problems, meshes)]
    zs = [P.cell_vector(prec) for P in B.problems]
    B.patch_inverse(rs, zs)
    for P, m, r, z in zip(B.problems, meshes, rs, zs):
        z1 = P.patch_inverse(r)
        assert bool((z1 == z).all()), f"patch inverse q{m.p} n{m.n}"
        zref = patches.SchwarzFactors(m)(operators.scatter(m, to_np(P.unpack(r)).astype(np.float64)))
        check_err(to_np(P.unpack(z)), zref[m.dofs], {0: 1e-12, 1: 1e-5}[prec], f"long-row batch q{m.p} prec={prec}")


def test_batch_autotune(F):
    wls = small_batch(count=9, seed=5)
    B = F.Batch([(w.p, w.n, None) for w in wls])
    xs = [P.gather(to_dev(w.x), F.F32) for P, w in zip(B.problems, wls)]
    ys = [P.cell_vector(F.F32) for P in B.problems]
    B.apply(xs, ys)
    before = [to_np(y).copy() for y in ys]
    note("autotune")
    choice = B.autotune(F.F32)
    assert set(choice) == {w.p for w in wls}
    B.apply(xs, ys)
    for y, y0 in zip(ys, before):
        assert rel_err(to_np(y), y0) <= 1e-6


def _requests(F, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        p = int(rng.choice([2, 3, 7]))
        n = int(rng.integers(3, 6 if p == 7 else 9))
        f = synth.request_rhs_nodal(p, (n, n, n), int(rng.integers(0, 2**31 - 1)))
        out.append((p, n, f))
    return out


@pytest.mark.parametrize("sp,pc", [(0, 0), (1, 0), (0, 3), (1, 3)])
def test_server_matches_standalone_solves(F, sp, pc):
    """Every served solution equals its standalone pcg_solve bit for bit and
    meets the 1e-8 target on the oracle's own residual ||b - A_D u|| / ||b||;
    a zero source is solved at once (u = 0, no iteration), as pcg_solve
    returns it."""
    reqs = _requests(F, 8, 11 + sp)
    reqs.insert(3, (3, 4, np.zeros(synth.global_len(3, (4, 4, 4)))))
    note(f"server sp={sp} pc={pc}: " + " ".join(f"q{p}n{n}" for p, n, _ in reqs))
    sweeps, omega = (2, 0.125) if pc == 0 else (1, 0.2)
    S = F.Server(hbm_budget=8 << 30, max_active=4, smoother_prec=sp, precond=pc, sweeps=sweeps, omega=omega)
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
    assert len(results) == len(tickets)
    for t, (p, n, f) in zip(tickets, reqs):
        u_srv, info = results[t]
        assert info["status"] == 0 and info["relres"] <= 1e-8
        P = F.Problem(p, n)
        b = P.mass_apply(P.gather(to_dev(f)))
        u, inf1 = P.pcg_solve(b, rtol=1e-8, maxit=800, smoother_prec=sp, precond=pc, sweeps=sweeps, omega=omega)
        assert inf1["iters"] == info["iters"]
        np.testing.assert_array_equal(u_srv, to_np(P.extract(u)))
        if not np.any(f):
            assert info["iters"] == 0 and not np.any(u_srv)
            continue
        m = Mesh(p, (n, n, n))
        b_glob = operators.mass_global(m, f)
        true = np.linalg.norm(b_glob - operators.apply_global(m, u_srv)) / np.linalg.norm(b_glob)
        print(f"served q{p} n{n}: {info['iters']} iterations, oracle residual {true:.2e}", flush=True)
        assert true <= 2e-8
    S.close()


def test_server_long_rows_fp64_smoother(F):
    """Requests of 48^3 cells with the FP64 smoother: two p = 3 solves share
    the batched launches, so the server's smoother takes the assembly with
    lanes over cells and the accumulating combine by global node rows; every
    solve equals its standalone pcg_solve bit for bit."""
    rng = np.random.default_rng(5)
    reqs = [(3, 48, synth.request_rhs_nodal(3, (48, 48, 48), int(rng.integers(0, 2**31 - 1)))),
            (3, 48, synth.request_rhs_nodal(3, (48, 48, 48), int(rng.integers(0, 2**31 - 1)))),
            (2, 48, synth.request_rhs_nodal(2, (48, 48, 48), int(rng.integers(0, 2**31 - 1))))]
    note("server long rows, FP64 smoother")
    S = F.Server(hbm_budget=16 << 30, max_active=4, smoother_prec=F.F64)
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
    assert len(results) == len(tickets)
    for t, (p, n, f) in zip(tickets, reqs):
        u_srv, info = results[t]
        assert info["status"] == 0 and info["relres"] <= 1e-8
        P = F.Problem(p, n)
        b = P.mass_apply(P.gather(to_dev(f)))
        u, inf1 = P.pcg_solve(b, rtol=1e-8, maxit=800, smoother_prec=F.F64)
        assert inf1["iters"] == info["iters"]
        np.testing.assert_array_equal(u_srv, to_np(P.extract(u)))
        m = Mesh(p, (n, n, n))
        b_glob = operators.mass_global(m, f)
        true = np.linalg.norm(b_glob - operators.apply_global(m, u_srv)) / np.linalg.norm(b_glob)
        assert true <= 2e-8, true
    S.close()


def test_server_admission_by_memory(F):
    reqs = _requests(F, 6, 21)
    fps = [F.footprint_bytes(p, n, F.F32) for p, n, _ in reqs]
    budget = int(max(fps) * 1.5)                     # at most one or two solves in flight
    S = F.Server(hbm_budget=budget, max_active=8, smoother_prec=F.F32)
    big = F.footprint_bytes(7, 48, F.F32)
    with pytest.raises(F.FemError) as e:
        S.submit(7, 48, np.zeros((48 * 7 + 1) ** 3))
    assert e.value.status == F.FEM_ENOMEM and big > budget
    tickets = [S.submit(p, n, f) for p, n, f in reqs]
    pending = set(tickets)
    max_active = 0
    for _ in range(100000):
        a, q, d = S.step()
        max_active = max(max_active, a)
        in_use, hw = S.memory()
        assert in_use <= budget
        fin = S.finished()
        assert fin == sorted(fin) and set(fin) <= pending
        for t in list(pending):
            r = S.poll(t, want_u=False)
            assert (r is not None) == (t in fin)
            if r is not None:
                assert r[1]["status"] == 0
                pending.discard(t)
        if not pending:
            break
    assert not pending
    assert S.memory()[1] <= budget
    S.close()


def test_threaded_stream_driver(F):
    """The stream driver steps the server on its own thread while the client
    thread submits and collects; every request of a short burst completes."""
    from paper_2607_02335_amd import serve
    reqs = synth.serve_stream(count=40, rate=400.0, seed=9, nmax=8)
    note("threaded stream of 40 requests")
    res = serve.run_stream(reqs, hbm_budget=4 << 30, max_active=16)
    assert res["requests"] == 40 and res["failures"] == 0
    assert res["mean_iters"] > 0 and res["p99_latency_s"] >= res["p50_latency_s"] > 0
    assert res["hbm_high_water_bytes"] <= 4 << 30
