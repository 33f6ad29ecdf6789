"""Parity at the benchmark's other full-size workloads, in the launch
configuration the benchmark times.

* Q2, 96^3 graded cells (seed 1; the same 193^3 nodes as Q3 64^3): the full
  FP64 apply against the oracle (13,824 storage blocks, so the register
  kernel's persistent grid wraps), and the FP64 patch inverse (the fused
  sweep from the assembled residual, the default for p = 2 in FP64) on
  sampled cells against dense LU of their corner patches.
* The batch of 256 independent problems (p uniform in {2, 3, 7}, n uniform
  in [4, 32], seed 3): autotuned kernel shapes, FP32 apply of every problem
  against the oracle's cell-wise apply, and the FP32 patch inverse on
  sampled cells of every problem (every fourth p = 7 problem: dense LU of a
  2197^2 patch is the oracle's slow step) against dense LU.
"""
import numpy as np
import pytest

import synth
from oracle import operators, patches
from oracle.mesh import Mesh
from tests.gpu_util import check_err, note, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2607_02335_amd import fem
    assert torch.cuda.is_available()
    return fem


def test_q2_96_apply_full_and_patch_inverse_sampled(F):
    wl = synth.workload_q2_graded()
    m = Mesh(2, wl.n, wl.widths)
    P = F.Problem(2, wl.n, wl.widths)
    note("q2 96^3 apply FP64")
    xd = P.gather(to_dev(wl.x))
    y = P.apply(xd)
    check_err(to_np(P.unpack(y)), operators.apply_cells(m, operators.gather(m, wl.x)), 1e-12, "q2 96^3 apply")
    note("q2 96^3 patch inverse FP64")
    z = P.patch_inverse(y)
    rng = np.random.default_rng(96)
    cells = np.unique(np.concatenate([[0, 95, 96 * 96 - 1, m.ncells // 2, m.ncells - 1],
                                      rng.integers(0, m.ncells, 40)]))
    r = operators.scatter(m, to_np(P.unpack(y)))
    ref = patches.additive_schwarz_at_cells(m, r, cells)
    check_err(to_np(P.unpack(z))[cells], ref, 1e-12, "q2 96^3 patch inverse")
    zz = P.unpack(P.gather(P.extract(z)))
    assert bool((zz == P.unpack(z)).all())


def test_batch_256_fp32_against_oracle(F):
    wls = synth.batch_problems(count=256, seed=3)
    note("batch of 256 problems, FP32, autotuned")
    B = F.Batch([(w.p, w.n, None) for w in wls])
    xs = [P.gather(to_dev(w.x), F.F32) for P, w in zip(B.problems, wls)]
    ys = [P.cell_vector(F.F32) for P in B.problems]
    zs = [P.cell_vector(F.F32) for P in B.problems]
    choice = B.autotune(F.F32)
    print(f"autotuned {choice}", flush=True)
    B.apply(xs, ys)
    B.patch_inverse(ys, zs)
    rng = np.random.default_rng(256)
    worst = {2: [0, 0], 3: [0, 0], 7: [0, 0]}
    k7 = 0
    for i, (P, w, x, y, z) in enumerate(zip(B.problems, wls, xs, ys, zs)):
        m = Mesh(w.p, w.n, w.widths)
        yc = to_np(P.unpack(y))
        mx, _ = check_err(yc, operators.apply_cells(m, to_np(P.unpack(x))), 1e-5, f"batch[{i}] apply q{w.p} n{w.n[0]}")
        worst[w.p][0] = max(worst[w.p][0], mx)
        if w.p == 7:
            k7 += 1
            if k7 % 4 != 1:
                continue
            cells = np.array([rng.integers(0, m.ncells)])
        else:
            cells = np.unique(np.concatenate([[0, m.ncells - 1], rng.integers(0, m.ncells, 6)]))
        ref = patches.additive_schwarz_at_cells(m, operators.scatter(m, yc), cells)
        mx, _ = check_err(to_np(P.unpack(z))[cells], ref, 1e-5, f"batch[{i}] patch inverse q{w.p} n{w.n[0]}")
        worst[w.p][1] = max(worst[w.p][1], mx)
    print(f"worst max-abs errors per degree (apply, patch inverse): {worst}", flush=True)
    B.close()
