"""The Python binding rejects caller buffers the library would read or write
out of bounds (length, dtype, layout, device), before any library call.

Runs on the CPU: the checks come before the handle is touched, so a
problem object with the sizes of a real one but no device handle is enough.
"""
import numpy as np
import pytest
import torch

from paper_2607_02335_amd import fem


def fake_problem(p=2, n=(3, 4, 5)):
    P = object.__new__(fem.Problem)
    P.p, P.n, P.h, P._owned = p, n, None, False
    P.num_cells = n[0] * n[1] * n[2]
    P.cell_len = -(-P.num_cells // 64) * 64 * (p + 1) ** 3
    P.global_len = (n[0] * p + 1) * (n[1] * p + 1) * (n[2] * p + 1)
    P.num_patches = (n[0] - 1) * (n[1] - 1) * (n[2] - 1)
    return P


def test_wrong_lengths_are_rejected():
    P = fake_problem()
    short = torch.zeros(P.cell_len - 1, dtype=torch.float64)
    for call in (lambda: P.apply(short), lambda: P.patch_inverse(short), lambda: P.smoother_step(short),
                 lambda: P.scatter(short), lambda: P.extract(short), lambda: P.dss(short),
                 lambda: P.dot(short, short), lambda: P.assembled_norm(short), lambda: P.pcg_solve(short),
                 lambda: P.mass_apply(short), lambda: P.unpack(short), lambda: P.convert(short, fem.F32),
                 lambda: P.gather(torch.zeros(P.global_len + 1, dtype=torch.float64)),
                 lambda: P.pack(torch.zeros(3, dtype=torch.float64))):
        with pytest.raises(ValueError, match="elements"):
            call()


def test_wrong_dtype_layout_and_output_are_rejected():
    P = fake_problem()
    x = torch.zeros(P.cell_len, dtype=torch.float64)
    with pytest.raises(ValueError, match="dtype"):
        P.apply(x, torch.zeros(P.cell_len, dtype=torch.float32))         # y must match x
    with pytest.raises(ValueError, match="dtype"):
        P.pcg_solve(torch.zeros(P.cell_len, dtype=torch.float32))       # b is FP64
    with pytest.raises(ValueError, match="dtype"):
        P.apply(torch.zeros(P.cell_len, dtype=torch.int64))
    with pytest.raises(ValueError, match="elements"):
        P.patch_inverse(x, torch.zeros(P.cell_len + 64, dtype=torch.float64))
    with pytest.raises(ValueError, match="contiguous"):
        P.apply(torch.zeros(2 * P.cell_len, dtype=torch.float64)[::2])
    with pytest.raises(ValueError, match="device memory"):
        P.apply(x)                                                       # host memory
    with pytest.raises(ValueError, match="torch tensor"):
        P.apply(np.zeros(P.cell_len))


def test_server_and_desc_checks():
    S = object.__new__(fem.Server)
    S.h, S.glen = None, {}
    with pytest.raises(ValueError, match="global nodes"):
        S.submit(2, 4, np.zeros(10))
    with pytest.raises(ValueError, match="entries"):
        fem.make_desc(2, (3, 3, 3), [np.ones(3), np.ones(2), np.ones(3)])
    B = object.__new__(fem.Batch)
    B.problems = [fake_problem(), fake_problem(3, (2, 2, 2))]
    B.h = None
    xs = [torch.zeros(P.cell_len, dtype=torch.float32) for P in B.problems]
    with pytest.raises(ValueError, match="vectors"):
        B.apply(xs[:1], xs[:1])
    with pytest.raises(ValueError, match="elements"):
        B.apply([xs[1], xs[0]], xs)
