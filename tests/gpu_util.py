"""Shared helpers of the GPU tests (device tensors <-> oracle arrays)."""
import sys

import numpy as np

from oracle.mesh import Mesh


def note(msg):
    """Name the case on stdout before a GPU step (flushed)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def cuda():
    import torch
    return torch


def to_dev(a):
    torch = cuda()
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def to_np(t):
    return t.detach().float().cpu().numpy().astype(np.float64) if t.dtype != cuda().float64 \
        else t.detach().cpu().numpy()


def graded(p, n, seed):
    rng = np.random.default_rng(seed)
    n3 = (n, n, n) if isinstance(n, int) else tuple(n)
    w = []
    for nd in n3:
        v = rng.uniform(0.5, 1.5, nd)
        w.append(v / v.sum())
    return Mesh(p, n3, w), w, rng


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def l2_rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def check_err(got, ref, tol, what):
    """Both error measures of a result against the oracle (max-abs error over
    the largest oracle entry, and the l2 norm of the error over the oracle's),
    printed, each at most `tol`."""
    mx = rel_err(got, ref)
    l2 = l2_rel(np.ravel(got), np.ravel(ref))
    print(f"[err] {what}: max-abs {mx:.3e}, l2 {l2:.3e} (bound {tol:.0e})", flush=True)
    assert mx <= tol and l2 <= tol, (what, mx, l2, tol)
    return mx, l2
