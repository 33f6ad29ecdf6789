"""Thin ctypes binding of libfem_mi355x.so (argument marshalling only).

PyTorch supplies device memory and the current stream; every step of the
computation runs in the library's HIP kernels.  The binding fails loudly if
the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfem_mi355x.so")
HEADER = os.path.join(HERE, "..", "include", "fem.h")

FEM_OK, FEM_EINVAL, FEM_ENOMEM, FEM_EHIP, FEM_ENOTCONV, FEM_EBREAKDOWN, FEM_EAGAIN, FEM_ENOTFOUND = range(8)
F64, F32, BF16, F16 = 0, 1, 2, 3
DIRICHLET, NEUMANN = 0, 1
CG_AUTO, CG_PCG, CG_FCG = 0, 1, 2
PC_SCHWARZ, PC_DSS, PC_JACOBI, PC_TWO_LEVEL = 0, 1, 2, 3
STATUS_NAMES = {0: "FEM_OK", 1: "FEM_EINVAL", 2: "FEM_ENOMEM", 3: "FEM_EHIP", 4: "FEM_ENOTCONV",
                5: "FEM_EBREAKDOWN", 6: "FEM_EAGAIN", 7: "FEM_ENOTFOUND"}


class FemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Desc(ct.Structure):
    _fields_ = [("p", ct.c_int), ("n", ct.c_int * 3), ("widths", ct.POINTER(ct.c_double) * 3),
                ("bc", ct.c_int)]


class TraceRec(ct.Structure):
    _fields_ = [("label", ct.c_char * 48), ("p", ct.c_int), ("prec", ct.c_int), ("launches", ct.c_int),
                ("total_ms", ct.c_double)]


class SolveInfo(ct.Structure):
    _fields_ = [("iters", ct.c_int), ("status", ct.c_int), ("relres", ct.c_double),
                ("seconds", ct.c_double)]


_lib = None


def lib():
    """Load the HIP library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2607_02335_amd.build first")
    L = ct.CDLL(LIB_PATH)
    vp, i, d, sz = ct.c_void_p, ct.c_int, ct.c_double, ct.c_size_t
    pp = ct.POINTER(vp)
    sigs = {
        "fem_problem_create": ([ct.POINTER(Desc), vp, pp], i),
        "fem_problem_destroy": ([vp], i),
        "fem_set_stream": ([vp, vp], i),
        "fem_cell_len": ([vp], sz), "fem_global_len": ([vp], sz),
        "fem_num_cells": ([vp], sz), "fem_num_patches": ([vp], sz),
        "fem_footprint_bytes": ([ct.POINTER(Desc), i], sz),
        "fem_prec_bytes": ([i], sz),
        "fem_gather": ([vp, vp, vp, i], i), "fem_scatter": ([vp, vp, vp, i], i),
        "fem_extract": ([vp, vp, vp, i], i), "fem_pack": ([vp, vp, vp, i], i),
        "fem_unpack": ([vp, vp, vp, i], i), "fem_convert": ([vp, vp, i, vp, i], i),
        "fem_distribute_assembled": ([vp, vp, vp, i], i),
        "fe_apply": ([vp, vp, vp, i], i), "fe_mass_apply": ([vp, vp, vp, i], i),
        "fem_dss": ([vp, vp, vp, i], i), "fem_dss_axis": ([vp, vp, i, i], i),
        "patch_inverse": ([vp, vp, vp, i], i),
        "smoother_step": ([vp, vp, vp, i, i, d], i),
        "fem_two_level": ([vp, vp, vp, i, i, d], i),
        "fem_dot": ([vp, vp, i, vp, i, ct.POINTER(d)], i),
        "fem_assembled_norm": ([vp, vp, i, ct.POINTER(d)], i),
        "pcg_solve": ([vp, vp, vp, d, i, i, i, d, i, ct.POINTER(SolveInfo)], i),
        "pcg_solve_pc": ([vp, vp, vp, d, i, i, i, i, d, i, ct.POINTER(SolveInfo)], i),
        "fem_precond_apply": ([vp, i, vp, vp, i], i),
        "pcg_solve_noalloc": ([vp, vp, vp, d, i, i, i, i, d, i, ct.POINTER(SolveInfo)], i),
        "fem_noalloc_scratch_bytes": ([], sz),
        "fem_batch_create": ([i, ct.POINTER(Desc), vp, pp], i),
        "fem_batch_destroy": ([vp], i),
        "fem_batch_problem": ([vp, i, pp], i),
        "fem_batch_apply": ([vp, pp, pp, i], i),
        "fem_batch_patch_inverse": ([vp, pp, pp, i], i),
        "fem_batch_autotune": ([vp, i, ct.POINTER(i)], i),
        "fem_batch_set_mixed": ([vp, i], i),
        "fem_batch_mixed": ([vp], i),
        "fem_server_set_mixed": ([vp, i], i),
        "fem_server_create": ([sz, i, i, i, d, vp, pp], i),
        "fem_server_destroy": ([vp], i),
        "fem_server_create_pc": ([sz, i, i, i, i, d, vp, pp], i),
        "fem_server_submit": ([vp, ct.POINTER(Desc), vp, d, i, ct.POINTER(ct.c_uint64)], i),
        "fem_server_step": ([vp, ct.POINTER(i), ct.POINTER(i), ct.POINTER(i)], i),
        "fem_server_poll": ([vp, ct.c_uint64, vp, ct.POINTER(SolveInfo)], i),
        "fem_server_memory": ([vp, ct.POINTER(sz), ct.POINTER(sz)], i),
        "fem_server_finished": ([vp, ct.POINTER(ct.c_uint64), i], i),
        "fem_server_stats": ([vp, ct.POINTER(d), i], i),
        "fem_mb_create": ([i, i, vp, vp, vp, pp], i),
        "fem_mb_destroy": ([vp], i),
        "fem_mb_cell_len": ([vp], sz),
        "fem_mb_block_offset": ([vp, i], sz),
        "fem_mb_pack": ([vp, vp, vp, i], i),
        "fem_mb_unpack": ([vp, vp, vp, i], i),
        "fem_mb_dss": ([vp, vp, i, i], i),
        "fem_mb_stats": ([vp, ct.POINTER(i), i], i),
        "fem_layout_len": ([i, vp, i], sz),
        "fem_layout_pack": ([i, vp, i, vp, vp, i, vp], i),
        "fem_layout_mass": ([i, vp, i, i, vp, vp, vp], i),
        "fem_layout_dss": ([i, vp, i, vp, vp], i),
        "fem_host_1d_matrices": ([i, vp, vp], i),
        "fem_host_fd_1d": ([i, d, d, vp, vp], i),
        "fem_host_gll_nodes": ([i, vp], i),
        "fem_set_option": ([i, i], i),
        "fem_trace_enable": ([i], i),
        "fem_trace_read": ([ct.POINTER(TraceRec), i], i),
        "fem_last_error": ([], ct.c_char_p),
        "fem_version": ([], ct.c_char_p),
    }
    for name, (args, res) in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def header_functions():
    """Names of the functions include/fem.h declares."""
    with open(HEADER) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b([A-Za-z_][A-Za-z0-9_]*)\s*\([^;{]*\)\s*;", src)) -
                  {"if", "while", "for", "return", "sizeof"})


def check(status, what=""):
    if status != FEM_OK:
        msg = lib().fem_last_error().decode()
        raise FemError(status, f"{what}: {msg}" if what else msg)
    return status


# ---------------------------------------------------------------- helpers
def _ptr(t):
    """Device address of a torch tensor (or None)."""
    if t is None:
        return None
    return ct.c_void_p(t.data_ptr())


def _torch():
    import torch
    return torch


def torch_dtype(prec):
    torch = _torch()
    return {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16, F16: torch.float16}[prec]


def prec_of(t):
    torch = _torch()
    return {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16, torch.float16: F16}[t.dtype]


def _check_vec(t, length, prec=None, name="vector"):
    """Reject a caller-supplied tensor the library would read or write out of
    bounds: it must be a contiguous tensor of `length` elements and, when
    given, of the dtype of precision `prec` (its device is checked by
    _require_cuda once every argument has passed this)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.numel() != length:
        raise ValueError(f"{name}: has {t.numel()} elements, expected {length}")
    if t.dtype not in (torch.float64, torch.float32, torch.bfloat16, torch.float16):
        raise ValueError(f"{name}: unsupported dtype {t.dtype}")
    if prec is not None and t.dtype != torch_dtype(prec):
        raise ValueError(f"{name}: dtype {t.dtype} does not match precision {prec} ({torch_dtype(prec)})")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    return t


def _require_cuda(*ts):
    """Every given tensor must live in device memory (checked after the
    sizes and dtypes of all arguments)."""
    for t in ts:
        if t is not None and t.device.type != "cuda":
            raise ValueError(f"vector on {t.device}: the library takes device memory")


def _stream():
    torch = _torch()
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_desc(p, n, widths=None, bc=DIRICHLET):
    if isinstance(n, int):
        n = (n, n, n)
    d = Desc()
    d.p = int(p)
    for k in range(3):
        d.n[k] = int(n[k])
    keep = []
    for k in range(3):
        if widths is None or widths[k] is None:
            d.widths[k] = ct.POINTER(ct.c_double)()
        else:
            w = np.ascontiguousarray(widths[k], dtype=np.float64)
            if w.ndim != 1 or w.size != int(n[k]):
                raise ValueError(f"widths[{k}]: has {w.size} entries, the mesh has {int(n[k])} cells")
            keep.append(w)
            d.widths[k] = w.ctypes.data_as(ct.POINTER(ct.c_double))
    d.bc = int(bc)
    d._keep = keep
    return d


OPT_PI_FUSED = 1
OPT_COMBINE_PER_CELL = 2
OPT_RESTRICT_FROM_CELLS = 3
OPT_PI_SLAB_MB = 4
OPT_APPLY_PLANES_P7 = 5


def set_option(option, value):
    check(lib().fem_set_option(option, value), "fem_set_option")


def trace_enable(on=True):
    """Start (or stop) recording per-launch HIP event pairs."""
    check(lib().fem_trace_enable(1 if on else 0), "fem_trace_enable")


def trace_read():
    """Aggregated launch durations since the last read: a list of dicts
    {label, p, prec, launches, total_ms, avg_us}."""
    cap = 512
    recs = (TraceRec * cap)()
    n = min(cap, lib().fem_trace_read(recs, cap))
    return [dict(label=r.label.decode(), p=r.p, prec=r.prec, launches=r.launches, total_ms=r.total_ms,
                 avg_us=r.total_ms * 1e3 / max(r.launches, 1)) for r in recs[:n]]


def host_1d_matrices(p):
    n1 = p + 1
    M = np.zeros((n1, n1))
    K = np.zeros((n1, n1))
    check(lib().fem_host_1d_matrices(p, M.ctypes.data, K.ctypes.data), "fem_host_1d_matrices")
    return M, K


def host_gll_nodes(p):
    x = np.zeros(p + 1)
    check(lib().fem_host_gll_nodes(p, x.ctypes.data), "fem_host_gll_nodes")
    return x


def node_coords(p, widths):
    """Coordinates of the global node planes along one direction."""
    xi = host_gll_nodes(p)
    w = np.asarray(widths, dtype=np.float64)
    v = np.concatenate(([0.0], np.cumsum(w)))
    X = np.empty(len(w) * p + 1)
    for i in range(len(w)):
        X[i * p:(i + 1) * p + 1] = v[i] + w[i] * xi
    X[::p] = v
    return X


def host_fd_1d(p, h0, h1):
    nP = 2 * p - 1
    S = np.zeros((nP, nP))
    lam = np.zeros(nP)
    check(lib().fem_host_fd_1d(p, h0, h1, S.ctypes.data, lam.ctypes.data), "fem_host_fd_1d")
    return S, lam


def footprint_bytes(p, n, smoother_prec=F32, widths=None):
    d = make_desc(p, n, widths)
    return lib().fem_footprint_bytes(ct.byref(d), smoother_prec)


class Problem:
    """A Q_p Poisson problem on a graded box mesh, resident on the GPU."""

    def __init__(self, p, n, widths=None, bc=DIRICHLET, _handle=None):
        self.p = int(p)
        self.n = (n, n, n) if isinstance(n, int) else tuple(int(v) for v in n)
        self.widths = widths
        self.bc = bc
        self._owned = _handle is None
        if _handle is None:
            d = make_desc(p, self.n, widths, bc)
            h = ct.c_void_p()
            check(lib().fem_problem_create(ct.byref(d), _stream(), ct.byref(h)), "fem_problem_create")
            self.h = h
        else:
            self.h = _handle
        L = lib()
        self.cell_len = L.fem_cell_len(self.h)
        self.global_len = L.fem_global_len(self.h)
        self.num_cells = L.fem_num_cells(self.h)
        self.num_patches = L.fem_num_patches(self.h)

    def close(self):
        if getattr(self, "h", None) and self._owned:
            lib().fem_problem_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self, *tensors):
        _require_cuda(*tensors)
        lib().fem_set_stream(self.h, _stream())

    def _cell(self, t, prec, name):
        """Check a caller's cell-wise vector (length, dtype, device, layout)."""
        return _check_vec(t, self.cell_len, prec, name)

    # vectors -------------------------------------------------------------
    def cell_vector(self, prec=F64):
        torch = _torch()
        return torch.zeros(self.cell_len, dtype=torch_dtype(prec), device="cuda")

    def gather(self, x_glob, prec=F64):
        _check_vec(x_glob, self.global_len, F64, "x_glob")
        self._sync_stream(x_glob)
        out = self.cell_vector(prec)
        check(lib().fem_gather(self.h, _ptr(x_glob), _ptr(out), prec), "fem_gather")
        return out

    def scatter(self, y_cell):
        self._cell(y_cell, None, "y_cell")
        self._sync_stream(y_cell)
        torch = _torch()
        out = torch.empty(self.global_len, dtype=torch.float64, device="cuda")
        check(lib().fem_scatter(self.h, _ptr(y_cell), _ptr(out), prec_of(y_cell)), "fem_scatter")
        return out

    def extract(self, u_cell):
        self._cell(u_cell, None, "u_cell")
        self._sync_stream(u_cell)
        torch = _torch()
        out = torch.empty(self.global_len, dtype=torch.float64, device="cuda")
        check(lib().fem_extract(self.h, _ptr(u_cell), _ptr(out), prec_of(u_cell)), "fem_extract")
        return out

    def pack(self, canon, prec=F64):
        _check_vec(canon, self.num_cells * (self.p + 1) ** 3, F64, "canon")
        self._sync_stream(canon)
        out = self.cell_vector(prec)
        check(lib().fem_pack(self.h, _ptr(canon), _ptr(out), prec), "fem_pack")
        return out

    def unpack(self, v_cell):
        self._cell(v_cell, None, "v_cell")
        self._sync_stream(v_cell)
        torch = _torch()
        nn = (self.p + 1) ** 3
        out = torch.empty(self.num_cells * nn, dtype=torch.float64, device="cuda")
        check(lib().fem_unpack(self.h, _ptr(v_cell), _ptr(out), prec_of(v_cell)), "fem_unpack")
        return out.view(self.num_cells, nn)

    def convert(self, src, prec):
        self._cell(src, None, "src")
        self._sync_stream(src)
        out = self.cell_vector(prec)
        check(lib().fem_convert(self.h, _ptr(src), prec_of(src), _ptr(out), prec), "fem_convert")
        return out

    def distribute_assembled(self, r, prec):
        """G^T r / multiplicity per copy in `prec` (r dual FP64)."""
        self._cell(r, F64, "r")
        self._sync_stream(r)
        out = self.cell_vector(prec)
        check(lib().fem_distribute_assembled(self.h, _ptr(r), _ptr(out), prec), "fem_distribute_assembled")
        return out

    # operators -----------------------------------------------------------
    def apply(self, x, y=None):
        self._cell(x, None, "x")
        if y is not None:
            self._cell(y, prec_of(x), "y")
        _require_cuda(x, y)
        y = self.cell_vector(prec_of(x)) if y is None else y
        self._sync_stream()
        check(lib().fe_apply(self.h, _ptr(x), _ptr(y), prec_of(x)), "fe_apply")
        return y

    def mass_apply(self, x, y=None):
        self._cell(x, None, "x")
        if y is not None:
            self._cell(y, prec_of(x), "y")
        _require_cuda(x, y)
        y = self.cell_vector(prec_of(x)) if y is None else y
        self._sync_stream()
        check(lib().fe_mass_apply(self.h, _ptr(x), _ptr(y), prec_of(x)), "fe_mass_apply")
        return y

    def dss(self, v, s=None):
        self._cell(v, None, "v")
        if s is not None:
            self._cell(s, prec_of(v), "s")
        _require_cuda(v, s)
        s = self.cell_vector(prec_of(v)) if s is None else s
        self._sync_stream()
        check(lib().fem_dss(self.h, _ptr(v), _ptr(s), prec_of(v)), "fem_dss")
        return s

    def dss_axis(self, v, axis):
        self._cell(v, None, "v")
        self._sync_stream(v)
        check(lib().fem_dss_axis(self.h, _ptr(v), axis, prec_of(v)), "fem_dss_axis")
        return v

    def patch_inverse(self, r, z=None):
        self._cell(r, None, "r")
        if z is not None:
            self._cell(z, prec_of(r), "z")
        _require_cuda(r, z)
        z = self.cell_vector(prec_of(r)) if z is None else z
        self._sync_stream()
        check(lib().patch_inverse(self.h, _ptr(r), _ptr(z), prec_of(r)), "patch_inverse")
        return z

    def smoother_step(self, r, z=None, sweeps=2, omega=0.125):
        self._cell(r, None, "r")
        if z is not None:
            self._cell(z, prec_of(r), "z")
        _require_cuda(r, z)
        z = self.cell_vector(prec_of(r)) if z is None else z
        self._sync_stream()
        check(lib().smoother_step(self.h, _ptr(r), _ptr(z), prec_of(r), sweeps, omega), "smoother_step")
        return z

    def two_level(self, r, z=None, sweeps=1, omega=0.2):
        """z = B r: smoothing sweeps, exact Q1 coarse correction, sweeps."""
        self._cell(r, None, "r")
        if z is not None:
            self._cell(z, prec_of(r), "z")
        _require_cuda(r, z)
        z = self.cell_vector(prec_of(r)) if z is None else z
        self._sync_stream()
        check(lib().fem_two_level(self.h, _ptr(r), _ptr(z), prec_of(r), sweeps, omega), "fem_two_level")
        return z

    def dot(self, a, b):
        self._cell(a, None, "a")
        self._cell(b, None, "b")
        self._sync_stream(a, b)
        out = ct.c_double()
        check(lib().fem_dot(self.h, _ptr(a), prec_of(a), _ptr(b), prec_of(b), ct.byref(out)), "fem_dot")
        return out.value

    def assembled_norm(self, r):
        self._cell(r, None, "r")
        self._sync_stream(r)
        out = ct.c_double()
        check(lib().fem_assembled_norm(self.h, _ptr(r), prec_of(r), ct.byref(out)), "fem_assembled_norm")
        return out.value

    def precond_apply(self, r, kind=PC_JACOBI, prec=F64, z=None):
        """z = S r (PC_DSS) or D_cell^{-1} S r (PC_JACOBI); r dual FP64."""
        self._cell(r, F64, "r")
        if z is not None:
            self._cell(z, prec, "z")
        _require_cuda(r, z)
        z = self.cell_vector(prec) if z is None else z
        self._sync_stream()
        check(lib().fem_precond_apply(self.h, kind, _ptr(r), _ptr(z), prec), "fem_precond_apply")
        return z

    def pcg_solve(self, b, u=None, rtol=1e-8, maxit=1000, smoother_prec=F64, sweeps=2,
                  omega=0.125, variant=CG_AUTO, raise_on_error=True, precond=PC_SCHWARZ):
        """Solve A u = b (b dual, FP64).  Returns (u, info dict)."""
        self._cell(b, F64, "b")
        if u is not None:
            self._cell(u, F64, "u")
        _require_cuda(b, u)
        u = self.cell_vector(F64) if u is None else u
        self._sync_stream()
        info = SolveInfo()
        if precond == PC_SCHWARZ:
            st = lib().pcg_solve(self.h, _ptr(b), _ptr(u), rtol, maxit, smoother_prec, sweeps, omega,
                                 variant, ct.byref(info))
        else:
            st = lib().pcg_solve_pc(self.h, _ptr(b), _ptr(u), rtol, maxit, precond, smoother_prec, sweeps,
                                    omega, variant, ct.byref(info))
        res = dict(iters=info.iters, status=info.status, relres=info.relres, seconds=info.seconds)
        if raise_on_error and st not in (FEM_OK,):
            check(st, "pcg_solve")
        return u, res

    def pcg_solve_noalloc(self, b, u, rtol=1e-8, maxit=1000, smoother_prec=F64, sweeps=2, omega=0.125,
                          variant=CG_AUTO, precond=PC_SCHWARZ, raise_on_error=True):
        """pcg_solve whose solver vectors live in the library's fixed device
        scratch (no allocation in the call): u (initial guess, solution) is
        the caller's."""
        self._cell(b, F64, "b")
        self._cell(u, F64, "u")
        _require_cuda(b, u)
        self._sync_stream()
        info = SolveInfo()
        st = lib().pcg_solve_noalloc(self.h, _ptr(b), _ptr(u), rtol, maxit, precond, smoother_prec, sweeps, omega,
                                     variant, ct.byref(info))
        res = dict(iters=info.iters, status=info.status, relres=info.relres, seconds=info.seconds)
        if raise_on_error and st not in (FEM_OK,):
            check(st, "pcg_solve")
        return u, res


class Batch:
    """Independent problems launched together: one mixed-degree launch per
    kernel phase when the degrees are two or three of {2, 3, 7}, else one
    launch per degree."""

    def __init__(self, problems):
        """problems: list of (p, n, widths-or-None) or (p, n, widths-or-None, bc)."""
        descs = (Desc * len(problems))()
        self._descs = []
        spec = [(t[0], t[1], t[2], t[3] if len(t) > 3 else DIRICHLET) for t in problems]
        for i, (p, n, w, bc) in enumerate(spec):
            d = make_desc(p, n, w, bc)
            self._descs.append(d)
            descs[i] = d
        h = ct.c_void_p()
        check(lib().fem_batch_create(len(problems), descs, _stream(), ct.byref(h)), "fem_batch_create")
        self.h = h
        self.problems = []
        for i, (p, n, w, bc) in enumerate(spec):
            ph = ct.c_void_p()
            check(lib().fem_batch_problem(self.h, i, ct.byref(ph)), "fem_batch_problem")
            self.problems.append(Problem(p, n, w, bc, _handle=ph))

    def close(self):
        if getattr(self, "h", None):
            lib().fem_batch_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _ptrs(ts):
        arr = (ct.c_void_p * len(ts))()
        for i, t in enumerate(ts):
            arr[i] = t.data_ptr()
        return arr

    def _check(self, xs, ys, nx, ny):
        if len(xs) != len(self.problems) or len(ys) != len(self.problems):
            raise ValueError(f"expected {len(self.problems)} vectors per argument")
        prec = prec_of(_check_vec(xs[0], self.problems[0].cell_len, None, nx + "[0]"))
        for i, P in enumerate(self.problems):
            P._cell(xs[i], prec, f"{nx}[{i}]")
            P._cell(ys[i], prec, f"{ny}[{i}]")
        return prec

    def apply(self, xs, ys):
        self._check(xs, ys, "xs", "ys")
        _require_cuda(*xs, *ys)
        check(lib().fem_batch_apply(self.h, self._ptrs(xs), self._ptrs(ys), prec_of(xs[0])), "fem_batch_apply")

    def patch_inverse(self, rs, zs):
        self._check(rs, zs, "rs", "zs")
        _require_cuda(*rs, *zs)
        check(lib().fem_batch_patch_inverse(self.h, self._ptrs(rs), self._ptrs(zs), prec_of(rs[0])),
              "fem_batch_patch_inverse")

    def autotune(self, prec):
        choice = (ct.c_int * 14)(*([-1] * 14))
        check(lib().fem_batch_autotune(self.h, prec, choice), "fem_batch_autotune")
        return {p: (choice[2 * (p - 1)], choice[2 * (p - 1) + 1]) for p in range(1, 8)
                if choice[2 * (p - 1)] >= 0}

    def set_mixed(self, mixed):
        check(lib().fem_batch_set_mixed(self.h, 1 if mixed else 0), "fem_batch_set_mixed")

    @property
    def mixed(self):
        """True if the batched calls run as mixed-degree launches."""
        return bool(lib().fem_batch_mixed(self.h))


class Server:
    """Continuous-batching Poisson solve server (device-resident solves)."""

    def __init__(self, hbm_budget, max_active=64, smoother_prec=F32, sweeps=2, omega=0.125, precond=PC_SCHWARZ):
        h = ct.c_void_p()
        check(lib().fem_server_create_pc(int(hbm_budget), max_active, precond, smoother_prec, sweeps, omega,
                                         _stream(), ct.byref(h)), "fem_server_create_pc")
        self.h = h
        self.glen = {}

    def close(self):
        if getattr(self, "h", None):
            lib().fem_server_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, p, n, f, widths=None, rtol=1e-8, maxit=2000):
        n3 = (n, n, n) if isinstance(n, int) else tuple(int(v) for v in n)
        f = np.ascontiguousarray(f, dtype=np.float64)
        need = (n3[0] * p + 1) * (n3[1] * p + 1) * (n3[2] * p + 1)
        if f.ndim != 1 or f.size != need:
            raise ValueError(f"f: has {f.size} values, the mesh has {need} global nodes")
        d = make_desc(p, n3, widths)
        t = ct.c_uint64()
        check(lib().fem_server_submit(self.h, ct.byref(d), f.ctypes.data, rtol, maxit, ct.byref(t)),
              "fem_server_submit")
        self.glen[t.value] = f.size
        return t.value

    def set_mixed(self, mixed):
        check(lib().fem_server_set_mixed(self.h, 1 if mixed else 0), "fem_server_set_mixed")

    def step(self):
        a, q, dn = ct.c_int(), ct.c_int(), ct.c_int()
        check(lib().fem_server_step(self.h, ct.byref(a), ct.byref(q), ct.byref(dn)), "fem_server_step")
        return a.value, q.value, dn.value

    def poll(self, ticket, want_u=True):
        """(u, info) when finished, else None."""
        info = SolveInfo()
        u = np.empty(self.glen[ticket]) if want_u else None
        st = lib().fem_server_poll(self.h, ticket, u.ctypes.data if want_u else None, ct.byref(info))
        if st == FEM_EAGAIN:
            return None
        check(st, "fem_server_poll")
        self.glen.pop(ticket, None)
        return u, dict(iters=info.iters, status=info.status, relres=info.relres, seconds=info.seconds)

    def finished(self):
        """Tickets of finished, not yet collected solves (ascending)."""
        L = lib()
        n = L.fem_server_finished(self.h, None, 0)
        if n <= 0:
            return []
        out = (ct.c_uint64 * n)()
        n = min(n, L.fem_server_finished(self.h, out, n))
        return [int(out[k]) for k in range(n)]

    def stats(self):
        """Host seconds per server-step phase and the step count."""
        out = (ct.c_double * 6)()
        check(lib().fem_server_stats(self.h, out, 6), "fem_server_stats")
        keys = ("admit", "launch", "wait_scalars", "retire_finish", "retire_start", "steps")
        return dict(zip(keys, list(out)))

    def memory(self):
        a, b = ct.c_size_t(), ct.c_size_t()
        check(lib().fem_server_memory(self.h, ct.byref(a), ct.byref(b)), "fem_server_memory")
        return a.value, b.value


class MultiBlockDss:
    """DSS on a multi-block mesh: blocks glued along whole faces in any
    orientation (structured cascade per block, then the inter-block
    skeleton)."""

    def __init__(self, p, block_n, corners):
        bn = np.ascontiguousarray(np.asarray(block_n, dtype=np.int32).ravel())
        cs = np.ascontiguousarray(np.asarray(corners, dtype=np.int32).ravel())
        if bn.size % 3 or cs.size != 8 * (bn.size // 3):
            raise ValueError("block_n needs 3 and corners 8 entries per block")
        self.p = int(p)
        self.nb = bn.size // 3
        self.block_n = bn.reshape(-1, 3)
        h = ct.c_void_p()
        check(lib().fem_mb_create(self.p, self.nb, bn.ctypes.data, cs.ctypes.data, _stream(), ct.byref(h)),
              "fem_mb_create")
        self.h = h
        self.cell_len = lib().fem_mb_cell_len(self.h)
        self.canon_len = int(sum(int(np.prod(n)) for n in self.block_n)) * (self.p + 1) ** 3

    def close(self):
        if getattr(self, "h", None):
            lib().fem_mb_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pack(self, canon, prec=F64):
        _check_vec(canon, self.canon_len, F64, "canon")
        _require_cuda(canon)
        torch = _torch()
        out = torch.zeros(self.cell_len, dtype=torch_dtype(prec), device="cuda")
        check(lib().fem_mb_pack(self.h, _ptr(canon), _ptr(out), prec), "fem_mb_pack")
        return out

    def unpack(self, v):
        _check_vec(v, self.cell_len, None, "v")
        _require_cuda(v)
        torch = _torch()
        out = torch.empty(self.canon_len, dtype=torch.float64, device="cuda")
        check(lib().fem_mb_unpack(self.h, _ptr(v), _ptr(out), prec_of(v)), "fem_mb_unpack")
        return out

    def dss(self, v, stages=3):
        """In place: v <- S v."""
        _check_vec(v, self.cell_len, None, "v")
        _require_cuda(v)
        check(lib().fem_mb_dss(self.h, _ptr(v), prec_of(v), stages), "fem_mb_dss")
        return v

    def stats(self):
        out = (ct.c_int * 6)()
        check(lib().fem_mb_stats(self.h, out, 6), "fem_mb_stats")
        keys = ("faces", "face_threads", "lines", "line_width", "vertices", "vertex_width")
        return dict(zip(keys, list(out)))


class LayoutStudy:
    """FP64 vectors of a uniform mesh in the blocked layout with block size B
    (the layout study): pack/unpack, mass apply, structured DSS."""

    def __init__(self, p, n, B):
        self.p, self.B = int(p), int(B)
        self.n = (n, n, n) if isinstance(n, int) else tuple(int(v) for v in n)
        self._n = (ct.c_int * 3)(*self.n)
        self.len = lib().fem_layout_len(self.p, self._n, self.B)
        if self.len == 0:
            raise ValueError("layout study: p in 2..5, n >= 1, B a power of two <= 128")
        self.canon_len = self.n[0] * self.n[1] * self.n[2] * (self.p + 1) ** 3

    def vector(self):
        torch = _torch()
        return torch.zeros(self.len, dtype=torch.float64, device="cuda")

    def pack(self, canon):
        _check_vec(canon, self.canon_len, F64, "canon")
        _require_cuda(canon)
        out = self.vector()
        check(lib().fem_layout_pack(self.p, self._n, self.B, _ptr(canon), _ptr(out), 0, _stream()), "fem_layout_pack")
        return out

    def unpack(self, v):
        _check_vec(v, self.len, F64, "v")
        _require_cuda(v)
        torch = _torch()
        out = torch.empty(self.canon_len, dtype=torch.float64, device="cuda")
        check(lib().fem_layout_pack(self.p, self._n, self.B, _ptr(v), _ptr(out), 1, _stream()), "fem_layout_pack")
        return out

    def mass(self, x, y=None, tile=32):
        _check_vec(x, self.len, F64, "x")
        if y is not None:
            _check_vec(y, self.len, F64, "y")
        _require_cuda(x, y)
        y = self.vector() if y is None else y
        check(lib().fem_layout_mass(self.p, self._n, self.B, tile, _ptr(x), _ptr(y), _stream()), "fem_layout_mass")
        return y

    def dss(self, v):
        _check_vec(v, self.len, F64, "v")
        _require_cuda(v)
        check(lib().fem_layout_dss(self.p, self._n, self.B, _ptr(v), _stream()), "fem_layout_dss")
        return v
