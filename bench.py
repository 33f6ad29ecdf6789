"""Benchmark of the cell-wise Q_p Laplacian hot path on one MI355X.

One step on the headline workload (Q3, 64^3 cells graded per direction with
widths U[0.5,1.5] (seed 1), FP64, x ~ U[-1,1]) is one pass of the operator
and the smoother's patch solve:  y = A x (fe_apply), then z = P_AS y
(patch_inverse).  The reported rate counts unique DoFs ((64*3+1)^3) per
second of that pass; the per-operation rates, the Q2 (96^3) and Q7 (24^3)
workloads and the Q7 solve times with FP64/FP32/BF16 smoothers are reported
beside it.

Inputs live in HBM before timing starts; the timed region rotates through
several independent (x, y, z) buffer sets larger than the 256 MB Infinity
Cache so repeated steps do not run out of cache.

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--quick]
       python bench.py --mode calib        (plain 1 GiB copy, for counters)
       python bench.py --mode serve        (continuous-batching stream)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def unique_dofs(p, n):
    return (n * p + 1) ** 3


def cell_dofs(p, n):
    return n ** 3 * (p + 1) ** 3


class Timer:
    """HIP events on the current stream (the stream the library launches on)."""

    def __init__(self, torch):
        self.torch = torch

    def time(self, fn, reps):
        t = self.torch
        s, e = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        s.record()
        for i in range(reps):
            fn(i)
        e.record()
        e.synchronize()
        return s.elapsed_time(e) / reps * 1e-3      # seconds per call


def setup(fem, torch, p, n, seed, prec=0, rotate_bytes=768 << 20):
    """Problem plus enough (x, y, z) sets to exceed the Infinity Cache."""
    import synth
    wl = synth._graded(f"q{p}_{n}", p, n, seed)
    P = fem.Problem(p, n, wl.widths)
    xg = torch.as_tensor(wl.x, device="cuda")
    x0 = P.gather(xg, prec)
    per_set = 3 * P.cell_len * fem.lib().fem_prec_bytes(prec)
    nsets = max(1, min(6, -(-rotate_bytes // per_set)))
    sets = []
    for _ in range(nsets):
        sets.append((x0.clone(), P.cell_vector(prec), P.cell_vector(prec)))
    torch.cuda.synchronize()
    return P, sets, wl


def measure_workload(fem, torch, p, n, seed, steps, warmup, prec=0):
    P, sets, wl = setup(fem, torch, p, n, seed, prec)
    ns = len(sets)

    def step(i):
        x, y, z = sets[i % ns]
        P.apply(x, y)
        P.patch_inverse(y, z)

    def apply_only(i):
        x, y, _ = sets[i % ns]
        P.apply(x, y)

    def pi_only(i):
        _, y, z = sets[i % ns]
        P.patch_inverse(y, z)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(i)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    tm = Timer(torch)
    t_apply = tm.time(apply_only, max(steps, 10))
    t_pi = tm.time(pi_only, max(steps, 10))
    # per-kernel durations of the same steps, from HIP event pairs the library
    # records around each launch on the stream it launches on
    fem.trace_enable(True)
    for i in range(steps):
        step(i)
    torch.cuda.synchronize()
    kernels = fem.trace_read()
    fem.trace_enable(False)
    u = unique_dofs(p, n)
    c = cell_dofs(p, n)
    es = {0: 8, 1: 4, 2: 2}[prec]
    cs = 8 if prec == 0 else 4
    res = dict(p=p, n=n, unique_dofs=u, cell_dofs=c, s_per_step=wall, kernels=kernels, esize=es, csize=cs,
               apply_s=t_apply, pi_s=t_pi,
               apply_unique_gdofs=u / t_apply / 1e9, pi_unique_gdofs=u / t_pi / 1e9,
               apply_cell_gdofs=c / t_apply / 1e9, pi_cell_gdofs=c / t_pi / 1e9,
               step_unique_gdofs=u / wall / 1e9,
               apply_gbs=2 * es * c / t_apply / 1e9, pi_gbs=2 * es * c / t_pi / 1e9)
    res["roofline_by_kernel"] = kernel_table(res)
    del sets
    P.close()
    torch.cuda.empty_cache()
    return res


def kernel_bytes(label, p, n, esize=8, csize=8):
    """Algorithmic HBM bytes of one launch of a traced kernel: each array it
    must read or write, once.  cell = cell-wise vector (storage precision,
    esize bytes), uniq = assembled global-node array, patch = patch-result
    buffer ((2p-1)^3 per patch), both in the compute precision (csize)."""
    cell = cell_dofs(p, n) * esize
    uniq = unique_dofs(p, n) * csize
    patch = (n - 1) ** 3 * (2 * p - 1) ** 3 * csize
    return {"apply": 2 * cell, "pi_assemble": cell + uniq, "pi_solve": uniq + patch,
            "pi_combine": patch + cell, "pi_sweep": 2 * cell + uniq}.get(label)


def kernel_flops(label, p, n):
    """Algorithmic flops of one launch (FMA = 2): the sum-factorised apply
    (7 one-dimensional contractions of (p+1) terms per cell DoF plus the
    3-term combination) and the fast-diagonalisation patch solve (two
    transforms of 3 one-dimensional passes over (2p-1)^3 values, 2(2p-1)
    flops each, plus the diagonal scaling)."""
    nP = 2 * p - 1
    if label == "apply":
        return cell_dofs(p, n) * (7 * 2 * (p + 1) + 4)
    if label == "pi_solve":
        return (n - 1) ** 3 * (12 * nP ** 4 + nP ** 3)
    return None


def measured_traffic(workload, label):
    """HBM bytes per launch of a traced kernel from the committed counter
    summary of the workload, or None when there is none or the kernel
    sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    from paper_2607_02335_amd import profiling
    with open(path) as f:
        rec = json.load(f)
    if rec.get("sources_sha256") != profiling.sources_hash():
        return None
    k = rec.get("kernels", {}).get(label)
    return None if k is None else int(round(k["bytes"]))


def kernel_table(rec):
    """Every traced kernel of a workload against the HBM roofline."""
    p, n = rec["p"], rec["n"]
    out = []
    for k in rec["kernels"]:
        b = kernel_bytes(k["label"], p, n, rec.get("esize", 8), rec.get("csize", 8))
        if b is None:
            continue
        gbs = b / (k["avg_us"] * 1e-6) / 1e9
        row = {"kernel": k["label"], "avg_us": round(k["avg_us"], 2), "algorithmic_bytes": b,
               "GB/s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        fl = kernel_flops(k["label"], p, n)
        if fl is not None:
            peak = FP64_PEAK_TFLOPS if rec.get("csize", 8) == 8 else FP32_PEAK_TFLOPS
            tf = fl / (k["avg_us"] * 1e-6) / 1e12
            row.update({"algorithmic_flops": fl, "TFLOP/s": round(tf, 2), "flop_frac": round(tf / peak, 4)})
        out.append(row)
    return out


def roofline(rec, workload="q3_64"):
    """Roofline record of the kernel with the largest share of the step."""
    p, n = rec["p"], rec["n"]
    es, cs = rec.get("esize", 8), rec.get("csize", 8)
    ks = [k for k in rec["kernels"] if kernel_bytes(k["label"], p, n, es, cs) is not None]
    dom = max(ks, key=lambda k: k["total_ms"])
    t = dom["avg_us"] * 1e-6
    byts = kernel_bytes(dom["label"], p, n, es, cs)
    gbs = byts / t / 1e9
    fl = kernel_flops(dom["label"], p, n)
    out = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(workload, dom["label"]),
           "kernel": dom["label"], "launch_avg_us": round(dom["avg_us"], 2), "launches": dom["launches"],
           "algorithmic_bytes_per_launch": byts}
    if fl is not None:
        tf = fl / t / 1e12
        out["fp64_tflops"] = round(tf, 2)
        out["fp64_frac"] = round(tf / FP64_PEAK_TFLOPS, 4)
    return out


def batch_times(fem, torch, steps, warmup, count=256, seed=3):
    """256 independent problems (p uniform in {2,3,7}, n uniform in [4,32],
    seed 3): FP32 apply + patch inverse of all of them, one launch per degree
    and operation, with the autotuned kernel shapes.  Rate = unique DoFs of
    the whole batch per second of one pass."""
    import synth
    wls = synth.batch_problems(count=count, seed=seed)
    B = fem.Batch([(w.p, w.n, None) for w in wls])
    xs = [P.gather(torch.as_tensor(w.x, device="cuda"), fem.F32) for P, w in zip(B.problems, wls)]
    ys = [P.cell_vector(fem.F32) for P in B.problems]
    zs = [P.cell_vector(fem.F32) for P in B.problems]
    choice = B.autotune(fem.F32)

    def step(i):
        B.apply(xs, ys)
        B.patch_inverse(ys, zs)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(i)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    uniq = sum(unique_dofs(w.p, w.n[0]) for w in wls)
    cell = sum(cell_dofs(w.p, w.n[0]) for w in wls)
    out = dict(problems=count, unique_dofs=uniq, cell_dofs=cell, s_per_pass=t,
               unique_gdofs=uniq / t / 1e9, cell_gdofs=cell / t / 1e9,
               autotuned={str(k): v for k, v in choice.items()})
    del xs, ys, zs
    B.close()
    torch.cuda.empty_cache()
    return out


def solve_times(fem, torch, reps):
    """Q7 24^3 graded solve to 1e-8 with FP64/FP32/BF16 smoothers."""
    import synth
    wl = synth.workload_q7_graded()
    P = fem.Problem(7, 24, wl.widths)
    X = [fem.node_coords(7, wl.widths[d]) for d in range(3)]
    f = np.kron(np.kron(np.sin(np.pi * X[2]), np.sin(np.pi * X[1])), np.sin(np.pi * X[0]))
    f = f + 0.01 * wl.noise
    b = P.mass_apply(P.gather(torch.as_tensor(f, device="cuda")))
    out = {}
    for name, sp in (("fp64", fem.F64), ("fp32", fem.F32), ("bf16", fem.BF16)):
        times, iters = [], None
        P.pcg_solve(b, smoother_prec=sp)                  # warm
        for _ in range(reps):
            u = P.cell_vector(fem.F64)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u, info = P.pcg_solve(b, u=u, rtol=1e-8, maxit=2000, smoother_prec=sp)
            times.append(time.perf_counter() - t0)
            iters = info["iters"]
        ts = np.sort(np.asarray(times))
        out[name] = dict(iters=iters, p50_s=float(np.percentile(ts, 50)), p99_s=float(np.percentile(ts, 99)),
                         relres=info["relres"])
    P.close()
    return out


def cpu_baseline(steps_budget_s=20.0):
    """The oracle on the host cores on a bounded sample of the headline
    workload: the full matrix-free apply, and dense-LU patch solves on a
    sample of patches, scaled to the whole mesh."""
    import synth
    from oracle import operators, patches
    from oracle.mesh import Mesh
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = 1
    wl = synth.workload_q3_graded()
    m = Mesh(3, wl.n, wl.widths)
    t0 = time.perf_counter()
    y = operators.apply_global(m, wl.x)
    t_apply = time.perf_counter() - t0
    verts = patches.interior_vertices(m)
    rng = np.random.default_rng(0)
    t0 = time.perf_counter()
    done = 0
    for v in verts[rng.permutation(len(verts))]:
        idx = patches.patch_nodes(m, v)
        patches.patch_solve(m, v, y[idx])
        done += 1
        if time.perf_counter() - t0 > steps_budget_s:
            break
    t_pi = (time.perf_counter() - t0) / done * len(verts)
    u = unique_dofs(3, 64)
    return dict(value=u / (t_apply + t_pi), unit="DoFs/s", cores=int(cores), kind="oracle",
                sample=f"Q3 64^3 graded: full matrix-free apply ({t_apply:.2f} s) + dense-LU solves of "
                       f"{done} of {len(verts)} vertex patches, extrapolated ({t_pi:.1f} s)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mode", default="bench", choices=["bench", "calib", "serve"])
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--only", choices=["q2_96", "q7_24", "q7_solve", "batch_256"], default=None,
                    help="run one secondary workload alone (for profiling) and print its record")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--solve-reps", type=int, default=5)
    ap.add_argument("--requests", type=int, default=10000, help="serving mode: stream length")
    ap.add_argument("--prec", choices=["f64", "f32", "bf16"], default="f64",
                    help="storage precision of --only q2_96 / q7_24")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU only (the library runs each problem on one device; "
              "splitting a mesh over several GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2607_02335_amd import fem
    fem.lib()
    torch.cuda.set_device(0)

    if a.mode == "calib":
        n = 1 << 27                       # 1 GiB of doubles
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes_read": n * 8, "calib_copy_bytes_written": n * 8}))
        return
    if a.mode == "serve":
        from paper_2607_02335_amd import serve
        print(json.dumps(serve.run_stream_bench(count=a.requests, log=log)))
        return

    if a.only:
        log(f"{a.only} alone")
        if a.only == "q7_solve":
            rec = solve_times(fem, torch, a.solve_reps)
        elif a.only == "batch_256":
            rec = batch_times(fem, torch, a.steps, a.warmup)
        else:
            p, n = (2, 96) if a.only == "q2_96" else (7, 24)
            prec = {"f64": fem.F64, "f32": fem.F32, "bf16": fem.BF16}[a.prec]
            rec = measure_workload(fem, torch, p, n, 1, a.steps, a.warmup, prec)
            rec["prec"] = a.prec
        print(json.dumps({a.only: rec}))
        return
    log("headline workload Q3 64^3 graded FP64")
    head = measure_workload(fem, torch, 3, 64, 1, a.steps, a.warmup)
    extra = {"q3_64": head}
    if not a.quick:
        log("Q2 96^3 graded")
        extra["q2_96"] = measure_workload(fem, torch, 2, 96, 1, a.steps, a.warmup)
        log("Q7 24^3 graded")
        extra["q7_24"] = measure_workload(fem, torch, 7, 24, 1, a.steps, a.warmup)
        log("Q7 24^3 solves")
        extra["q7_solve"] = solve_times(fem, torch, a.solve_reps)
        log("batch of 256 problems")
        extra["batch_256"] = batch_times(fem, torch, a.steps, a.warmup)

    roof = roofline(head)
    cpu = None
    if not a.no_cpu:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline()
    line = {
        "metric": "unique DoFs/s of one apply + vertex-patch inverse pass (Q3 64^3 graded, FP64)",
        "value": head["step_unique_gdofs"] * 1e9,
        "unit": "DoFs/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": head["s_per_step"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "Q3 Laplacian, 64^3 cells, per-direction widths U[0.5,1.5] seed 1, "
                               "Dirichlet, x~U[-1,1]; step = fe_apply + patch_inverse",
                   "p": 3, "cells": 64 ** 3, "unique_dofs": head["unique_dofs"],
                   "cell_dofs": head["cell_dofs"], "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
