"""Benchmark of the cell-wise Q_p Laplacian hot path on one MI355X.

One step on the headline workload (Q3, 64^3 cells graded per direction with
widths U[0.5,1.5] (seed 1), FP64, x ~ U[-1,1]) is one pass of the operator
and the smoother's patch solve:  y = A x (fe_apply), then z = P_AS y
(patch_inverse).  The reported rate counts unique DoFs ((64*3+1)^3) per
second of that pass; the per-operation rates, the Q2 (96^3) and Q7 (24^3)
workloads, the Q7 solve times with FP64/FP32/BF16/FP16 smoothers, the 256-problem
batch, the paper's own kernels (mass operator, structured DSS, assembled
mass) and the 10,000-request serving stream (p50/p99 latency, solved DoF/s)
are reported beside it.

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
    # hot: one buffer set over and over (what fits of it stays in the
    # Infinity Cache between launches)
    t_apply_hot = tm.time(lambda i: apply_only(0), max(steps, 10))
    t_pi_hot = tm.time(lambda i: pi_only(0), max(steps, 10))
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
               apply_gbs=2 * es * c / t_apply / 1e9, pi_gbs=2 * es * c / t_pi / 1e9,
               hot=dict(apply_s=t_apply_hot, pi_s=t_pi_hot, apply_gbs=2 * es * c / t_apply_hot / 1e9,
                        pi_gbs=2 * es * c / t_pi_hot / 1e9, step_unique_gdofs=u / (t_apply_hot + t_pi_hot) / 1e9))
    res["roofline_by_kernel"] = kernel_table(res)
    res["ops"] = op_table(res, f"q{p}_{n}" if prec == 0 else None)
    del sets
    P.close()
    torch.cuda.empty_cache()
    return res


# Launch-trace label -> the operation of the hot path it belongs to.
OP_OF = {"apply": "apply", "mass": "mass", "pi_assemble": "patch_inverse", "pi_solve": "patch_inverse",
         "pi_combine": "patch_inverse", "pi_sweep": "patch_inverse", "dss_axis": "dss"}


def op_bytes(op, p, n, esize=8):
    """Algorithmic HBM bytes of one operation on an n^3 mesh: the per-unit
    figure of the measurement model times the units.  The apply, the mass
    apply and the patch inverse read one cell-wise vector and write one
    (2 x esize bytes per cell DoF; geometry and eigen-data are O(n) and not
    counted); the structured DSS reads and writes both coincident copies of
    every face pair of every axis pass (4 x esize per pair)."""
    cell = cell_dofs(p, n) * esize
    if op in ("apply", "mass", "patch_inverse"):
        return 2 * cell
    if op == "dss":
        return 4 * esize * (p + 1) ** 2 * 3 * (n - 1) * n * n
    return None


def op_flops(op, p, n):
    """Algorithmic flops of one operation (FMA = 2).  Apply: 14(p+1) per cell
    DoF, the useful work of the paper's Laplace table (seven 1D contractions
    of p+1 terms); mass: 6(p+1) (three contractions); patch inverse: per
    vertex patch two transforms of three 1D passes over (2p-1)^3 values
    (2(2p-1) flops each) plus the diagonal scaling, 12 (2p-1)^4 + (2p-1)^3."""
    nP = 2 * p - 1
    if op == "apply":
        return cell_dofs(p, n) * 14 * (p + 1)
    if op == "mass":
        return cell_dofs(p, n) * 6 * (p + 1)
    if op == "patch_inverse":
        return (n - 1) ** 3 * (12 * nP ** 4 + nP ** 3)
    return None


def kernel_bytes(label, p, n, esize=8, csize=8):
    """Algorithmic bytes charged to one launch of a traced kernel: the bytes
    of the whole operation it is a phase of (a phase processes every cell
    DoF of the operation), so its fraction of the HBM peak says how far the
    operation would be from its roofline if this kernel were all of it."""
    op = OP_OF.get(label)
    return None if op is None else op_bytes(op, p, n, esize)


def design_bytes(label, p, n, esize=8, csize=8):
    """Bytes one launch must move given the design's own intermediate arrays
    (cell = cell-wise vector in the storage precision, uniq = assembled
    global-node array, patch = patch-result buffer, both in the compute
    precision): the floor of that kernel's traffic, not the operation's."""
    cell = cell_dofs(p, n) * esize
    uniq = unique_dofs(p, n) * csize
    patch = (n - 1) ** 3 * (2 * p - 1) ** 3 * csize
    return {"apply": 2 * cell, "pi_assemble": cell + uniq, "pi_solve": uniq + patch,
            "pi_combine": patch + cell, "pi_sweep": uniq + cell}.get(label)


def kernel_flops(label, p, n):
    """Flops of one launch: the apply's, and the patch solves' for the
    phase that runs them (pi_solve, or the fused pi_sweep)."""
    if label == "apply":
        return op_flops("apply", p, n)
    if label in ("pi_solve", "pi_sweep"):
        return op_flops("patch_inverse", p, n)
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


def _peak_flops(csize):
    return FP64_PEAK_TFLOPS if csize == 8 else FP32_PEAK_TFLOPS


def kernel_table(rec):
    """Every traced kernel of a workload against the HBM roofline, charged
    its operation's algorithmic bytes (and, beside, its design floor)."""
    p, n = rec["p"], rec["n"]
    es, cs = rec.get("esize", 8), rec.get("csize", 8)
    out = []
    for k in rec["kernels"]:
        b = kernel_bytes(k["label"], p, n, es, cs)
        if b is None:
            continue
        t = k["avg_us"] * 1e-6
        gbs = b / t / 1e9
        row = {"kernel": k["label"], "op": OP_OF[k["label"]], "avg_us": round(k["avg_us"], 2),
               "algorithmic_bytes": b, "GB/s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        db = design_bytes(k["label"], p, n, es, cs)
        if db is not None:
            row["design_bytes"] = db
            row["design_hbm_frac"] = round(db / t / 1e9 / HBM_PEAK_GBS, 4)
        fl = kernel_flops(k["label"], p, n)
        if fl is not None:
            tf = fl / t / 1e12
            row.update({"algorithmic_flops": fl, "TFLOP/s": round(tf, 2), "flop_frac": round(tf / _peak_flops(cs), 4)})
        out.append(row)
    return out


def op_table(rec, workload=None):
    """Each operation of the step as one unit: its kernels' summed average
    launch time against its algorithmic bytes and flops, and the counter
    traffic of its kernels over the algorithmic bytes (null when absent or
    stale)."""
    p, n = rec["p"], rec["n"]
    es, cs = rec.get("esize", 8), rec.get("csize", 8)
    ops = {}
    for k in rec["kernels"]:
        op = OP_OF.get(k["label"])
        if op is None:
            continue
        o = ops.setdefault(op, {"kernels": [], "time_us": 0.0, "traffic": 0})
        o["kernels"].append(k["label"])
        o["time_us"] += k["avg_us"]
        tr = measured_traffic(workload, k["label"]) if workload else None
        o["traffic"] = None if (tr is None or o["traffic"] is None) else o["traffic"] + tr
    out = {}
    for op, o in ops.items():
        t = o["time_us"] * 1e-6
        b = op_bytes(op, p, n, es)
        gbs = b / t / 1e9
        row = {"kernels": o["kernels"], "time_us": round(o["time_us"], 2), "algorithmic_bytes": b,
               "GB/s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
               "roofline_time_us": round(b / (HBM_PEAK_GBS * 1e9) * 1e6, 2)}
        fl = op_flops(op, p, n)
        if fl is not None:
            tf = fl / t / 1e12
            row.update({"algorithmic_flops": fl, "TFLOP/s": round(tf, 2), "flop_frac": round(tf / _peak_flops(cs), 4)})
        if o["traffic"]:
            row["traffic_bytes"] = o["traffic"]
            row["traffic_over_algorithmic"] = round(o["traffic"] / b, 3)
        out[op] = row
    return out


def roofline(rec, workload="q3_64", copy_gbs=None):
    """Roofline record of the kernel with the largest share of the step,
    charged its operation's algorithmic bytes per launch, with the step's
    operations as whole units beside it."""
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
           "kernel": dom["label"], "op": OP_OF[dom["label"]], "launch_avg_us": round(dom["avg_us"], 2),
           "launches": dom["launches"], "algorithmic_bytes_per_launch": byts,
           "design_bytes_per_launch": design_bytes(dom["label"], p, n, es, cs)}
    if fl is not None:
        tf = fl / t / 1e12
        out["algorithmic_flops_per_launch"] = fl
        out["tflops"] = round(tf, 2)
        out["flop_frac"] = round(tf / _peak_flops(cs), 4)
    if copy_gbs:
        out["copy_peak_GB/s"] = round(copy_gbs, 1)
        out["frac_of_copy_peak"] = round(gbs / copy_gbs, 4)
    out["ops"] = op_table(rec, workload)
    return out


def copy_peak(torch, nbytes=1 << 30, reps=10):
    """Measured device copy bandwidth: read + write of a plain 1 GiB copy,
    (2 x bytes) / time, timed with HIP events."""
    n = nbytes // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    t = Timer(torch).time(lambda i: dst.copy_(src), reps)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / t / 1e9


def paper_kernels(fem, torch, reps=10, n_dss=128, degrees=(2, 3, 7)):
    """The paper's own measured kernels on uniform unit-cube meshes, FP64:
    the mass operator (one volumetric apply, Table "mass operator"), the
    structured DSS in place (three axis passes, Table "DSS throughput") and
    the entire assembled mass operator (volumetric apply + DSS, Table
    "entire mass operator", 128^3 cells).  Rates in unique DoFs per second,
    bytes by the algorithmic model; cold (two rotating buffer pairs)."""
    out = {}
    for p in degrees:
        n = n_dss
        P = fem.Problem(p, n)
        x = P.gather(torch.ones(P.global_len, dtype=torch.float64, device="cuda"))
        pairs = [(x, P.cell_vector()), (x.clone(), P.cell_vector())]
        tm = Timer(torch)
        for i in range(2):
            P.mass_apply(*pairs[i % 2])
            P.dss(pairs[i % 2][1], pairs[i % 2][1])
        torch.cuda.synchronize()
        t_vol = tm.time(lambda i: P.mass_apply(*pairs[i % 2]), reps)
        t_dss = tm.time(lambda i: P.dss(pairs[i % 2][1], pairs[i % 2][1]), reps)

        def both(i):
            P.mass_apply(*pairs[i % 2])
            P.dss(pairs[i % 2][1], pairs[i % 2][1])
        t_op = tm.time(both, reps)
        u, c = unique_dofs(p, n), cell_dofs(p, n)
        bm, bd = op_bytes("mass", p, n), op_bytes("dss", p, n)
        out[f"q{p}_{n}"] = dict(
            p=p, n=n, unique_dofs=u, cell_dofs=c,
            mass=dict(s=t_vol, unique_gdofs=u / t_vol / 1e9, cell_gdofs=c / t_vol / 1e9,
                      algorithmic_bytes=bm, gbs=bm / t_vol / 1e9, hbm_frac=bm / t_vol / 1e9 / HBM_PEAK_GBS),
            dss=dict(s=t_dss, unique_gdofs=u / t_dss / 1e9, algorithmic_bytes=bd, gbs=bd / t_dss / 1e9,
                     hbm_frac=bd / t_dss / 1e9 / HBM_PEAK_GBS),
            assembled_mass=dict(s=t_op, unique_gdofs=u / t_op / 1e9))
        del x, pairs
        P.close()
        torch.cuda.empty_cache()
    return out


def layout_sweep(fem, torch, reps=5, blocks=(1, 2, 4, 8, 16, 32, 64, 128)):
    """The layout study (block size B of the blocked element-fastest layout,
    FP64, uniform unit-cube meshes of about 1e8 cell DoFs): volumetric mass
    apply (best of two tile shapes) and structured DSS, in unique DoFs per
    second, per degree and B."""
    sizes = {2: 160, 3: 128, 4: 96, 5: 80}
    out = {}
    tm = Timer(torch)
    for p, n in sizes.items():
        u, c = unique_dofs(p, n), cell_dofs(p, n)
        canon = torch.rand(c, dtype=torch.float64, device="cuda")
        rows = []
        for B in blocks:
            L = fem.LayoutStudy(p, n, B)
            xs = [L.pack(canon), L.pack(canon)]
            ys = [L.vector(), L.vector()]
            best = None
            for tile in (16, 32):
                L.mass(xs[0], ys[0], tile=tile)
                t = tm.time(lambda i: L.mass(xs[i % 2], ys[i % 2], tile=tile), reps)
                best = (t, tile) if best is None or t < best[0] else best
            L.dss(ys[0])
            t_dss = tm.time(lambda i: L.dss(ys[i % 2]), reps)
            rows.append(dict(B=B, mass_s=best[0], mass_tile=best[1], mass_unique_gdofs=u / best[0] / 1e9,
                             mass_gbs=2 * 8 * c / best[0] / 1e9, dss_s=t_dss, dss_unique_gdofs=u / t_dss / 1e9,
                             dss_gbs=op_bytes("dss", p, n) / t_dss / 1e9))
            del xs, ys
        out[f"q{p}_{n}"] = rows
        del canon
        torch.cuda.empty_cache()
    return out


def batch_times(fem, torch, steps, warmup, count=256, seed=3):
    """256 independent problems (p uniform in {2,3,7}, n uniform in [4,32],
    seed 3): FP32 apply + patch inverse of all of them.  Timed both ways:
    one mixed-degree launch per kernel phase (default shapes), and one
    launch per degree with the autotuned shapes; the rate is that of the way
    the autotuner keeps.  Rate = unique DoFs of the whole batch per second of
    one pass."""
    import synth
    wls = synth.batch_problems(count=count, seed=seed)
    B = fem.Batch([(w.p, w.n, None) for w in wls])
    xs = [P.gather(torch.as_tensor(w.x, device="cuda"), fem.F32) for P, w in zip(B.problems, wls)]
    ys = [P.cell_vector(fem.F32) for P in B.problems]
    zs = [P.cell_vector(fem.F32) for P in B.problems]
    choice = B.autotune(fem.F32)
    kept = B.mixed

    def step(i):
        B.apply(xs, ys)
        B.patch_inverse(ys, zs)

    def timed():
        for i in range(warmup):
            step(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(i)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    ways = {}
    for mixed in (True, False):
        B.set_mixed(mixed)
        ways["mixed" if mixed else "per_degree"] = timed()
    B.set_mixed(kept)
    t = ways["mixed" if kept else "per_degree"]
    uniq = sum(unique_dofs(w.p, w.n[0]) for w in wls)
    cell = sum(cell_dofs(w.p, w.n[0]) for w in wls)
    out = dict(problems=count, unique_dofs=uniq, cell_dofs=cell, s_per_pass=t,
               unique_gdofs=uniq / t / 1e9, cell_gdofs=cell / t / 1e9,
               launches="mixed" if kept else "per_degree",
               s_per_pass_mixed=ways["mixed"], s_per_pass_per_degree=ways["per_degree"],
               autotuned={str(k): v for k, v in choice.items()})
    del xs, ys, zs
    B.close()
    torch.cuda.empty_cache()
    return out


def solve_times(fem, torch, reps):
    """Q7 24^3 graded solve to 1e-8 with FP64/FP32/BF16/FP16 smoothers, for the
    Schwarz smoother alone and for the two-level preconditioner."""
    import synth
    wl = synth.workload_q7_graded()
    P = fem.Problem(7, 24, wl.widths)
    X = [fem.node_coords(7, wl.widths[d]) for d in range(3)]
    f = np.kron(np.kron(np.sin(np.pi * X[2]), np.sin(np.pi * X[1])), np.sin(np.pi * X[0]))
    f = f + 0.01 * wl.noise
    b = P.mass_apply(P.gather(torch.as_tensor(f, device="cuda")))
    out = {}
    # the Schwarz smoother (2 sweeps, omega 1/8) and the two-level method
    # (1 + 1 sweeps, omega 1/5, exact FP64 coarse correction)
    for pre, pc, sweeps, omega in (("", fem.PC_SCHWARZ, 2, 0.125), ("two_level_", fem.PC_TWO_LEVEL, 1, 0.2)):
        for name, sp in (("fp64", fem.F64), ("fp32", fem.F32), ("bf16", fem.BF16), ("fp16", fem.F16)):
            times, iters = [], None
            P.pcg_solve(b, smoother_prec=sp, precond=pc, sweeps=sweeps, omega=omega)          # warm
            for _ in range(reps):
                u = P.cell_vector(fem.F64)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                u, info = P.pcg_solve(b, u=u, rtol=1e-8, maxit=2000, smoother_prec=sp, precond=pc, sweeps=sweeps,
                                      omega=omega)
                times.append(time.perf_counter() - t0)
                iters = info["iters"]
            ts = np.sort(np.asarray(times))
            out[pre + name] = dict(iters=iters, p50_s=float(np.percentile(ts, 50)),
                                   p99_s=float(np.percentile(ts, 99)), relres=info["relres"])
    P.close()
    return out


def cpu_baseline(steps_budget_s=20.0):
    """The oracle on the host cores on a bounded sample of the headline
    workload: the full matrix-free apply, and dense-LU patch solves on a
    sample of patches, scaled to the whole mesh."""
    import synth
    from oracle import operators, patches
    from oracle.mesh import Mesh
    from threadpoolctl import threadpool_limits
    wl = synth.workload_q3_graded()
    m = Mesh(3, wl.n, wl.widths)
    # the oracle is a serial program (a Python loop over patches); its BLAS
    # calls are held to one thread too, so `cores` is what actually ran
    with threadpool_limits(limits=1):
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
    return dict(value=u / (t_apply + t_pi), unit="DoFs/s", cores=1, kind="oracle",
                sample=f"Q3 64^3 graded, one thread: full matrix-free apply ({t_apply:.2f} s) + dense-LU "
                       f"solves of {done} of {len(verts)} vertex patches, extrapolated ({t_pi:.1f} s)",
                host_cpus=os.cpu_count())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--mode", default="bench", choices=["bench", "calib", "serve"])
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--only", choices=["q2_96", "q7_24", "q7_solve", "batch_256", "paper_kernels", "layout"], default=None,
                    help="run one secondary workload alone (for profiling) and print its record")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--solve-reps", type=int, default=5)
    ap.add_argument("--requests", type=int, default=10000, help="serving mode: stream length")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests of the serving stream in the default run (0: skip)")
    ap.add_argument("--prec", choices=["f64", "f32", "bf16", "f16"], default="f64",
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
        elif a.only == "paper_kernels":
            rec = paper_kernels(fem, torch)
        elif a.only == "layout":
            rec = layout_sweep(fem, torch)
        else:
            p, n = (2, 96) if a.only == "q2_96" else (7, 24)
            prec = {"f64": fem.F64, "f32": fem.F32, "bf16": fem.BF16, "f16": fem.F16}[a.prec]
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
        log("mass operator, structured DSS, assembled mass at 128^3")
        extra["paper_kernels"] = paper_kernels(fem, torch)
        log("layout study: block size sweep")
        extra["layout_sweep"] = layout_sweep(fem, torch)
        if a.serve_requests > 0:
            from paper_2607_02335_amd import serve
            log(f"serving stream of {a.serve_requests} requests at 200/s")
            extra["serve"] = serve.run_stream_bench(count=a.serve_requests, log=log)

    log("copy peak")
    copy_gbs = copy_peak(torch)
    roof = roofline(head, "q3_64", copy_gbs)
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
