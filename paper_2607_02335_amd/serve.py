"""Serving driver: a Poisson-arrival stream of solve requests replayed in
real time against the continuous-batching server of the library.

Each request (degree p, n^3 cells of the unit cube, nodal source f ~ U[-1,1])
is submitted when its arrival time has passed on the wall clock; the host
loop alternates server steps (every admitted solve advances one iteration in
batched launches) with polling.  Latency is completion minus arrival.
"""
from __future__ import annotations

import time

import numpy as np

import synth
from paper_2607_02335_amd import fem


def run_stream(requests, hbm_budget=64 << 30, max_active=256, smoother_prec=fem.F32, rtol=1e-8,
               maxit=3000, log_every=5.0, log=None):
    S = fem.Server(hbm_budget=hbm_budget, max_active=max_active, smoother_prec=smoother_prec)
    t0 = time.perf_counter()
    nxt = 0
    pending = {}
    lat, iters, udofs = [], [], 0
    failures = 0
    steps = 0
    last_log = t0
    peak_active = 0
    while nxt < len(requests) or pending:
        now = time.perf_counter() - t0
        while nxt < len(requests) and requests[nxt]["t"] <= now:
            r = requests[nxt]
            f = synth.request_rhs_nodal(r["p"], (r["n"],) * 3, r["seed"])
            tk = S.submit(r["p"], r["n"], f, rtol=rtol, maxit=maxit)
            pending[tk] = r
            nxt += 1
        a, q, d = S.step()
        steps += 1
        peak_active = max(peak_active, a)
        tnow = time.perf_counter() - t0
        for tk in (S.finished() if d else []):
            res = S.poll(tk, want_u=False)
            if res is None:
                continue
            r = pending.pop(tk)
            info = res[1]
            if info["status"] != 0:
                failures += 1
            lat.append(tnow - r["t"])
            iters.append(info["iters"])
            udofs += (r["n"] * r["p"] + 1) ** 3
        if not pending and nxt < len(requests):
            time.sleep(max(0.0, min(0.001, requests[nxt]["t"] - (time.perf_counter() - t0))))
        if log and time.perf_counter() - last_log > log_every:
            last_log = time.perf_counter()
            log(f"t={tnow:7.1f}s submitted={nxt} done={len(lat)} active={a} queued={q} steps={steps}")
    wall = time.perf_counter() - t0
    in_use, high = S.memory()
    S.close()
    lat = np.asarray(lat)
    return dict(requests=len(requests), wall_s=wall, steps=steps, failures=failures,
                p50_latency_s=float(np.percentile(lat, 50)), p99_latency_s=float(np.percentile(lat, 99)),
                mean_iters=float(np.mean(iters)), solved_unique_dofs_per_s=udofs / wall,
                peak_active=peak_active, hbm_high_water_bytes=int(high), hbm_budget_bytes=int(hbm_budget))


def run_stream_bench(count=10000, rate=200.0, seed=4, log=None):
    reqs = synth.serve_stream(count=count, rate=rate, seed=seed)
    res = run_stream(reqs, log=log)
    res.update(metric="p50/p99 solve latency and solved unique DoFs/s under Poisson arrivals",
               config=dict(workload=f"{count} Poisson solve requests at {rate:g}/s, p in {{2,3,7}} "
                                    f"w=(0.4,0.4,0.2), n lognormal median 12 clipped [4,48], seed {seed}",
                           smoother="FP32 additive Schwarz, 2 sweeps, FCG to 1e-8"))
    return res
