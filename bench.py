#!/usr/bin/env python3
"""Benchmark of the DEM force step on one MI355X.

Workload (default): 1,000,000 polydisperse spheres (lognormal radii, median
4 um, sigma_log 0.15, clipped to [2, 8] um) in a walled box at volume fraction
0.1 under gravity, half of them seeded touching a neighbour; FP32 contact
force arithmetic with FP64 overlap, history and integration; 200 steps.  The
FP64 path on the same input is timed beside it.

Prints one JSON line: particle-steps/s (whole job), the roofline of the
dominant kernel (algorithmic bytes / HIP-event-timed launch duration), and
the FP64 CPU oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "particle-steps/s at 1M (FP32 batched vs FP64 plain); p50/p99 job latency"


def kernel_bytes(phase, n, m, m_old, fp64, key_bits, force_out=False):
    """Algorithmic HBM bytes of one launch (each record counted once)."""
    if phase == "detect":
        # own record 32, cell range 8, row write 8; partner index 4 per contact
        return 48 * n + 4 * m
    if phase == "force":
        # reads: state 80, rows 8, prev 4, old row 8, cell bound 4;
        # writes: integrated state 80, key+index 8, F/T 24 (48 in FP64) when
        # stored; per contact: partner index 4 + new history 28; per old
        # contact 28
        fo = (48 if fp64 else 24) if force_out else 0
        return (104 + 88 + fo) * n + 32 * m + 28 * m_old
    if phase == "sort":
        passes = max(1, (key_bits + 7) // 8)
        return 20 * n * passes
    if phase == "reorder":
        # keys+index 8, gather 80, write 80, prev 4, cell bounds ~8
        return 180 * n
    return 0


def run_gpu(sc, precision, steps, warmup, stream):
    import torch
    from paper_1503_03553_amd import FLAG_NO_FORCE_OUTPUT, Sim
    sim = Sim.from_scene(sc, precision=precision, stream=stream, flags=FLAG_NO_FORCE_OUTPUT)
    sim.step(warmup)
    sim.sync()
    info0 = sim.info()
    sim.profile(True)
    sim.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sim.profile_read()
    info1 = sim.info()
    sim.close()
    k = info1["steps_done"] - info0["steps_done"]
    m = (info1["sum_contacts"] - info0["sum_contacts"]) / max(k, 1)
    m_old = (info1["sum_old"] - info0["sum_old"]) / max(k, 1)
    matched = (info1["sum_matched"] - info0["sum_matched"]) / max(k, 1)
    return dict(seconds=t1 - t0, steps=steps, prof=prof, contacts=m, contacts_old=m_old,
                matched=matched, info=info1)


def roofline(res, n, fp64):
    key_bits = res["info"]["key_bits"]
    rows = {}
    for ph, (ms, cnt) in res["prof"].items():
        if cnt == 0:
            continue
        avg_s = ms / cnt * 1e-3
        b = kernel_bytes(ph, n, res["contacts"], res["contacts_old"], fp64, key_bits)
        rows[ph] = dict(avg_us=avg_s * 1e6, bytes=b, gbs=b / avg_s / 1e9)
    dom = max(rows, key=lambda p: rows[p]["avg_us"])
    r = rows[dom]
    out = {"bound": "hbm", "kernel": "k_" + dom, "achieved": round(r["gbs"], 1),
           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(r["gbs"] / HBM_PEAK_GBS, 4),
           "traffic": None, "bytes_per_launch": int(r["bytes"]),
           "avg_launch_us": round(r["avg_us"], 2)}
    return out, rows


def cpu_baseline(sc, dt, budget_s):
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    threads = min(threads, 16)
    s = oracle.Sim(sc, dt=dt, mode=1, threads=threads)
    t0 = time.perf_counter()
    s.step(1)
    t1 = time.perf_counter() - t0
    k = max(1, min(50, int(budget_s / max(t1, 1e-6))))
    t0 = time.perf_counter()
    s.step(k)
    el = time.perf_counter() - t0
    return {"value": round(sc.n * k / el, 1), "unit": "particle-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d steps (after 1 untimed) of the same %d-particle workload, cell-list mode, "
                      "OpenMP over particles" % (k, sc.n)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--verbose", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(got --gpus %d)" % a.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import gen
    from paper_1503_03553_amd import PREC_FP64, PREC_MIXED
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    def log(*x):
        if a.verbose:
            print(*x, file=sys.stderr, flush=True)

    t = time.perf_counter()
    sc = gen.config_dilute(n=a.n)
    log("generated %d spheres in %.1fs" % (sc.n, time.perf_counter() - t))

    mixed = run_gpu(sc, PREC_MIXED, a.steps, a.warmup, stream)
    n = sc.n
    value = n * a.steps / mixed["seconds"]
    roof, rows = roofline(mixed, n, fp64=False)
    log("mixed", json.dumps(rows))

    extra = {}
    if not a.no_fp64:
        f64 = run_gpu(sc, PREC_FP64, a.steps, a.warmup, stream)
        roof64, rows64 = roofline(f64, n, fp64=True)
        log("fp64", json.dumps(rows64))
        extra["fp64_plain"] = {"value": round(n * a.steps / f64["seconds"], 1),
                               "ms_per_step": round(f64["seconds"] / a.steps * 1e3, 4),
                               "roofline": roof64}

    step_bytes = sum(r["bytes"] for r in rows.values())
    step_time = sum(r["avg_us"] for r in rows.values()) * 1e-6
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(mixed["seconds"] / a.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": "dilute-1m: %d polydisperse spheres, phi 0.1, walls, gravity, "
                               "single simulation" % n,
                   "precision": "mixed: fp32 contact force, fp64 overlap/history/integration",
                   "contacts_per_particle": round(mixed["contacts"] / n, 4),
                   "history_matched_per_step": round(mixed["matched"], 1),
                   "cells": list(mixed["info"]["cells"]), "key_bits": mixed["info"]["key_bits"]},
        "roofline": roof,
        "kernels": {k: {"avg_us": round(v["avg_us"], 2), "GBps": round(v["gbs"], 1)}
                    for k, v in rows.items()},
        "step_roofline_frac": round(step_bytes / step_time / 1e9 / HBM_PEAK_GBS, 4),
    }
    out.update(extra)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(sc, None, a.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
