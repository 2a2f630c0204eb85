#!/usr/bin/env python3
"""Benchmark of the DEM step on one MI355X.

Headline workload (`value`): 1,000,000 polydisperse spheres (lognormal radii,
median 4 um, sigma_log 0.15, clipped to [2, 8] um) in a walled box at volume
fraction 0.1 under gravity, half of them seeded touching a neighbour; FP32
contact force arithmetic with FP64 overlap, history and integration; 200
steps (the default), one simulation.  Beside it, on the same GPU and in the
same run:
  fp64_plain      the same input with every operation in FP64;
  plain_2000_fp64 2,000 monodisperse spheres at volume fraction 0.3, FP64,
                  1000 steps;
  dense_shear_8m  8M spheres grown to volume fraction 0.55 (not timed), then
                  Lees-Edwards shear: throughput and contact-table churn;
  batched         256 independent jobs, N log-uniform in [1k, 200k], volume
                  fraction U[0.1, 0.5], run in one pool (one set of launches
                  per step), cell factor and job layout picked by the
                  autotuner;
  serving         1,000 requests arriving as a Poisson stream (20 jobs/s),
                  jobs of 1k-1M particles and 100-2000 steps, served by
                  continuous batching; p50/p99 latency split into queueing
                  and service, and aggregate throughput;
  cpu_baseline    the FP64 CPU oracle on a bounded sample of the headline
                  workload, on all cores of the process's share and on one.

Prints one JSON line.  The roofline object is that of the dominant kernel of
the headline run: the method's bytes per launch / its average duration from
HIP events recorded on the stream the kernels run on.
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

HBM_PEAK_GBS = 8000.0
METRIC = "particle-steps/s at 1M (FP32 batched vs FP64 plain); p50/p99 job latency"


def kernel_bytes(phase, n, m, m_old, fp64, key_bits, force_out=False, half=True, merge=True):
    """Bytes one launch of the phase's kernels reads and writes as
    implemented (each record counted once); `half`: the default half search,
    whose lists the force kernel turns into rows (else the full search
    writes the rows); `merge`: the default sort (merge of the particles that
    changed cell) rather than the radix sort."""
    if phase == "detect":
        if half:
            # own FP32 record 16 + FP64 position 32, cell bounds 8 (as
            # below); per contact: list entry 8 and its counter 4
            return 56 * n + 12 * m
        # own FP32 record 16 + FP64 position 32, 9 cell-row bounds read as
        # 27 cells x 8 (cache-resident, counted once per particle: 8), row
        # write 8; partner index 4 per contact
        return 48 * n + 4 * m
    if phase == "force":
        # reads: sorted position 32, velocities 48 and old row 8 through the
        # permutation 4, new row 8; writes: integrated state 80, F/T 24 (48 in
        # FP64) when stored; the sort's input: with the merge sort the key
        # before the step 4, with the radix sort key and index 8 and the old
        # cell's bound read 4; per contact: partner index 4, partner
        # permutation 4, new history 28; per old contact 28.  With the half
        # search also the list counter read and reset 8 per particle, and per
        # contact the list entry 8 and the partner index written 4.
        fo = (48 if fp64 else 24) if force_out else 0
        extra = 8 * n + 12 * m if half else 0
        sort_in = 4 if merge else 12
        return (100 + 80 + sort_in + fo) * n + 36 * m + 28 * m_old + extra
    if phase == "sort":
        if merge:
            # keys before the step and the new state's positions read 36; at
            # each new position the sorted key, the FP32 record and the
            # permutation written 24; plus the few movers (negligible)
            return 60 * n
        passes = max(1, (key_bits + 7) // 8)
        return 20 * n * passes
    if phase == "reorder":
        if merge:
            # the sorted keys (neighbours from the cache) 4, cell bounds ~8
            return 12 * n
        # sorted key and source index 8, gathered position 32, FP32 record
        # written 16, permutation 4, cell bounds ~8
        return 68 * n
    return 0


def method_bytes(phase, n, m, m_old, fp64, key_bits, force_out=False, merge=True):
    """Algorithmic bytes of one launch: what the method's step needs of HBM
    for the work the phase's kernels do, each particle's record and each
    contact's entry counted once, independent of how the kernels organise
    it.  Per particle with c directed contacts (c' of the step before):
      detect  (contact search)          40 + 4c: position and radius 28, cell
              ranges 8, row start/count 4; partner index 4 per contact
      force   (history match, contact law, per-particle sums, integration
              and hashing in one pass)  176 + 32c + 28c': own and partner
              records once 80 (position, velocity, angular velocity,
              radius, id), permutation and old row 8, row 8, integrated
              state written 72, key and index 8; per contact partner index 4
              and new id and displacement 28; per old contact id and
              displacement 28; F and T 24 (48 in FP64) only when stored
      sort    (stable sort of (key, index))  the implementation's bytes (the
              merge sort's placement also writes the FP32 records)
      reorder (gather into cell order, cell bounds)  at most 168 (index 4,
              record gathered 80 and written 80, bounds 4); the kernels move
              only positions, so their own smaller count applies
    """
    impl = kernel_bytes(phase, n, m, m_old, fp64, key_bits, force_out=force_out, merge=merge)
    if phase == "detect":
        return min(40 * n + 4 * m, impl)
    if phase == "force":
        fo = (48 if fp64 else 24) if force_out else 0
        return (176 + fo) * n + 32 * m + 28 * m_old
    if phase == "reorder":
        return min(168 * n, impl)
    return impl


def phase_rows(prof, n, m, m_old, fp64, key_bits, half=True, merge=True):
    rows = {}
    for ph, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        avg_s = ms / cnt * 1e-3
        b = method_bytes(ph, n, m, m_old, fp64, key_bits, merge=merge)
        bi = kernel_bytes(ph, n, m, m_old, fp64, key_bits, half=half, merge=merge)
        rows[ph] = dict(avg_us=avg_s * 1e6, bytes=b, impl_bytes=bi, gbs=b / avg_s / 1e9)
    return rows


def measured_traffic(kernel, precision_tag):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes scaled by a plain copy of known size),
    or None when the kernels have changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_dilute_1m.json")
    src = os.path.join(ROOT, "paper_1503_03553_amd", "csrc", "dem_kernels.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernels_source_sha256") != sha:
        return None
    for k, v in rec["per_launch_bytes"].items():
        if kernel_is(k, kernel, precision_tag):
            return int(v)
    return None


def kernel_is(name, kernel, precision_tag):
    """Whether a profiled kernel name ("k_force<float, 8>") is the headline
    path's instantiation of `kernel`: the force kernel in the given precision
    over the half search's lists (list slots after the type, not 0)."""
    if name.split("<")[0] != kernel:
        return False
    if kernel == "k_force":
        return precision_tag in name and not name.replace(" ", "").endswith(",0>")
    return True


# Peak VALU issue rate: each CU's four SIMDs issue one wave64 VALU
# instruction every four cycles (16 lanes per cycle), so a CU issues one per
# cycle: 256 CUs x 2.4 GHz.
VALU_PEAK = 256 * 2.4e9
PHASE_KERNELS = {"detect": ("k_detect_half",), "force": ("k_force",),
                 "sort": ("k_mov_sort", "k_place"), "reorder": ("k_reorder", "k_tick")}


def valu_insts(phase, precision_tag):
    """VALU wave-instructions per step of a phase (its kernels' SQ_INSTS_VALU
    per launch, summed) from the committed counter summary, or None when the
    kernels have changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "valu_dilute_1m.json")
    src = os.path.join(ROOT, "paper_1503_03553_amd", "csrc", "dem_kernels.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernels_source_sha256") != sha:
        return None
    tot, found = 0.0, False
    for k, v in rec["per_launch"].items():
        if any(kernel_is(k, b, precision_tag) for b in PHASE_KERNELS.get(phase, ())):
            tot += v["SQ_INSTS_VALU"]
            found = True
    return tot if found else None


def valu_of(phase, avg_us, precision_tag):
    n = valu_insts(phase, precision_tag)
    if n is None:
        return None
    rate = n / (avg_us * 1e-6)
    return {"insts_per_launch": int(n), "achieved": round(rate / 1e9, 2), "peak": VALU_PEAK / 1e9,
            "unit": "G wave-instr/s", "frac": round(rate / VALU_PEAK, 4)}


def roofline_of(rows, precision_tag="float"):
    """The dominant kernel against the HBM peak: `achieved` is its
    algorithmic bytes (method_bytes) per launch over its average launch
    duration; `implementation_bytes_per_launch` is what the kernel moves as
    written, `overhead_bytes_per_launch` the difference."""
    dom = max(rows, key=lambda p: rows[p]["avg_us"])
    r = rows[dom]
    kern = PHASE_KERNELS[dom][0] if dom in PHASE_KERNELS else "k_" + dom
    return {"bound": "hbm", "kernel": kern, "achieved": round(r["gbs"], 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(r["gbs"] / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(kern, precision_tag),
            "bytes_per_launch": int(r["bytes"]), "avg_launch_us": round(r["avg_us"], 2),
            "implementation_bytes_per_launch": int(r["impl_bytes"]),
            "overhead_bytes_per_launch": int(r["impl_bytes"] - r["bytes"]),
            "valu_issue": valu_of(dom, r["avg_us"], precision_tag)}


def contact_kernels_of(rows):
    """The contact search and the force kernel together (the force/contact
    kernels) against the HBM peak: their algorithmic bytes over the sum of
    their average launch durations, beside the 0.5 target."""
    if "detect" not in rows or "force" not in rows:
        return None
    b = rows["detect"]["bytes"] + rows["force"]["bytes"]
    us = rows["detect"]["avg_us"] + rows["force"]["avg_us"]
    gbs = b / (us * 1e-6) / 1e9
    return {"bytes_per_step": int(b), "us_per_step": round(us, 2), "achieved": round(gbs, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "target_frac": 0.5}


def kernels_of(rows, precision_tag="float", headline=True):
    """Per-phase duration and algorithmic GB/s; VALU issue utilisation only
    for the headline workload, whose instruction counts were taken."""
    out = {}
    for k, v in rows.items():
        va = valu_of(k, v["avg_us"], precision_tag) if headline else None
        out[k] = {"avg_us": round(v["avg_us"], 2), "GBps": round(v["gbs"], 1),
                  "bytes": int(v["bytes"]), "implementation_bytes": int(v["impl_bytes"]),
                  "valu_frac": None if va is None else va["frac"]}
    return out


# ------------------------------------------------------------ single sim
def run_single(sc, precision, steps, warmup, stream, flags=0):
    """Warm-up, then `steps` timed steps without instrumentation (the
    throughput); then the same again from the same initial state with HIP
    events at the phase boundaries (the per-kernel durations, over the same
    steps)."""
    import torch
    from paper_1503_03553_amd import FLAG_NO_FORCE_OUTPUT, Sim
    out = {}
    for profiled in (False, True):
        sim = Sim.from_scene(sc, precision=precision, stream=stream,
                             flags=FLAG_NO_FORCE_OUTPUT | flags)
        sim.step(warmup)
        sim.sync()
        info0 = sim.info()
        if profiled:
            sim.profile(True)
            sim.profile_read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.sync()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if profiled:
            out["prof"] = sim.profile_read()
            out["seconds_profiled"] = t1 - t0
        else:
            out["seconds"] = t1 - t0
        info1 = sim.info()
        sim.close()
    k = max(info1["steps_done"] - info0["steps_done"], 1)
    out.update(steps=steps, info=info1,
               contacts=(info1["sum_contacts"] - info0["sum_contacts"]) / k,
               contacts_old=(info1["sum_old"] - info0["sum_old"]) / k,
               matched=(info1["sum_matched"] - info0["sum_matched"]) / k)
    return out


# -------------------------------------------------------------- ablation
def run_ablation(sizes, steps, warmup, stream, log):
    """The fused single loop (section 3.4; the comparison of section 4) and
    the action-reaction variant (section 3.3) against the split path on the
    grid inputs of gen.config_ablation, in mixed precision.  "split" is the
    split with the full per-particle search of Algorithm 1, as the variants
    have it; "half_search" the default path (each pair tested once).
    "collide" is the contact search plus the force kernels: detect + force
    for the split paths, the fused kernel plus the clearing of the old cell
    bounds for the fused one, detect + pair forces + sums for
    action-reaction."""
    import gen
    from paper_1503_03553_amd import (FLAG_ACTION_REACTION, FLAG_FULL_DETECT, FLAG_FUSED,
                                      FLAG_THREAD_SPLIT, PREC_MIXED)
    rows = []
    for n in sizes:
        for regime in ("dense", "sparse"):
            sc = gen.config_ablation(n, regime)
            row = {"n": sc.n, "regime": regime}
            for name, flag in (("split", FLAG_FULL_DETECT), ("half_search", 0),
                               ("fused", FLAG_FUSED),
                               ("thread_split", FLAG_THREAD_SPLIT),
                               ("action_reaction", FLAG_ACTION_REACTION)):
                r = run_single(sc, PREC_MIXED, steps, warmup, stream, flags=flag)
                ph = {p: ms / c * 1e3 for p, (ms, c) in r["prof"].items() if c}
                row["contacts_per_particle"] = round(r["contacts"] / sc.n, 3)
                row[name] = {"ms_per_step": round(r["seconds"] / steps * 1e3, 4),
                             "collide_us": round(ph.get("detect", 0.0) + ph.get("force", 0.0), 2),
                             "phases_us": {p: round(v, 2) for p, v in ph.items()}}
            row["collide_fused_over_split"] = round(row["fused"]["collide_us"] /
                                                    row["split"]["collide_us"], 3)
            row["step_fused_over_split"] = round(row["fused"]["ms_per_step"] /
                                                 row["split"]["ms_per_step"], 3)
            row["collide_thread_split_over_split"] = round(row["thread_split"]["collide_us"] /
                                                           row["split"]["collide_us"], 3)
            row["step_half_search_over_split"] = round(row["half_search"]["ms_per_step"] /
                                                       row["split"]["ms_per_step"], 3)
            row["step_action_reaction_over_split"] = round(
                row["action_reaction"]["ms_per_step"] / row["split"]["ms_per_step"], 3)
            log("ablation %s" % json.dumps(row))
            rows.append(row)
    return rows


# --------------------------------------------------------------- batched
def pool_for(scenes, precision, stream, slack_jobs=0, flags=0):
    from paper_1503_03553_amd import Pool
    from paper_1503_03553_amd.binding import job_cells
    parts = sum(((s.n + 127) // 128) * 128 for s in scenes)
    cells = sum(job_cells(s) for s in scenes)
    return Pool(max_particles=max(parts, 128), max_cells=max(cells, 1),
                max_jobs=len(scenes) + slack_jobs, precision=precision, stream=stream, flags=flags)


def run_batched(scenes, steps, warmup, stream, tune_steps, log):
    """Autotune, then `steps` timed steps of the whole pool without
    instrumentation (the throughput), then the same again in a fresh pool
    with HIP events at the phase boundaries (the kernel durations)."""
    import torch
    from paper_1503_03553_amd import FLAG_NO_FORCE_OUTPUT, PREC_MIXED, tune
    make = lambda c: pool_for(scenes, PREC_MIXED, stream, flags=FLAG_NO_FORCE_OUTPUT)
    t = time.perf_counter()
    best, table = tune.autotune(make, scenes, steps=tune_steps, warmup=2, log=log)
    tune_s = time.perf_counter() - t
    out = {}
    for profiled in (False, True):
        pool = make(best)
        tune.fill_pool(pool, scenes, warmup + steps, best)
        pool.step(warmup)
        pool.sync()
        if profiled:
            pool.profile(True)
            pool.profile_read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pool.step(steps)
        pool.sync()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if profiled:
            out["prof"] = pool.profile_read()
            out["seconds_profiled"] = t1 - t0
        else:
            out["seconds"] = t1 - t0
            out["finished"] = len(pool.poll())
        pool.close()
    out.update(n=sum(s.n for s in scenes), best=best, tune_s=tune_s,
               table=[(c, round(s * 1e3, 4)) for c, s in table])
    return out


def run_one_at_a_time(scenes, precision, steps, warmup, stream):
    """The same jobs through the plain single-simulation path, one after
    another: seconds per step of each job alone (no instrumentation), summed."""
    import torch
    from paper_1503_03553_amd import FLAG_NO_FORCE_OUTPUT, Sim
    total = 0.0
    for sc in scenes:
        sim = Sim.from_scene(sc, precision=precision, stream=stream, flags=FLAG_NO_FORCE_OUTPUT)
        sim.step(warmup)
        sim.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.sync()
        torch.cuda.synchronize()
        total += (time.perf_counter() - t0) / steps
        sim.close()
    return total


# --------------------------------------------------------------- serving
def run_serving(scenes, arr, steps, stream, budget_particles, superstep, log, at_once_too=False):
    """Serve the requests (request q: scenes[q] for steps[q] steps, arriving
    at arr[q]) at their arrival times; the same requests all arriving at once
    give the throughput of a pool that is never idle."""
    from paper_1503_03553_amd import FLAG_NO_FORCE_OUTPUT, PREC_MIXED, Pool
    from paper_1503_03553_amd.serve import Request, Server
    max_jobs = 256
    out = []
    for at_once in ((False, True) if at_once_too else (False,)):
        pool = Pool(max_particles=budget_particles, max_cells=4 * budget_particles + 4096 * 64,
                    max_jobs=max_jobs, precision=PREC_MIXED, stream=stream,
                    flags=FLAG_NO_FORCE_OUTPUT)
        reqs = [Request(q, scenes[q], int(steps[q]), 0.0 if at_once else float(arr[q]))
                for q in range(len(arr))]
        srv = Server(pool, superstep=superstep, target_s=0.05)
        st = srv.run(reqs, deadline=900.0)
        pool.close()
        log("serving%s: %s" % (" (all at once)" if at_once else "", json.dumps(st)))
        out.append(st)
    return out


# ----------------------------------------------------------- cpu oracle
def cpu_model():
    """The host CPU's model name (/proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def host_threads():
    """Threads for the all-core oracle run: the CPUs this process may use,
    at most 16 (a one-GPU share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    env = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    if env:
        n = min(n, env)
    return max(1, min(n, 16))


def oracle_rate(sc, threads, budget_s, max_steps=50, steps=None):
    """particle-steps/s of the oracle (cell-list mode) on `sc` with `threads`
    OpenMP threads: one untimed step, then `steps` (or as many as fit
    budget_s, at most max_steps) timed."""
    import oracle
    s = oracle.Sim(sc, mode=1, threads=threads)
    t0 = time.perf_counter()
    s.step(1)
    t1 = time.perf_counter() - t0
    k = steps if steps else max(1, min(max_steps, int(budget_s / max(t1, 1e-6))))
    t0 = time.perf_counter()
    s.step(k)
    el = time.perf_counter() - t0
    return sc.n * k / el, k


def cpu_baseline(sc, budget_s, plain=None):
    """The oracle on the host's cores: the headline workload (a bounded
    number of steps) on all cores of the process's share and on one core,
    and the 2,000-sphere plain workload over its 1000 steps on both."""
    th = host_threads()
    rate, k = oracle_rate(sc, th, budget_s)
    rate1, k1 = oracle_rate(sc, 1, budget_s, max_steps=20)
    out = {"value": round(rate, 1), "unit": "particle-steps/s", "cores": th, "kind": "oracle",
           "sample": "%d steps (after 1 untimed) of the same %d-particle workload, cell-list mode, "
                     "OpenMP over particles" % (k, sc.n),
           "single_core": {"value": round(rate1, 1), "cores": 1,
                           "sample": "%d steps (after 1 untimed), one thread" % k1},
           "cpu_model": cpu_model(), "cpus_visible": os.cpu_count()}
    if plain is not None:
        pa, ka = oracle_rate(plain, th, 0, steps=1000)
        p1, k1 = oracle_rate(plain, 1, 0, steps=1000)
        out["plain_2000_fp64"] = {"all_cores": round(pa, 1), "single_core": round(p1, 1),
                                  "cores": th, "steps": ka, "unit": "particle-steps/s"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the action-reaction and full-search legs beside the headline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--batch-jobs", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--tune-steps", type=int, default=10)
    ap.add_argument("--alone-steps", type=int, default=100,
                    help="steps per job when the batched jobs run one at a time (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-all-at-once", action="store_true",
                    help="also serve the same requests all arriving at once")
    ap.add_argument("--serve-gen-threads", type=int, default=12,
                    help="host threads drawing the served scenes during the GPU legs")
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-budget", type=int, default=8_000_000)
    ap.add_argument("--superstep", type=int, default=20)
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="first run a plain device-to-device copy of this many MiB 5 times "
                         "(reference reads/writes for HBM traffic counters)")
    ap.add_argument("--no-ablation", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--dense-n", type=int, default=8_000_000)
    ap.add_argument("--dense-steps", type=int, default=100)
    ap.add_argument("--grow-increments", type=int, default=200,
                    help="radius increments of the dense pack's growth")
    ap.add_argument("--grow-steps", type=int, default=20,
                    help="DEM steps after each radius increment")
    ap.add_argument("--ablation-sizes", default="131072,524288,2097152")
    ap.add_argument("--ablation-steps", type=int, default=20)
    ap.add_argument("--only", choices=("all", "single", "batch", "serve", "ablation", "dense"),
                    default="all",
                    help="run one part only (for profiling); the JSON line then lacks the others")
    ap.add_argument("--verbose", action="store_true")
    a = ap.parse_args()
    if a.only != "all":
        a.no_fp64 = a.no_fp64 or a.only != "single"
        a.no_cpu = True
        a.no_batch = a.only != "batch"
        a.no_serve = a.only != "serve"
        a.no_ablation = a.only != "ablation"
        a.no_dense = a.only != "dense"
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(got --gpus %d)" % a.gpus, file=sys.stderr)
        sys.exit(2)

    def log(*x):
        if a.verbose:
            print(*x, file=sys.stderr, flush=True)

    import gen
    # every input is drawn before anything touches the GPU (the generators
    # fork worker processes)
    t = time.perf_counter()
    sc = gen.config_dilute(n=a.n) if a.only in ("all", "single") or not a.no_cpu else None
    if sc is not None:
        log("headline input: %d spheres in %.1fs" % (sc.n, time.perf_counter() - t))
    batch = []
    if not a.no_batch:
        t = time.perf_counter()
        sizes = gen.batch_sizes(0, a.batch_jobs)
        batch = gen.generate_many(gen.config_batch_job,
                                  [(0, m, int(sizes[m])) for m in range(a.batch_jobs)])
        log("batched input: %d jobs, %d spheres in %.1fs (%d to grow)" % (
            len(batch), sum(s.n for s in batch), time.perf_counter() - t,
            sum(1 for s in batch if s.meta.get("grow"))))
    dense = None
    if not a.no_dense:
        t = time.perf_counter()
        dense = gen.config_dense_start(n=a.dense_n)
        log("dense start: %d spheres in %.1fs" % (dense.n, time.perf_counter() - t))
    serve_in = None
    if not a.no_serve:
        # the served requests' scenes are drawn on host threads while the
        # GPU legs run (the serving clock starts once all are there); the
        # process pools above are done by then
        import concurrent.futures as cf
        arr, sizes, steps = gen.serve_requests(gen.SEED_BASE + 9000, a.serve_requests,
                                               rate=a.serve_rate)
        gen.build_helper()
        ex = cf.ThreadPoolExecutor(max(1, min(a.serve_gen_threads, os.cpu_count() or 1)))
        futs = [ex.submit(gen.config_serve_job, q, int(sizes[q])) for q in range(len(sizes))]
        serve_in = (futs, arr, steps, ex, time.perf_counter())

    import torch
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if a.calibrate_copy_mb:
        src = torch.ones(a.calibrate_copy_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    out = {}
    if a.only in ("all", "single"):
        out = headline(a, sc, stream, log)
    run_others(a, out, sc, batch, serve_in, stream, log, dense)
    print(json.dumps(out), flush=True)


def headline(a, sc, stream, log):
    from paper_1503_03553_amd import PREC_FP64, PREC_MIXED
    mixed = run_single(sc, PREC_MIXED, a.steps, a.warmup, stream)
    n = sc.n
    value = n * a.steps / mixed["seconds"]
    rows = phase_rows(mixed["prof"], n, mixed["contacts"], mixed["contacts_old"], False,
                      mixed["info"]["key_bits"])
    log("mixed", json.dumps(rows))

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(mixed["seconds"] / a.steps * 1e3, 4),
        # a second pass of as many steps with HIP events at the phase
        # boundaries gives the kernel durations below
        "ms_per_step_with_events": round(mixed["seconds_profiled"] / a.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": "dilute-1m: %d polydisperse spheres, phi 0.1, walls, gravity, "
                               "one simulation, %d steps" % (n, a.steps),
                   "precision": "mixed: fp32 contact force, fp64 overlap/history/integration",
                   "contact_search": "half stencil, each pair tested once",
                   "contacts_per_particle": round(mixed["contacts"] / n, 4),
                   "history_matched_per_step": round(mixed["matched"], 1),
                   "cells": list(mixed["info"]["cells"]), "key_bits": mixed["info"]["key_bits"]},
        "roofline": roofline_of(rows),
        "contact_kernels_roofline": contact_kernels_of(rows),
        "kernels": kernels_of(rows),
    }
    step_bytes = sum(r["bytes"] for r in rows.values())
    step_time = sum(r["avg_us"] for r in rows.values()) * 1e-6
    out["step_roofline_frac"] = round(step_bytes / step_time / 1e9 / HBM_PEAK_GBS, 4)

    if not a.no_variants:
        from paper_1503_03553_amd import FLAG_ACTION_REACTION
        ar = run_single(sc, PREC_MIXED, a.steps, a.warmup, stream, flags=FLAG_ACTION_REACTION)
        rows_ar = phase_rows(ar["prof"], n, ar["contacts"], ar["contacts_old"], False,
                             ar["info"]["key_bits"], half=False)
        out["action_reaction"] = {"value": round(n * a.steps / ar["seconds"], 1),
                                  "unit": "particle-steps/s",
                                  "ms_per_step": round(ar["seconds"] / a.steps * 1e3, 4),
                                  "phases_us": {k: round(v["avg_us"], 2) for k, v in rows_ar.items()}}
        # the full per-particle search of Algorithm 1 in place of the half search
        from paper_1503_03553_amd import FLAG_FULL_DETECT
        fd = run_single(sc, PREC_MIXED, a.steps, a.warmup, stream, flags=FLAG_FULL_DETECT)
        rows_fd = phase_rows(fd["prof"], n, fd["contacts"], fd["contacts_old"], False,
                             fd["info"]["key_bits"], half=False)
        out["full_detect"] = {"value": round(n * a.steps / fd["seconds"], 1),
                              "unit": "particle-steps/s",
                              "ms_per_step": round(fd["seconds"] / a.steps * 1e3, 4),
                              "kernels": kernels_of(rows_fd, headline=False)}

    if not a.no_fp64:
        f64 = run_single(sc, PREC_FP64, a.steps, a.warmup, stream)
        rows64 = phase_rows(f64["prof"], n, f64["contacts"], f64["contacts_old"], True,
                            f64["info"]["key_bits"])
        log("fp64", json.dumps(rows64))
        out["fp64_plain"] = {"value": round(n * a.steps / f64["seconds"], 1),
                             "unit": "particle-steps/s",
                             "ms_per_step": round(f64["seconds"] / a.steps * 1e3, 4),
                             "ms_per_step_with_events":
                                 round(f64["seconds_profiled"] / a.steps * 1e3, 4),
                             "roofline": roofline_of(rows64, "double"),
                             "kernels": kernels_of(rows64, "double")}
        # the 2,000-sphere plain workload in FP64 over its 1000 steps (launch
        # latency bound at this size)
        import gen
        pl = gen.config_plain()
        r = run_single(pl, PREC_FP64, 1000, a.warmup, stream)
        out["plain_2000_fp64"] = {"value": round(pl.n * 1000 / r["seconds"], 1),
                                  "unit": "particle-steps/s", "steps": 1000,
                                  "ms_per_step": round(r["seconds"] / 1000 * 1e3, 4),
                                  "contacts_per_particle": round(r["contacts"] / pl.n, 4)}

    return out


def gen_dense_run(start, g):
    import gen
    return gen.dense_run_scene(start, g["x"], g["v"], g["w"])


def run_others(a, out, sc, batch, serve_in, stream, log, dense=None):
    if dense is not None:
        # the 8M dense sheared pack: grown to phi 0.55 on the GPU (not timed),
        # then the sheared run: throughput and contact-table churn
        from paper_1503_03553_amd import PREC_MIXED, pack
        t = time.perf_counter()
        g = pack.grown(dense, increments=a.grow_increments, steps_per_increment=a.grow_steps,
                       stream=stream, log=log)
        grow_s = time.perf_counter() - t
        run = gen_dense_run(dense, g)
        log("dense pack grown in %.1fs: %s" % (grow_s, json.dumps(g["stats"])))
        r = run_single(run, PREC_MIXED, a.dense_steps, a.warmup, stream)
        rows = phase_rows(r["prof"], run.n, r["contacts"], r["contacts_old"], False,
                          r["info"]["key_bits"])
        m = r["contacts"]
        out["dense_shear_8m"] = {
            "value": round(run.n * a.dense_steps / r["seconds"], 1), "unit": "particle-steps/s",
            "particles": run.n, "steps": a.dense_steps, "warmup": a.warmup,
            "ms_per_step": round(r["seconds"] / a.dense_steps * 1e3, 4),
            "workload": "%d spheres, phi %.2f grown on the GPU from RSA at phi %.2f, Lees-Edwards "
                        "shear %g/s, mixed precision" % (run.n, dense.meta["phi"],
                                                         dense.meta["phi0"], run.shear_rate),
            "growth": dict(g["stats"], seconds=round(grow_s, 2)),
            "contacts_per_particle": round(m / run.n, 4),
            "churn_per_step": {"created": round(m - r["matched"], 1),
                               "broken": round(r["contacts_old"] - r["matched"], 1),
                               "created_frac": round((m - r["matched"]) / max(m, 1), 5)},
            "contact_kernels_roofline": contact_kernels_of(rows),
            "kernels": kernels_of(rows, headline=False)}
    if batch:
        from paper_1503_03553_amd import PREC_FP64, PREC_MIXED, pack
        # jobs above the volume fraction RSA reaches quickly are grown to it
        # first, all in one pool (not timed)
        t = time.perf_counter()
        gi = [k for k, sc in enumerate(batch) if sc.meta.get("grow")]
        grown = pack.grow_pool([batch[k] for k in gi], increments=a.grow_increments,
                               steps_per_increment=a.grow_steps, stream=stream)
        import gen
        for k, st in zip(gi, grown):
            batch[k] = gen.grown_scene(batch[k], st["x"], st["v"], st["w"])
        grow_s = time.perf_counter() - t
        log("batched: %d jobs grown in %.1fs" % (len(gi), grow_s))
        b = run_batched(batch, a.batch_steps, a.warmup, stream, a.tune_steps, log)
        brows = phase_rows(b["prof"], b["n"], 0, 0, False, 24)
        value = b["n"] * a.batch_steps / b["seconds"]
        phis = [sc.meta.get("phi", 0.0) for sc in batch]
        out["batched"] = {"value": round(value, 1),
                          "unit": "particle-steps/s",
                          "jobs": len(batch), "particles": b["n"], "steps": a.batch_steps,
                          "phi_range": [round(min(phis), 3), round(max(phis), 3)],
                          "grown_jobs": len(gi), "growth_seconds": round(grow_s, 2),
                          "ms_per_step": round(b["seconds"] / a.batch_steps * 1e3, 4),
                          "ms_per_step_with_events":
                              round(b["seconds_profiled"] / a.batch_steps * 1e3, 4),
                          "finished": b["finished"],
                          "autotuned": b["best"], "tune_seconds": round(b["tune_s"], 2),
                          "tune_table_ms_per_step": b["table"],
                          "kernels_avg_us": {k: round(v["avg_us"], 2) for k, v in brows.items()}}
        if "fp64_plain" in out:
            out["batched"]["vs_fp64_plain"] = round(value / out["fp64_plain"]["value"], 3)
        if a.alone_steps:
            # the same 256 jobs through the plain single-simulation path
            alone = {}
            for name, prec in (("fp64", PREC_FP64), ("mixed", PREC_MIXED)):
                sec = run_one_at_a_time(batch, prec, a.alone_steps, 5, stream)
                alone[name] = {"value": round(b["n"] / sec, 1), "unit": "particle-steps/s",
                               "ms_per_step_all_jobs": round(sec * 1e3, 4)}
                log("alone %s: %.3f ms per step of all jobs" % (name, sec * 1e3))
            out["batched"]["same_jobs_one_at_a_time"] = dict(alone, steps=a.alone_steps)
            out["batched"]["vs_fp64_plain_same_jobs"] = round(value / alone["fp64"]["value"], 3)

    if not a.no_ablation:
        sizes = [int(v) for v in a.ablation_sizes.split(",") if v]
        out["ablation_fused_vs_split"] = {
            "what": "collide = contact search + force kernels per step, mixed precision; "
                    "fused = the single loop before the split of section 3.4; "
                    "thread_split = that split within each particle's thread; "
                    "action_reaction = each pair's force once, applied to both",
            "steps": a.ablation_steps, "warmup": 5,
            "rows": run_ablation(sizes, a.ablation_steps, 5, stream, log)}

    if serve_in is not None:
        futs, arr, steps, ex, t = serve_in
        scenes = [f.result() for f in futs]
        ex.shutdown()
        log("serving input: %d requests over %.0fs, %d spheres, ready %.1fs after the start" % (
            len(arr), float(arr[-1]) if len(arr) else 0.0, sum(sc.n for sc in scenes),
            time.perf_counter() - t))
        res = run_serving(scenes, arr, steps, stream, a.serve_budget, a.superstep, log,
                          at_once_too=a.serve_all_at_once)
        st = res[0]
        out["serving"] = {"rate_jobs_per_s": a.serve_rate,
                          "arrival_span_s": round(float(arr[-1]), 2) if len(arr) else 0.0,
                          "requests": int(len(arr)),
                          "particles_total": int(sum(sc.n for sc in scenes)),
                          "offered_particle_steps_per_s":
                              round(sum(sc.n * int(k) for sc, k in zip(scenes, steps)) /
                                    max(float(arr[-1]), 1e-9), 1) if len(arr) else 0.0,
                          "budget_particles": a.serve_budget,
                          "superstep": "adaptive, %d to start, about 50 ms each" % a.superstep,
                          "p50_latency_s": round(st["p50_s"], 4),
                          "p99_latency_s": round(st["p99_s"], 4),
                          "wait_p50_s": round(st["wait_p50_s"], 4),
                          "wait_p99_s": round(st["wait_p99_s"], 4),
                          "service_p50_s": round(st["service_p50_s"], 4),
                          "service_p99_s": round(st["service_p99_s"], 4),
                          "value": round(st["particle_steps_per_s"], 1),
                          "unit": "particle-steps/s", "makespan_s": round(st["makespan_s"], 3),
                          "failed": st["failed"]}
        if len(res) > 1:
            sat = res[1]
            out["serving"]["all_at_once"] = {"value": round(sat["particle_steps_per_s"], 1),
                                             "makespan_s": round(sat["makespan_s"], 3),
                                             "p50_latency_s": round(sat["p50_s"], 4),
                                             "p99_latency_s": round(sat["p99_s"], 4)}

    if not a.no_cpu:
        import gen
        out["cpu_baseline"] = cpu_baseline(sc, a.cpu_budget, gen.config_plain())


if __name__ == "__main__":
    main()
