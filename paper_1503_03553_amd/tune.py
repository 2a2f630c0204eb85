"""Autotuner of the batched form: picks the cell size factor and the tile
schedule (the order in which jobs are laid out in the pool) by timing a
few steps of the real workload for each candidate.

Neither choice changes any result: a job's trajectory is bitwise the same for
every admissible cell size and wherever it sits in the pool, so the tuner
only trades time.  Host policy only; every step runs in the HIP library.
"""
from __future__ import annotations

import time

import numpy as np

ORDERS = ("given", "size_desc", "density_desc")


def job_order(scenes, order):
    """Indices of `scenes` in the layout order named by `order`."""
    idx = list(range(len(scenes)))
    if order == "given":
        return idx
    if order == "size_desc":
        return sorted(idx, key=lambda k: -scenes[k].n)
    if order == "density_desc":
        def phi(sc):
            vol = float(np.prod(np.asarray(sc.hi) - np.asarray(sc.lo)))
            return float(np.sum(4.0 / 3.0 * np.pi * np.asarray(sc.r, np.float64) ** 3)) / vol
        return sorted(idx, key=lambda k: -phi(scenes[k]))
    raise ValueError(order)


def cell_size_for(sc, factor):
    """Cell size `factor` times the job's largest contact distance (0 = the
    library default, which is factor 1)."""
    if factor == 1.0 or len(sc.r) == 0:
        return 0.0
    return float(factor * 2.0 * float(np.max(np.asarray(sc.r, np.float32))))


def candidates(factors=(1.0, 1.25, 1.5), orders=ORDERS):
    return [dict(cell_factor=f, order=o) for f in factors for o in orders]


def fill_pool(pool, scenes, steps, cand, add_kw=None):
    """Add every scene (in the candidate's order, with its cell size) and
    return the job ids in the order of `scenes`."""
    ids = [None] * len(scenes)
    for k in job_order(scenes, cand["order"]):
        kw = dict(add_kw or {})
        kw["cell_size"] = cell_size_for(scenes[k], cand["cell_factor"])
        ids[k] = pool.add_scene(scenes[k], steps=steps, **kw)
    return ids


def autotune(make_pool, scenes, cands=None, steps=10, warmup=3, clock=time.perf_counter,
             log=None):
    """Time `steps` steps (after `warmup`) of the whole workload for every
    candidate; returns (best candidate, [(candidate, seconds per step)])."""
    cands = cands or candidates()
    table = []
    for c in cands:
        pool = make_pool(c)
        try:
            fill_pool(pool, scenes, warmup + steps + 1, c)
            pool.step(warmup)
            pool.sync()
            t0 = clock()
            pool.step(steps)
            pool.sync()
            sec = (clock() - t0) / steps
        finally:
            pool.close()
        table.append((c, sec))
        if log:
            log("tune %s: %.3f ms/step" % (c, sec * 1e3))
    best = min(table, key=lambda t: t[1])[0]
    return best, table
