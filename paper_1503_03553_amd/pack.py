"""Dense packings by growth on the GPU.

The paper's dense measurements start from particles "warmed up until dense"
(section 5.2); without gravity a dense pack is made by inflating the
particles of a looser random packing while the simulation runs, so that
overlaps push them apart as they grow.  This module drives that growth
through the library (dem_set_radii between steps); every step is the same
DEM step the simulator runs.  The result can be cached on disk, keyed by the
start's name, seed and the schedule, for a second use in the same run.
"""
from __future__ import annotations

import os

import numpy as np

from .binding import FLAG_NO_FORCE_OUTPUT, PREC_MIXED, Sim


def grow(start, increments=200, steps_per_increment=20, precision=PREC_MIXED, stream=None,
         log=None):
    """Inflate the particles of `start` (a scene whose meta holds r_full, the
    radii to reach) from its radii to r_full in `increments` equal steps of
    the radius scale, running `steps_per_increment` DEM steps after each.
    The grid is laid out for the full radii from the start.  Returns a dict
    with the grown state (x, v, w in pid order), the contact pairs (i, j)
    of the last step and the time step the growth ran at."""
    r_full = np.asarray(start.meta["r_full"], np.float64)
    r0 = np.asarray(start.r, np.float64)
    s0 = float(np.median(r0 / r_full))
    cell = 2.0 * float(r_full.max()) * (1.0 + 1e-5)
    sim = Sim.from_scene(start, precision=precision, stream=stream, cell_size=cell,
                         flags=FLAG_NO_FORCE_OUTPUT)
    try:
        for k in range(1, increments + 1):
            s = s0 + (1.0 - s0) * k / increments
            r = r_full if k == increments else np.minimum(r_full * s, r_full)
            sim.set_radii(r)
            sim.step(steps_per_increment)
            if log and (k % max(1, increments // 4) == 0):
                sim.sync()
                inf = sim.info()
                log("growth %d/%d: %.3f directed contacts per particle" % (
                    k, increments, inf["contacts"] / max(start.n, 1)))
        sim.sync()
        st = sim.get_state(forces=False)
        i, j, _ = sim.get_contacts()
        dt = sim.info()["dt"]
    finally:
        sim.close()
    return dict(x=st["x"], v=st["v"], w=st["w"], i=i, j=j, dt=dt)


def overlaps(scene, x, i, j):
    """Overlap r_i + r_j - |x_j - x_i| of particle contacts (i, j) (minimum
    image on the periodic axes; the shear offset is taken as zero, as at the
    end of a growth without shear)."""
    i = np.asarray(i, np.int64)
    j = np.asarray(j, np.int64)
    keep = j < 0xFFFFFFF0
    i, j = i[keep], j[keep]
    d = x[j] - x[i]
    L = np.asarray(scene.hi, np.float64) - np.asarray(scene.lo, np.float64)
    for a in range(3):
        if scene.periodic & (1 << a):
            d[:, a] -= L[a] * np.rint(d[:, a] / L[a])
    r = np.asarray(scene.meta.get("r_full", scene.r), np.float64)
    return i, r[i] + r[j] - np.linalg.norm(d, axis=1)


def grown(start, increments=200, steps_per_increment=20, precision=PREC_MIXED, stream=None,
          cache_dir=None, log=None):
    """grow() with an on-disk cache (cache_dir, else $DEM_PACK_CACHE, else
    none) and the pack's statistics: directed contacts per particle, the
    largest count of one particle, and the largest and median overlap over
    the radius of the particle."""
    cache_dir = cache_dir or os.environ.get("DEM_PACK_CACHE")
    key = "%s-s%d-%dx%d-p%d.npz" % (start.name, int(start.meta.get("seed", 0)), increments,
                                    steps_per_increment, precision)
    path = os.path.join(cache_dir, key) if cache_dir else None
    if path and os.path.exists(path):
        z = np.load(path)
        g = {k: z[k] for k in z.files}
        g["dt"] = float(g["dt"])
    else:
        g = grow(start, increments, steps_per_increment, precision, stream, log)
        if path:
            os.makedirs(cache_dir, exist_ok=True)
            np.savez(path + ".tmp.npz", **g)
            os.replace(path + ".tmp.npz", path)
    n = start.n
    ii, dn = overlaps(start, g["x"], g["i"], g["j"])
    rr = np.asarray(start.meta["r_full"], np.float64)[ii]
    per = np.bincount(np.asarray(g["i"], np.int64), minlength=n) if n else np.zeros(0)
    g["stats"] = {"contacts_per_particle": float(len(g["i"]) / max(n, 1)),
                  "max_contacts_of_a_particle": int(per.max()) if n else 0,
                  "max_overlap_over_r": float((dn / rr).max()) if dn.size else 0.0,
                  "median_overlap_over_r": float(np.median(dn / rr)) if dn.size else 0.0,
                  "increments": increments, "steps_per_increment": steps_per_increment}
    return g


def grow_pool(starts, increments=200, steps_per_increment=20, precision=PREC_MIXED,
              stream=None):
    """grow() for many jobs at once: the starts run as the jobs of one pool,
    each inflated to its own r_full in `increments` equal steps of its radius
    scale with `steps_per_increment` steps after each increment.  Returns,
    per start, the grown state (x, v, w in pid order)."""
    from .binding import Pool, job_cells
    if not starts:
        return []
    cells_of = [2.0 * float(np.max(sc.meta["r_full"])) * (1.0 + 1e-5) for sc in starts]
    parts = sum(((sc.n + 127) // 128) * 128 for sc in starts)
    ncell = sum(job_cells(sc, c) for sc, c in zip(starts, cells_of))
    total = increments * steps_per_increment
    pool = Pool(max_particles=max(parts, 128), max_cells=max(ncell, 1), max_jobs=len(starts),
                precision=precision, stream=stream, flags=FLAG_NO_FORCE_OUTPUT)
    try:
        ids = [pool.add_scene(sc, steps=total + 1, cell_size=c) for sc, c in zip(starts, cells_of)]
        s0 = [float(np.median(np.asarray(sc.r) / np.asarray(sc.meta["r_full"]))) for sc in starts]
        for k in range(1, increments + 1):
            for jid, sc, s in zip(ids, starts, s0):
                rf = np.asarray(sc.meta["r_full"], np.float64)
                r = rf if k == increments else np.minimum(rf * (s + (1.0 - s) * k / increments), rf)
                pool.set_radii(jid, r)
            pool.step(steps_per_increment)
        pool.sync()
        return [pool.get_state(jid) for jid in ids]
    finally:
        pool.close()
