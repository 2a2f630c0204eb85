"""Shared helpers of the GPU parity tests: run the HIP library and the oracle
on the same seeded scene and compare them to the tolerances of the contract.

Tolerances (relative, per step): forces and torques 1e-5 of the natural
scale (sum of |F_ij| over a particle's contacts plus |m g|; in mixed
precision the sum over its contacts of the magnitudes of the four terms of
Eq. (1), elastic and damping normal, spring and damping tangential, plus
|m g|), tangential displacement 1e-5 of the larger of its magnitude and the
contact's overlap (in mixed precision, for a contact on the sliding cap, also
of that rounding scale over k_t: Eq. (4) resets the displacement from the
capped FP32 force), contact sets bit-exact; trajectories 1e-4 of the largest
displacement after 100 steps.  In mixed precision the contacts that sit on
the sliding cap within an FP32 rounding bound (cap ties) and their owners
are counted instead of held to the tolerance.
"""
import sys

import numpy as np

import gen
import oracle
from paper_1503_03553_amd import PREC_FP64, PREC_MIXED, Sim

FACE = 0xFFFFFFF0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_pair(scene, precision, dt=None, **kw):
    """GPU sim and oracle sim of one scene with the oracle's time step."""
    o = oracle.Sim(scene, dt=dt, mode=1)
    g = Sim.from_scene(scene, precision=precision, dt=o.dt, **kw)
    return g, o


def contact_key(i, j):
    return (np.asarray(i, np.uint64) << np.uint64(32)) | np.asarray(j, np.uint64)


def compare_contacts(g_i, g_j, o_i, o_j):
    a = contact_key(g_i, g_j)
    b = contact_key(o_i, o_j)
    assert a.shape == b.shape, "contact count %d (gpu) vs %d (oracle)" % (a.size, b.size)
    assert np.array_equal(a, b), "contact sets differ"


def natural_force_scale(o, scene, terms=False):
    """Per particle: sum_j |F_ij| + |m_i g|, and sum_j r_i |F_ij| (the lever
    arm times the force: a torque of a nearly head-on contact is a small
    difference of products of that size).  With `terms`, |F_ij| is replaced
    by the sum of the magnitudes of the terms of Eq. (1) (the oracle's
    rounding scale of the force): an FP32 evaluation errs by a few rounding
    units of those, and where the elastic and the damping normal force of a
    separating contact nearly cancel, |F_ij| is thousands of times smaller."""
    n = scene.n
    sF = np.zeros(n)
    sT = np.zeros(n)
    if o.cF is not None and len(o.hist):
        ii = o.hist.i.astype(np.int64)
        f = o.cQ[:, 3] if terms else np.linalg.norm(o.cF, axis=1)
        np.add.at(sF, ii, f)
        np.add.at(sT, ii, scene.r[ii] * f)
    dens = np.array([scene.materials[k].density for k in scene.mat])
    m = dens * 4.0 / 3.0 * np.pi * scene.r ** 3
    sF = sF + m * np.linalg.norm(np.asarray(scene.gravity))
    return sF, sT


def contact_overlaps(scene, x, i, j, time):
    """Overlap of each contact (i, j) at positions x: the natural length of
    its tangential displacement (the tangential spring force over the normal
    force scales as their ratio).  Minimum image on periodic axes, with the
    shear offset across y."""
    i = np.asarray(i, np.int64)
    j = np.asarray(j, np.int64)
    r = np.asarray(scene.r, np.float64)
    out = np.zeros(i.size)
    face = j >= FACE
    pi = i[~face]
    pj = j[~face]
    d = x[pj] - x[pi]
    L = np.asarray(scene.hi, float) - np.asarray(scene.lo, float)
    per = int(scene.periodic)
    if per & 2:
        ky = -np.rint(d[:, 1] / L[1])
        d[:, 1] += ky * L[1]
        if scene.shear_rate:
            shift = np.fmod(scene.shear_rate * L[1] * time, L[0])
            d[:, 0] += ky * shift
    if per & 1:
        d[:, 0] -= L[0] * np.rint(d[:, 0] / L[0])
    if per & 4:
        d[:, 2] -= L[2] * np.rint(d[:, 2] / L[2])
    out[~face] = r[pi] + r[pj] - np.linalg.norm(d, axis=1)
    f = (j[face] - FACE).astype(np.int64)
    fi = i[face]
    box = f < 6
    ax = np.where(box, f // 2, 0)
    p = x[fi, ax]
    lo = np.asarray(scene.lo, float)[ax]
    hi = np.asarray(scene.hi, float)[ax]
    ov = r[fi] - np.where(f % 2 == 1, hi - p, p - lo)
    # extra walls: distance to the closest point of the rectangle or segment
    for k in np.nonzero(~box)[0]:
        wl = scene.extra_walls[f[k] - 6]
        c = x[fi[k]]
        pw, u, v = (np.asarray(a, float) for a in (wl.p, wl.u, wl.v))
        q = pw + np.clip(np.dot(c - pw, u) / np.dot(u, u), 0, 1) * u
        if wl.kind == 0:
            q = q + np.clip(np.dot(c - pw, v) / np.dot(v, v), 0, 1) * v
        ov[k] = r[fi[k]] - np.linalg.norm(q - c)
    out[face] = ov
    return out


# A contact whose sliding test the oracle decides by less than this many
# units of the magnitudes of the terms that enter it (k_t |dt|, eta |v|,
# mu |F_n|, ...) can go either way when those terms are rounded to FP32
# (2^-18 = 64 FP32 rounding units): such a "cap tie" may switch between
# the capped and the uncapped branch of Eq. (4).  The force stays
# continuous there, but the displacement jumps by eta v_t / k_t (the
# paper's reset folds the damping in), so in mixed precision those contacts'
# displacements and their owners' totals are reported, not held to the
# tolerance.  Every other contact and particle is.
CAP_BAND = 2.0 ** -18


def cap_ties(o):
    """Mask of the oracle's contacts (o.hist order) that are cap ties."""
    q = o.cQ
    return np.abs(q[:, 0] - q[:, 1]) <= CAP_BAND * q[:, 2]


def _stats(rel):
    rel = np.asarray(rel, float)
    if rel.size == 0:
        return (0.0, 0.0)
    return (float(rel.max()), float(np.median(rel)))


def check_step(o, scene, st, ci, cj, cdt, tol, ties=False, x0=None, time=0.0):
    """Compare one GPU step (new state `st` with F, T; contacts ci, cj, cdt)
    with the oracle `o` that took the same step with keep_contact_forces.
    Tangential displacements are compared against the larger of their own
    magnitude and the contact's overlap at the start of the step (positions
    x0, default the scene's).  With `ties` (mixed precision) the cap ties and
    the particles that own them are exempt from the tolerance and counted.
    Returns the counts and the (max, median) relative errors."""
    compare_contacts(ci, cj, o.hist.i, o.hist.j)
    # tangential displacement per contact
    ref = o.hist.dt
    err = np.linalg.norm(cdt - ref, axis=1)
    scale = np.linalg.norm(ref, axis=1)
    dn = contact_overlaps(scene, scene.x if x0 is None else x0, o.hist.i, o.hist.j, time)
    floor = np.maximum(dn, 1e-9 * (scale.max() if scale.size else 0.0)) + 1e-300
    if ties:
        # a capped contact's displacement is reset from the FP32 capped force:
        # its rounding is that of the force terms, over k_t
        capped = o.cQ[:, 0] > o.cQ[:, 1]
        floor = np.where(capped, np.maximum(floor, o.cQ[:, 3] / np.maximum(o.cQ[:, 4], 1e-300)),
                         floor)
    rel_dt = err / np.maximum(scale, floor)
    tie = cap_ties(o) if ties else np.zeros(len(ref), bool)
    bad = (rel_dt > tol) & ~tie
    assert not bad.any(), "%d of %d tangential displacements off (max rel %.3g)" % (
        int(bad.sum()), len(ref), float(rel_dt[~tie].max()))
    # per-particle force and torque (in mixed precision against the rounding
    # scale of the FP32 force arithmetic; the largest error against the net
    # contact forces is reported beside it)
    sF, sT = natural_force_scale(o, scene, terms=ties)
    sFn, _ = natural_force_scale(o, scene)
    relF = np.linalg.norm(st["F"] - o.F, axis=1) / np.maximum(sF, 1e-300)
    relT = np.linalg.norm(st["T"] - o.T, axis=1) / np.maximum(sT, 1e-300)
    relT[sT == 0] = np.where(np.linalg.norm(st["T"][sT == 0], axis=1) == 0, 0.0, np.inf)
    owner = np.zeros(scene.n, bool)
    owner[o.hist.i[tie].astype(np.int64)] = True
    badF = (relF > tol) & ~owner
    badT = (relT > tol) & ~owner
    assert not badF.any(), "force off: max rel %.3g" % float(relF[~owner].max())
    assert not badT.any(), "torque off: max rel %.3g" % float(relT[~owner].max())
    return dict(contacts=len(ref), cap_ties=int(tie.sum()),
                tie_dt_off=int(((rel_dt > tol) & tie).sum()),
                tie_owners=int(owner.sum()),
                tie_owners_off=int((((relF > tol) | (relT > tol)) & owner).sum()),
                err_dt=_stats(rel_dt[~tie]), err_F=_stats(relF[~owner]),
                err_T=_stats(relT[~owner]),
                err_F_net=_stats((np.linalg.norm(st["F"] - o.F, axis=1) /
                                  np.maximum(sFn, 1e-300))[~owner]))


def step_parity(scene, precision, history=None, tol=1e-5, dt=None, ties=None, **kw):
    """One step from identical state and history; compares contact set,
    tangential displacements, per-particle F and T and the new state.  Cap
    ties are exempt in mixed precision only (ties=None)."""
    if ties is None:
        ties = precision == PREC_MIXED
    g, o = make_pair(scene, precision, dt=dt, **kw)
    try:
        if history is not None:
            hi, hj, hdt = history
            g.set_contacts(hi, hj, hdt)
            o.hist = oracle.History(hi, hj, hdt)
            order = np.lexsort((o.hist.j, o.hist.i))
            o.hist = oracle.History(o.hist.i[order], o.hist.j[order], o.hist.dt[order])
        g.step(1)
        st = g.get_state()
        ci, cj, cdt = g.get_contacts()
        o.step(keep_contact_forces=True)
        rep = check_step(o, scene, st, ci, cj, cdt, tol, ties, x0=scene.x, time=0.0)
        return g, o, st, rep
    finally:
        g.close()


def trajectory_parity(scene, precision, steps=100, tol=1e-4, dt=None, chunk=None, **kw):
    g, o = make_pair(scene, precision, dt=dt, **kw)
    try:
        x0, v0, w0 = scene.x.copy(), scene.v.copy(), scene.w.copy()
        if chunk:
            k = 0
            while k < steps:
                c = min(chunk, steps - k)
                g.step(c)
                k += c
        else:
            g.step(steps)
        st = g.get_state(forces=False)
        o.step(steps)
        out = {}
        for name, gv, ov, base in (("x", st["x"], o.x, x0), ("v", st["v"], o.v, v0),
                                    ("w", st["w"], o.w, w0)):
            d_ref = ov - base
            if name == "x" and scene.periodic:
                # compare displacements modulo the box
                L = scene.hi - scene.lo
                d_ref = d_ref - L * np.round(d_ref / L)
                diff = gv - ov
                diff = diff - L * np.round(diff / L)
            else:
                diff = gv - ov
            scale = np.linalg.norm(d_ref, axis=1).max()
            e = np.linalg.norm(diff, axis=1)
            err = e.max()
            out[name] = (err, scale)
            # per particle, relative to the largest change: (max, median)
            out[name + "_rel"] = _stats(e / max(scale, 1e-300))
            assert err <= tol * scale + 1e-300, "%s: max err %.3g vs scale %.3g" % (name, err, scale)
        return out
    finally:
        g.close()


def random_history(scene, seed, frac=0.8, scale=None):
    """A plausible tangential history for most current contacts (and a few
    stale pairs that no longer touch, which must be dropped)."""
    i, j = oracle.contacts(scene, mode=1)
    rng = np.random.default_rng(seed)
    keep = rng.random(i.size) < frac
    i, j = i[keep], j[keep]
    if scale is None:
        scale = 1e-3 * float(np.median(scene.r))
    dt = rng.normal(0, scale, size=(i.size, 3))
    # antisymmetric for particle pairs, as a real history is
    idx = {(a, b): k for k, (a, b) in enumerate(zip(i.tolist(), j.tolist()))}
    for (a, b), k in idx.items():
        if b < FACE and (b, a) in idx and a > b:
            dt[k] = -dt[idx[(b, a)]]
    # stale entries
    n = scene.n
    si = rng.integers(0, n, 10).astype(np.uint32)
    sj = ((si + 7) % n).astype(np.uint32)
    pairs = set(zip(i.tolist(), j.tolist()))
    extra = [(a, b) for a, b in zip(si.tolist(), sj.tolist()) if a != b and (a, b) not in pairs]
    extra = list(dict.fromkeys(extra))
    if extra:
        ei = np.array([a for a, _ in extra], np.uint32)
        ej = np.array([b for _, b in extra], np.uint32)
        i = np.concatenate([i, ei])
        j = np.concatenate([j, ej])
        dt = np.concatenate([dt, rng.normal(0, scale, size=(len(extra), 3))])
    return i.astype(np.uint32), j.astype(np.uint32), dt


SCENES = {
    "cluster64": lambda: gen.scene_cluster(seed=1, n_side=4, vel_sigma=0.2, polydisperse=True),
    "random3000": lambda: gen.scene_random(seed=21, n=3000, phi=0.22, p_touch=0.7, vel_sigma=0.2),
    "periodic1500": lambda: gen.scene_random(seed=22, n=1500, phi=0.22, p_touch=0.7, walls=0,
                                             periodic=7, gravity=(0, 0, 0)),
    "shear1500": lambda: gen.scene_random(seed=23, n=1500, phi=0.22, p_touch=0.7, walls=0,
                                          periodic=7, gravity=(0, 0, 0), shear_rate=2000.0),
    "mixedwall": lambda: gen.scene_random(seed=24, n=1200, phi=0.22, p_touch=0.7,
                                          walls=gen.WALL_ALL & ~3, periodic=1),
    "materials": lambda: gen.scene_random(seed=25, n=1000, phi=0.22, p_touch=0.7, n_materials=3),
}


def symmetric_history(sc, seed):
    """random_history with both directions of every particle pair present:
    the lower id's entry is kept and the other direction carries its
    negative, as in a history the method itself builds."""
    i, j, dt = random_history(sc, seed)
    part = j < FACE
    own = part & (i < j)
    keep_i = np.concatenate([i[~part], i[own], j[own]])
    keep_j = np.concatenate([j[~part], j[own], i[own]])
    keep_dt = np.concatenate([dt[~part], dt[own], -dt[own]])
    return keep_i.astype(np.uint32), keep_j.astype(np.uint32), keep_dt
