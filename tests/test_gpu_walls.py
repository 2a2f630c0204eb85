"""GPU parity with extra static walls (closed rectangles and segments, the
"CollideRectangle" / "CollideLine" walls of the paper's kernel list) against
the FP64 oracle: the contact set (wall ids included) bit for bit, forces and
history within the single-step tolerances, trajectories within 1e-4 after
100 steps; a pool job with walls equals the same job alone; malformed walls
are rejected.
"""
import math

import numpy as np
import pytest

import gen
import oracle
from gpu_util import (FACE, random_history, say, step_parity, symmetric_history,
                      trajectory_parity)
from paper_1503_03553_amd import FLAG_FUSED, PREC_FP64, PREC_MIXED, DemError, Pool, Sim

pytestmark = pytest.mark.gpu

PRECS = [("fp64", PREC_FP64), ("mixed", PREC_MIXED)]


def _rotation(axis, angle):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * K @ K


def wall_scene(seed, n_free=1200):
    """A 150 um box with a tilted plate through its centre, a rod across it
    and a small plate near the floor; spheres resting on both sides of the
    tilted plate and along the rod at 0.99 r, plus free spheres that touch
    neither a wall nor a placed sphere."""
    rng = np.random.default_rng(seed)
    L, r = 150e-6, 5e-6
    C = np.full(3, L / 2)
    R = _rotation((1.0, 2.0, 3.0), 0.6)
    u, v = R @ np.array([80e-6, 0, 0]), R @ np.array([0, 60e-6, 0])
    p = C - (u + v) / 2
    nrm = R @ np.array([0.0, 0.0, 1.0])
    rod_p, rod_u = np.array([10e-6, 20e-6, 30e-6]), np.array([130e-6, 110e-6, 20e-6])
    walls = [gen.Wall(gen.RECT, tuple(p), tuple(u), tuple(v)),
             gen.Wall(gen.SEGMENT, tuple(rod_p), tuple(rod_u)),
             gen.Wall(gen.RECT, (40e-6, 40e-6, 12e-6), (60e-6, 0.0, 0.0), (0.0, 50e-6, 0.0))]
    placed = []
    for i in range(6):
        for j in range(5):
            for side in (1.0, -1.0):
                placed.append(p + (i + 0.5) / 6 * u + (j + 0.5) / 5 * v + side * 0.99 * r * nrm)
    rod_dir = rod_u / np.linalg.norm(rod_u)
    perp = np.cross(rod_dir, [0.0, 0.0, 1.0])
    perp /= np.linalg.norm(perp)
    for k in range(8):
        placed.append(rod_p + (k + 0.5) / 8 * rod_u + 0.99 * r * perp)
    placed = np.array(placed)
    free = gen.rsa(gen.f32(np.full(n_free, r)), np.zeros(3), np.full(3, L), seed=seed)
    x = np.vstack([placed, free])
    n = x.shape[0]
    vel = 0.05 * rng.standard_normal((n, 3))
    vel[:len(placed)] = 0.0  # resting on their wall
    sc = gen.Scene(lo=np.zeros(3), hi=np.full(3, L), x=x, v=vel,
                   w=np.zeros((n, 3)), r=gen.f32(np.full(n, r)), mat=np.zeros(n, np.uint16),
                   materials=[gen.Material.make(restitution=0.5, mu=0.3)], walls=gen.WALL_ALL,
                   extra_walls=walls)
    # drop free spheres that touch a wall or a placed sphere (placed ones all
    # touch their wall only)
    ci, cj = oracle.contacts(sc, mode=1)
    bad = set()
    for a, b in zip(ci.tolist(), cj.tolist()):
        if a >= len(placed) and (b >= FACE + 6 or (b < FACE and b < len(placed))):
            bad.add(a)
    keep = np.array([k for k in range(n) if k not in bad])
    sc.x, sc.v, sc.w = sc.x[keep], sc.v[keep], sc.w[keep]
    sc.r, sc.mat = sc.r[keep], sc.mat[keep]
    return sc


def wall_contacts(sc):
    i, j = oracle.contacts(sc, mode=1)
    return int(np.sum(j >= FACE + 6))


@pytest.mark.parametrize("prec_name,prec", PRECS)
def test_walls_one_step_parity(prec_name, prec):
    say("case walls one_step", prec_name)
    sc = wall_scene(31)
    assert wall_contacts(sc) >= 60
    hist = random_history(sc, seed=6)
    tol = 1e-9 if prec == PREC_FP64 else 1e-5
    _, _, _, rep = step_parity(sc, prec, history=hist, tol=tol)
    say("  contacts", rep["contacts"])


@pytest.mark.parametrize("prec_name,prec", PRECS)
def test_walls_trajectory_100_steps(prec_name, prec):
    say("case walls trajectory", prec_name)
    out = trajectory_parity(wall_scene(32), prec, steps=100, tol=1e-4)
    say("  ", out)


def test_walls_fused_one_step_parity():
    say("case walls fused")
    sc = wall_scene(33)
    hist = random_history(sc, seed=7)
    step_parity(sc, PREC_FP64, history=hist, tol=1e-9, flags=FLAG_FUSED)


def test_walls_pool_job_equals_job_alone():
    say("case walls pool")
    a, b = wall_scene(34, n_free=600), gen.scene_random(seed=35, n=700, phi=0.2, p_touch=0.7)
    dts = [oracle.Sim(s, mode=1).dt for s in (a, b)]
    pool = Pool(max_particles=a.n + b.n + 256, max_cells=max(4 * a.n, 4096) + max(4 * b.n, 4096),
                max_jobs=2, precision=PREC_MIXED)
    try:
        jb = pool.add_scene(b, steps=20, dt=dts[1])
        ja = pool.add_scene(a, steps=20, dt=dts[0])
        pool.step(20)
        pool.sync()
        for s, j, dt in ((a, ja, dts[0]), (b, jb, dts[1])):
            g = Sim.from_scene(s, precision=PREC_MIXED, dt=dt)
            g.step(20)
            ref = g.get_state()
            g.close()
            got = pool.get_state(j)
            for k in ("x", "v", "w"):
                assert np.array_equal(got[k], ref[k]), k
    finally:
        pool.close()


def test_malformed_walls_are_rejected():
    base = gen.scene_cluster(seed=1, n_side=2)
    good = gen.Wall(gen.RECT, (0.0, 0.0, 1e-6), (1e-5, 0.0, 0.0), (0.0, 1e-5, 0.0))
    cases = [
        [gen.Wall(gen.RECT, (0.0, 0.0, 1e-6), (1e-5, 0.0, 0.0), (1e-6, 1e-5, 0.0))],  # not orthogonal
        [gen.Wall(gen.SEGMENT, (0.0, 0.0, 1e-6), (0.0, 0.0, 0.0))],                    # zero length
        [gen.Wall(7, (0.0, 0.0, 1e-6), (1e-5, 0.0, 0.0), (0.0, 1e-5, 0.0))],           # unknown kind
        [gen.Wall(gen.RECT, (np.nan, 0.0, 1e-6), (1e-5, 0.0, 0.0), (0.0, 1e-5, 0.0))],
        [good] * 11,                                                                   # too many
    ]
    for walls in cases:
        sc = base.copy()
        sc.extra_walls = walls
        with pytest.raises(DemError):
            Sim.from_scene(sc, precision=PREC_MIXED)
    sc = base.copy()
    sc.extra_walls = [good] * 10
    Sim.from_scene(sc, precision=PREC_MIXED).close()


def test_walls_action_reaction_one_step_parity():
    say("case walls action-reaction")
    from paper_1503_03553_amd import FLAG_ACTION_REACTION
    sc = wall_scene(36)
    step_parity(sc, PREC_FP64, history=symmetric_history(sc, seed=8), tol=1e-9,
                flags=FLAG_ACTION_REACTION)
