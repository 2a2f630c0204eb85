"""The two contact searches: the default one, which tests each pair once
(each particle scans the upper half of its cell stencil) and enters each
contact in both particles' rows, and the full per-particle search of
Algorithm 1 (DEM_FLAG_FULL_DETECT).

The contact test is symmetric in the two particles, so both searches give the
same rows bit for bit at every step (partner order included), and with them
every later result: states, forces and history are bitwise equal.  The other
GPU tests run the default search against the oracle; here the full search
meets the same single-step and trajectory tolerances, and the two are
compared with each other along churning runs, in pools, with walls and when a
row outgrows its buffer.
"""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import SCENES, random_history, say, step_parity, trajectory_parity
from paper_1503_03553_amd import FLAG_FULL_DETECT, PREC_FP64, PREC_MIXED, Pool, Sim
from test_gpu_walls import wall_scene

pytestmark = pytest.mark.gpu

PRECS = [("fp64", PREC_FP64), ("mixed", PREC_MIXED)]


@pytest.mark.parametrize("prec_name,prec", PRECS)
@pytest.mark.parametrize("name", ["cluster64", "random3000", "periodic1500", "shear1500",
                                  "mixedwall", "materials"])
def test_full_detect_one_step_parity(name, prec_name, prec):
    say("case full one_step", name, prec_name)
    sc = SCENES[name]()
    tol = 1e-9 if prec == PREC_FP64 else 1e-5
    _, _, _, rep = step_parity(sc, prec, history=random_history(sc, seed=5), tol=tol, flags=FLAG_FULL_DETECT)
    assert rep["contacts"] > 0


@pytest.mark.parametrize("name", ["random3000", "shear1500"])
def test_full_detect_trajectory_100_steps(name):
    say("case full trajectory", name)
    trajectory_parity(SCENES[name](), PREC_MIXED, steps=100, tol=1e-4, flags=FLAG_FULL_DETECT)


def _same_runs(sc, steps, prec=PREC_MIXED, min_changed=1):
    dt = oracle.Sim(sc, mode=1).dt
    gs = [Sim.from_scene(sc, precision=prec, dt=dt, flags=f) for f in (0, FLAG_FULL_DETECT)]
    try:
        changed, prev = 0, None
        for step in range(steps):
            for g in gs:
                g.step(1)
            a, b = gs[0].get_contacts(), gs[1].get_contacts()
            for k in range(3):
                assert np.array_equal(a[k], b[k]), "step %d" % step
            key = set(zip(a[0].tolist(), a[1].tolist()))
            if prev is not None:
                changed += len(key ^ prev)
            prev = key
        assert changed >= min_changed
        sa, sb = gs[0].get_state(), gs[1].get_state()
        for k in ("x", "v", "w", "F", "T"):
            assert np.array_equal(sa[k], sb[k]), k
        return [g.info() for g in gs]
    finally:
        for g in gs:
            g.close()


@pytest.mark.parametrize("name", ["random3000", "shear1500", "periodic1500", "materials"])
def test_half_and_full_detect_agree_every_step(name):
    # contacts made and broken along the run; rows and every state bit equal
    say("case half vs full", name)
    sc = SCENES[name]()
    sc.v *= 20.0
    _same_runs(sc, 30)


def test_half_and_full_detect_agree_with_walls():
    say("case half vs full walls")
    _same_runs(wall_scene(37), 20, prec=PREC_FP64, min_changed=0)


def test_half_detect_row_overflow_regrows():
    # a big sphere touched by more spheres than the first row buffer holds:
    # the step is redone with longer rows (and longer adjacency lists), and
    # matches the oracle and the full search
    say("case half row overflow")
    rng = np.random.default_rng(3)
    R, r = 8e-6, 2e-6
    c = np.array([50e-6] * 3)
    dirs = rng.normal(size=(60, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    keep = [0]
    for k in range(1, 60):
        if all(np.dot(dirs[k], dirs[q]) < np.cos(0.5) for q in keep):
            keep.append(k)
    dirs = dirs[keep]
    x = np.vstack([c, c + dirs * (R + r - 1e-9)])
    n = x.shape[0]
    assert n - 1 > 16
    sc = gen.Scene(lo=np.zeros(3), hi=np.full(3, 100e-6), x=x, v=np.zeros((n, 3)),
                   w=np.zeros((n, 3)), r=gen.f32([R] + [r] * (n - 1)), mat=np.zeros(n, np.uint16),
                   materials=[gen.Material.make()], walls=gen.WALL_ALL, gravity=(0, 0, 0))
    _, _, _, rep = step_parity(sc, PREC_FP64, tol=1e-9)
    assert rep["contacts"] >= 2 * (n - 1)
    infos = _same_runs(sc, 3, prec=PREC_FP64, min_changed=0)
    assert infos[0]["contacts"] == infos[1]["contacts"]


def test_half_detect_pool_jobs_equal_full_detect_pool():
    say("case half pool")
    scs = [gen.scene_random(seed=421, n=700, phi=0.22, p_touch=0.7, vel_sigma=0.2),
           gen.scene_random(seed=422, n=129, phi=0.2, p_touch=0.8, vel_sigma=0.3),
           gen.scene_random(seed=423, n=600, phi=0.22, p_touch=0.7, walls=0, periodic=7,
                            gravity=(0, 0, 0), shear_rate=2000.0),
           gen.scene_random(seed=424, n=500, phi=0.22, p_touch=0.7, n_materials=3)]
    dts = [oracle.Sim(s, mode=1).dt for s in scs]
    steps = [30, 12, 30, 21]
    states = []
    for flags in (0, FLAG_FULL_DETECT):
        pool = Pool(max_particles=sum(s.n for s in scs) + 128 * len(scs),
                    max_cells=sum(max(4 * s.n, 4096) for s in scs), max_jobs=len(scs),
                    precision=PREC_MIXED, flags=flags)
        try:
            ids = [pool.add_scene(s, steps=k, dt=dt) for s, k, dt in zip(scs, steps, dts)]
            pool.step(32)
            pool.sync()
            states.append([pool.get_state(j) for j in ids])
        finally:
            pool.close()
    for a, b in zip(*states):
        for k in ("x", "v", "w"):
            assert np.array_equal(a[k], b[k]), k


def test_full_detect_flag_with_variants_changes_nothing():
    # the force-path variants always run the full search: adding the flag
    # gives bitwise the same run
    from paper_1503_03553_amd import FLAG_ACTION_REACTION, FLAG_FUSED
    say("case full flag with variants")
    sc = SCENES["random3000"]()
    dt = oracle.Sim(sc, mode=1).dt
    for v in (FLAG_FUSED, FLAG_ACTION_REACTION):
        states = []
        for flags in (v, v | FLAG_FULL_DETECT):
            g = Sim.from_scene(sc, precision=PREC_MIXED, dt=dt, flags=flags)
            g.step(10)
            states.append(g.get_state())
            g.close()
        for k in ("x", "v", "w", "F", "T"):
            assert np.array_equal(states[0][k], states[1][k]), (v, k)


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_half_and_full_detect_agree_on_small_periodic_grids(k):
    # sheared periodic boxes of k cells per axis: at 5 cells and more the
    # waves away from every periodic boundary take the plain filter and
    # exact test of the half search, below that every wave shifts images
    say("case half vs full periodic grid", k)
    sc = gen.scene_random(seed=431, n=1000, phi=0.22, p_touch=0.8, walls=0, periodic=7,
                          gravity=(0, 0, 0), shear_rate=5000.0)
    sc.v *= 10.0
    L = float(sc.hi[0] - sc.lo[0])
    cell = L / (k + 0.5)
    assert cell >= 2.0 * float(np.max(sc.r))
    dt = oracle.Sim(sc, mode=1).dt
    gs = [Sim.from_scene(sc, precision=PREC_FP64, dt=dt, cell_size=cell, flags=f)
          for f in (0, FLAG_FULL_DETECT)]
    try:
        assert tuple(gs[0].info()["cells"]) == (k, k, k)
        for step in range(20):
            for g in gs:
                g.step(1)
            a, b = gs[0].get_contacts(), gs[1].get_contacts()
            for q in range(3):
                assert np.array_equal(a[q], b[q]), "step %d" % step
        sa, sb = gs[0].get_state(), gs[1].get_state()
        for key in ("x", "v", "w", "F", "T"):
            assert np.array_equal(sa[key], sb[key]), key
        assert a[0].size > 0
    finally:
        for g in gs:
            g.close()
