"""GPU parity of the action-reaction variant (each particle pair's force
computed once by the particle with the lower id and applied with opposite
signs to both), the scheme section 3.3 avoids.

Against the FP64 oracle (which computes every directed contact) it meets the
single-step and trajectory tolerances of the split path: in exact arithmetic
F_ji = -F_ij, since the relative velocity, the normal and a pair's
tangential history all change sign with the direction.  Its contact set is
the split path's bit for bit; a job in a pool gives bitwise the results of
the same scene run alone with the variant.
"""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import SCENES, say, step_parity, symmetric_history, trajectory_parity
from paper_1503_03553_amd import (FLAG_ACTION_REACTION, FLAG_FUSED, PREC_FP64, PREC_MIXED,
                                  DemError, Pool, Sim)

pytestmark = pytest.mark.gpu

PRECS = [("fp64", PREC_FP64), ("mixed", PREC_MIXED)]


@pytest.mark.parametrize("prec_name,prec", PRECS)
@pytest.mark.parametrize("name", ["cluster64", "random3000", "shear1500", "mixedwall",
                                  "materials"])
def test_action_reaction_one_step_parity(name, prec_name, prec):
    say("case action-reaction one_step", name, prec_name)
    sc = SCENES[name]()
    hist = symmetric_history(sc, seed=5)
    tol = 1e-9 if prec == PREC_FP64 else 1e-5
    _, _, _, rep = step_parity(sc, prec, history=hist, tol=tol,
                               flags=FLAG_ACTION_REACTION)
    say("  ", rep)
    assert rep["contacts"] > 0


@pytest.mark.parametrize("prec_name,prec", PRECS)
@pytest.mark.parametrize("name", ["random3000", "shear1500"])
def test_action_reaction_trajectory_100_steps(name, prec_name, prec):
    say("case action-reaction trajectory", name, prec_name)
    out = trajectory_parity(SCENES[name](), prec, steps=100, tol=1e-4,
                            flags=FLAG_ACTION_REACTION)
    say("  ", out)


def test_action_reaction_and_split_find_the_same_contacts_every_step():
    say("case action-reaction vs split contacts")
    sc = SCENES["random3000"]()
    sc.v *= 20.0
    dt = oracle.Sim(sc, mode=1).dt
    gs = [Sim.from_scene(sc, precision=PREC_FP64, dt=dt, flags=f)
          for f in (0, FLAG_ACTION_REACTION)]
    try:
        scale = float(np.median(sc.r))
        for step in range(30):
            for g in gs:
                g.step(1)
            (ai, aj, adt), (bi, bj, bdt) = gs[0].get_contacts(), gs[1].get_contacts()
            assert np.array_equal(ai, bi) and np.array_equal(aj, bj), "step %d" % step
            assert np.abs(adt - bdt).max(initial=0.0) <= 1e-9 * scale
        a, b = gs[0].get_state(), gs[1].get_state()
        for k in ("x", "v", "w"):
            d = np.abs(a[k] - b[k]).max()
            assert d <= 1e-9 * max(np.abs(a[k]).max(), 1e-300), k
    finally:
        for g in gs:
            g.close()


def test_action_reaction_conserves_momentum():
    # periodic box, no gravity, no walls: every pair adds +F and -F, so the
    # forces sum to zero up to the rounding of the per-particle sums
    say("case action-reaction momentum")
    sc = SCENES["periodic1500"]()
    g = Sim.from_scene(sc, precision=PREC_FP64, flags=FLAG_ACTION_REACTION)
    try:
        g.step(5)
        F = g.get_state()["F"]
        assert np.abs(F).sum() > 0
        assert np.abs(F.sum(axis=0)).max() <= 1e-12 * np.abs(F).sum()
    finally:
        g.close()


def test_action_reaction_pool_jobs_equal_jobs_alone():
    say("case action-reaction pool")
    scs = [gen.scene_random(seed=411, n=700, phi=0.22, p_touch=0.7, vel_sigma=0.2),
           gen.scene_random(seed=412, n=129, phi=0.2, p_touch=0.8, vel_sigma=0.3),
           gen.scene_random(seed=413, n=600, phi=0.22, p_touch=0.7, walls=0, periodic=7,
                            gravity=(0, 0, 0), shear_rate=2000.0),
           gen.scene_random(seed=414, n=500, phi=0.22, p_touch=0.7, n_materials=3)]
    dts = [oracle.Sim(s, mode=1).dt for s in scs]
    steps = [30, 12, 30, 21]
    pool = Pool(max_particles=sum(s.n for s in scs) + 128 * len(scs),
                max_cells=sum(max(4 * s.n, 4096) for s in scs), max_jobs=len(scs),
                precision=PREC_MIXED, flags=FLAG_ACTION_REACTION)
    try:
        ids = [pool.add_scene(s, steps=k, dt=dt) for s, k, dt in zip(scs, steps, dts)]
        pool.step(32)
        pool.sync()
        assert sorted(pool.poll()) == sorted(ids)
        for s, k, dt, j in zip(scs, steps, dts, ids):
            g = Sim.from_scene(s, precision=PREC_MIXED, dt=dt, flags=FLAG_ACTION_REACTION)
            g.step(k)
            ref = g.get_state()
            g.close()
            got = pool.get_state(j)
            for key in ("x", "v", "w"):
                assert np.array_equal(got[key], ref[key]), "job n=%d: %s" % (s.n, key)
    finally:
        pool.close()


def test_action_reaction_capacity_regrow_is_transparent():
    say("case action-reaction regrow")
    sc = SCENES["random3000"]()
    dt = oracle.Sim(sc, mode=1).dt
    g1 = Sim.from_scene(sc, precision=PREC_MIXED, dt=dt, flags=FLAG_ACTION_REACTION)
    g2 = Sim.from_scene(sc, precision=PREC_MIXED, dt=dt, flags=FLAG_ACTION_REACTION,
                        max_contacts=16)
    try:
        g1.step(20)
        g2.step(20)
        assert g2.info()["regrows"] >= 1
        a, b = g1.get_state(), g2.get_state()
        for k in ("x", "v", "w", "F", "T"):
            assert np.array_equal(a[k], b[k]), k
    finally:
        g1.close()
        g2.close()


def test_fused_with_action_reaction_is_rejected():
    sc = SCENES["cluster64"]()
    with pytest.raises(DemError):
        Sim.from_scene(sc, precision=PREC_MIXED, flags=FLAG_FUSED | FLAG_ACTION_REACTION)
