"""GPU parity of the fused single loop, the ablation of the split of section
3.4: one kernel whose lane per particle runs the contact law as soon as it
finds a contact.

Against the FP64 oracle it meets the single-step and trajectory tolerances of
the split path; against the split path its contact set is the same bit for
bit at every step.  Its per-particle sums follow the order in which the
contacts were found, so its states differ from the split path's only by the
rounding of that order.  A job in a fused pool gives bitwise the results of
the same scene run alone with the fused kernel.
"""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import SCENES, random_history, say, step_parity, trajectory_parity
from paper_1503_03553_amd import FLAG_FUSED, PREC_FP64, PREC_MIXED, Pool, Sim

pytestmark = pytest.mark.gpu

PRECS = [("fp64", PREC_FP64), ("mixed", PREC_MIXED)]


@pytest.mark.parametrize("prec_name,prec", PRECS)
@pytest.mark.parametrize("name", ["cluster64", "random3000", "shear1500", "mixedwall",
                                  "materials"])
def test_fused_one_step_parity(name, prec_name, prec):
    say("case fused one_step", name, prec_name)
    sc = SCENES[name]()
    hist = random_history(sc, seed=5)
    tol = 1e-9 if prec == PREC_FP64 else 1e-5
    _, _, _, rep = step_parity(sc, prec, history=hist, tol=tol,
                               flags=FLAG_FUSED)
    say("  ", rep)
    assert rep["contacts"] > 0


@pytest.mark.parametrize("prec_name,prec", PRECS)
@pytest.mark.parametrize("name", ["random3000", "shear1500"])
def test_fused_trajectory_100_steps(name, prec_name, prec):
    say("case fused trajectory", name, prec_name)
    out = trajectory_parity(SCENES[name](), prec, steps=100, tol=1e-4, flags=FLAG_FUSED)
    say("  ", out)


def test_fused_and_split_find_the_same_contacts_every_step():
    say("case fused vs split contacts")
    sc = SCENES["random3000"]()
    sc.v *= 20.0  # contacts made and broken during the run
    dt = oracle.Sim(sc, mode=1).dt
    gs = [Sim.from_scene(sc, precision=PREC_FP64, dt=dt, flags=f) for f in (0, FLAG_FUSED)]
    try:
        scale = float(np.median(sc.r))
        changed = 0
        prev = None
        for step in range(30):
            for g in gs:
                g.step(1)
            (ai, aj, adt), (bi, bj, bdt) = gs[0].get_contacts(), gs[1].get_contacts()
            assert np.array_equal(ai, bi) and np.array_equal(aj, bj), "step %d" % step
            # the tangential displacements differ by the summation order only
            assert np.abs(adt - bdt).max(initial=0.0) <= 1e-9 * scale
            key = set(zip(ai.tolist(), aj.tolist()))
            if prev is not None:
                changed += len(key ^ prev)
            prev = key
        assert changed > 0, "no contact was made or broken"
        a, b = gs[0].get_state(forces=False), gs[1].get_state(forces=False)
        for k in ("x", "v", "w"):
            d = np.abs(a[k] - b[k]).max()
            assert d <= 1e-9 * max(np.abs(a[k]).max(), 1e-300), k
    finally:
        for g in gs:
            g.close()


def test_fused_slab_overflow_regrows():
    # a big sphere with more contacts than a particle's slab holds: the step
    # is redone with wider slabs, and the result is the oracle's
    say("case fused slab overflow")
    rng = np.random.default_rng(3)
    R, r = 8e-6, 2e-6
    c = np.array([50e-6] * 3)
    dirs = rng.normal(size=(40, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    keep = [0]
    for k in range(1, 40):
        if all(np.dot(dirs[k], dirs[q]) < np.cos(0.5) for q in keep):
            keep.append(k)
    dirs = dirs[keep]
    x = np.vstack([c, c + dirs * (R + r - 1e-9)])
    n = x.shape[0]
    assert n > 9
    sc = gen.Scene(lo=np.zeros(3), hi=np.full(3, 100e-6), x=x, v=np.zeros((n, 3)),
                   w=np.zeros((n, 3)), r=gen.f32([R] + [r] * (n - 1)), mat=np.zeros(n, np.uint16),
                   materials=[gen.Material.make()], walls=gen.WALL_ALL, gravity=(0, 0, 0))
    g, _, _, rep = step_parity(sc, PREC_FP64, tol=1e-9, flags=FLAG_FUSED)
    assert rep["contacts"] >= 2 * (n - 1)


def test_fused_pool_jobs_equal_jobs_alone():
    say("case fused pool")
    scs = [gen.scene_random(seed=401, n=700, phi=0.22, p_touch=0.7, vel_sigma=0.2),
           gen.scene_random(seed=402, n=129, phi=0.2, p_touch=0.8, vel_sigma=0.3),
           gen.scene_random(seed=403, n=600, phi=0.22, p_touch=0.7, walls=0, periodic=7,
                            gravity=(0, 0, 0), shear_rate=2000.0),
           gen.scene_random(seed=404, n=500, phi=0.22, p_touch=0.7, n_materials=3)]
    dts = [oracle.Sim(s, mode=1).dt for s in scs]
    steps = [30, 12, 30, 21]
    pool = Pool(max_particles=sum(s.n for s in scs) + 128 * len(scs),
                max_cells=sum(max(4 * s.n, 4096) for s in scs), max_jobs=len(scs),
                precision=PREC_MIXED, flags=FLAG_FUSED)
    try:
        ids = [pool.add_scene(s, steps=k, dt=dt) for s, k, dt in zip(scs, steps, dts)]
        pool.step(32)
        pool.sync()
        assert sorted(pool.poll()) == sorted(ids)
        for s, k, dt, j in zip(scs, steps, dts, ids):
            g = Sim.from_scene(s, precision=PREC_MIXED, dt=dt, flags=FLAG_FUSED)
            g.step(k)
            ref = g.get_state()
            g.close()
            got = pool.get_state(j)
            for key in ("x", "v", "w"):
                assert np.array_equal(got[key], ref[key]), "job n=%d: %s" % (s.n, key)
    finally:
        pool.close()


# ------------------------------------------------ the paper's per-thread split
@pytest.mark.parametrize("prec_name,prec", PRECS)
@pytest.mark.parametrize("name", ["random3000", "shear1500", "materials"])
def test_thread_split_equals_compacted_split(name, prec_name, prec):
    # the same per-contact terms summed in the same order: the per-thread
    # second loop gives the compacted force kernel's results up to the
    # rounding the compiler's contraction choices may change
    say("case thread split", name, prec_name)
    from paper_1503_03553_amd import FLAG_THREAD_SPLIT
    sc = SCENES[name]()
    dt = oracle.Sim(sc, mode=1).dt
    runs = []
    for flags in (0, FLAG_THREAD_SPLIT):
        g = Sim.from_scene(sc, precision=prec, dt=dt, flags=flags)
        g.step(25)
        runs.append((g.get_state(), g.get_contacts()))
        g.close()
    (a, ca), (b, cb) = runs
    assert np.array_equal(ca[0], cb[0]) and np.array_equal(ca[1], cb[1])
    tol = 1e-9 if prec == PREC_FP64 else 1e-5
    assert np.abs(ca[2] - cb[2]).max(initial=0.0) <= tol * max(np.abs(ca[2]).max(), 1e-300)
    for k in ("x", "v", "w", "F", "T"):
        scale = max(np.abs(a[k]).max(), 1e-300)
        assert np.abs(a[k] - b[k]).max() <= tol * scale, k


def test_thread_split_one_step_parity():
    say("case thread split oracle")
    from paper_1503_03553_amd import FLAG_THREAD_SPLIT
    sc = SCENES["random3000"]()
    step_parity(sc, PREC_MIXED, history=random_history(sc, seed=9), tol=1e-5, flags=FLAG_THREAD_SPLIT)
