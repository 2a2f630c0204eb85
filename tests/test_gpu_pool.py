"""GPU tests of the job pool: many simulations of uneven sizes advanced by
shared launches.

The contract is isolation: a job in any mix, admitted at any time, gives
bitwise the results of the same scene run alone (whose parity with the
oracle the single-simulation tests establish), runs exactly its own number
of steps and is then frozen.
"""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import say
from paper_1503_03553_amd import PREC_FP64, PREC_MIXED, DemError, Pool, Sim

pytestmark = pytest.mark.gpu


def mixed_scenes():
    """Scenes of different sizes, boxes, boundaries and materials."""
    return [
        gen.scene_random(seed=301, n=700, phi=0.22, p_touch=0.7, vel_sigma=0.2),
        gen.scene_cluster(seed=302, n_side=4, vel_sigma=0.2, polydisperse=True),
        gen.scene_random(seed=303, n=129, phi=0.2, p_touch=0.8, vel_sigma=0.3),
        gen.scene_random(seed=304, n=900, phi=0.22, p_touch=0.7, walls=0, periodic=7,
                         gravity=(0, 0, 0)),
        gen.scene_random(seed=305, n=600, phi=0.22, p_touch=0.7, walls=0, periodic=7,
                         gravity=(0, 0, 0), shear_rate=2000.0),
        gen.scene_random(seed=306, n=500, phi=0.22, p_touch=0.7, n_materials=3),
        gen.scene_random(seed=307, n=2500, phi=0.25, p_touch=0.7, vel_sigma=0.2),
        gen.scene_random(seed=308, n=1, phi=0.03, vel_sigma=0.3),
    ]


def cells_bound(scenes):
    # a job's grid has at most max(4 n, 4096) cells
    return sum(max(4 * s.n, 4096) for s in scenes)


def alone(sc, precision, dt, steps):
    g = Sim.from_scene(sc, precision=precision, dt=dt)
    g.step(steps)
    st = g.get_state()
    g.close()
    return st


def assert_same(a, b, what):
    for k in ("x", "v", "w"):
        assert np.array_equal(a[k], b[k]), "%s: %s differs" % (what, k)


@pytest.mark.parametrize("prec_name,prec", [("mixed", PREC_MIXED), ("fp64", PREC_FP64)])
def test_jobs_in_a_mix_equal_jobs_alone(prec_name, prec):
    say("case pool mix", prec_name)
    scs = mixed_scenes()
    dts = [oracle.Sim(s, mode=1).dt for s in scs]
    steps = [40, 25, 40, 33, 40, 17, 40, 5]
    pool = Pool(max_particles=sum(s.n for s in scs) + 128 * len(scs),
                max_cells=cells_bound(scs), max_jobs=len(scs), precision=prec)
    ids = [pool.add_scene(s, steps=k, dt=dt) for s, k, dt in zip(scs, steps, dts)]
    pool.step(45)
    pool.sync()
    done = pool.poll()
    assert sorted(done) == sorted(ids)
    for s, k, dt, j in zip(scs, steps, dts, ids):
        inf = pool.job_info(j)
        assert inf["status"] == "done" and inf["steps_done"] == k and inf["steps_left"] == 0
        assert inf["time"] == pytest.approx(k * dt, rel=1e-12)
        assert_same(pool.get_state(j), alone(s, prec, dt, k), "job n=%d" % s.n)
    pool.close()


def test_admission_and_removal_between_steps():
    say("case pool admission")
    scs = mixed_scenes()
    dts = [oracle.Sim(s, mode=1).dt for s in scs]
    cap = scs[0].n + scs[6].n + 3 * 128
    pool = Pool(max_particles=cap, max_cells=cells_bound(scs[:1] + scs[6:7]) + 8192, max_jobs=3,
                precision=PREC_MIXED)
    a = pool.add_scene(scs[0], steps=10, dt=dts[0])
    b = pool.add_scene(scs[6], steps=30, dt=dts[6])
    # no room for another 2500-particle job
    with pytest.raises(DemError) as e:
        pool.add_scene(scs[6], steps=5, dt=dts[6])
    assert e.value.code == -6
    pool.step(4)
    c = pool.add_scene(scs[2], steps=12, dt=dts[2])  # joins while a and b run
    pool.step(8)
    assert sorted(pool.poll()) == [a]
    pool.remove(a)
    d = pool.add_scene(scs[5], steps=9, dt=dts[5])  # reuses a's tiles
    pool.step(20)
    assert sorted(pool.poll()) == sorted([b, c, d])
    assert_same(pool.get_state(b), alone(scs[6], PREC_MIXED, dts[6], 30), "b")
    assert_same(pool.get_state(c), alone(scs[2], PREC_MIXED, dts[2], 12), "c")
    assert_same(pool.get_state(d), alone(scs[5], PREC_MIXED, dts[5], 9), "d")
    for j in (b, c, d):
        pool.remove(j)
    free = pool.capacity()
    assert free["jobs"] == 3 and free["particles"] >= cap - 127
    pool.close()


def test_failed_job_does_not_disturb_the_others():
    say("case pool failure isolation")
    scs = mixed_scenes()
    good = scs[0]
    dt = oracle.Sim(good, mode=1).dt
    pool = Pool(max_particles=good.n + scs[1].n + 256, max_cells=cells_bound([good, scs[1]]),
                max_jobs=2, precision=PREC_MIXED)
    g = pool.add_scene(good, steps=20, dt=dt)
    bad = pool.add_scene(scs[1], steps=20, dt=1e30)  # overflows within a few steps
    pool.step(20)
    pool.sync()
    assert pool.job_info(bad)["status"] == "failed"
    assert pool.job_info(g)["status"] == "done"
    assert_same(pool.get_state(g), alone(good, PREC_MIXED, dt, 20), "good job")
    pool.close()


def test_pool_job_trajectory_matches_oracle():
    # directly against the oracle too, with another job beside it
    say("case pool vs oracle")
    sc = gen.scene_random(seed=311, n=1000, phi=0.22, p_touch=0.7, vel_sigma=0.2)
    other = gen.scene_random(seed=312, n=300, phi=0.2, p_touch=0.7)
    o = oracle.Sim(sc, mode=1)
    pool = Pool(max_particles=1300 + 256, max_cells=cells_bound([sc, other]), max_jobs=2,
                precision=PREC_MIXED)
    pool.add_scene(other, steps=100)
    j = pool.add_scene(sc, steps=100, dt=o.dt)
    pool.step(100)
    got = pool.get_state(j)
    pool.close()
    o.step(100)
    # the single-simulation trajectory bar: error within 1e-4 of the largest change
    for k, base in (("x", sc.x), ("v", sc.v), ("w", sc.w)):
        ref = getattr(o, k)
        scale = np.linalg.norm(ref - base, axis=1).max()
        err = np.linalg.norm(got[k] - ref, axis=1).max()
        assert err <= 1e-4 * scale, "%s: %.3g vs %.3g" % (k, err, scale)


def test_pool_argument_errors():
    say("case pool errors")
    sc = mixed_scenes()[2]
    pool = Pool(max_particles=512, max_cells=8192, max_jobs=1, precision=PREC_MIXED)
    with pytest.raises(DemError):
        pool.add_scene(sc, steps=0)
    j = pool.add_scene(sc, steps=3)
    with pytest.raises(DemError):  # no free slot
        pool.add_scene(sc, steps=3)
    with pytest.raises(DemError):
        pool.job_info(j + 100)
    pool.step(3)
    assert pool.poll() == [j]
    assert pool.poll() == []
    pool.close()


def test_served_requests_equal_requests_alone():
    # continuous batching with real arrivals: requests join while others run,
    # and each result is bitwise that of the request run alone
    say("case serving")
    from paper_1503_03553_amd.serve import Request, Server
    scs = mixed_scenes()
    dts = [oracle.Sim(s, mode=1).dt for s in scs]
    for s, dt in zip(scs, dts):
        s.dt = dt
    steps = [60, 15, 30, 45, 25, 35, 50, 10]
    reqs = [Request(k, scs[k], steps[k], 0.002 * k) for k in range(len(scs))]
    got = {}

    def keep(req, pool):
        got[req.rid] = pool.get_state(req.job)

    # room for about half of the jobs at a time
    pool = Pool(max_particles=3800, max_cells=cells_bound(scs), max_jobs=4, precision=PREC_MIXED)
    srv = Server(pool, superstep=7, on_done=keep)
    st = srv.run(reqs, deadline=120.0)
    pool.close()
    say("  ", st)
    assert st["jobs"] == len(scs) and st["failed"] == 0
    assert srv.supersteps >= 2
    for k, s in enumerate(scs):
        assert_same(got[k], alone(s, PREC_MIXED, dts[k], steps[k]), "request %d" % k)
