"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Every input is seeded; sizes span several 128-particle tiles with a ragged
tail.  The contact set must be bit-exact; forces, torques and tangential
displacements within 1e-5 of their natural scale after one step from the
same state and history; trajectories within 1e-4 after 100 steps.
"""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import SCENES, make_pair, random_history, say, step_parity, trajectory_parity
from paper_1503_03553_amd import PREC_FP64, PREC_MIXED, DemError, Sim

pytestmark = pytest.mark.gpu

PRECS = [("fp64", PREC_FP64), ("mixed", PREC_MIXED)]


@pytest.mark.parametrize("prec_name,prec", PRECS)
@pytest.mark.parametrize("name", list(SCENES))
def test_one_step_parity(name, prec_name, prec):
    say("case one_step", name, prec_name)
    sc = SCENES[name]()
    hist = random_history(sc, seed=5)
    # FP32 force arithmetic may flip the sliding-cap branch of a contact
    # sitting on the cap within FP32 rounding (a cap tie); those and their
    # owners are counted, every other contact and particle is held to tol
    tol = 1e-9 if prec == PREC_FP64 else 1e-5
    _, _, _, rep = step_parity(sc, prec, history=hist, tol=tol)
    say("  ", rep)
    assert rep["contacts"] > 0


@pytest.mark.parametrize("prec_name,prec", PRECS)
@pytest.mark.parametrize("name", ["cluster64", "random3000", "shear1500"])
def test_trajectory_100_steps(name, prec_name, prec):
    say("case trajectory", name, prec_name)
    sc = SCENES[name]()
    rep = trajectory_parity(sc, prec, steps=100, tol=1e-4)
    say("  ", {k: "%.2e/%.2e" % v for k, v in rep.items()})


def test_plain_config_small_contact_rich():
    # the plain FP64 workload (2,000 monodisperse spheres, phi 0.3, walls,
    # gravity) with velocities x100 so that contacts form within the run
    say("case plain 2000 x100 velocities")
    sc = gen.config_plain()
    sc.v *= 100.0
    rep = trajectory_parity(sc, PREC_FP64, steps=200, tol=1e-4)
    say("  ", rep)


@pytest.mark.parametrize("n", [1, 2, 127, 128, 129, 257])
def test_ragged_sizes(n):
    say("case ragged", n)
    sc = gen.scene_random(seed=100 + n, n=n, phi=0.2 if n > 16 else 0.03, p_touch=0.8,
                          vel_sigma=0.3)
    step_parity(sc, PREC_FP64, tol=1e-9)
    trajectory_parity(sc, PREC_MIXED, steps=30, tol=1e-4)


def test_empty_simulation():
    say("case empty")
    m = gen.Material.make()
    s = Sim(lo=[0, 0, 0], hi=[1e-4] * 3, x=np.zeros((0, 3)), v=np.zeros((0, 3)),
            w=np.zeros((0, 3)), r=np.zeros(0), materials=[m], dt=1e-9)
    s.step(5)
    st = s.get_state()
    assert st["x"].shape == (0, 3)
    i, j, dt = s.get_contacts()
    assert i.size == 0
    assert s.info()["steps_done"] == 5
    s.close()


def test_all_in_one_cell_and_outside_box():
    # a clump bigger than a cell's share, plus a particle that left the box
    say("case clump")
    sc = gen.scene_cluster(seed=4, n_side=3, vel_sigma=0.1)
    sc.x[0] = sc.lo - 3e-6  # outside the box: sits in a border cell
    step_parity(sc, PREC_FP64, tol=1e-9)


def test_capacity_regrow_is_transparent():
    say("case regrow")
    sc = SCENES["random3000"]()
    g1, o = make_pair(sc, PREC_MIXED)
    g2 = Sim.from_scene(sc, precision=PREC_MIXED, dt=o.dt, max_contacts=16)
    g1.step(20)
    g2.step(20)
    a, b = g1.get_state(), g2.get_state()
    assert g2.info()["regrows"] >= 1
    for k in ("x", "v", "w", "F", "T"):
        assert np.array_equal(a[k], b[k]), k
    ca, cb = g1.get_contacts(), g2.get_contacts()
    for u, v in zip(ca, cb):
        assert np.array_equal(u, v)
    g1.close()
    g2.close()


def test_row_overflow_switches_kernel():
    # a particle with more than 16 contacts (a big sphere in a crowd of small ones)
    say("case row overflow")
    rng = np.random.default_rng(3)
    R, r = 8e-6, 2e-6
    c = np.array([50e-6] * 3)
    dirs = rng.normal(size=(40, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    # keep directions well separated so the small spheres do not overlap each other
    keep = [0]
    for k in range(1, 40):
        if all(np.dot(dirs[k], dirs[q]) < np.cos(0.5) for q in keep):
            keep.append(k)
    dirs = dirs[keep]
    x = np.vstack([c, c + dirs * (R + r - 1e-9)])
    n = x.shape[0]
    assert n > 17
    sc = gen.Scene(lo=np.zeros(3), hi=np.full(3, 100e-6), x=x, v=np.zeros((n, 3)),
                   w=np.zeros((n, 3)), r=gen.f32([R] + [r] * (n - 1)), mat=np.zeros(n, np.uint16),
                   materials=[gen.Material.make()], walls=gen.WALL_ALL, gravity=(0, 0, 0))
    step_parity(sc, PREC_FP64, tol=1e-9)


def test_deterministic_and_cell_size_invariant():
    say("case determinism")
    sc = SCENES["random3000"]()
    o = oracle.Sim(sc, mode=1)
    runs = []
    for cs in (0.0, 0.0, 3.0 * sc.r.max(), 5.0 * sc.r.max()):
        g = Sim.from_scene(sc, precision=PREC_MIXED, dt=o.dt, cell_size=cs)
        g.step(25)
        runs.append((g.get_state(), g.get_contacts()))
        g.close()
    for st, ct in runs[1:]:
        for k in ("x", "v", "w", "F", "T"):
            assert np.array_equal(st[k], runs[0][0][k]), k
        for u, v in zip(ct, runs[0][1]):
            assert np.array_equal(u, v)


def test_checkpoint_restore_bitwise():
    say("case checkpoint")
    sc = SCENES["random3000"]()
    o = oracle.Sim(sc, mode=1)
    g = Sim.from_scene(sc, precision=PREC_MIXED, dt=o.dt)
    g.step(10)
    st = g.get_state()
    ci, cj, cdt = g.get_contacts()
    g.step(10)
    ref = g.get_state()
    g.close()
    sc2 = sc.copy()
    sc2.x, sc2.v, sc2.w = st["x"], st["v"], st["w"]
    h = Sim.from_scene(sc2, precision=PREC_MIXED, dt=o.dt)
    h.set_contacts(ci, cj, cdt)
    h.step(10)
    got = h.get_state()
    h.close()
    for k in ("x", "v", "w"):
        assert np.array_equal(got[k], ref[k]), k


def test_set_state_keeps_history():
    say("case set_state")
    sc = SCENES["cluster64"]()
    o = oracle.Sim(sc, mode=1)
    g = Sim.from_scene(sc, precision=PREC_FP64, dt=o.dt)
    g.step(3)
    st = g.get_state()
    c0 = g.get_contacts()
    g.set_state(st["x"], st["v"], st["w"])
    c1 = g.get_contacts()
    for u, v in zip(c0, c1):
        assert np.array_equal(u, v)
    g.step(2)
    a = g.get_state()
    g.close()
    h = Sim.from_scene(sc, precision=PREC_FP64, dt=o.dt)
    h.step(5)
    b = h.get_state()
    h.close()
    for k in ("x", "v", "w"):
        assert np.array_equal(a[k], b[k]), k


def test_auto_dt_matches_oracle_rule():
    say("case auto dt")
    sc = gen.config_plain()
    g = Sim.from_scene(sc, precision=PREC_FP64)
    dt = g.info()["dt"]
    g.close()
    ref = oracle.dt_rule(sc)
    assert abs(dt - ref) <= 1e-12 * ref


def test_nonfinite_is_reported():
    say("case nonfinite")
    sc = SCENES["cluster64"]()
    # an absurd time step drives the state to overflow within a few steps
    g = Sim.from_scene(sc, precision=PREC_MIXED, dt=1e30)
    g.step(5)
    with pytest.raises(DemError) as e:
        g.sync()
    assert e.value.code == -4
    g.close()


def test_invalid_arguments_rejected():
    say("case invalid")
    m = gen.Material.make()
    x = np.full((4, 3), 50e-6) + np.arange(4)[:, None] * 20e-6
    z = np.zeros((4, 3))
    with pytest.raises(DemError):
        Sim(lo=[0, 0, 0], hi=[1e-4] * 3, x=x, v=z, w=z, r=[-1e-6] * 4, materials=[m])
    with pytest.raises(DemError):  # wall on a periodic axis
        Sim(lo=[0, 0, 0], hi=[1e-4] * 3, x=x, v=z, w=z, r=[1e-6] * 4, materials=[m], periodic=1,
            walls=0x3F)
    with pytest.raises(DemError):  # fewer than 3 cells along a periodic axis
        Sim(lo=[0, 0, 0], hi=[1e-4] * 3, x=x, v=z, w=z, r=[2e-5] * 4, materials=[m], periodic=7,
            walls=0)


def drifting_scene(n, seed):
    # a dilute periodic cloud translating as a whole: about one cell per
    # step, so most particles change cell every step, and no new contacts
    sc = gen.scene_random(seed=seed, n=n, phi=0.02, p_touch=0.0, walls=0, periodic=7,
                          gravity=(0, 0, 0), vel_sigma=1e-3)
    sc.v += np.array([12.0, 7.0, 5.0])
    return sc


@pytest.mark.parametrize("n", [6000, 20000])
def test_many_cell_changes_per_step(n):
    # n = 6000: thousands of particles change cell per step and are merged
    # into the unchanged ones; n = 20000: more than the merge takes, so the
    # steps are redone with the radix sort
    say("case many cell changes", n)
    sc = drifting_scene(n, seed=31)
    rep = trajectory_parity(sc, PREC_MIXED, steps=6, tol=1e-4, dt=1e-6)
    say("  ", rep)


def test_particle_far_outside_the_box():
    # a particle far outside the box (its FP32 search record is not usable)
    # passes every pre-filter comparison; the exact re-walk keeps its row
    say("case far outside")
    sc = gen.scene_random(seed=32, n=3000, phi=0.2, p_touch=0.7, vel_sigma=0.2)
    L = sc.hi - sc.lo
    sc.x[5] = sc.lo + np.array([0.5, 0.5, 5.0]) * L
    step_parity(sc, PREC_FP64, tol=1e-9)


@pytest.mark.parametrize("name", ["random3000", "shear1500"])
def test_merge_sort_equals_radix_sort(name):
    # the order of every step, hence every result, is the same whether the
    # particles that changed cell are merged or all keys are radix sorted
    say("case merge vs radix", name)
    from paper_1503_03553_amd import FLAG_RADIX_SORT
    sc = SCENES[name]()
    sc.v *= 50.0  # many cell changes per step
    o = oracle.Sim(sc, mode=1)
    runs = []
    for flags in (0, FLAG_RADIX_SORT):
        g = Sim.from_scene(sc, precision=PREC_MIXED, dt=o.dt, flags=flags)
        g.step(40)
        runs.append((g.get_state(), g.get_contacts()))
        g.close()
    for k in ("x", "v", "w", "F", "T"):
        assert np.array_equal(runs[0][0][k], runs[1][0][k]), k
    for u, v in zip(runs[0][1], runs[1][1]):
        assert np.array_equal(u, v)


def test_mover_into_the_first_cell():
    # one particle crosses into the corner cell, whose key sorts before every
    # other particle's: the merge must place it first
    say("case mover into first cell")
    sc = gen.scene_cluster(seed=5, n_side=3, vel_sigma=0.05)
    o = oracle.Sim(sc, mode=1)
    cell = 2.0 * float(sc.r.max())
    sc.x[0] = sc.lo + 1.0005 * cell
    sc.v[0] = -0.002 * cell / o.dt
    trajectory_parity(sc, PREC_MIXED, steps=2, tol=1e-4)


def test_redone_step_keeps_contacts():
    # a periodic pack of touching pairs translating by about a cell per step:
    # the first step has more cell changes than the merge takes and is redone
    # with the radix sort after the force kernel has started; the redone
    # step must find every contact, so histories match the oracle's
    say("case redone step")
    sc = gen.scene_random(seed=33, n=20000, phi=0.1, p_touch=0.9, walls=0, periodic=7,
                          gravity=(0, 0, 0), vel_sigma=1e-4)
    o = oracle.Sim(sc, mode=1)
    sc.v += 1.5 * 2.0 * float(sc.r.max()) / o.dt * np.array([1.0, 0.6, 0.3])
    o = oracle.Sim(sc, dt=o.dt, mode=1)
    g = Sim.from_scene(sc, precision=PREC_FP64, dt=o.dt)
    g.step(4)
    ci, cj, cdt = g.get_contacts()
    g.close()
    o.step(4)
    compare_contacts_full = (ci.size, o.hist.i.size)
    assert compare_contacts_full[0] == compare_contacts_full[1] and ci.size > 1000
    assert np.array_equal(ci, o.hist.i) and np.array_equal(cj, o.hist.j)
    scale = np.linalg.norm(o.hist.dt, axis=1).max()
    assert np.abs(cdt - o.hist.dt).max() <= 1e-9 * scale
