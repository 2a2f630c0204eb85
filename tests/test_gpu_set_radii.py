"""dem_set_radii (include/dem.h): new radii between steps, keeping state and
contact history.  A simulation whose radii are replaced after some steps
continues bitwise like a simulation created from its state, history and the
new radii; radii beyond the grid or not finite are refused; a pack grown to
volume fraction 0.55 this way is a valid input whose next step matches the
oracle."""
import numpy as np
import pytest

import gen
from gpu_util import SCENES, say
from paper_1503_03553_amd import DemError, PREC_FP64, PREC_MIXED, Sim, pack

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec_name,prec", [("mixed", PREC_MIXED), ("fp64", PREC_FP64)])
@pytest.mark.parametrize("name", ["random3000", "periodic1500"])
def test_new_radii_continue_like_a_fresh_simulation(name, prec_name, prec):
    say("case set_radii", name, prec_name)
    sc = SCENES[name]()
    r1 = gen.f32(sc.r * 1.01)
    cell = 2.0 * float(r1.max()) * 1.0001
    a = Sim.from_scene(sc, precision=prec, cell_size=cell)
    try:
        dt = a.info()["dt"]
        a.step(5)
        st = a.get_state(forces=False)
        hi, hj, hdt = a.get_contacts()
        a.set_radii(r1)
        a.step(5)
        ra = a.get_state()
        ca = a.get_contacts()
    finally:
        a.close()
    b_sc = sc.copy()
    b_sc.x, b_sc.v, b_sc.w, b_sc.r = st["x"], st["v"], st["w"], r1
    with Sim.from_scene(b_sc, precision=prec, dt=dt) as b:
        b.set_contacts(hi, hj, hdt)
        b.step(5)
        rb = b.get_state()
        cb = b.get_contacts()
    for k in ("x", "v", "w", "F", "T"):
        assert np.array_equal(ra[k], rb[k]), k
    for u, v in zip(ca, cb):
        assert np.array_equal(u, v)
    # the larger radii made new contacts
    assert ca[0].size > hi.size


def test_radii_beyond_the_grid_or_not_finite_are_refused():
    sc = SCENES["random3000"]()
    with Sim.from_scene(sc, precision=PREC_MIXED) as g:
        cell = min(g.info()["cells"])  # counts; the widths follow from the box
        width = float(np.min((sc.hi - sc.lo) / np.array(g.info()["cells"])))
        assert cell > 0
        big = sc.r.copy()
        # wider than a cell: beyond even the two-level search's wide scan
        big[0] = gen.f32(np.array([1.01 * width]))[0]
        with pytest.raises(DemError) as e:
            g.set_radii(big)
        assert e.value.code == -1
        bad = sc.r.copy()
        bad[3] = np.nan
        with pytest.raises(DemError) as e:
            g.set_radii(bad)
        assert e.value.code == -1
        # nothing changed: the simulation still steps
        g.step(2)
        g.sync()


def test_grown_pack_steps_like_the_oracle():
    from test_gpu_fullsize import last_step_parity
    say("case grown pack 30000")
    start = gen.config_dense_start(n=30000)
    g = pack.grown(start)
    say("  grown:", g["stats"])
    st = g["stats"]
    assert st["contacts_per_particle"] > 1.0
    assert st["max_overlap_over_r"] < 0.1
    sc = gen.dense_run_scene(start, g["x"], g["v"], g["w"])
    phi = float(np.sum(4.0 / 3.0 * np.pi * sc.r ** 3) / np.prod(sc.hi - sc.lo))
    assert abs(phi - 0.55) < 1e-6
    rep = last_step_parity(sc, steps=20, tol=1e-5, threads=8)
    say("  ", rep)
    assert rep["contacts"] > sc.n
