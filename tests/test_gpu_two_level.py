"""Two-level contact search (the default search's grid of twice the radius
cut, the few larger particles scanning a two-cell stencil themselves; here
with the cut given, radius_cut): the
contact set of one step equals the oracle's brute force, and over many steps
the two-level search gives bitwise the contacts, forces and states of the
one-level grid (cells of twice the largest radius) and of the paper's full
search, in walled, periodic and sheared boxes, with big particles of twice
the small radius (contact distance of two big ones = two cells) and with a
lognormal radius law."""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import say, step_parity
from paper_1503_03553_amd import FLAG_FULL_DETECT, PREC_FP64, PREC_MIXED, Sim

pytestmark = pytest.mark.gpu

# scene -> radius cut: the small radius of the bimodal scenes (their big
# spheres have twice it, so two big ones touch across exactly two cells), and
# about the 98th percentile of the lognormal law
CUT = {"bimodal_walls": 4.0e-6, "bimodal_sheared": 4.0e-6, "lognormal_periodic": 5.45e-6}

SCENES = {
    "bimodal_walls": lambda: gen.scene_random(seed=501, n=6000, phi=0.22, p_touch=0.8,
                                              polydisperse=False, big_frac=0.015,
                                              vel_sigma=0.3),
    "bimodal_sheared": lambda: gen.scene_random(seed=502, n=6000, phi=0.22, p_touch=0.8,
                                                polydisperse=False, big_frac=0.015, walls=0,
                                                periodic=7, gravity=(0, 0, 0),
                                                shear_rate=4000.0, vel_sigma=0.3),
    "lognormal_periodic": lambda: gen.scene_random(seed=503, n=8000, phi=0.22, p_touch=0.8,
                                                   walls=gen.WALL_ALL & ~3, periodic=1,
                                                   vel_sigma=0.3),
}


def _info(sc, prec, **kw):
    with Sim.from_scene(sc, precision=prec, **kw) as g:
        return g.info()


@pytest.mark.parametrize("prec_name,prec", [("mixed", PREC_MIXED), ("fp64", PREC_FP64)])
@pytest.mark.parametrize("name", list(SCENES))
def test_two_level_step_matches_the_oracle(name, prec_name, prec):
    say("case two-level oracle", name, prec_name)
    sc = SCENES[name]()
    inf = _info(sc, prec, radius_cut=CUT[name])
    assert inf["big"] > 0 and inf["radius_cut"] < float(np.max(sc.r))
    tol = 1e-9 if prec == PREC_FP64 else 1e-5
    _, _, _, rep = step_parity(sc, prec, tol=tol, radius_cut=CUT[name])
    # the big particles' contacts are part of the exact set
    assert rep["contacts"] > sc.n // 2


@pytest.mark.parametrize("name", list(SCENES))
def test_two_level_equals_one_level_and_full_search(name):
    say("case two-level vs one-level vs full", name)
    sc = SCENES[name]()
    dt = oracle.Sim(sc, mode=1).dt
    one = 2.0 * float(np.max(sc.r)) * 1.0001
    gs = [Sim.from_scene(sc, precision=PREC_MIXED, dt=dt, radius_cut=CUT[name]),
          Sim.from_scene(sc, precision=PREC_MIXED, dt=dt, cell_size=one),
          Sim.from_scene(sc, precision=PREC_MIXED, dt=dt, flags=FLAG_FULL_DETECT)]
    try:
        assert gs[0].info()["big"] > 0 and gs[1].info()["big"] == 0
        for step in range(30):
            for g in gs:
                g.step(1)
            ref = gs[0].get_contacts()
            for g in gs[1:]:
                got = g.get_contacts()
                for q in range(3):
                    assert np.array_equal(ref[q], got[q]), "step %d" % step
        s0 = gs[0].get_state()
        for g in gs[1:]:
            s = g.get_state()
            for k in ("x", "v", "w", "F", "T"):
                assert np.array_equal(s0[k], s[k]), k
    finally:
        for g in gs:
            g.close()


def test_automatic_cut_one_level_when_dilute_two_level_when_dense():
    say("case automatic radius cut")
    dilute = gen.scene_random(seed=504, n=5000, phi=0.1, p_touch=0.5)
    with Sim.from_scene(dilute, precision=PREC_MIXED) as g:
        assert g.info()["big"] == 0
    start = gen.config_dense_start(n=20000)
    dense = gen.dense_run_scene(start, start.x, start.v, start.w)  # full radii: phi 0.55
    dense.x = start.x  # overlapping, but only the grid is looked at
    with Sim.from_scene(dense, precision=PREC_MIXED) as g:
        inf = g.info()
        assert 0 < inf["big"] <= 0.002 * dense.n + 1
        assert inf["radius_cut"] < float(np.max(dense.r))
