"""Regression test: pairs that touch by rounding only (tests/grazing.py).
The force kernels must take the contact geometry from the predicate's own
squared distance (no fused multiply-add), so that the overlap of such a pair
is zero or positive, never negative: finite forces equal to the oracle's, in
both precisions, in every force-path variant."""
import numpy as np
import pytest

from gpu_util import say, step_parity
from grazing import grazing_scene
from paper_1503_03553_amd import (FLAG_ACTION_REACTION, FLAG_FULL_DETECT, FLAG_FUSED,
                                  FLAG_THREAD_SPLIT, PREC_FP64, PREC_MIXED, Sim)

pytestmark = pytest.mark.gpu

VARIANTS = [("half", 0), ("full", FLAG_FULL_DETECT), ("fused", FLAG_FUSED),
            ("thread", FLAG_THREAD_SPLIT), ("action_reaction", FLAG_ACTION_REACTION)]


@pytest.mark.parametrize("prec_name,prec", [("fp64", PREC_FP64), ("mixed", PREC_MIXED)])
@pytest.mark.parametrize("vname,flags", VARIANTS)
def test_grazing_pairs_one_step(vname, flags, prec_name, prec):
    say("case grazing one step", vname, prec_name)
    sc = grazing_scene(seed=3, npairs=64)
    tol = 1e-9 if prec == PREC_FP64 else 1e-5
    _, o, st, rep = step_parity(sc, prec, tol=tol, flags=flags)
    say("  ", rep)
    assert rep["contacts"] == 128
    assert np.isfinite(st["F"]).all() and np.isfinite(st["x"]).all()


@pytest.mark.parametrize("prec_name,prec", [("fp64", PREC_FP64), ("mixed", PREC_MIXED)])
def test_grazing_pairs_stay_finite(prec_name, prec):
    say("case grazing 50 steps", prec_name)
    sc = grazing_scene(seed=4, npairs=64)
    with Sim.from_scene(sc, precision=prec) as g:
        g.step(50)
        g.sync()
        st = g.get_state()
    for k in ("x", "v", "w", "F", "T"):
        assert np.isfinite(st[k]).all(), k
