"""The accuracy statement of the two precisions against the FP64 oracle: for
each seeded scene, the largest and the median relative error of the
tangential displacements, forces and torques after one step from identical
state and history, and of positions, velocities and angular velocities after
100 steps (relative to the natural scales of the parity tests).  The test
holds every figure to the tolerances and prints the table; with
DEM_ACCURACY_OUT set it also writes it there as JSON."""
import json
import os

import pytest

from gpu_util import SCENES, random_history, say, step_parity, trajectory_parity
from paper_1503_03553_amd import PREC_FP64, PREC_MIXED

pytestmark = pytest.mark.gpu

ROWS = {}


@pytest.mark.parametrize("prec_name,prec", [("fp64", PREC_FP64), ("mixed", PREC_MIXED)])
@pytest.mark.parametrize("name", list(SCENES))
def test_accuracy_row(name, prec_name, prec):
    say("case accuracy", name, prec_name)
    sc = SCENES[name]()
    tol = 1e-9 if prec == PREC_FP64 else 1e-5
    _, _, _, rep = step_parity(sc, prec, history=random_history(sc, seed=5), tol=tol)
    tr = trajectory_parity(sc, prec, steps=100, tol=1e-4)
    row = {"contacts": rep["contacts"], "cap_ties": rep["cap_ties"],
           "tie_owners": rep["tie_owners"], "tie_owners_off": rep["tie_owners_off"],
           "step1": {"dt": rep["err_dt"], "F": rep["err_F"], "T": rep["err_T"]},
           "steps100": {"x": tr["x_rel"], "v": tr["v_rel"], "w": tr["w_rel"]}}
    ROWS["%s/%s" % (name, prec_name)] = row
    say("  ", json.dumps(row))


def test_accuracy_table_written():
    if not ROWS:
        pytest.skip("no rows (run with the rows above)")
    say("accuracy table (max / median relative error)")
    for k, r in sorted(ROWS.items()):
        s1, s100 = r["step1"], r["steps100"]
        say("  %-22s dt %.1e/%.1e F %.1e/%.1e T %.1e/%.1e | x %.1e/%.1e v %.1e/%.1e w %.1e/%.1e"
            " | ties %d" % ((k,) + s1["dt"] + s1["F"] + s1["T"] + s100["x"] + s100["v"] +
                             s100["w"] + (r["cap_ties"],)))
    out = os.environ.get("DEM_ACCURACY_OUT")
    if out:
        os.makedirs(os.path.dirname(out) or ".", exist_ok=True)
        with open(out, "w") as fh:
            json.dump(ROWS, fh, indent=1, sort_keys=True)
