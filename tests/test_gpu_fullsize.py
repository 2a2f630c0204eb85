"""Parity at the full sizes of the workloads, in the launch configuration the
benchmark times: the GPU runs the workload; after its last step the
oracle takes that same step from the GPU's own state and contact history
(the state before the step is copied out), and the contact set, the
tangential displacements, the per-particle forces (recovered from the
velocity change, since the benchmark does not store forces) and the new
positions and velocities are compared to the single-step tolerances.

The dense workload size can be lowered with DEM_FULL_N for quick runs.
"""
import os

import numpy as np
import pytest

import gen
import oracle
from gpu_util import check_step, say
from paper_1503_03553_amd import FLAG_NO_FORCE_OUTPUT, PREC_MIXED, Sim

pytestmark = pytest.mark.gpu


def last_step_parity(sc, steps, tol, threads=16):
    g = Sim.from_scene(sc, precision=PREC_MIXED, flags=FLAG_NO_FORCE_OUTPUT)
    dt = g.info()["dt"]
    g.step(steps - 1)
    st0 = g.get_state(forces=False)
    hi, hj, hdt = g.get_contacts()
    t0 = g.info()["time"]
    g.step(1)
    st1 = g.get_state(forces=False)
    ci, cj, cdt = g.get_contacts()
    g.close()
    say("  gpu done: %d contacts before, %d after" % (hi.size, ci.size))

    o = oracle.Sim(sc, dt=dt, mode=1, threads=threads)
    o.x, o.v, o.w = st0["x"].copy(), st0["v"].copy(), st0["w"].copy()
    o.time = t0
    o.hist = oracle.History(hi, hj, hdt)
    o.step(keep_contact_forces=True)
    say("  oracle step done")

    # forces and torques from the velocity changes (semi-implicit Euler)
    dens = np.array([sc.materials[k].density for k in sc.mat])
    m = dens * 4.0 / 3.0 * np.pi * sc.r.astype(np.float64) ** 3
    inertia = 0.4 * m * sc.r.astype(np.float64) ** 2
    st1 = dict(st1)
    st1["F"] = (st1["v"] - st0["v"]) * (m / dt)[:, None]
    st1["T"] = (st1["w"] - st0["w"]) * (inertia / dt)[:, None]
    # the velocity change is a difference of nearby FP64 numbers: its own
    # rounding is far below the tolerance (checked against the oracle's too)
    rep = check_step(o, sc, st1, ci, cj, cdt, tol, True, x0=st0["x"], time=t0)
    # positions: each moved by dt times the new velocity
    dx = st1["x"] - o.x
    if sc.periodic:
        L = sc.hi - sc.lo
        dx -= L * np.round(dx / L)
    move = np.abs(o.x - st0["x"])
    if sc.periodic:
        move = np.minimum(move, np.abs(L - move))
    assert np.abs(dx).max() <= tol * move.max() + 1e-12 * np.abs(sc.hi).max()
    return rep


def test_dense_sheared_pack_full_size():
    from paper_1503_03553_amd import pack
    n = int(os.environ.get("DEM_FULL_N", "8000000"))
    say("case dense shear", n)
    start = gen.config_dense_start(n=n)
    say("  generated, box %.4g m" % (start.hi[0] - start.lo[0]))
    g = pack.grown(start, log=say)
    say("  grown:", g["stats"])
    sc = gen.dense_run_scene(start, g["x"], g["v"], g["w"])
    rep = last_step_parity(sc, steps=100, tol=1e-5)
    say("  ", rep)
    # the grown pack at phi 0.55: more than one directed contact per particle
    assert rep["contacts"] > n


def test_dilute_headline_workload_full_size():
    say("case dilute 1M")
    sc = gen.config_dilute()
    rep = last_step_parity(sc, steps=200, tol=1e-5)
    say("  ", rep)
