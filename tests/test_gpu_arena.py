"""Device memory lent by the caller (include/dem.h, dem_create and
dem_pool_create): a simulation or a pool whose every device buffer is carved
from a torch tensor gives bitwise the results of one whose memory the library
allocates; a too small arena is refused; the contact table grows inside the
arena's spare room and fails cleanly without it; a pool sized by an HBM
budget fits it."""
import numpy as np
import pytest

import gen
from gpu_util import FACE, SCENES, say
from paper_1503_03553_amd import DemError, Pool, PREC_FP64, PREC_MIXED, Sim
from paper_1503_03553_amd.binding import footprint, make_params, pool_footprint

pytestmark = pytest.mark.gpu


def _run(sc, prec, steps, **kw):
    with Sim.from_scene(sc, precision=prec, **kw) as g:
        g.step(steps)
        g.sync()
        st = g.get_state()
        c = g.get_contacts()
        info = g.info()
    return st, c, info


def _params_of(sc, prec, max_contacts=0):
    return make_params(sc.lo, sc.hi, sc.walls, sc.periodic, sc.gravity, sc.shear_rate, sc.dt,
                       0.0, prec, sc.kn_form, 0.0, max_contacts)


def _same(a, b):
    for k in ("x", "v", "w", "F", "T"):
        assert np.array_equal(a[0][k], b[0][k]), k
    for u, v in zip(a[1], b[1]):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("prec_name,prec", [("fp64", PREC_FP64), ("mixed", PREC_MIXED)])
def test_step_in_a_torch_arena_equals_library_memory(prec_name, prec):
    import torch
    say("case arena", prec_name)
    sc = SCENES["random3000"]()
    need = footprint(_params_of(sc, prec), sc.n)
    arena = torch.empty(need, dtype=torch.uint8, device="cuda")
    a = _run(sc, prec, 30, arena=arena)
    b = _run(sc, prec, 30)
    _same(a, b)
    assert a[2]["device_bytes"] <= need
    assert a[1][0].size > 1000


def test_too_small_or_misaligned_arena_is_refused():
    import torch
    sc = SCENES["cluster64"]()
    need = footprint(_params_of(sc, PREC_MIXED), sc.n)
    arena = torch.empty(need, dtype=torch.uint8, device="cuda")
    with pytest.raises(DemError) as e:
        Sim.from_scene(sc, precision=PREC_MIXED, arena=arena[: need - 1])
    assert e.value.code == -1
    with pytest.raises(DemError) as e:
        Sim.from_scene(sc, precision=PREC_MIXED, arena=(arena.data_ptr() + 8, need - 8))
    assert e.value.code == -1


def test_contact_table_grows_inside_the_arena_or_fails_cleanly():
    import torch
    sc = gen.scene_cluster(seed=2, n_side=6, vel_sigma=0.2, polydisperse=True)
    # one contact slot per particle: the first step must grow the table
    need = footprint(_params_of(sc, PREC_MIXED, max_contacts=sc.n), sc.n)
    room = torch.empty(4 * need, dtype=torch.uint8, device="cuda")
    a = _run(sc, PREC_MIXED, 10, arena=room, max_contacts=sc.n)
    b = _run(sc, PREC_MIXED, 10, max_contacts=sc.n)
    _same(a, b)
    assert a[2]["regrows"] >= 1 and a[2]["device_bytes"] <= 4 * need
    tight = torch.empty(need, dtype=torch.uint8, device="cuda")
    g = Sim.from_scene(sc, precision=PREC_MIXED, arena=tight, max_contacts=sc.n)
    try:
        g.step(1)
        with pytest.raises(DemError) as e:
            g.sync()
        assert e.value.code == -3  # DEM_ECAPACITY: no room left to grow
    finally:
        g.close()


def test_pool_sized_by_budget_and_in_an_arena():
    import torch
    jobs = [SCENES["random3000"](), SCENES["materials"](), SCENES["cluster64"]()]
    budget = 64 << 20
    alone = [_run(sc, PREC_MIXED, 20) for sc in jobs]
    for use_arena in (False, True):
        arena = torch.empty(budget, dtype=torch.uint8, device="cuda") if use_arena else None
        pool = Pool(precision=PREC_MIXED, max_jobs=8, hbm_budget=0 if use_arena else budget,
                    arena=arena)
        try:
            assert pool_footprint(pool.params) <= budget
            ids = [pool.add_scene(sc, steps=20) for sc in jobs]
            pool.step(25)
            pool.sync()
            assert sorted(pool.poll()) == sorted(ids)
            for jid, ref in zip(ids, alone):
                st = pool.get_state(jid)
                for k in ("x", "v", "w"):
                    assert np.array_equal(st[k], ref[0][k]), k
        finally:
            pool.close()
