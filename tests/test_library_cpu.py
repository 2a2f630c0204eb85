"""Host-side checks of the C-ABI library (no GPU needed, no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1503_03553_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dem.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dem_[a-z_]+)\s*\(", src)))


def test_header_declares_exactly_the_binding_exports():
    assert declared_functions() == sorted(binding.EXPORTS)


def test_library_loads_and_exports_every_symbol():
    assert os.path.exists(binding.library_path()), "build libdem.so first"
    L = ctypes.CDLL(binding.library_path())
    for name in declared_functions():
        assert hasattr(L, name), name
    out = subprocess.check_output(["nm", "-D", "--defined-only", binding.library_path()]).decode()
    for name in declared_functions():
        assert re.search(r"\bT %s\b" % name, out), name


def test_status_strings_and_footprint_without_gpu():
    L = binding.lib()
    assert binding.status_str(0) == "ok"
    assert binding.status_str(-3) == "contact capacity exceeded"
    P = binding.make_params([0, 0, 0], [1e-3] * 3, precision=binding.PREC_MIXED)
    f1 = binding.footprint(P, 1000)
    f2 = binding.footprint(P, 1_000_000)
    assert 0 < f1 < f2
    assert L.dem_create(None, None, 0, 0, None, None, None, None, None, None, 0, None,
                        ctypes.byref(ctypes.c_void_p())) == -1


def test_ctypes_layouts_match_the_header(tmp_path):
    prog = tmp_path / "sizes.c"
    prog.write_text('#include "dem.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n",'
                    ' sizeof(dem_params), sizeof(dem_material), sizeof(dem_info),'
                    ' offsetof(dem_params, precision), offsetof(dem_params, max_contacts),'
                    ' offsetof(dem_info, cells), sizeof(dem_wall), offsetof(dem_wall, v),'
                    ' offsetof(dem_params, extra_walls));return 0;}\n')
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(binding.Params), ctypes.sizeof(binding.Material),
            ctypes.sizeof(binding.Info), binding.Params.precision.offset,
            binding.Params.max_contacts.offset, binding.Info.cells.offset,
            ctypes.sizeof(binding.Wall), binding.Wall.v.offset,
            binding.Params.extra_walls.offset]
    assert got == want


def test_pool_ctypes_layouts_match_the_header(tmp_path):
    prog = tmp_path / "psizes.c"
    prog.write_text('#include "dem.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(dem_pool_params),'
                    ' sizeof(dem_job_info), offsetof(dem_pool_params, precision),'
                    ' offsetof(dem_job_info, n), offsetof(dem_job_info, dt),'
                    ' offsetof(dem_pool_params, hbm_budget));return 0;}\n')
    exe = tmp_path / "psizes"
    subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(binding.PoolParams), ctypes.sizeof(binding.JobInfo),
            binding.PoolParams.precision.offset, binding.JobInfo.n.offset,
            binding.JobInfo.dt.offset, binding.PoolParams.hbm_budget.offset]
    assert got == want


def test_pool_footprint_and_argument_checks_without_gpu():
    L = binding.lib()
    pp = binding.make_pool_params(100_000, 400_000, 64, binding.PREC_MIXED)
    small = binding.make_pool_params(1_000, 4_096, 4, binding.PREC_MIXED)
    assert 0 < binding.pool_footprint(small) < binding.pool_footprint(pp)
    h = ctypes.c_void_p()
    assert L.dem_pool_create(None, None, 0, None, ctypes.byref(h)) == -1
    bad = binding.make_pool_params(1000, 4096, 0, binding.PREC_MIXED)  # no job slots
    assert L.dem_pool_create(ctypes.byref(bad), None, 0, None, ctypes.byref(h)) == -1
    bad = binding.make_pool_params(1000, 4096, 4, 7)  # unknown precision
    assert L.dem_pool_create(ctypes.byref(bad), None, 0, None, ctypes.byref(h)) == -1
    # neither capacities nor a budget
    bad = binding.make_pool_params(0, 0, 4, binding.PREC_MIXED)
    assert L.dem_pool_create(ctypes.byref(bad), None, 0, None, ctypes.byref(h)) == -1
    # a budget below the footprint of the given capacities
    bad = binding.make_pool_params(100_000, 400_000, 64, binding.PREC_MIXED,
                                   hbm_budget=binding.pool_footprint(pp) - 1)
    assert L.dem_pool_create(ctypes.byref(bad), None, 0, None, ctypes.byref(h)) == -1
    assert binding.status_str(-6) == "pool full"


def test_binding_raises_without_gpu_instead_of_falling_back():
    import gen
    from paper_1503_03553_amd import DemError, Sim
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    sc = gen.scene_cluster(seed=1, n_side=2)
    with pytest.raises(DemError):
        Sim.from_scene(sc)


def test_binding_constants_match_the_header():
    # flags, precisions, wall kinds and limits: every DEM_* integer constant
    # the header defines has the binding's value under the same name
    src = open(HEADER).read()
    defs = dict(re.findall(r"#define\s+DEM_([A-Z0-9_]+)\s+(0x[0-9a-fA-F]+|\d+)u?\b", src))
    names = {"FLAG_" + k[5:]: v for k, v in defs.items() if k.startswith("FLAG_")}
    assert {"FLAG_FUSED", "FLAG_ACTION_REACTION", "FLAG_THREAD_SPLIT",
            "FLAG_FULL_DETECT"} <= set(names)
    for name, v in names.items():
        assert getattr(binding, name) == int(v, 0), name


def test_budget_sized_pool_footprint_without_gpu():
    # with max_particles = 0 the pool takes the largest capacities whose
    # footprint fits the budget
    for budget in (64 << 20, 1 << 30, 20 << 30):
        pp = binding.make_pool_params(0, 0, 0, binding.PREC_MIXED, hbm_budget=budget)
        f = binding.pool_footprint(pp)
        assert 0.9 * budget < f <= budget
        pp64 = binding.make_pool_params(0, 0, 0, binding.PREC_FP64, hbm_budget=budget)
        assert 0.9 * budget < binding.pool_footprint(pp64) <= budget
    tiny = binding.make_pool_params(0, 0, 0, binding.PREC_MIXED, hbm_budget=4096)
    assert binding.pool_footprint(tiny) == 0  # not even one tile fits


def test_job_prepare_rejects_positions_outside_a_periodic_box():
    # a position beyond [lo, hi] along a periodic axis would be clamped into a
    # border cell whose stencil misses the partners of its periodic image
    import numpy as np
    import gen
    from paper_1503_03553_amd import DemError, PREC_MIXED
    from paper_1503_03553_amd.binding import PreparedJob
    sc = gen.scene_random(seed=22, n=300, phi=0.2, p_touch=0.5, walls=0, periodic=7,
                          gravity=(0, 0, 0))
    PreparedJob.from_scene(sc, PREC_MIXED).close()
    L = sc.hi[0] - sc.lo[0]
    for a in range(3):
        bad = sc.copy()
        bad.x[5, a] = sc.hi[a] + 1e-3 * L
        with pytest.raises(DemError):
            PreparedJob.from_scene(bad, PREC_MIXED)
    edge = sc.copy()
    edge.x[5, 0] = sc.hi[0]  # on the boundary itself: accepted
    PreparedJob.from_scene(edge, PREC_MIXED).close()
    walled = sc.copy()
    walled.periodic, walled.walls = 0, gen.WALL_ALL
    walled.x[5, 0] = sc.hi[0] + 1e-3 * L  # no periodic axis: a wall pushes it back
    PreparedJob.from_scene(walled, PREC_MIXED).close()
