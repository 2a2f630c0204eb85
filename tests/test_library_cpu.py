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
    assert L.dem_create(None, None, 0, 0, None, None, None, None, None, None,
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
                    'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(dem_pool_params),'
                    ' sizeof(dem_job_info), offsetof(dem_pool_params, precision),'
                    ' offsetof(dem_job_info, n), offsetof(dem_job_info, dt));return 0;}\n')
    exe = tmp_path / "psizes"
    subprocess.check_call(["gcc", "-I" + os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(binding.PoolParams), ctypes.sizeof(binding.JobInfo),
            binding.PoolParams.precision.offset, binding.JobInfo.n.offset,
            binding.JobInfo.dt.offset]
    assert got == want


def test_pool_footprint_and_argument_checks_without_gpu():
    L = binding.lib()
    pp = binding.make_pool_params(100_000, 400_000, 64, binding.PREC_MIXED)
    small = binding.make_pool_params(1_000, 4_096, 4, binding.PREC_MIXED)
    assert 0 < binding.pool_footprint(small) < binding.pool_footprint(pp)
    h = ctypes.c_void_p()
    assert L.dem_pool_create(None, None, ctypes.byref(h)) == -1
    bad = binding.make_pool_params(1000, 4096, 0, binding.PREC_MIXED)  # no job slots
    assert L.dem_pool_create(ctypes.byref(bad), None, ctypes.byref(h)) == -1
    bad = binding.make_pool_params(1000, 4096, 4, 7)  # unknown precision
    assert L.dem_pool_create(ctypes.byref(bad), None, ctypes.byref(h)) == -1
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
