"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle's C source is built once more with both sanitizers and run in a
child process with the ASan runtime preloaded (the Python interpreter is not
instrumented).  The child steps small scenes that reach every code path of
a step: the cell list and the brute-force pair loop, box faces and extra
walls (rectangle and segment), periodic axes with a sheared y boundary,
several materials, and history carried over steps.  Any sanitizer report
aborts the child.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import numpy as np
import gen, oracle

def run(sc, steps, mode):
    s = oracle.Sim(sc, mode=mode, threads=2)
    s.step(steps, keep_contact_forces=True)
    assert np.isfinite(s.x).all() and np.isfinite(s.v).all() and np.isfinite(s.w).all()
    return s

# walled box, polydisperse, gravity, several materials: cell list and all pairs
sc = gen.scene_random(11, 300, phi=0.3, n_materials=3)
a, b = run(sc, 5, 1), run(sc, 5, 0)
assert np.array_equal(a.hist.i, b.hist.i) and np.array_equal(a.hist.j, b.hist.j)
# periodic on all axes with a Lees-Edwards boundary
run(gen.scene_random(12, 250, phi=0.3, walls=0, periodic=7, gravity=(0, 0, 0),
                     shear_rate=1e4), 5, 1)
# extra walls: a rectangle and a segment inside a walled box
sc = gen.scene_random(13, 200, phi=0.2)
L = float(sc.hi[0] - sc.lo[0])
sc.extra_walls = [gen.Wall(gen.RECT, (0.2 * L, 0.2 * L, 0.5 * L), (0.6 * L, 0, 0), (0, 0.6 * L, 0)),
                  gen.Wall(gen.SEGMENT, (0.1 * L, 0.5 * L, 0.3 * L), (0.8 * L, 0, 0))]
run(sc, 5, 1)
# the closed forms and the contact count of a few pairs
oracle.contacts(gen.scene_cluster(seed=4, n_side=3))
oracle.alpha(0.5)
print("sanitized oracle: ok")
"""


def _runtime(name):
    cc = shutil.which("gcc")
    if not cc:
        return None
    p = subprocess.run([cc, "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return p if p and os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(_runtime("libasan.so") is None, reason="gcc without the ASan runtime")
def test_oracle_runs_clean_under_asan_and_ubsan():
    sys.path.insert(0, ROOT)
    import oracle
    so = oracle.build_sanitized()
    env = dict(os.environ)
    env.update(DEM_ORACLE_SO=so, LD_PRELOAD=_runtime("libasan.so"),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               PYTHONPATH=ROOT + os.pathsep + env.get("PYTHONPATH", ""), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "sanitized oracle: ok" in r.stdout
