"""The grazing-pair scene (tests/grazing.py) has the property the GPU
regression test relies on, and the oracle handles it: every pair is in the
contact set, with a non-negative overlap and finite forces."""
import numpy as np

import oracle
from grazing import grazing_scene, is_grazing


def test_grazing_pairs_touch_by_rounding_only():
    sc = grazing_scene(seed=3, npairs=16)
    s = float(sc.r[0] + sc.r[1])
    for k in range(16):
        assert is_grazing(sc.x[2 * k], sc.x[2 * k + 1], s)
    i, j = oracle.contacts(sc, mode=0)
    want = sorted([(2 * k, 2 * k + 1) for k in range(16)] + [(2 * k + 1, 2 * k) for k in range(16)])
    assert sorted(zip(i.tolist(), j.tolist())) == want
    o = oracle.Sim(sc, mode=0)
    o.step(keep_contact_forces=True)
    assert np.isfinite(o.cF).all() and np.isfinite(o.x).all() and np.isfinite(o.v).all()
