"""FP64 CPU oracle of the DEM step (ctypes shim over oracle/dem_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the simulator package.  It shares no
code with the GPU path; both sides only share the seeded input generators in
gen/.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_LIB = None
MAXMAT = 8
FACE_ID = 0xFFFFFFF0  # partner id of box face f is FACE_ID + f
MAX_WALLS = 10        # extra wall k has partner id FACE_ID + 6 + k


def build(force: bool = False) -> str:
    src = os.path.join(_HERE, "dem_oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class Wall(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("pad", ctypes.c_int32), ("p", ctypes.c_double * 3),
                ("u", ctypes.c_double * 3), ("v", ctypes.c_double * 3)]


class Params(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("walls", ctypes.c_uint32), ("periodic", ctypes.c_uint32),
                ("gravity", ctypes.c_double * 3), ("shear_rate", ctypes.c_double),
                ("time", ctypes.c_double), ("dt", ctypes.c_double),
                ("kn_form", ctypes.c_int32), ("n_mats", ctypes.c_int32),
                ("E", ctypes.c_double * MAXMAT), ("poisson", ctypes.c_double * MAXMAT),
                ("G", ctypes.c_double * MAXMAT), ("density", ctypes.c_double * MAXMAT),
                ("restitution", ctypes.c_double * MAXMAT), ("mu", ctypes.c_double * MAXMAT),
                ("n_extra", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("extra", Wall * MAX_WALLS)]


_P = ctypes.POINTER(Params)
_vp = ctypes.c_void_p


def build_sanitized() -> str:
    """The same source built with AddressSanitizer and UndefinedBehaviorSanitizer
    (for tests that run the oracle under them: load it with DEM_ORACLE_SO set to
    the returned path, libasan preloaded)."""
    src = os.path.join(_HERE, "dem_oracle.c")
    so = os.path.join(_HERE, "liboracle_san.so")
    if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        tmp = so + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined",
                               "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                               "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared",
                               "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, so)
    return so


def lib():
    global _LIB
    if _LIB is None:
        L = ctypes.CDLL(os.environ.get("DEM_ORACLE_SO") or build())
        L.orc_alpha.restype = ctypes.c_double
        L.orc_alpha.argtypes = [ctypes.c_double]
        L.orc_mass.restype = ctypes.c_double
        L.orc_mass.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_kn.restype = ctypes.c_double
        L.orc_kn.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.orc_kt.restype = ctypes.c_double
        L.orc_kt.argtypes = [_P, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double]
        L.orc_contact_time.restype = ctypes.c_double
        L.orc_contact_time.argtypes = [ctypes.c_double] * 3
        L.orc_dt_rule.restype = ctypes.c_double
        L.orc_dt_rule.argtypes = [_P, ctypes.c_long, _vp, _vp]
        L.orc_le_offset.restype = ctypes.c_double
        L.orc_le_offset.argtypes = [_P, ctypes.c_double]
        L.orc_contacts.restype = ctypes.c_long
        L.orc_contacts.argtypes = [_P, ctypes.c_long, _vp, _vp, ctypes.c_int, ctypes.c_long, _vp, _vp]
        L.orc_pair.restype = None
        L.orc_pair.argtypes = [_P, _vp, _vp, _vp, ctypes.c_double, ctypes.c_int, _vp, _vp, _vp,
                               ctypes.c_double, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp,
                               _vp, _vp]
        L.orc_step.restype = ctypes.c_int
        L.orc_step.argtypes = [_P, ctypes.c_long, _vp, _vp, _vp, _vp, _vp, ctypes.c_long, _vp,
                               _vp, _vp, ctypes.c_long, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                               _vp, ctypes.c_int, ctypes.c_int]
        _LIB = L
    return _LIB


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def params(scene, time=0.0, dt=None) -> Params:
    P = Params()
    for a in range(3):
        P.lo[a] = float(scene.lo[a])
        P.hi[a] = float(scene.hi[a])
        P.gravity[a] = float(scene.gravity[a])
    P.walls = int(scene.walls)
    P.periodic = int(scene.periodic)
    P.shear_rate = float(scene.shear_rate)
    P.time = float(time)
    P.kn_form = int(scene.kn_form)
    P.n_mats = len(scene.materials)
    assert 1 <= P.n_mats <= MAXMAT
    for k, m in enumerate(scene.materials):
        P.E[k], P.poisson[k], P.G[k] = m.E, m.poisson, m.G
        P.density[k], P.restitution[k], P.mu[k] = m.density, m.restitution, m.mu
    walls = list(getattr(scene, "extra_walls", []) or [])
    assert len(walls) <= MAX_WALLS
    P.n_extra = len(walls)
    for k, wl in enumerate(walls):
        P.extra[k].kind = int(wl.kind)
        for a in range(3):
            P.extra[k].p[a] = float(wl.p[a])
            P.extra[k].u[a] = float(wl.u[a])
            P.extra[k].v[a] = float(wl.v[a])
    if dt is None:
        dt = scene.dt if scene.dt else dt_rule(scene, P)
    P.dt = float(dt)
    return P


def alpha(eps: float) -> float:
    return lib().orc_alpha(float(eps))


def mass(rho, r):
    return lib().orc_mass(float(rho), float(r))


def kn(P, mi, mj, ri, rj):
    return lib().orc_kn(ctypes.byref(P), mi, mj, float(ri), float(rj))


def kt(P, mi, mj, ri, rj, dn):
    return lib().orc_kt(ctypes.byref(P), mi, mj, float(ri), float(rj), float(dn))


def contact_time(mstar, kn_, v0):
    return lib().orc_contact_time(float(mstar), float(kn_), float(v0))


def dt_rule(scene, P=None) -> float:
    if P is None:
        P = params(scene, dt=1.0)
    r = _c(scene.r, np.float64)
    mat = _c(scene.mat, np.uint16)
    return lib().orc_dt_rule(ctypes.byref(P), r.shape[0], r.ctypes.data, mat.ctypes.data)


def le_offset(P, t):
    return lib().orc_le_offset(ctypes.byref(P), float(t))


def contacts(scene, x=None, mode=1, time=0.0):
    """Contact set as two uint32 arrays (i, j), sorted by (i, j)."""
    P = params(scene, time=time, dt=1.0)
    x = _c(scene.x if x is None else x, np.float64)
    r = _c(scene.r, np.float64)
    n = r.shape[0]
    cap = max(64, 16 * n)
    oi = np.zeros(cap, np.uint32)
    oj = np.zeros(cap, np.uint32)
    m = lib().orc_contacts(ctypes.byref(P), n, x.ctypes.data, r.ctypes.data, mode, cap,
                           oi.ctypes.data, oj.ctypes.data)
    if m < 0:
        raise RuntimeError("orc_contacts failed (%d)" % m)
    return oi[:m].copy(), oj[:m].copy()


def pair(P, xi, vi, wi, ri, mi, xj=None, vj=None, wj=None, rj=0.0, mj=0, face=-1, dt_old=(0, 0, 0)):
    """Force, torque, new tangential displacement, overlap, capped flag of one contact on i."""
    z = np.zeros(3)
    xi, vi, wi = _c(xi, np.float64), _c(vi, np.float64), _c(wi, np.float64)
    xj = _c(z if xj is None else xj, np.float64)
    vj = _c(z if vj is None else vj, np.float64)
    wj = _c(z if wj is None else wj, np.float64)
    dto = _c(dt_old, np.float64)
    F, T, dtn = np.zeros(3), np.zeros(3), np.zeros(3)
    dn = ctypes.c_double()
    cap = ctypes.c_int()
    lib().orc_pair(ctypes.byref(P), xi.ctypes.data, vi.ctypes.data, wi.ctypes.data, float(ri), mi,
                   xj.ctypes.data, vj.ctypes.data, wj.ctypes.data, float(rj), mj, face,
                   dto.ctypes.data, F.ctypes.data, T.ctypes.data, dtn.ctypes.data,
                   ctypes.addressof(dn), ctypes.addressof(cap))
    return F, T, dtn, dn.value, bool(cap.value)


class History:
    """Pair history: (i, j) sorted, tangential displacement per directed contact."""

    def __init__(self, i=None, j=None, dt=None):
        self.i = np.zeros(0, np.uint32) if i is None else _c(i, np.uint32)
        self.j = np.zeros(0, np.uint32) if j is None else _c(j, np.uint32)
        self.dt = np.zeros((0, 3)) if dt is None else _c(dt, np.float64).reshape(-1, 3)

    def __len__(self):
        return int(self.i.shape[0])

    def as_dict(self):
        return {(int(a), int(b)): self.dt[k] for k, (a, b) in enumerate(zip(self.i, self.j))}


class Sim:
    """A plain oracle simulation: state, history, time; `step()` advances one step."""

    def __init__(self, scene, dt=None, mode=1, threads=0):
        self.scene = scene
        self.x = _c(scene.x, np.float64).copy()
        self.v = _c(scene.v, np.float64).copy()
        self.w = _c(scene.w, np.float64).copy()
        self.r = _c(scene.r, np.float64)
        self.mat = _c(scene.mat, np.uint16)
        self.time = 0.0
        self.P = params(scene, time=0.0, dt=dt)
        self.dt = self.P.dt
        self.hist = History()
        self.mode = mode
        self.threads = threads
        self.F = np.zeros_like(self.x)
        self.T = np.zeros_like(self.x)
        self.cF = None
        self.cT = None
        # per contact: |F_t| before the cap, mu |F_n|, rounding scale of the
        # sliding test, sum of the magnitudes of the terms of Eq. (1), k_t
        self.cQ = None

    def step(self, k=1, keep_contact_forces=False):
        n = self.r.shape[0]
        for _ in range(k):
            self.P.time = self.time
            cap = max(64, 2 * len(self.hist) + 16 * n)
            oi = np.zeros(cap, np.uint32)
            oj = np.zeros(cap, np.uint32)
            odt = np.zeros((cap, 3))
            cF = np.zeros((cap, 3)) if keep_contact_forces else None
            cT = np.zeros((cap, 3)) if keep_contact_forces else None
            cQ = np.zeros((cap, 5)) if keep_contact_forces else None
            m = ctypes.c_long()
            h = self.hist
            rc = lib().orc_step(ctypes.byref(self.P), n, self.x.ctypes.data, self.v.ctypes.data,
                                self.w.ctypes.data, self.r.ctypes.data, self.mat.ctypes.data,
                                len(h), h.i.ctypes.data, h.j.ctypes.data, h.dt.ctypes.data, cap,
                                ctypes.addressof(m), oi.ctypes.data, oj.ctypes.data,
                                odt.ctypes.data, self.F.ctypes.data, self.T.ctypes.data,
                                None if cF is None else cF.ctypes.data,
                                None if cT is None else cT.ctypes.data,
                                None if cQ is None else cQ.ctypes.data, self.mode, self.threads)
            if rc != 0:
                raise RuntimeError("orc_step failed (%d)" % rc)
            mm = m.value
            self.hist = History(oi[:mm].copy(), oj[:mm].copy(), odt[:mm].copy())
            if keep_contact_forces:
                self.cF, self.cT, self.cQ = cF[:mm].copy(), cT[:mm].copy(), cQ[:mm].copy()
            self.time = self.time + self.dt
        return self
