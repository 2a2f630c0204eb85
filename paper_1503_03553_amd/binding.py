"""ctypes binding of libdem.so with the names of include/dem.h.

Argument marshalling only: every step of the simulation runs in the HIP
library.  PyTorch is used, when given, only to supply the HIP stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libdem.so")

DEM_FACE_ID = 0xFFFFFFF0
MAX_MATERIALS = 8
PREC_FP64 = 0
PREC_MIXED = 1
FLAG_NO_FORCE_OUTPUT = 1
FLAG_RADIX_SORT = 2
FLAG_FUSED = 4
FLAG_ACTION_REACTION = 8
FLAG_THREAD_SPLIT = 16
FLAG_FULL_DETECT = 32
NPHASE = 4
PHASES = ("detect", "force", "sort", "reorder")

STATUS = {0: "DEM_OK", -1: "DEM_EINVAL", -2: "DEM_ENOMEM", -3: "DEM_ECAPACITY",
          -4: "DEM_ENONFINITE", -5: "DEM_EDEVICE", -6: "DEM_EBUSY", -7: "DEM_ESCRATCH"}
STATIC_BYTES = 64 << 20  # DEM_STATIC_BYTES

# every symbol include/dem.h declares
EXPORTS = ("dem_create", "dem_create_static", "dem_step", "dem_sync", "dem_get_state",
           "dem_get_contacts",
           "dem_set_contacts", "dem_set_state", "dem_set_radii", "dem_get_info", "dem_destroy",
           "dem_status_str",
           "dem_footprint", "dem_profile", "dem_profile_read", "dem_pool_footprint",
           "dem_pool_create", "dem_pool_add", "dem_pool_step", "dem_pool_sync", "dem_pool_poll",
           "dem_pool_job_info", "dem_pool_get_state", "dem_pool_remove", "dem_pool_capacity",
           "dem_job_cells", "dem_job_prepare", "dem_job_prep_cells", "dem_pool_add_prepared",
           "dem_pool_set_radii",
           "dem_job_prep_free",
           "dem_pool_profile", "dem_pool_profile_read", "dem_pool_destroy")

JOB_RUNNING, JOB_DONE, JOB_FAILED = 0, 1, 2
JOB_STATUS = {JOB_RUNNING: "running", JOB_DONE: "done", JOB_FAILED: "failed"}


class DemError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, STATUS.get(code, "?"), code))


class Material(ctypes.Structure):
    _fields_ = [("E", ctypes.c_double), ("poisson", ctypes.c_double), ("G", ctypes.c_double),
                ("density", ctypes.c_double), ("restitution", ctypes.c_double),
                ("mu", ctypes.c_double)]


class Wall(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_uint32),
                ("p", ctypes.c_double * 3), ("u", ctypes.c_double * 3), ("v", ctypes.c_double * 3)]


class Params(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("walls", ctypes.c_uint32), ("periodic", ctypes.c_uint32),
                ("gravity", ctypes.c_double * 3), ("shear_rate", ctypes.c_double),
                ("dt", ctypes.c_double), ("time", ctypes.c_double),
                ("precision", ctypes.c_int32), ("kn_form", ctypes.c_int32),
                ("cell_size", ctypes.c_double), ("max_contacts", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("n_extra_walls", ctypes.c_uint32),
                ("extra_walls", ctypes.c_void_p), ("radius_cut", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("steps_done", ctypes.c_uint64), ("dt", ctypes.c_double),
                ("time", ctypes.c_double), ("contacts", ctypes.c_uint64),
                ("capacity", ctypes.c_uint64), ("regrows", ctypes.c_uint64),
                ("sum_contacts", ctypes.c_uint64), ("sum_matched", ctypes.c_uint64),
                ("sum_old", ctypes.c_uint64), ("cells", ctypes.c_uint32 * 3),
                ("key_bits", ctypes.c_uint32), ("device_bytes", ctypes.c_uint64),
                ("radius_cut", ctypes.c_double), ("big", ctypes.c_uint64)]


class PoolParams(ctypes.Structure):
    _fields_ = [("max_particles", ctypes.c_uint64), ("max_cells", ctypes.c_uint64),
                ("max_jobs", ctypes.c_uint32), ("precision", ctypes.c_int32),
                ("contact_slots", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("hbm_budget", ctypes.c_uint64)]


class JobInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("reserved", ctypes.c_uint32), ("n", ctypes.c_uint64),
                ("steps_done", ctypes.c_uint64), ("steps_left", ctypes.c_uint64),
                ("time", ctypes.c_double), ("dt", ctypes.c_double)]


_LIB = None
_vp = ctypes.c_void_p


def library_path() -> str:
    return _SO


def lib():
    """Load libdem.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        # PyTorch ships its own HIP and HSA runtimes under the sonames of
        # ROCm's.  Loaded first, they are the ones libdem.so binds to, so the
        # process has one runtime and torch's device memory and streams are
        # valid handles for the library; loaded after libdem.so, torch would
        # bring a second HSA runtime that cannot open the GPU.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(_SO):
            raise RuntimeError("libdem.so not found at %s; run __graft_entry__.build() or "
                               "python paper_1503_03553_amd/build.py" % _SO)
        L = ctypes.CDLL(_SO)
        P = ctypes.POINTER(Params)
        L.dem_create.restype = ctypes.c_int
        L.dem_create.argtypes = [P, _vp, ctypes.c_uint32, ctypes.c_uint64, _vp, _vp, _vp, _vp, _vp,
                                 _vp, ctypes.c_uint64, _vp, ctypes.POINTER(_vp)]
        L.dem_create_static.restype = ctypes.c_int
        L.dem_create_static.argtypes = [P, _vp, ctypes.c_uint32, ctypes.c_uint64, _vp, _vp, _vp,
                                        _vp, _vp, _vp, ctypes.POINTER(_vp)]
        L.dem_step.restype = ctypes.c_int
        L.dem_step.argtypes = [_vp, ctypes.c_uint32]
        L.dem_sync.restype = ctypes.c_int
        L.dem_sync.argtypes = [_vp]
        L.dem_get_state.restype = ctypes.c_int
        L.dem_get_state.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
        L.dem_get_contacts.restype = ctypes.c_int
        L.dem_get_contacts.argtypes = [_vp, ctypes.c_uint64, _vp, _vp, _vp,
                                       ctypes.POINTER(ctypes.c_uint64)]
        L.dem_set_contacts.restype = ctypes.c_int
        L.dem_set_contacts.argtypes = [_vp, ctypes.c_uint64, _vp, _vp, _vp]
        L.dem_set_state.restype = ctypes.c_int
        L.dem_set_state.argtypes = [_vp, _vp, _vp, _vp]
        L.dem_set_radii.restype = ctypes.c_int
        L.dem_set_radii.argtypes = [_vp, _vp]
        L.dem_get_info.restype = ctypes.c_int
        L.dem_get_info.argtypes = [_vp, ctypes.POINTER(Info)]
        L.dem_destroy.restype = None
        L.dem_destroy.argtypes = [_vp]
        L.dem_status_str.restype = ctypes.c_char_p
        L.dem_status_str.argtypes = [ctypes.c_int]
        L.dem_footprint.restype = ctypes.c_uint64
        L.dem_footprint.argtypes = [P, ctypes.c_uint64]
        L.dem_profile.restype = ctypes.c_int
        L.dem_profile.argtypes = [_vp, ctypes.c_int]
        L.dem_profile_read.restype = ctypes.c_int
        L.dem_profile_read.argtypes = [_vp, _vp, _vp]
        PP = ctypes.POINTER(PoolParams)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.dem_pool_footprint.restype = ctypes.c_uint64
        L.dem_pool_footprint.argtypes = [PP]
        L.dem_pool_create.restype = ctypes.c_int
        L.dem_pool_create.argtypes = [PP, _vp, ctypes.c_uint64, _vp, ctypes.POINTER(_vp)]
        L.dem_pool_add.restype = ctypes.c_int
        L.dem_pool_add.argtypes = [_vp, P, _vp, ctypes.c_uint32, ctypes.c_uint64, _vp, _vp, _vp,
                                   _vp, _vp, ctypes.c_uint32, u64p]
        L.dem_pool_step.restype = ctypes.c_int
        L.dem_pool_step.argtypes = [_vp, ctypes.c_uint32]
        L.dem_pool_sync.restype = ctypes.c_int
        L.dem_pool_sync.argtypes = [_vp]
        L.dem_pool_poll.restype = ctypes.c_int
        L.dem_pool_poll.argtypes = [_vp, _vp, ctypes.c_uint32, u32p]
        L.dem_pool_job_info.restype = ctypes.c_int
        L.dem_pool_job_info.argtypes = [_vp, ctypes.c_uint64, ctypes.POINTER(JobInfo)]
        L.dem_pool_get_state.restype = ctypes.c_int
        L.dem_pool_get_state.argtypes = [_vp, ctypes.c_uint64, _vp, _vp, _vp]
        L.dem_pool_set_radii.restype = ctypes.c_int
        L.dem_pool_set_radii.argtypes = [_vp, ctypes.c_uint64, _vp]
        L.dem_pool_remove.restype = ctypes.c_int
        L.dem_pool_remove.argtypes = [_vp, ctypes.c_uint64]
        L.dem_pool_capacity.restype = ctypes.c_int
        L.dem_pool_capacity.argtypes = [_vp, u64p, u64p, u32p]
        L.dem_job_prepare.restype = ctypes.c_int
        L.dem_job_prepare.argtypes = [P, _vp, ctypes.c_uint32, ctypes.c_uint64, _vp, _vp, _vp, _vp,
                                      _vp, ctypes.POINTER(_vp)]
        L.dem_job_prep_cells.restype = ctypes.c_uint64
        L.dem_job_prep_cells.argtypes = [_vp]
        L.dem_pool_add_prepared.restype = ctypes.c_int
        L.dem_pool_add_prepared.argtypes = [_vp, _vp, ctypes.c_uint32, u64p]
        L.dem_job_prep_free.restype = None
        L.dem_job_prep_free.argtypes = [_vp]
        L.dem_job_cells.restype = ctypes.c_uint64
        L.dem_job_cells.argtypes = [P, ctypes.c_uint64, ctypes.c_double]
        L.dem_pool_profile.restype = ctypes.c_int
        L.dem_pool_profile.argtypes = [_vp, ctypes.c_int]
        L.dem_pool_profile_read.restype = ctypes.c_int
        L.dem_pool_profile_read.argtypes = [_vp, _vp, _vp]
        L.dem_pool_destroy.restype = None
        L.dem_pool_destroy.argtypes = [_vp]
        _LIB = L
    return _LIB


def status_str(code: int) -> str:
    return lib().dem_status_str(code).decode()


def _check(code, what):
    if code != 0:
        raise DemError(code, what)


def _c(a, dtype, shape=None):
    a = np.ascontiguousarray(a, dtype=dtype)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _arena_handle(arena):
    """(device pointer, bytes) of a lent device arena: a torch tensor on the
    GPU (any dtype, contiguous) or a (pointer, bytes) pair; None for none."""
    if arena is None:
        return None, 0
    if isinstance(arena, tuple):
        return int(arena[0]), int(arena[1])
    if not arena.is_cuda or not arena.is_contiguous():
        raise ValueError("the arena must be a contiguous tensor on the GPU")
    return int(arena.data_ptr()), int(arena.numel() * arena.element_size())


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


def make_params(lo, hi, walls=0x3F, periodic=0, gravity=(0.0, 0.0, -9.81), shear_rate=0.0,
                dt=0.0, time=0.0, precision=PREC_FP64, kn_form=0, cell_size=0.0, max_contacts=0,
                flags=0, extra_walls=(), radius_cut=0.0) -> Params:
    """dem_params; extra_walls holds objects with kind, p, u, v (e.g. gen.Wall),
    kept alive by the returned structure."""
    P = Params()
    for a in range(3):
        P.lo[a] = float(lo[a])
        P.hi[a] = float(hi[a])
        P.gravity[a] = float(gravity[a])
    P.walls = int(walls)
    P.periodic = int(periodic)
    P.shear_rate = float(shear_rate)
    P.dt = float(dt)
    P.time = float(time)
    P.precision = int(precision)
    P.kn_form = int(kn_form)
    P.cell_size = float(cell_size)
    P.max_contacts = int(max_contacts)
    P.flags = int(flags)
    P.radius_cut = float(radius_cut)
    ws = list(extra_walls or ())
    arr = (Wall * max(1, len(ws)))()
    for k, wl in enumerate(ws):
        arr[k].kind = int(wl.kind)
        for a in range(3):
            arr[k].p[a] = float(wl.p[a])
            arr[k].u[a] = float(wl.u[a])
            arr[k].v[a] = float(wl.v[a])
    P._walls = arr
    P.n_extra_walls = len(ws)
    P.extra_walls = ctypes.addressof(arr) if ws else None
    return P


def footprint(params: Params, n: int) -> int:
    return int(lib().dem_footprint(ctypes.byref(params), int(n)))


class Sim:
    """One simulation on the GPU (dem_create ... dem_destroy)."""

    def __init__(self, lo, hi, x, v, w, r, materials, mat=None, walls=0x3F, periodic=0,
                 gravity=(0.0, 0.0, -9.81), shear_rate=0.0, dt=0.0, time=0.0,
                 precision=PREC_FP64, kn_form=0, cell_size=0.0, max_contacts=0, flags=0,
                 stream=None, extra_walls=(), arena=None, static=False, radius_cut=0.0):
        """arena: device memory lent for every device buffer of the simulation
        (a torch tensor on the GPU, or (pointer, bytes)); it must hold at least
        footprint(params, n) bytes and is kept referenced by the handle.
        static: create with dem_create_static (no device allocation; the
        library's static scratch of STATIC_BYTES, one such simulation per
        device at a time); not with an arena."""
        if static and arena is not None:
            raise ValueError("a static simulation takes no arena")
        L = lib()
        self.params = make_params(lo, hi, walls, periodic, gravity, shear_rate, dt, time,
                                  precision, kn_form, cell_size, max_contacts, flags, extra_walls,
                                  radius_cut)
        x = _c(x, np.float64, (-1, 3))
        n = x.shape[0]
        v = _c(v, np.float64, (n, 3))
        w = _c(w, np.float64, (n, 3))
        r32 = _c(r, np.float32, (n,))
        mats = (Material * len(materials))()
        for k, m in enumerate(materials):
            mats[k] = Material(m.E, m.poisson, m.G, m.density, m.restitution, m.mu)
        mat16 = None if mat is None else _c(mat, np.uint16, (n,))
        self.n = n
        self._h = _vp()
        self._arena = arena  # a lent arena must outlive the handle
        aptr, abytes = _arena_handle(arena)
        self._keep = (x, v, w, r32, mats, mat16)
        m16 = None if mat16 is None else mat16.ctypes.data
        if static:
            code = L.dem_create_static(ctypes.byref(self.params), ctypes.cast(mats, _vp),
                                       len(materials), n, x.ctypes.data, v.ctypes.data,
                                       w.ctypes.data, r32.ctypes.data, m16,
                                       _stream_handle(stream), ctypes.byref(self._h))
        else:
            code = L.dem_create(ctypes.byref(self.params), ctypes.cast(mats, _vp), len(materials),
                                n, x.ctypes.data, v.ctypes.data, w.ctypes.data, r32.ctypes.data,
                                m16, aptr, abytes, _stream_handle(stream), ctypes.byref(self._h))
        self._keep = None
        _check(code, "dem_create_static" if static else "dem_create")

    @classmethod
    def from_scene(cls, sc, precision=PREC_FP64, **kw):
        """Build from any object with the attributes of gen.Scene."""
        args = dict(lo=sc.lo, hi=sc.hi, x=sc.x, v=sc.v, w=sc.w, r=sc.r, materials=sc.materials,
                    mat=sc.mat if len(sc.materials) > 1 else None, walls=sc.walls,
                    periodic=sc.periodic, gravity=sc.gravity, shear_rate=sc.shear_rate, dt=sc.dt,
                    kn_form=sc.kn_form, precision=precision,
                    extra_walls=getattr(sc, "extra_walls", ()))
        args.update(kw)
        return cls(**args)

    # -------------------------------------------------------------- calls
    def _handle(self):
        if not self._h:
            raise RuntimeError("simulation destroyed")
        return self._h

    def step(self, k=1):
        _check(lib().dem_step(self._handle(), int(k)), "dem_step")
        return self

    def sync(self):
        _check(lib().dem_sync(self._handle()), "dem_sync")
        return self

    def get_state(self, forces=True):
        n = self.n
        x, v, w = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 3))
        F = np.zeros((n, 3)) if forces else None
        T = np.zeros((n, 3)) if forces else None
        code = lib().dem_get_state(self._handle(), x.ctypes.data, v.ctypes.data, w.ctypes.data,
                                   None if F is None else F.ctypes.data,
                                   None if T is None else T.ctypes.data)
        _check(code, "dem_get_state")
        return dict(x=x, v=v, w=w, F=F, T=T)

    def get_contacts(self):
        m = ctypes.c_uint64()
        _check(lib().dem_get_contacts(self._handle(), 0, None, None, None, ctypes.byref(m)),
               "dem_get_contacts")
        k = m.value
        i = np.zeros(max(k, 1), np.uint32)
        j = np.zeros(max(k, 1), np.uint32)
        dt = np.zeros((max(k, 1), 3))
        _check(lib().dem_get_contacts(self._handle(), k, i.ctypes.data, j.ctypes.data,
                                      dt.ctypes.data, ctypes.byref(m)), "dem_get_contacts")
        return i[:k], j[:k], dt[:k]

    def set_contacts(self, i, j, dt):
        i = _c(i, np.uint32)
        j = _c(j, np.uint32)
        dt = _c(dt, np.float64, (-1, 3))
        _check(lib().dem_set_contacts(self._handle(), i.shape[0], i.ctypes.data, j.ctypes.data,
                                      dt.ctypes.data), "dem_set_contacts")

    def set_state(self, x, v, w):
        x = _c(x, np.float64, (self.n, 3))
        v = _c(v, np.float64, (self.n, 3))
        w = _c(w, np.float64, (self.n, 3))
        _check(lib().dem_set_state(self._handle(), x.ctypes.data, v.ctypes.data, w.ctypes.data),
               "dem_set_state")

    def set_radii(self, r):
        """New radii (pid order), rounded to FP32; state and history kept."""
        r32 = _c(r, np.float32, (self.n,))
        _check(lib().dem_set_radii(self._handle(), r32.ctypes.data), "dem_set_radii")

    def info(self) -> dict:
        inf = Info()
        _check(lib().dem_get_info(self._handle(), ctypes.byref(inf)), "dem_get_info")
        out = {f: getattr(inf, f) for f, _ in Info._fields_}
        out["cells"] = tuple(inf.cells)
        return out

    def profile(self, enable=True):
        _check(lib().dem_profile(self._handle(), 1 if enable else 0), "dem_profile")

    def profile_read(self) -> dict:
        ms = np.zeros(NPHASE)
        cnt = np.zeros(NPHASE, np.uint64)
        _check(lib().dem_profile_read(self._handle(), ms.ctypes.data, cnt.ctypes.data),
               "dem_profile_read")
        return {p: (float(ms[k]), int(cnt[k])) for k, p in enumerate(PHASES)}

    def close(self):
        if self._h:
            lib().dem_destroy(self._h)
            self._h = _vp()
        self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def make_pool_params(max_particles, max_cells, max_jobs, precision=PREC_MIXED, contact_slots=0,
                     flags=0, hbm_budget=0) -> PoolParams:
    pp = PoolParams()
    pp.hbm_budget = int(hbm_budget)
    pp.max_particles = int(max_particles)
    pp.max_cells = int(max_cells)
    pp.max_jobs = int(max_jobs)
    pp.precision = int(precision)
    pp.contact_slots = int(contact_slots)
    pp.flags = int(flags)
    return pp


def pool_footprint(pp: PoolParams) -> int:
    return int(lib().dem_pool_footprint(ctypes.byref(pp)))


def job_cells(sc, cell_size=0.0) -> int:
    """Cells a job of this scene takes from a pool (dem_job_cells)."""
    P = make_params(sc.lo, sc.hi, sc.walls, sc.periodic, sc.gravity, sc.shear_rate, sc.dt,
                    0.0, PREC_MIXED, sc.kn_form, cell_size)
    rmax = float(np.max(np.asarray(sc.r, np.float32))) if len(sc.r) else 0.0
    if rmax <= 0.0:
        rmax = float(np.min(np.asarray(sc.hi) - np.asarray(sc.lo))) / 6.1
    return int(lib().dem_job_cells(ctypes.byref(P), int(len(sc.r)), rmax))


def job_fits(sc, cap, cell_size=0.0) -> bool:
    """Whether a scene fits the free capacity `cap` (dict of Pool.capacity)."""
    n = int(len(sc.r))
    tiles = (n + 127) // 128
    c = job_cells(sc, cell_size)
    return c > 0 and tiles * 128 <= cap["particles"] and c <= cap["cells"]


class PreparedJob:
    """A job validated and placed in cell order on the host (dem_job_prepare),
    waiting for admission into a pool; safe to create on another thread."""

    def __init__(self, lo, hi, x, v, w, r, materials, precision, mat=None, walls=0x3F,
                 periodic=0, gravity=(0.0, 0.0, -9.81), shear_rate=0.0, dt=0.0, time=0.0,
                 kn_form=0, cell_size=0.0, extra_walls=(), radius_cut=0.0):
        P = make_params(lo, hi, walls, periodic, gravity, shear_rate, dt, time, precision,
                        kn_form, cell_size, extra_walls=extra_walls, radius_cut=radius_cut)
        x = _c(x, np.float64, (-1, 3))
        n = x.shape[0]
        v = _c(v, np.float64, (n, 3))
        w = _c(w, np.float64, (n, 3))
        r32 = _c(r, np.float32, (n,))
        mats = (Material * len(materials))()
        for k, m in enumerate(materials):
            mats[k] = Material(m.E, m.poisson, m.G, m.density, m.restitution, m.mu)
        mat16 = None if mat is None else _c(mat, np.uint16, (n,))
        self.n = n
        self._h = _vp()
        _check(lib().dem_job_prepare(ctypes.byref(P), ctypes.cast(mats, _vp), len(materials), n,
                                     x.ctypes.data, v.ctypes.data, w.ctypes.data,
                                     r32.ctypes.data, None if mat16 is None else mat16.ctypes.data,
                                     ctypes.byref(self._h)), "dem_job_prepare")

    @classmethod
    def from_scene(cls, sc, precision, **kw):
        args = dict(lo=sc.lo, hi=sc.hi, x=sc.x, v=sc.v, w=sc.w, r=sc.r, materials=sc.materials,
                    mat=sc.mat if len(sc.materials) > 1 else None, walls=sc.walls,
                    periodic=sc.periodic, gravity=sc.gravity, shear_rate=sc.shear_rate, dt=sc.dt,
                    kn_form=sc.kn_form, extra_walls=getattr(sc, "extra_walls", ()))
        args.update(kw)
        return cls(precision=precision, **args)

    def cells(self) -> int:
        return int(lib().dem_job_prep_cells(self._h)) if self._h else 0

    def close(self):
        if self._h:
            lib().dem_job_prep_free(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pool:
    """Many simulations advanced by shared launches (dem_pool_*)."""

    def __init__(self, max_particles=0, max_cells=0, max_jobs=0, precision=PREC_MIXED,
                 contact_slots=0, flags=0, stream=None, hbm_budget=0, arena=None):
        """Capacities as given, or with max_particles = 0 the largest that fit
        hbm_budget bytes (or the lent arena)."""
        self.params = make_pool_params(max_particles, max_cells, max_jobs, precision,
                                       contact_slots, flags, hbm_budget)
        self.precision = int(precision)
        self._h = _vp()
        self._n = {}
        self._arena = arena
        aptr, abytes = _arena_handle(arena)
        _check(lib().dem_pool_create(ctypes.byref(self.params), aptr, abytes,
                                     _stream_handle(stream), ctypes.byref(self._h)),
               "dem_pool_create")

    def _handle(self):
        if not self._h:
            raise RuntimeError("pool destroyed")
        return self._h

    def add(self, lo, hi, x, v, w, r, materials, steps, mat=None, walls=0x3F, periodic=0,
            gravity=(0.0, 0.0, -9.81), shear_rate=0.0, dt=0.0, time=0.0, kn_form=0,
            cell_size=0.0, extra_walls=(), radius_cut=0.0) -> int:
        P = make_params(lo, hi, walls, periodic, gravity, shear_rate, dt, time, self.precision,
                        kn_form, cell_size, extra_walls=extra_walls, radius_cut=radius_cut)
        x = _c(x, np.float64, (-1, 3))
        n = x.shape[0]
        v = _c(v, np.float64, (n, 3))
        w = _c(w, np.float64, (n, 3))
        r32 = _c(r, np.float32, (n,))
        mats = (Material * len(materials))()
        for k, m in enumerate(materials):
            mats[k] = Material(m.E, m.poisson, m.G, m.density, m.restitution, m.mu)
        mat16 = None if mat is None else _c(mat, np.uint16, (n,))
        job = ctypes.c_uint64()
        _check(lib().dem_pool_add(self._handle(), ctypes.byref(P), ctypes.cast(mats, _vp),
                                  len(materials), n, x.ctypes.data, v.ctypes.data, w.ctypes.data,
                                  r32.ctypes.data, None if mat16 is None else mat16.ctypes.data,
                                  int(steps), ctypes.byref(job)), "dem_pool_add")
        self._n[job.value] = n
        return job.value

    def add_scene(self, sc, steps, **kw) -> int:
        args = dict(lo=sc.lo, hi=sc.hi, x=sc.x, v=sc.v, w=sc.w, r=sc.r, materials=sc.materials,
                    mat=sc.mat if len(sc.materials) > 1 else None, walls=sc.walls,
                    periodic=sc.periodic, gravity=sc.gravity, shear_rate=sc.shear_rate, dt=sc.dt,
                    kn_form=sc.kn_form, extra_walls=getattr(sc, "extra_walls", ()))
        args.update(kw)
        return self.add(steps=steps, **args)

    def prepare_scene(self, sc, **kw) -> PreparedJob:
        """Host-side preparation of a job for this pool (any thread)."""
        return PreparedJob.from_scene(sc, self.precision, **kw)

    def add_prepared(self, prep, steps) -> int:
        job = ctypes.c_uint64()
        _check(lib().dem_pool_add_prepared(self._handle(), prep._h, int(steps), ctypes.byref(job)),
               "dem_pool_add_prepared")
        self._n[job.value] = prep.n
        prep.close()
        return job.value

    def step(self, k=1):
        _check(lib().dem_pool_step(self._handle(), int(k)), "dem_pool_step")
        return self

    def sync(self):
        _check(lib().dem_pool_sync(self._handle()), "dem_pool_sync")
        return self

    def poll(self, cap=None):
        cap = len(self._n) if cap is None else int(cap)
        out = np.zeros(max(cap, 1), np.uint64)
        k = ctypes.c_uint32()
        _check(lib().dem_pool_poll(self._handle(), out.ctypes.data, cap, ctypes.byref(k)),
               "dem_pool_poll")
        return [int(j) for j in out[:k.value]]

    def job_info(self, job) -> dict:
        inf = JobInfo()
        _check(lib().dem_pool_job_info(self._handle(), int(job), ctypes.byref(inf)),
               "dem_pool_job_info")
        out = {f: getattr(inf, f) for f, _ in JobInfo._fields_ if f != "reserved"}
        out["status"] = JOB_STATUS.get(inf.status, inf.status)
        return out

    def get_state(self, job):
        n = self._n[int(job)]
        x, v, w = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 3))
        _check(lib().dem_pool_get_state(self._handle(), int(job), x.ctypes.data, v.ctypes.data,
                                        w.ctypes.data), "dem_pool_get_state")
        return dict(x=x, v=v, w=w)

    def set_radii(self, job, r):
        """New radii of a job (pid order), rounded to FP32; state and history kept."""
        r32 = _c(r, np.float32, (self._n[int(job)],))
        _check(lib().dem_pool_set_radii(self._handle(), int(job), r32.ctypes.data),
               "dem_pool_set_radii")

    def remove(self, job):
        _check(lib().dem_pool_remove(self._handle(), int(job)), "dem_pool_remove")
        self._n.pop(int(job), None)

    def capacity(self) -> dict:
        p, c = ctypes.c_uint64(), ctypes.c_uint64()
        j = ctypes.c_uint32()
        _check(lib().dem_pool_capacity(self._handle(), ctypes.byref(p), ctypes.byref(c),
                                       ctypes.byref(j)), "dem_pool_capacity")
        return dict(particles=p.value, cells=c.value, jobs=j.value)

    def fits(self, sc, cell_size=0.0) -> bool:
        """Whether a job of this scene fits in the pool now."""
        cap = self.capacity()
        return cap["jobs"] >= 1 and job_fits(sc, cap, cell_size)

    def profile(self, enable=True):
        _check(lib().dem_pool_profile(self._handle(), 1 if enable else 0), "dem_pool_profile")

    def profile_read(self) -> dict:
        ms = np.zeros(NPHASE)
        cnt = np.zeros(NPHASE, np.uint64)
        _check(lib().dem_pool_profile_read(self._handle(), ms.ctypes.data, cnt.ctypes.data),
               "dem_pool_profile_read")
        return {p: (float(ms[k]), int(cnt[k])) for k, p in enumerate(PHASES)}

    def close(self):
        if self._h:
            lib().dem_pool_destroy(self._h)
            self._h = _vp()
        self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
