"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package only draws initial configurations (positions, radii, velocities,
materials, box descriptions).  It holds none of the simulated method's
arithmetic: no contact law, no time-step rule, no integrator.  A time step of
0.0 in a scene means "let the simulator pick it" and each side applies its own
rule.

Workloads follow the paper's set-up (Section "Performance evaluation"):
spheres placed without initial overlap in a box, optionally seeded with
touching pairs so that contacts exist from the first step.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 150303553
WALL_ALL = 0x3F  # six faces: bit 2a = low face of axis a, bit 2a+1 = high face

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def build_helper(force: bool = False) -> str:
    """Compile gen/rsa.c into gen/librsa.so (gcc, host code only)."""
    src = os.path.join(_HERE, "rsa.c")
    out = os.path.join(_HERE, "librsa.so")
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


def _lib():
    global _LIB
    if _LIB is None:
        lib = ctypes.CDLL(build_helper())
        lib.rsa_place.restype = ctypes.c_int
        lib.rsa_place.argtypes = [
            ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
            ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p]
        _LIB = lib
    return _LIB


@dataclass
class Material:
    E: float = 3.0e9          # Young's modulus [Pa]
    poisson: float = 0.3
    G: float = 3.0e9 / (2 * 1.3)  # shear modulus [Pa]
    density: float = 1200.0   # [kg/m^3]
    restitution: float = 0.5
    mu: float = 0.3           # sliding friction coefficient

    @staticmethod
    def make(E=3.0e9, poisson=0.3, density=1200.0, restitution=0.5, mu=0.3, G=None):
        return Material(E=E, poisson=poisson, G=E / (2 * (1 + poisson)) if G is None else G,
                        density=density, restitution=restitution, mu=mu)


@dataclass
class Wall:
    """A static wall inside the box besides its faces: kind RECT is the
    rectangle p + s u + t v (u orthogonal to v), kind SEGMENT the segment
    p + s u; s, t in [0, 1].  Lengths in metres."""
    kind: int
    p: tuple
    u: tuple
    v: tuple = (0.0, 0.0, 0.0)


RECT, SEGMENT = 0, 1


@dataclass
class Scene:
    """One simulation's inputs, in SI units.  Arrays are in particle-id order."""
    lo: np.ndarray
    hi: np.ndarray
    x: np.ndarray            # (n,3) float64
    v: np.ndarray            # (n,3) float64
    w: np.ndarray            # (n,3) float64 angular velocity
    r: np.ndarray            # (n,)  float64 holding float32-representable values
    mat: np.ndarray          # (n,)  uint16 material index
    materials: list
    walls: int = WALL_ALL
    periodic: int = 0
    gravity: tuple = (0.0, 0.0, -9.81)
    shear_rate: float = 0.0
    dt: float = 0.0          # 0 = simulator's own rule
    steps: int = 1
    kn_form: int = 0         # 0 = as printed, 1 = textbook Hertz
    extra_walls: list = field(default_factory=list)   # Wall entries, at most 10
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.r.shape[0])

    def copy(self) -> "Scene":
        import copy
        return copy.deepcopy(self)


def f32(a):
    """Round to float32-representable values (kept in float64)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def lognormal_radii(rng, n, median=4e-6, sigma=0.15, rmin=2e-6, rmax=8e-6):
    r = median * np.exp(sigma * rng.standard_normal(n))
    return f32(np.clip(r, rmin, rmax))


def rsa(r, lo, hi, periodic=0, p_touch=0.0, touch_max=2e-3, seed=0, max_attempts=100000,
        big_first=False):
    """Random sequential addition; returns (n,3) positions (raises if it jams).

    big_first places the spheres in order of decreasing radius (stable), which
    reaches higher volume fractions before jamming; positions are returned in
    the order of r either way."""
    if big_first:
        r64 = np.asarray(r, dtype=np.float64)
        order = np.argsort(-r64, kind="stable")
        xs = rsa(r64[order], lo, hi, periodic, p_touch, touch_max, seed, max_attempts)
        x = np.empty_like(xs)
        x[order] = xs
        return x
    r = np.ascontiguousarray(r, dtype=np.float64)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    n = r.shape[0]
    x = np.zeros((n, 3), dtype=np.float64)
    got = _lib().rsa_place(n, r.ctypes.data, lo.ctypes.data, hi.ctypes.data, periodic,
                           float(p_touch), float(touch_max), int(seed) & (2**64 - 1),
                           int(max_attempts), x.ctypes.data)
    if got != n:
        raise RuntimeError("RSA placed only %d of %d spheres" % (got, n))
    return x


def box_side(r, phi):
    """Side of the cube holding spheres r at volume fraction phi."""
    return float((np.sum(4.0 / 3.0 * np.pi * np.asarray(r) ** 3) / phi) ** (1.0 / 3.0))


def _finish(rng, x, r, lo, hi, materials, vel_sigma=0.1, **kw):
    n = r.shape[0]
    v = vel_sigma * rng.standard_normal((n, 3))
    w = np.zeros((n, 3))
    mat = np.zeros(n, dtype=np.uint16)
    return Scene(lo=np.asarray(lo, float), hi=np.asarray(hi, float), x=x, v=v, w=w, r=r,
                 mat=mat, materials=materials, **kw)


def config_plain(seed=None, n=2000):
    """Monodisperse r = 5 um, phi = 0.3, six walls, gravity, 1000 steps.

    The stated 200 um box would give phi = 0.131 for 2,000 spheres; N and phi
    are kept and the box side follows from them (151.7 um at N = 2000)."""
    seed = SEED_BASE + 0 if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    r = f32(np.full(n, 5e-6))
    L = box_side(r, 0.3)
    lo, hi = np.zeros(3), np.full(3, L)
    x = rsa(r, lo, hi, seed=seed)
    mats = [Material.make(restitution=0.5, mu=0.3)]
    return _finish(rng, x, r, lo, hi, mats, steps=1000, name="plain-2k-fp64",
                   meta=dict(phi=0.3))


def config_dilute(seed=None, n=1_000_000, p_touch=0.5, touch_max=2e-3):
    """1M polydisperse spheres (lognormal, median 4 um, sigma_log 0.15, clipped
    to [2, 8] um), walled box at phi = 0.1, gravity, 200 steps.  Half of the
    spheres are placed touching an earlier one so that about one contact per
    particle exists from the first step."""
    seed = SEED_BASE + 1 if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    r = lognormal_radii(rng, n)
    L = box_side(r, 0.1)
    lo, hi = np.zeros(3), np.full(3, L)
    x = rsa(r, lo, hi, p_touch=p_touch, touch_max=touch_max, seed=seed)
    mats = [Material.make(restitution=0.5, mu=0.3)]
    return _finish(rng, x, r, lo, hi, mats, steps=200, name="dilute-1m-mixed",
                   meta=dict(phi=0.1, p_touch=p_touch))


def config_batch_job(k, m, n=None, phi_lo=0.1, phi_hi=0.5, n_lo=1e3, n_hi=2e5, rsa_max=0.35,
                     phi0=0.30):
    """Job m of a batched workload: N log-uniform in [n_lo, n_hi], phi ~
    U[phi_lo, phi_hi], restitution ~ U[0.3, 0.9], mu ~ U[0.1, 0.5], walls,
    gravity, 500 steps.  Up to rsa_max the spheres are placed at phi by RSA
    (touch-seeded, largest first); above it (where RSA slows down and jams
    short of 0.5) they are placed by RSA at phi0 with radii shrunk by
    (phi0 / phi)^(1/3) and marked for growth to their full radii (meta
    r_full; the scene then carries the growth material, restitution 0.1 and
    no friction, without gravity, and meta the job's own material and
    gravity for dense_run_scene)."""
    seed = SEED_BASE + 1000 * k + m
    rng = np.random.Generator(np.random.PCG64(seed))
    if n is None:
        n = int(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
    phi = float(rng.uniform(phi_lo, phi_hi))
    eps = float(rng.uniform(0.3, 0.9))
    mu = float(rng.uniform(0.1, 0.5))
    r = lognormal_radii(rng, n)
    L = box_side(r, phi)
    lo, hi = np.zeros(3), np.full(3, L)
    mats = [Material.make(restitution=eps, mu=mu)]
    g = (0.0, 0.0, -9.81)
    if phi <= rsa_max:
        x = rsa(r, lo, hi, p_touch=0.5, seed=seed, big_first=True)
        return _finish(rng, x, r, lo, hi, mats, steps=500, name="batch-job-%d" % m,
                       gravity=g, meta=dict(phi=phi, seed=seed))
    r0 = f32(r * (phi0 / phi) ** (1.0 / 3.0))
    x = rsa(r0, lo, hi, p_touch=0.5, seed=seed, big_first=True)
    z = np.zeros((n, 3))
    return Scene(lo=lo, hi=hi, x=x, v=z.copy(), w=z.copy(), r=r0, mat=np.zeros(n, np.uint16),
                 materials=[Material.make(restitution=0.1, mu=0.0)], walls=WALL_ALL,
                 gravity=(0.0, 0.0, 0.0), steps=500, name="batch-job-%d" % m,
                 meta=dict(phi=phi, phi0=phi0, seed=seed, r_full=r, run_materials=mats,
                           run_gravity=g, grow=True))


def grown_scene(start, x, v, w):
    """The run of a job grown from `start` (config_batch_job above rsa_max):
    the grown state with the full radii, the job's own material and gravity."""
    m = start.meta
    return Scene(lo=start.lo.copy(), hi=start.hi.copy(), x=np.array(x, np.float64, copy=True),
                 v=np.array(v, np.float64, copy=True), w=np.array(w, np.float64, copy=True),
                 r=m["r_full"].copy(), mat=np.zeros(start.n, np.uint16),
                 materials=list(m["run_materials"]), walls=start.walls, periodic=start.periodic,
                 gravity=m["run_gravity"], steps=start.steps, name=start.name,
                 meta=dict(phi=m["phi"], seed=m["seed"], grown=True))


def rsa_tiled(r, lo, hi, splits=(4, 4, 4), p_touch=0.0, touch_max=2e-3, seed=0, threads=16,
              big_first=True):
    """RSA in a grid of sub-boxes filled in parallel threads (the C helper
    releases the interpreter lock).  Particle k goes to sub-box k mod the
    number of sub-boxes and lies wholly inside it, so spheres of different
    sub-boxes never overlap, nor do periodic images of the whole box."""
    import concurrent.futures as cf
    r = np.asarray(r, np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    nx, ny, nz = splits
    nsub = nx * ny * nz
    h = (hi - lo) / np.array(splits, np.float64)
    x = np.empty((r.size, 3))
    build_helper()

    def fill(s):
        ix, iy, iz = s % nx, (s // nx) % ny, s // (nx * ny)
        sl = lo + h * np.array([ix, iy, iz])
        idx = np.arange(s, r.size, nsub)
        if idx.size:
            x[idx] = rsa(r[idx], sl, sl + h, periodic=0, p_touch=p_touch, touch_max=touch_max,
                         seed=seed + 7919 * s, big_first=big_first)

    with cf.ThreadPoolExecutor(max(1, min(threads, os.cpu_count() or 1))) as ex:
        list(ex.map(fill, range(nsub)))
    return x


def config_dense_start(seed=None, n=8_000_000, phi=0.55, phi0=0.30, shear_rate=100.0,
                       splits=(4, 4, 4)):
    """Start of the dense sheared pack: N polydisperse spheres (the radius law
    of the dilute workload) in the periodic cube that holds them at volume
    fraction phi, placed by RSA with their radii shrunk by (phi0/phi)^(1/3)
    (volume fraction phi0, which RSA reaches).  The returned scene carries
    the shrunk radii, zero velocities and the material of the growth
    (restitution 0.1, no friction, no gravity); meta holds the full radii
    (r_full), phi, phi0, and the material and shear rate of the sheared run
    that follows the growth."""
    seed = SEED_BASE + 3 if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    r = lognormal_radii(rng, n)
    L = box_side(r, phi)
    lo, hi = np.zeros(3), np.full(3, L)
    r0 = f32(r * (phi0 / phi) ** (1.0 / 3.0))
    x = rsa_tiled(r0, lo, hi, splits=splits, seed=seed) if n > 200_000 else \
        rsa(r0, lo, hi, periodic=7, seed=seed, big_first=True)
    grow_mat = Material.make(restitution=0.1, mu=0.0)
    run_mat = Material.make(restitution=0.5, mu=0.3)
    z = np.zeros((n, 3))
    return Scene(lo=lo, hi=hi, x=x, v=z.copy(), w=z.copy(), r=r0, mat=np.zeros(n, np.uint16),
                 materials=[grow_mat], walls=0, periodic=7, gravity=(0.0, 0.0, 0.0),
                 steps=100, name="dense-shear-%d" % n,
                 meta=dict(phi=phi, phi0=phi0, r_full=r, run_material=run_mat,
                           shear_rate=shear_rate, seed=seed))


def dense_run_scene(start, x, v, w):
    """The sheared run of the dense pack: the grown positions, velocities and
    angular velocities (pid order) with the full radii, the run's material,
    and the Lees-Edwards shear (the affine profile shear_rate * (y - lo_y)
    added to v_x)."""
    m = start.meta
    v = np.array(v, np.float64, copy=True)
    v[:, 0] += m["shear_rate"] * (np.asarray(x)[:, 1] - start.lo[1])
    return Scene(lo=start.lo.copy(), hi=start.hi.copy(), x=np.array(x, np.float64, copy=True),
                 v=v, w=np.array(w, np.float64, copy=True), r=m["r_full"].copy(),
                 mat=np.zeros(start.n, np.uint16), materials=[m["run_material"]], walls=0,
                 periodic=7, gravity=(0.0, 0.0, 0.0), shear_rate=m["shear_rate"], steps=100,
                 name=start.name, meta=dict(phi=m["phi"]))


def config_ablation(n, regime, seed=None, r=5e-6):
    """Inputs of the fused-versus-split comparison of section 4 (N from
    131,072 up to 2M): monodisperse spheres on a simple cubic grid with small
    random offsets, six walls, gravity.

    "dense" stands in for the packed state after the warm-up: spacing
    2 r (1 - 1e-3) and offsets U(-2e-3 r, 2e-3 r) per coordinate, so that
    most grid neighbours overlap (about five directed contacts per sphere,
    varying from sphere to sphere).  "sparse" is the initial state with no
    contacts: spacing 2.2 r and offsets U(-0.05 r, 0.05 r)."""
    seed = SEED_BASE + 7000 + (0 if regime == "dense" else 1) if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    if regime == "dense":
        h, jit = 2.0 * r * (1.0 - 1e-3), 2e-3 * r
    elif regime == "sparse":
        h, jit = 2.2 * r, 0.05 * r
    else:
        raise ValueError(regime)
    m = int(round(n ** (1.0 / 3.0)))
    nz = -(-n // (m * m))
    k = np.arange(n)
    ijk = np.stack([k % m, (k // m) % m, k // (m * m)], axis=1).astype(np.float64)
    lo = np.zeros(3)
    hi = np.array([m, m, nz], np.float64) * h + 2.0 * r
    x = r + 0.5 * (h - 2.0 * r) + ijk * h + rng.uniform(-jit, jit, size=(n, 3))
    x = np.clip(x, lo + r, hi - r)
    mats = [Material.make(restitution=0.5, mu=0.3)]
    return _finish(rng, x, f32(np.full(n, r)), lo, hi, mats, steps=20,
                   name="ablation-%s-%d" % (regime, n), meta=dict(regime=regime))


def batch_sizes(k, jobs, lo=1e3, hi=2e5):
    """Particle counts of a batched workload: log-uniform in [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 7000 + k))
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=jobs)).astype(np.int64)


def serve_requests(seed, n_requests=1000, rate=20.0, n_lo=1e3, n_hi=1e6, steps_lo=100,
                   steps_hi=2000):
    """A Poisson arrival stream of simulation requests: arrival times [s] of
    n_requests requests at `rate` jobs/s (exponential gaps), and per request
    its particle count (log-uniform in [n_lo, n_hi]) and steps (uniform
    integers in [steps_lo, steps_hi]).  Request q's scene is
    config_serve_job(q, n[q])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    arr = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    sizes = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=n_requests)).astype(np.int64)
    steps = rng.integers(steps_lo, steps_hi + 1, size=n_requests)
    return arr, sizes, steps


def config_serve_job(q, n):
    """The scene of serving request q: a batched-workload job of n particles
    (own seed) with phi ~ U[0.1, 0.3], placed by RSA."""
    return config_batch_job(2, q, n=int(n), phi_lo=0.1, phi_hi=0.3)


def generate_threaded(fn, args, threads=16):
    """fn(*a) for every a in args on a pool of threads (the RSA helper runs
    without the interpreter lock), in order; no copies between processes."""
    import concurrent.futures as cf
    build_helper()
    with cf.ThreadPoolExecutor(max(1, min(threads, os.cpu_count() or 1))) as ex:
        return list(ex.map(lambda a: fn(*a), args))


def generate_many(fn, args, workers=None):
    """fn(*a) for every a in args in a pool of processes (CPU only: call it
    before anything in the process has touched a GPU)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    workers = workers or min(16, os.cpu_count() or 1)
    if workers <= 1 or len(args) <= 1:
        return [fn(*a) for a in args]
    build_helper()
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
        futs = [ex.submit(fn, *a) for a in args]
        return [f.result() for f in futs]


# ---------------------------------------------------------------- tiny scenes
def scene_pair(r1=5e-6, r2=5e-6, gap=-1e-9, v1=(0.1, 0, 0), v2=(-0.1, 0, 0), w1=(0, 0, 0),
               w2=(0, 0, 0), material=None, walls=0, L=100e-6, gravity=(0.0, 0.0, 0.0),
               offset=(0.0, 0.0, 0.0)):
    """Two spheres on the x axis, centre distance r1 + r2 + gap."""
    material = material or Material.make()
    c = np.full(3, L / 2) + np.asarray(offset, float)
    d = r1 + r2 + gap
    x = np.array([c - [d / 2, 0, 0], c + [d / 2, 0, 0]])
    return Scene(lo=np.zeros(3), hi=np.full(3, L), x=x, v=np.array([v1, v2], float),
                 w=np.array([w1, w2], float), r=f32([r1, r2]), mat=np.zeros(2, np.uint16),
                 materials=[material], walls=walls, periodic=0, gravity=tuple(gravity),
                 name="pair")


def scene_cluster(seed, n_side=4, r=5e-6, overlap_max=2e-3, vel_sigma=0.05, jitter=0.0,
                  walls=WALL_ALL, gravity=(0.0, 0.0, -9.81), polydisperse=False):
    """A compressed simple-cubic cluster: neighbours overlap by dn/r in
    U[0, overlap_max) so that every particle has several contacts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = n_side ** 3
    rr = lognormal_radii(rng, n, median=r, sigma=0.05, rmin=0.8 * r, rmax=1.2 * r) \
        if polydisperse else f32(np.full(n, r))
    spacing = 2 * r * (1 - overlap_max / 2)
    idx = np.stack(np.meshgrid(np.arange(n_side), np.arange(n_side), np.arange(n_side),
                               indexing="ij"), -1).reshape(-1, 3)
    x = (idx + 0.5) * spacing + 3 * r
    x = x + jitter * r * rng.uniform(-1, 1, size=x.shape)
    L = n_side * spacing + 6 * r
    mats = [Material.make()]
    return _finish(rng, x, rr, np.zeros(3), np.full(3, L), mats, vel_sigma=vel_sigma,
                   walls=walls, gravity=tuple(gravity), name="cluster")


def scene_random(seed, n, phi=0.3, p_touch=0.7, touch_max=2e-3, walls=WALL_ALL,
                 periodic=0, gravity=(0.0, 0.0, -9.81), polydisperse=True, vel_sigma=0.1,
                 shear_rate=0.0, n_materials=1, big_frac=0.0, big_r=8e-6):
    """Seeded random RSA fill with touch seeding; optionally periodic or several
    materials; with big_frac, that fraction of the spheres (chosen at random)
    gets radius big_r."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = lognormal_radii(rng, n) if polydisperse else f32(np.full(n, 4e-6))
    if big_frac > 0.0:
        r = r.copy()
        r[rng.random(n) < big_frac] = f32(np.array([big_r]))[0]
    L = box_side(r, phi)
    lo, hi = np.zeros(3), np.full(3, L)
    x = rsa(r, lo, hi, periodic=periodic, p_touch=p_touch, touch_max=touch_max, seed=seed)
    mats = [Material.make(restitution=0.5, mu=0.3)]
    for k in range(1, n_materials):
        mats.append(Material.make(E=float(rng.uniform(1e9, 5e9)),
                                  poisson=float(rng.uniform(0.2, 0.4)),
                                  density=float(rng.uniform(800, 2500)),
                                  restitution=float(rng.uniform(0.3, 0.9)),
                                  mu=float(rng.uniform(0.1, 0.5))))
    sc = _finish(rng, x, r, lo, hi, mats, vel_sigma=vel_sigma, walls=walls, periodic=periodic,
                 gravity=tuple(gravity), shear_rate=shear_rate, name="random")
    if n_materials > 1:
        sc.mat = rng.integers(0, n_materials, size=n).astype(np.uint16)
    if shear_rate:
        # affine shear profile u = shear_rate * y along x
        sc.v[:, 0] += shear_rate * (x[:, 1] - lo[1])
    return sc
