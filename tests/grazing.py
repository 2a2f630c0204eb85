"""Pairs of spheres that touch by rounding only: the contact predicate
((dx^2 + dy^2) + dz^2) < (r_i + r_j)^2, evaluated in FP64 without fused
multiply-add, accepts them, while their exact squared distance is at least
(r_i + r_j)^2.  A force computation that re-evaluated the distance more
exactly (a fused multiply-add) would find a non-positive overlap for them
and take the square root of a negative number."""
from fractions import Fraction

import numpy as np

import gen


def rounded_d2(dx, dy, dz):
    # Python floats are IEEE doubles with no fused multiply-add
    d2 = dx * dx + dy * dy
    return d2 + dz * dz


def is_grazing(xi, xj, s):
    dx, dy, dz = (float(xj[a] - xi[a]) for a in range(3))
    exact = Fraction(dx) ** 2 + Fraction(dy) ** 2 + Fraction(dz) ** 2
    return rounded_d2(dx, dy, dz) < s * s and exact >= Fraction(s) ** 2


def grazing_scene(seed=0, npairs=16, r=4e-6, vel_sigma=0.05):
    """npairs grazing pairs on a coarse grid (no other contacts), random
    velocities and spins, no walls, no gravity."""
    rng = np.random.default_rng(seed)
    r = float(np.float32(r))
    s = r + r
    side = int(np.ceil(npairs ** (1 / 3)))
    pitch = 8.0 * s
    L = side * pitch
    x = np.zeros((2 * npairs, 3))
    for k in range(npairs):
        c = (np.array([k % side, (k // side) % side, k // (side * side)]) + 0.5) * pitch
        while True:
            u = rng.normal(size=3)
            u /= np.linalg.norm(u)
            d = s * (1.0 + float(rng.integers(-3, 4)) * 2.0 ** -53)
            xj = c + d * u
            if is_grazing(c, xj, s):
                break
        x[2 * k], x[2 * k + 1] = c, xj
    n = 2 * npairs
    mats = [gen.Material.make(restitution=0.5, mu=0.3)]
    sc = gen.Scene(lo=np.zeros(3), hi=np.full(3, L), x=x,
                   v=vel_sigma * rng.standard_normal((n, 3)),
                   w=1e4 * rng.standard_normal((n, 3)), r=gen.f32(np.full(n, r)),
                   mat=np.zeros(n, np.uint16), materials=mats, walls=0, gravity=(0.0, 0.0, 0.0),
                   name="grazing")
    return sc
