"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own code: closed forms of the
Hertz contact (evaluated with scipy's quadrature / ODE integrators), textbook
special cases, conservation and balance laws that hold exactly for the
semi-implicit Euler step, brute force on tiny inputs, a hand-worked fixture,
and library neighbour search (scipy cKDTree).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, spatial

import gen
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------- helpers
def nondim_collision(alpha):
    """Head-on collision s'' = -s^1.5 - alpha s^0.25 s', s(0)=0, s'(0)=1 in the
    time unit (m*/k_n)^(2/5) v0^(-1/5): returns (contact time, restitution,
    max overlap) from scipy's DOP853."""
    def f(t, y):
        s = max(y[0], 0.0)
        return [y[1], -s ** 1.5 - alpha * s ** 0.25 * y[1]]

    def out(t, y):
        return y[0]
    out.terminal = True
    out.direction = -1
    sol = integrate.solve_ivp(f, [0, 50], [0.0, 1.0], method="DOP853", rtol=1e-12, atol=1e-14,
                              events=out, dense_output=True)
    tc = sol.t_events[0][0]
    e = -sol.y_events[0][0][1]
    ts = np.linspace(0, tc, 20001)
    smax = sol.sol(ts)[0].max()
    return tc, e, smax


def hertz_time_constant():
    """Elastic contact time from the energy integral
    t = 2 int_0^smax ds / sqrt(1 - 4/5 s^(5/2)), smax = (5/4)^(2/5)."""
    smax = 1.25 ** 0.4
    val, _ = integrate.quad(lambda s: 1.0 / math.sqrt(max(1.0 - 0.8 * s ** 2.5, 1e-300)), 0, smax,
                            limit=200)
    return 2.0 * val


def textbook_hertz_kn(E1, nu1, E2, nu2, r1, r2):
    """Hertz: F = 4/3 E* sqrt(R*) d^(3/2), 1/E* = (1-nu1^2)/E1 + (1-nu2^2)/E2 (Johnson, Contact Mechanics, ch. 4)."""
    Es = 1.0 / ((1 - nu1 ** 2) / E1 + (1 - nu2 ** 2) / E2)
    Rs = r1 * r2 / (r1 + r2) if r2 else r1
    return 4.0 / 3.0 * Es * math.sqrt(Rs)


def run_collision(scene, dt, max_steps=200000):
    """Run the oracle until the (only) contact ends; returns the sim, the number
    of steps in contact and the largest overlap seen."""
    s = oracle.Sim(scene, dt=dt, mode=0)
    steps_in = 0
    dmax = 0.0
    for _ in range(max_steps):
        s.step(keep_contact_forces=False)
        if len(s.hist):
            steps_in += 1
            d = np.linalg.norm(s.x[1] - s.x[0]) if scene.n == 2 else 0
            dmax = max(dmax, float(scene.r[0] + scene.r[-1] - d) if scene.n == 2 else 0.0)
        elif steps_in:
            break
    return s, steps_in, dmax


# --------------------------------------------------------- the contact law
@pytest.mark.parametrize("eps", [0.1, 0.3, 0.5, 0.7, 0.9, 0.99])
def test_alpha_restitutes_eps_exactly(eps):
    # The damping prefactor must make the model's head-on restitution equal eps.
    _, e, _ = nondim_collision(oracle.alpha(eps))
    assert abs(e - eps) < 1e-7


def test_hertz_time_constant_matches_beta_form():
    # 3.2180654597 = (4/5) B(2/5, 1/2) (5/4)^(2/5); the oracle's own constant
    # comes from that form, the test from the energy integral and the ODE.
    c_quad = hertz_time_constant()
    c_ode, e, smax = nondim_collision(0.0)
    assert abs(c_quad - c_ode) < 1e-8
    assert abs(e - 1.0) < 1e-9
    assert abs(smax - 1.25 ** 0.4) < 1e-6
    assert abs(oracle.contact_time(1.0, 1.0, 1.0) - c_quad) < 1e-9


@pytest.mark.parametrize("v0", [0.02, 0.2])
def test_elastic_headon_contact_time_and_overlap_textbook(v0):
    # kn_form 1 must be textbook Hertz; contact time and peak overlap follow.
    mat = gen.Material.make(restitution=1.0, mu=0.3)
    sc = gen.scene_pair(r1=5e-6, r2=4e-6, gap=1e-13, v1=(v0 / 2, 0, 0), v2=(-v0 / 2, 0, 0),
                        material=mat)
    sc.kn_form = 1
    kn = textbook_hertz_kn(mat.E, mat.poisson, mat.E, mat.poisson, 5e-6, 4e-6)
    m1 = 1200 * 4 / 3 * math.pi * (5e-6) ** 3
    m2 = 1200 * 4 / 3 * math.pi * (4e-6) ** 3
    ms = m1 * m2 / (m1 + m2)
    tc = hertz_time_constant() * (ms / kn) ** 0.4 * v0 ** -0.2
    dmax = (5 * ms * v0 ** 2 / (4 * kn)) ** 0.4
    s, n_in, dmax_sim = run_collision(sc, dt=tc / 1000)
    assert abs(n_in * s.dt - tc) / tc < 2e-3
    assert abs(dmax_sim - dmax) / dmax < 2e-3
    vrel = s.v[1, 0] - s.v[0, 0]
    assert abs(vrel / v0 - 1.0) < 2e-3  # elastic


def test_printed_kn_is_paper_factor_times_textbook():
    # As printed, k_n uses (2 - sigma^2)/E where Hertz has (1 - sigma^2)/E, so
    # the contact time scales by ((2 - s^2)/(1 - s^2))^(2/5).
    mat = gen.Material.make(restitution=1.0)
    sc = gen.scene_pair(gap=1e-13, v1=(0.05, 0, 0), v2=(-0.05, 0, 0), material=mat)
    sc1 = sc.copy()
    sc1.kn_form = 1
    tc0 = hertz_time_constant()
    kn1 = textbook_hertz_kn(mat.E, mat.poisson, mat.E, mat.poisson, 5e-6, 5e-6)
    kn0 = kn1 * (1 - 0.09) / (2 - 0.09)
    m = 1200 * 4 / 3 * math.pi * (5e-6) ** 3
    t_print = tc0 * (m / 2 / kn0) ** 0.4 * 0.1 ** -0.2
    s, n_in, _ = run_collision(sc, dt=t_print / 1000)
    assert abs(n_in * s.dt - t_print) / t_print < 2e-3


@pytest.mark.parametrize("eps,v0", [(0.3, 0.01), (0.5, 0.1), (0.5, 1.0), (0.9, 0.1)])
def test_restitution_equals_eps_independent_of_speed(eps, v0):
    mat = gen.Material.make(restitution=eps)
    sc = gen.scene_pair(gap=1e-13, v1=(v0 / 2, 0, 0), v2=(-v0 / 2, 0, 0), material=mat)
    P = oracle.params(sc, dt=1.0)
    m = oracle.mass(1200, 5e-6)
    tc = hertz_time_constant() * (m / 2 / oracle.kn(P, 0, 0, 5e-6, 5e-6)) ** 0.4 * v0 ** -0.2
    s, n_in, _ = run_collision(sc, dt=tc / 1000)
    e = (s.v[1, 0] - s.v[0, 0]) / v0
    assert abs(e - eps) < 2e-3
    # damped contact time from the nondimensional ODE
    tcd, _, _ = nondim_collision(oracle.alpha(eps))
    tdim = tcd * (m / 2 / oracle.kn(P, 0, 0, 5e-6, 5e-6)) ** 0.4 * v0 ** -0.2
    assert abs(n_in * s.dt - tdim) / tdim < 3e-3


def test_wall_headon_uses_particle_mass_and_radius():
    # A face is a sphere of infinite radius and mass: m* = m, r* = r.
    v0 = 0.1
    mat = gen.Material.make(restitution=1.0)
    L = 100e-6
    r = 5e-6
    sc = gen.Scene(lo=np.zeros(3), hi=np.full(3, L), x=np.array([[L / 2, L / 2, r + 1e-13]]),
                   v=np.array([[0, 0, -v0]]), w=np.zeros((1, 3)), r=gen.f32([r]),
                   mat=np.zeros(1, np.uint16), materials=[mat], walls=gen.WALL_ALL,
                   gravity=(0, 0, 0))
    sc.kn_form = 1
    kn = textbook_hertz_kn(mat.E, mat.poisson, mat.E, mat.poisson, r, 0)
    m = 1200 * 4 / 3 * math.pi * r ** 3
    tc = hertz_time_constant() * (m / kn) ** 0.4 * v0 ** -0.2
    s = oracle.Sim(sc, dt=tc / 1000, mode=0)
    n_in = 0
    for _ in range(5000):
        s.step()
        if len(s.hist):
            assert int(s.hist.j[0]) == oracle.FACE_ID + 4  # low z face
            n_in += 1
        elif n_in:
            break
    assert abs(n_in * s.dt - tc) / tc < 2e-3
    assert abs(s.v[0, 2] - v0) / v0 < 2e-3


def test_tangential_stick_oscillation_period():
    # A sphere pressed on a face by a constant load, no damping, no sliding:
    # the contact point's slip u obeys u'' = -(k_t (1/m + r^2/I)) u, so the
    # period is 2 pi sqrt(m / (3.5 k_t)) with Mindlin's k_t = 8 G* sqrt(r dn),
    # 1/G* = (2 - nu)/G + (2 - nu)/G.  A sign error in the rotational term of
    # Eq. (2), the lever arm or k_t changes the period (or makes it grow).
    mat = gen.Material.make(restitution=1.0, mu=100.0)
    r = 5e-6
    L = 100e-6
    g = 1e4
    m = 1200 * 4 / 3 * math.pi * r ** 3
    kn = textbook_hertz_kn(mat.E, mat.poisson, mat.E, mat.poisson, r, 0) * (1 - 0.09) / (2 - 0.09)
    d0 = (m * g / kn) ** (2 / 3)
    Gs = 1.0 / (2 * (2 - mat.poisson) / mat.G)
    kt = 8 * Gs * math.sqrt(r * d0)
    T = 2 * math.pi * math.sqrt(m / (3.5 * kt))
    u0 = 1e-6
    sc = gen.Scene(lo=np.zeros(3), hi=np.full(3, L), x=np.array([[L / 2, L / 2, r - d0]]),
                   v=np.array([[u0, 0, 0]]), w=np.zeros((1, 3)), r=gen.f32([r]),
                   mat=np.zeros(1, np.uint16), materials=[mat], walls=gen.WALL_ALL,
                   gravity=(0, 0, -g))
    dt = T / 2000
    r = float(sc.r[0])
    s = oracle.Sim(sc, dt=dt, mode=0)
    slip = []
    for _ in range(3000):
        s.step()
        # contact-point velocity along x for n = -z: v_x + (w x (-r z))_x = v_x - r w_y
        slip.append(s.v[0, 0] - r * s.w[0, 1])
    slip = np.array(slip)
    # zero crossings of the slip velocity (it starts at +u0 as a cosine)
    zc = np.where(np.sign(slip[:-1]) != np.sign(slip[1:]))[0]
    assert len(zc) >= 2
    period = 2 * (zc[1] - zc[0]) * dt
    assert abs(period - T) / T < 5e-3
    assert np.abs(slip).max() < 1.01 * u0  # bounded: no growth


def test_gross_sliding_spin_ratio_and_speed_loss():
    # Sliding on a face, the tangential impulse each step is mu |F_n| dt along a
    # fixed direction, so r dw / |dv_t| = m r^2 / I = 5/2 exactly, and the
    # speed drop is mu sum |F_n| dt / m.
    mat = gen.Material.make(restitution=0.5, mu=0.3)
    r = 5e-6
    L = 100e-6
    g = 1e4
    m = 1200 * 4 / 3 * math.pi * r ** 3
    P0 = oracle.params(gen.scene_pair(material=mat), dt=1.0)
    kn = oracle.kn(P0, 0, 0, r, 0)
    d0 = (m * g / kn) ** (2 / 3)
    sc = gen.Scene(lo=np.zeros(3), hi=np.full(3, L), x=np.array([[L / 2, L / 2, r - d0]]),
                   v=np.array([[0.05, 0, 0]]), w=np.zeros((1, 3)), r=gen.f32([r]),
                   mat=np.zeros(1, np.uint16), materials=[mat], walls=gen.WALL_ALL,
                   gravity=(0, 0, -g))
    r = float(sc.r[0])  # the stored radius is float32-representable
    m = 1200 * 4 / 3 * math.pi * r ** 3
    s = oracle.Sim(sc, dt=1e-9, mode=0)
    v0, w0 = s.v[0].copy(), s.w[0].copy()
    fn_sum = 0.0
    for _ in range(200):
        s.step(keep_contact_forces=True)
        fn_sum += abs(s.cF[0, 2])
    dv = s.v[0, 0] - v0[0]
    dw = s.w[0, 1] - w0[1]
    assert dv < 0 < dw  # friction slows it and spins it towards rolling (w_y > 0)
    assert abs(r * dw / dv + 2.5) < 1e-9
    assert abs(-dv - 0.3 * fn_sum * s.dt / m) / (-dv) < 1e-9


def _pair_normals(x, hist):
    i = hist.i.astype(np.int64)
    j = hist.j.astype(np.int64)
    part = hist.j < oracle.FACE_ID
    d = np.zeros((len(i), 3))
    d[part] = x[j[part]] - x[i[part]]
    return part, d


def test_cap_on_particle_contacts():
    sc = gen.scene_cluster(seed=11, n_side=4, vel_sigma=1.0, polydisperse=True, walls=0,
                           gravity=(0, 0, 0))
    s = oracle.Sim(sc, mode=0)
    seen_capped = 0
    for _ in range(10):
        x0 = s.x.copy()
        s.step(keep_contact_forces=True)
        part, d = _pair_normals(x0, s.hist)
        n = d[part] / np.linalg.norm(d[part], axis=1)[:, None]
        F = s.cF[part]
        fn = np.abs(np.sum(F * n, 1))
        ft = np.linalg.norm(F - np.sum(F * n, 1)[:, None] * n, axis=1)
        assert np.all(ft <= 0.3 * fn * (1 + 1e-9) + 1e-30)
        seen_capped += int(np.sum(ft > 0.3 * fn * (1 - 1e-9)))
    assert seen_capped > 0  # the cap was actually exercised


def test_newton_third_law_bitwise():
    sc = gen.scene_cluster(seed=3, n_side=4, vel_sigma=0.3, polydisperse=True, walls=0,
                           gravity=(0, 0, 0))
    sc.w = np.random.default_rng(1).normal(0, 1e4, size=sc.w.shape)
    s = oracle.Sim(sc, mode=0)
    for _ in range(15):
        s.step(keep_contact_forces=True)
        h = s.hist
        idx = {(int(a), int(b)): k for k, (a, b) in enumerate(zip(h.i, h.j))}
        assert len(idx) > 50
        for (a, b), k in idx.items():
            kk = idx[(b, a)]
            assert np.array_equal(s.cF[k], -s.cF[kk])
            assert np.array_equal(h.dt[k], -h.dt[kk])
            # T_ij / r_i and T_ji / r_j are both n x F
            np.testing.assert_allclose(s.cT[k] / sc.r[a], s.cT[kk] / sc.r[b], rtol=1e-13,
                                       atol=1e-30)


def test_linear_momentum_conserved_periodic():
    sc = gen.scene_random(seed=5, n=300, phi=0.25, walls=0, periodic=7, gravity=(0, 0, 0))
    s = oracle.Sim(sc, mode=1)
    m = 1200 * 4 / 3 * np.pi * sc.r ** 3
    p0 = (m[:, None] * s.v).sum(0)
    scale = (m[:, None] * np.abs(s.v)).sum(0)
    for _ in range(30):
        s.step()
    p1 = (m[:, None] * s.v).sum(0)
    assert len(s.hist) > 100
    assert np.all(np.abs(p1 - p0) <= 1e-13 * scale)


def test_angular_momentum_balance_exact():
    # For the semi-implicit step, L(n+1) - L(n) = dt sum_i (x_i x F_i + T_i)
    # with x_i at the start of the step, and pairwise that sum equals
    # dt sum_{i<j} dn_ij (n_ij x F_ij) (lever arm the full radius).
    sc = gen.scene_cluster(seed=9, n_side=4, vel_sigma=0.3, polydisperse=True, walls=0,
                           gravity=(0, 0, 0))
    s = oracle.Sim(sc, mode=0)
    m = 1200 * 4 / 3 * np.pi * sc.r ** 3
    I = 0.4 * m * sc.r ** 2

    def L(s):
        return (m[:, None] * np.cross(s.x, s.v)).sum(0) + (I[:, None] * s.w).sum(0)

    for _ in range(5):
        x0 = s.x.copy()
        L0 = L(s)
        s.step(keep_contact_forces=True)
        dL = L(s) - L0
        pred = s.dt * (np.cross(x0, s.F).sum(0) + s.T.sum(0))
        h = s.hist
        part, d = _pair_normals(x0, h)
        assert part.all()
        dist = np.linalg.norm(d, axis=1)
        n = d / dist[:, None]
        dn = sc.r[h.i] + sc.r[h.j] - dist
        pair = s.dt * 0.5 * (dn[:, None] * np.cross(n, s.cF)).sum(0)
        scale = s.dt * np.abs(np.cross(x0, s.F)).sum()
        assert np.all(np.abs(dL - pred) <= 1e-9 * scale)
        assert np.all(np.abs(pred - pair) <= 1e-9 * scale)


def test_free_flight_closed_form():
    sc = gen.scene_random(seed=2, n=50, phi=0.002, p_touch=0.0, walls=0, gravity=(0.3, -1.0, -9.81),
                          vel_sigma=0.01)
    s = oracle.Sim(sc, dt=1e-6, mode=1)
    x0, v0 = sc.x.copy(), sc.v.copy()
    g = np.array(sc.gravity)
    k = 40
    for _ in range(k):
        s.step()
        assert len(s.hist) == 0
    np.testing.assert_allclose(s.v, v0 + k * 1e-6 * g, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(s.x, x0 + k * 1e-6 * v0 + g * 1e-12 * k * (k + 1) / 2,
                               rtol=1e-12, atol=1e-15)


def test_frictionless_elastic_oblique_energy():
    mat = gen.Material.make(restitution=1.0, mu=0.0)
    sc = gen.scene_pair(r1=5e-6, r2=4e-6, gap=1e-13, v1=(0.1, 0, 0), v2=(-0.05, 0.02, 0),
                        material=mat, offset=(0, 0, 0))
    sc.x[1, 1] += 3e-6  # oblique impact
    sc.x[1, 0] -= 0.5e-6
    m = 1200 * 4 / 3 * np.pi * sc.r ** 3
    ke0 = 0.5 * (m[:, None] * sc.v ** 2).sum()
    s = oracle.Sim(sc, dt=2e-11, mode=0)
    seen = False
    for _ in range(200000):
        s.step()
        if len(s.hist):
            seen = True
        elif seen:
            break
    assert seen
    ke1 = 0.5 * (m[:, None] * s.v ** 2).sum()
    assert abs(ke1 - ke0) / ke0 < 1e-5
    assert np.allclose(s.w, 0)  # no tangential force, no spin


# ---------------------------------------------------------- contact set
def _pairs_from_kdtree(x, r, walls, lo, hi):
    """Contact set via scipy's k-d tree (library neighbour search) then the
    overlap predicate on the few candidates."""
    tree = spatial.cKDTree(x)
    cand = tree.query_pairs(2 * r.max(), output_type="ndarray")
    out = set()
    for a, b in cand:
        d = x[b] - x[a]
        d2 = d[0] * d[0] + d[1] * d[1]
        d2 = d2 + d[2] * d[2]
        if d2 < (r[a] + r[b]) ** 2:
            out.add((int(a), int(b)))
            out.add((int(b), int(a)))
    for i in range(len(r)):
        for f in range(6):
            if walls & (1 << f):
                a = f >> 1
                dist = hi[a] - x[i, a] if f & 1 else x[i, a] - lo[a]
                if dist < r[i]:
                    out.add((i, oracle.FACE_ID + f))
    return out


def test_contact_chain_fixture():
    with open(os.path.join(GOLD, "contact_chain.json")) as fh:
        g = json.load(fh)
    sc = gen.Scene(lo=np.array(g["box_lo"]), hi=np.array(g["box_hi"]), x=np.array(g["positions"]),
                   v=np.zeros((5, 3)), w=np.zeros((5, 3)), r=gen.f32(g["radii"]),
                   mat=np.zeros(5, np.uint16), materials=[gen.Material.make()], walls=g["walls"])
    want = set()
    for a, b in g["expected_pairs"]:
        want.add((a, oracle.FACE_ID + int(b[4:]) if isinstance(b, str) else b))
    for mode in (0, 1):
        i, j = oracle.contacts(sc, mode=mode)
        assert set(zip(i.tolist(), j.tolist())) == want


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_brute_force_matches_kdtree(seed):
    sc = gen.scene_random(seed=seed, n=800, phi=0.22, p_touch=0.6)
    i, j = oracle.contacts(sc, mode=0)
    got = set(zip(i.tolist(), j.tolist()))
    assert got == _pairs_from_kdtree(sc.x, sc.r, sc.walls, sc.lo, sc.hi)
    assert len(got) > 400


@pytest.mark.parametrize("periodic,shear", [(0, 0.0), (7, 0.0), (5, 0.0), (7, 100.0)])
def test_cells_match_brute_force(periodic, shear):
    walls = 0 if periodic == 7 else (gen.WALL_ALL & ~(3 | 48) if periodic == 5 else gen.WALL_ALL)
    sc = gen.scene_random(seed=17, n=600, phi=0.25, p_touch=0.6, walls=walls, periodic=periodic,
                          shear_rate=shear)
    for t in (0.0, 1.234e-3, 7.7e-2):
        a = oracle.contacts(sc, mode=0, time=t)
        b = oracle.contacts(sc, mode=1, time=t)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        assert len(a[0]) > 300


def test_lees_edwards_image_contact_and_velocity():
    # Two spheres across the y boundary: j's image at y_j - Ly sits at
    # x_j - D(t) and moves with v_j - shear Ly along x.
    L = 60e-6
    shear = 1000.0
    r = float(gen.f32([4e-6])[0])
    t = 2.5e-4
    D = (shear * L * t) % L
    dn0 = 1e-9
    d = np.array([1e-6, -math.sqrt((2 * r - dn0) ** 2 - 1e-12), 0.0])  # image minus i
    xi = np.array([10e-6, 1e-6, 30e-6])
    xj = np.array([(xi[0] + D + d[0]) % L, L + xi[1] + d[1], 30e-6])
    sc = gen.Scene(lo=np.zeros(3), hi=np.full(3, L), x=np.array([xi, xj]), v=np.zeros((2, 3)),
                   w=np.zeros((2, 3)), r=gen.f32([r, r]), mat=np.zeros(2, np.uint16),
                   materials=[gen.Material.make(restitution=0.5, mu=0.0)], walls=0, periodic=7,
                   gravity=(0, 0, 0), shear_rate=shear)
    i, j = oracle.contacts(sc, mode=0, time=t)
    assert set(zip(i.tolist(), j.tolist())) == {(0, 1), (1, 0)}
    i2, j2 = oracle.contacts(sc, mode=1, time=t)
    assert np.array_equal(i, i2) and np.array_equal(j, j2)
    # frictionless, both at rest: the image moves at -shear*L along x, so
    # v = v_i - v_image = +shear*L e_x and the damping term is -eta (v.n) n
    s = oracle.Sim(sc, dt=1e-10, mode=0)
    s.time = t
    s.step(keep_contact_forces=True)
    dd = (sc.x[1] - sc.x[0]) + np.array([-D, -L, 0.0])
    dist = np.linalg.norm(dd)
    n = dd / dist
    F = s.cF[0]
    m = 1200 * 4 / 3 * np.pi * r ** 3
    P = oracle.params(sc, dt=1.0)
    kn = oracle.kn(P, 0, 0, r, r)
    dn = 2 * r - dist
    eta = oracle.alpha(0.5) * np.sqrt(m / 2 * kn * np.sqrt(dn))
    v = np.array([shear * L, 0, 0])
    want = -kn * dn ** 1.5 * n - eta * (v @ n) * n
    np.testing.assert_allclose(F, want, rtol=1e-5)
    assert abs(eta * (v @ n)) > 0.05 * kn * dn ** 1.5  # the image velocity matters
    np.testing.assert_array_equal(s.cF[1], -s.cF[0])


def test_history_forgotten_and_restarted():
    mat = gen.Material.make(restitution=0.9, mu=0.5)
    sc = gen.scene_pair(gap=-2e-9, v1=(0.0, 0.05, 0), v2=(0.0, -0.05, 0), material=mat)
    s = oracle.Sim(sc, dt=1e-9, mode=0)
    s.step()
    assert len(s.hist) == 2 and np.abs(s.hist.dt).max() > 0
    s.x[1, 0] += 1e-6  # pull apart: the contact ends and its history is dropped
    s.step()
    assert len(s.hist) == 0
    s.x[1, 0] -= 1e-6
    s.v[:] = 0
    s.w[:] = 0
    s.step()
    # restarted history: only this step's v_t dt with zero velocity -> zero
    assert len(s.hist) == 2 and np.abs(s.hist.dt).max() == 0.0


def test_dt_rule_closed_form():
    sc = gen.scene_pair()
    mat = sc.materials[0]
    r = float(sc.r[0])
    m = 1200 * 4 / 3 * math.pi * r ** 3
    kn = textbook_hertz_kn(mat.E, mat.poisson, mat.E, mat.poisson, r, r) * 0.91 / 1.91
    want = hertz_time_constant() * (m / 2 / kn) ** 0.4 * 0.1 ** -0.2 / 50
    assert abs(oracle.dt_rule(sc) - want) / want < 1e-9


# --------------------------------------------------------------- extra walls
def _one_sphere(x, v, r=5e-6, L=100e-6, walls=gen.WALL_ALL, extra=(), gravity=(0.0, 0.0, 0.0)):
    mat = gen.Material.make()
    return gen.Scene(lo=np.zeros(3), hi=np.full(3, L), x=np.array([x], float),
                     v=np.array([v], float), w=np.zeros((1, 3)), r=gen.f32([r]),
                     mat=np.zeros(1, np.uint16), materials=[mat], walls=walls, gravity=gravity,
                     extra_walls=list(extra))


def test_rectangle_on_a_face_plane_acts_as_that_face():
    # A rectangle covering the low z face, with that face switched off, gives
    # the bounce (with friction and spin) of the face itself, which the
    # head-on and sliding pins above fix.
    L, r = 100e-6, 5e-6
    rect = gen.Wall(gen.RECT, (0.0, 0.0, 0.0), (L, 0.0, 0.0), (0.0, L, 0.0))
    x, v = (0.37 * L, 0.61 * L, r + 1e-13), (0.02, -0.01, -0.1)
    a = _one_sphere(x, v, gravity=(0, 0, -9.81))
    b = _one_sphere(x, v, walls=gen.WALL_ALL & ~(1 << 4), extra=[rect], gravity=(0, 0, -9.81))
    dt = oracle.Sim(a).dt
    sa, sb = oracle.Sim(a, dt=dt, mode=0), oracle.Sim(b, dt=dt, mode=0)
    steps_in = 0
    for _ in range(300):
        sa.step()
        sb.step()
        assert len(sa.hist) == len(sb.hist)
        if len(sa.hist):
            steps_in += 1
            assert int(sa.hist.j[0]) == oracle.FACE_ID + 4
            assert int(sb.hist.j[0]) == oracle.FACE_ID + 6
    assert 20 < steps_in < 300
    for k in ("x", "v", "w"):
        ref = getattr(sa, k)
        assert np.abs(getattr(sb, k) - ref).max() <= 1e-10 * max(np.abs(ref).max(), 1e-300), k
    assert np.abs(sa.w).max() > 0  # friction did act


def test_rectangle_edge_contact_closed_form():
    # Centre beside an edge: the contact point is on the edge, the normal
    # points from the centre to it, and at rest without history the force is
    # the Hertz normal force with the face stiffness (r* = r).
    r = 5e-6
    rect = gen.Wall(gen.RECT, (30e-6, 20e-6, 50e-6), (40e-6, 0.0, 0.0), (0.0, 60e-6, 0.0))
    e, h = 3e-6, 2e-6
    x = np.array([30e-6 - e, 50e-6, 50e-6 + h])
    sc = _one_sphere(x, (0, 0, 0), walls=0, extra=[rect])
    r = float(sc.r[0])
    P = oracle.params(sc, dt=1e-9)
    F, T, _, dn, _ = oracle.pair(P, x, np.zeros(3), np.zeros(3), r, 0, face=6)
    d = math.hypot(e, h)
    n = np.array([e, 0.0, -h]) / d
    kn = oracle.kn(P, 0, 0, r, 0)
    assert abs(dn - (r - d)) <= 1e-14 * r
    np.testing.assert_allclose(F, -kn * (r - d) ** 1.5 * n, rtol=1e-12, atol=1e-25)
    assert np.abs(T).max() <= 1e-12 * r * np.abs(F).max()  # F along n: no torque
    # inside and outside the radius along the same direction
    for scale, touching in ((0.999, True), (1.001, False)):
        y = np.array([30e-6, 50e-6, 50e-6]) + (x - np.array([30e-6, 50e-6, 50e-6])) * (r * scale / d)
        sc2 = _one_sphere(y, (0, 0, 0), walls=0, extra=[rect])
        i, j = oracle.contacts(sc2, mode=0)
        assert (len(i) == 1) == touching


def test_segment_contact_closed_form():
    r = 5e-6
    seg = gen.Wall(gen.SEGMENT, (20e-6, 50e-6, 50e-6), (60e-6, 0.0, 0.0))
    cases = [
        # beside the middle: normal perpendicular to the segment
        (np.array([50e-6, 54e-6, 50e-6]), np.array([0.0, -4e-6, 0.0])),
        # beyond the far end: normal towards the end point
        (np.array([83e-6, 50e-6, 52e-6]), np.array([-3e-6, 0.0, -2e-6])),
    ]
    for x, w in cases:
        sc = _one_sphere(x, (0, 0, 0), walls=0, extra=[seg])
        rr = float(sc.r[0])
        P = oracle.params(sc, dt=1e-9)
        F, _, _, dn, _ = oracle.pair(P, x, np.zeros(3), np.zeros(3), rr, 0, face=6)
        d = np.linalg.norm(w)
        kn = oracle.kn(P, 0, 0, rr, 0)
        assert abs(dn - (rr - d)) <= 1e-14 * rr
        np.testing.assert_allclose(F, -kn * (rr - d) ** 1.5 * w / d, rtol=1e-12, atol=1e-25)
        i, j = oracle.contacts(sc, mode=0)
        assert list(j) == [oracle.FACE_ID + 6]
    # a centre on the segment, and one just beyond the radius: no contact
    for x in (np.array([40e-6, 50e-6, 50e-6]), np.array([40e-6, 50e-6 + 1.0001 * r, 50e-6])):
        i, j = oracle.contacts(_one_sphere(x, (0, 0, 0), walls=0, extra=[seg]), mode=0)
        assert len(i) == 0


def _rotation(axis, angle):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * K @ K


def test_tilted_rectangle_is_a_rotated_floor():
    # The same oblique bounce (friction, spin) on an axis-aligned rectangle and
    # on the rectangle rotated by R about the box centre: the motion is R
    # times the other at every step, and the contact begins and ends on the
    # same steps.
    r = 5e-6
    C = np.full(3, 50e-6)
    p, u, v = np.array([30e-6, 30e-6, 40e-6]), np.array([40e-6, 0, 0]), np.array([0, 40e-6, 0])
    x0, v0 = np.array([52e-6, 47e-6, 40e-6 + r + 1e-12]), np.array([0.03, 0.01, -0.1])
    R = _rotation((1.0, 2.0, 3.0), 0.7)
    flat = _one_sphere(x0, v0, walls=0, extra=[gen.Wall(gen.RECT, tuple(p), tuple(u), tuple(v))])
    tilt = _one_sphere(C + R @ (x0 - C), R @ v0, walls=0,
                       extra=[gen.Wall(gen.RECT, tuple(C + R @ (p - C)), tuple(R @ u),
                                       tuple(R @ v))])
    dt = oracle.Sim(flat).dt
    sa, sb = oracle.Sim(flat, dt=dt, mode=0), oracle.Sim(tilt, dt=dt, mode=0)
    steps_in = 0
    for _ in range(200):
        sa.step()
        sb.step()
        assert len(sa.hist) == len(sb.hist)
        steps_in += len(sa.hist)
    assert 20 < steps_in < 200
    np.testing.assert_allclose(sb.x[0] - C, R @ (sa.x[0] - C), rtol=0, atol=1e-12 * 50e-6)
    np.testing.assert_allclose(sb.v[0], R @ sa.v[0], rtol=0, atol=1e-9 * np.abs(v0).max())
    np.testing.assert_allclose(sb.w[0], R @ sa.w[0], rtol=0, atol=1e-9 * np.abs(sa.w).max())
    assert sa.v[0, 2] > 0 and np.abs(sa.w).max() > 0


# ------------------------------------- Eq. 3 projection, tangential damping,
# -------------------------------------- Eq. 4 displacement, shear wrap
def _printed_kn(mat, ri, rj=0.0):
    """k_n with the paper's (2 - sigma^2)/E factor: the textbook Hertz
    stiffness (Johnson) scaled by (1 - s^2)/(2 - s^2) (pinned by the contact
    time tests above)."""
    s2 = mat.poisson ** 2
    return textbook_hertz_kn(mat.E, mat.poisson, mat.E, mat.poisson, ri, rj) * (1 - s2) / (2 - s2)


def _mindlin_kt(mat, ri, rj, dn):
    """Mindlin's tangential stiffness 8 G* sqrt(r* dn), 1/G* = (2 - nu)/G twice
    (one material); rj = 0 is a wall (r* = ri)."""
    Gs = 1.0 / (2.0 * (2.0 - mat.poisson) / mat.G)
    rs = ri * rj / (ri + rj) if rj else ri
    return 8.0 * Gs * math.sqrt(rs * dn)


def test_eq3_projection_fixture_oblique_wall():
    # Hand-worked fixture: the old displacement has a component along an
    # oblique normal; Eq. (3) removes exactly that component.
    with open(os.path.join(GOLD, "projection_oblique_wall.json")) as fh:
        g = json.load(fh)
    m = g["material"]
    mat = gen.Material.make(E=m["E"], poisson=m["poisson"], density=m["density"],
                            restitution=m["restitution"], mu=m["mu"])
    wl = g["wall"]
    r, dn = g["radius"], g["overlap"]
    q = np.array(g["wall_centre"])
    c = q + (r - dn) * np.array(g["outward_direction"])
    sc = gen.Scene(lo=np.array(g["box_lo"]), hi=np.array(g["box_hi"]), x=c[None, :],
                   v=np.zeros((1, 3)), w=np.zeros((1, 3)), r=gen.f32([r]),
                   mat=np.zeros(1, np.uint16), materials=[mat], walls=0, gravity=(0, 0, 0),
                   extra_walls=[gen.Wall(gen.RECT, tuple(wl["p"]), tuple(wl["u"]), tuple(wl["v"]))])
    assert float(sc.r[0]) == r  # 2^-17 is a float32 number
    P = oracle.params(sc, dt=1e-9)
    F, T, dtn, dn_o, capped = oracle.pair(P, c, np.zeros(3), np.zeros(3), r, 0, face=6,
                                          dt_old=g["dt_old"])
    e = g["expected"]
    kn = _printed_kn(mat, r)
    kt = _mindlin_kt(mat, r, 0.0, dn)
    assert abs(dn_o - dn) <= 1e-9 * dn
    assert capped == e["capped"]
    np.testing.assert_allclose(dtn, e["dt_new"], rtol=0, atol=1e-9 * 2e-9)
    want_F = kn * dn ** 1.5 * np.array(e["F_over_kn_dn15"]) + kt * np.array(e["F_over_kt"])
    np.testing.assert_allclose(F, want_F, rtol=0, atol=1e-9 * np.abs(want_F).max())
    want_T = r * kt * np.array(e["T_over_r_kt"])
    np.testing.assert_allclose(T, want_T, rtol=0, atol=1e-9 * np.abs(want_T).max())


def test_eq3_history_stays_in_the_rotating_tangent_plane():
    # Every stored displacement is perpendicular to the normal of the step
    # that produced it (Eq. 3 projects the old one and v_t is tangential; a
    # capped one is -F_t / k_t, also tangential), while the normals turn from
    # step to step.  Without the projection, or with its sign reversed, the
    # old displacement's component along the turned normal survives.
    sc = gen.scene_cluster(seed=13, n_side=4, vel_sigma=1.0, polydisperse=True, walls=0,
                           gravity=(0, 0, 0))
    sc.w = np.random.default_rng(4).normal(0, 3e5, size=sc.w.shape)
    s = oracle.Sim(sc, mode=0)
    turned = 0.0
    n_prev = {}
    for _ in range(30):
        x0, v0, w0 = s.x.copy(), s.v.copy(), s.w.copy()
        hist0 = s.hist.as_dict()
        s.step()
        h = s.hist
        part, d = _pair_normals(x0, h)
        assert part.all()
        n = d / np.linalg.norm(d, axis=1)[:, None]
        along = np.abs(np.sum(h.dt * n, axis=1))
        ii, jj = h.i.astype(np.int64), h.j.astype(np.int64)
        # rounding scale of the three terms of Eq. (3)
        vel = (np.linalg.norm(v0[ii], axis=1) + np.linalg.norm(v0[jj], axis=1) +
               sc.r[ii] * np.linalg.norm(w0[ii], axis=1) + sc.r[jj] * np.linalg.norm(w0[jj], axis=1))
        old = np.array([np.linalg.norm(hist0.get((a, b), np.zeros(3))) for a, b in zip(ii, jj)])
        bound = 1e-12 * (old + np.linalg.norm(h.dt, axis=1) + vel * s.dt)
        assert np.all(along <= bound), float((along / np.maximum(bound, 1e-300)).max())
        for k, key in enumerate(zip(ii.tolist(), jj.tolist())):
            if key in n_prev and key in hist0:
                turned = max(turned, float(np.linalg.norm(hist0[key]) *
                                           abs(np.dot(n_prev[key], n[k]) - 1.0) ** 0.5))
        n_prev = {key: n[k] for k, key in enumerate(zip(ii.tolist(), jj.tolist()))}
    # the normals did turn under old displacements: the check had something to see
    assert turned > 1e-6 * 1e-9


def _damped_slip(u0, gamma, wd, t):
    """Slip velocity of the damped contact spring u'' + 2 gamma u' + w0^2 u = 0
    with u(0) = 0, u'(0) = u0."""
    return u0 * np.exp(-gamma * t) * (np.cos(wd * t) - gamma / wd * np.sin(wd * t))


def test_tangential_damping_of_the_stick_oscillation():
    # A sphere pressed on a face, sticking (mu large), damped (eps < 1).  The
    # contact point's tangential displacement u obeys
    #   m u'' = (1 + m r^2 / I) (-k_t u - eta u') = 3.5 (-k_t u - eta u'),
    # so the slip decays at gamma = 1.75 eta / m and turns at
    # wd = sqrt(3.5 k_t / m - gamma^2), with eta = alpha(eps) sqrt(m k_n sqrt(dn))
    # (Eq. 1: the tangential damping uses the same eta as the normal one).
    mat = gen.Material.make(restitution=0.9, mu=100.0)
    L, g = 100e-6, 1e4
    r = float(gen.f32([5e-6])[0])
    m = 1200 * 4 / 3 * math.pi * r ** 3
    kn = _printed_kn(mat, r)
    d0 = (m * g / kn) ** (2 / 3)
    kt = _mindlin_kt(mat, r, 0.0, d0)
    eta = oracle.alpha(0.9) * math.sqrt(m * kn * math.sqrt(d0))
    gamma = 1.75 * eta / m
    wd = math.sqrt(3.5 * kt / m - gamma ** 2)
    T = 2 * math.pi / wd
    u0 = 1e-5
    sc = gen.Scene(lo=np.zeros(3), hi=np.full(3, L), x=np.array([[L / 2, L / 2, r - d0]]),
                   v=np.array([[u0, 0, 0]]), w=np.zeros((1, 3)), r=gen.f32([r]),
                   mat=np.zeros(1, np.uint16), materials=[mat], walls=gen.WALL_ALL,
                   gravity=(0, 0, -g))
    dt = T / 8000
    s = oracle.Sim(sc, dt=dt, mode=0)
    k = int(3 * T / dt)
    slip = np.empty(k)
    for q in range(k):
        s.step()
        slip[q] = s.v[0, 0] - r * s.w[0, 1]
    # semi-implicit Euler samples the velocity at the end of each step
    t = dt * np.arange(1, k + 1)
    want = _damped_slip(u0, gamma, wd, t)
    assert np.abs(slip - want).max() < 5e-3 * u0
    # the oscillation really decays over the three periods
    assert np.abs(slip[-int(T / dt):]).max() < 0.6 * u0


def _capped_invariant(F, dt_new, n, kt):
    """|F_t + k_t dt_new| relative to |F_t| for contact forces F, normals n."""
    Ft = F - np.sum(F * n, axis=1)[:, None] * n
    return np.linalg.norm(Ft + kt[:, None] * dt_new, axis=1) / np.linalg.norm(Ft, axis=1)


def test_eq4_displacement_recomputed_from_the_capped_force_on_a_face():
    # Gross sliding on a face with damping (eps = 0.5): every step is capped,
    # and Eq. (4) resets the displacement so that F_t = -k_t dt holds for the
    # capped force itself (the damping term folded in, as the paper states
    # it).  Reading -(F_t + eta v_t) / k_t instead, or keeping the uncapped
    # displacement, breaks the identity by eta |v_t| / |F_t| (order one here).
    mat = gen.Material.make(restitution=0.5, mu=0.3)
    L, g = 100e-6, 1e4
    r = float(gen.f32([5e-6])[0])
    m = 1200 * 4 / 3 * math.pi * r ** 3
    kn = _printed_kn(mat, r)
    d0 = (m * g / kn) ** (2 / 3)
    sc = gen.Scene(lo=np.zeros(3), hi=np.full(3, L), x=np.array([[L / 2, L / 2, r - d0]]),
                   v=np.array([[0.05, 0.01, 0]]), w=np.zeros((1, 3)), r=gen.f32([r]),
                   mat=np.zeros(1, np.uint16), materials=[mat], walls=gen.WALL_ALL,
                   gravity=(0, 0, -g))
    s = oracle.Sim(sc, dt=1e-9, mode=0)
    n = np.array([[0.0, 0.0, -1.0]])
    worst, eta_share = 0.0, 0.0
    for _ in range(100):
        x0, v0, w0 = s.x.copy(), s.v.copy(), s.w.copy()
        s.step(keep_contact_forces=True)
        assert len(s.hist) == 1
        dn = r - x0[0, 2]
        kt = _mindlin_kt(mat, r, 0.0, dn)
        F = s.cF
        Ft = F - np.sum(F * n, axis=1)[:, None] * n
        fn = abs(float(np.sum(F * n)))
        assert abs(np.linalg.norm(Ft) - 0.3 * fn) <= 1e-12 * fn  # capped
        worst = max(worst, float(_capped_invariant(F, s.hist.dt, n, np.array([kt]))[0]))
        vt = np.array([v0[0, 0] - r * w0[0, 1], v0[0, 1] + r * w0[0, 0], 0.0])
        eta = oracle.alpha(0.5) * math.sqrt(m * kn * math.sqrt(dn))
        eta_share = max(eta_share, eta * np.linalg.norm(vt) / np.linalg.norm(Ft))
    assert worst < 1e-10
    assert eta_share > 0.1  # the damping term is large: the two readings differ


def test_eq4_displacement_recomputed_on_capped_particle_contacts():
    # The same identity on every capped particle-particle contact of a
    # shaken polydisperse cluster, with k_t = 8 G* sqrt(r* dn) from the
    # geometry at the start of each step.
    mat = gen.Material.make(restitution=0.5, mu=0.3)
    sc = gen.scene_cluster(seed=11, n_side=4, vel_sigma=1.0, polydisperse=True, walls=0,
                           gravity=(0, 0, 0))
    sc.materials = [mat]
    s = oracle.Sim(sc, mode=0)
    seen = 0
    for _ in range(10):
        x0 = s.x.copy()
        s.step(keep_contact_forces=True)
        h = s.hist
        part, d = _pair_normals(x0, h)
        dist = np.linalg.norm(d, axis=1)
        n = d / dist[:, None]
        ri, rj = sc.r[h.i], sc.r[h.j]
        dn = ri + rj - dist
        kt = np.array([_mindlin_kt(mat, a, b, c) for a, b, c in zip(ri, rj, dn)])
        F = s.cF
        fn = np.abs(np.sum(F * n, axis=1))
        Ft = np.linalg.norm(F - np.sum(F * n, axis=1)[:, None] * n, axis=1)
        cap = Ft >= 0.3 * fn * (1 - 1e-12)
        seen += int(cap.sum())
        if cap.any():
            assert _capped_invariant(F[cap], h.dt[cap], n[cap], kt[cap]).max() < 1e-9
    assert seen > 20


def _peculiar_momentum(s, m, shear, lo_y):
    return (m * (s.v[:, 0] - shear * (s.x[:, 1] - lo_y))).sum()


def test_lees_edwards_wrap_keeps_peculiar_momentum():
    # Simple shear u = shear (y - lo_y) along x: a particle crossing the high y
    # boundary re-enters at the low one with x shifted back by the image
    # offset and v_x lowered by shear L_y, so its velocity relative to the
    # flow is unchanged.  Pair forces cancel (images included), so with zero
    # total momentum along y the total momentum relative to the flow,
    # sum m (v_x - shear (y - lo_y)), stays constant through the wraps.
    shear = 2000.0
    sc = gen.scene_random(seed=31, n=1000, phi=0.25, p_touch=0.7, walls=0, periodic=7,
                          gravity=(0, 0, 0), shear_rate=shear, vel_sigma=10.0)
    m = 1200 * 4 / 3 * np.pi * sc.r ** 3
    sc.v[:, 1] -= (m * sc.v[:, 1]).sum() / m.sum()  # no net motion across y
    s = oracle.Sim(sc, mode=1)
    q0 = _peculiar_momentum(s, m, shear, sc.lo[1])
    scale = (m * (np.abs(s.v[:, 0]) + shear * (sc.hi[1] - sc.lo[1]))).sum()
    Ly = sc.hi[1] - sc.lo[1]
    wraps = 0
    for _ in range(100):
        y0 = s.x[:, 1].copy()
        s.step()
        wraps += int(np.sum(np.abs(s.x[:, 1] - y0) > 0.5 * Ly))
        assert abs(_peculiar_momentum(s, m, shear, sc.lo[1]) - q0) <= 1e-12 * scale
    assert wraps >= 5 and len(s.hist) > 100


def test_lees_edwards_shifted_copy_follows_the_same_motion():
    # A sheared periodic box is unchanged by moving everything by b along y
    # while adding shear * b to v_x (a boost with the flow).  A compressed
    # cluster in the middle of the box (no boundary involved) and the same
    # cluster moved across the y boundary (pairs in contact through the
    # sheared image, particles wrapping during the run) must follow the same
    # motion once the second is brought back.
    shear, t0 = 5000.0, 3.7e-4
    a = gen.scene_cluster(seed=5, n_side=4, vel_sigma=0.05, polydisperse=True, walls=0,
                          gravity=(0, 0, 0))
    Lb = 3.0 * (a.hi[0] - a.lo[0])
    a.x += (Lb - (a.hi[0] - a.lo[0])) / 2
    a.hi = np.full(3, Lb)
    a.periodic = 7
    a.shear_rate = shear
    a.materials = [gen.Material.make(restitution=0.5, mu=0.3)]
    sa = oracle.Sim(a, mode=0)
    dt = sa.dt
    k = 150
    D = lambda t: math.fmod(shear * Lb * t, Lb)
    # move the cluster so that the particle with the largest upward speed
    # among those in its middle layer sits just below the boundary (the
    # particles above it start across): it crosses about a third of the way
    # through the run
    mid = np.argsort(np.abs(a.x[:, 1] - np.median(a.x[:, 1])))[:16]
    p = mid[np.argmax(a.v[mid, 1])]
    assert a.v[p, 1] > 0
    b = (Lb - a.x[p, 1]) - 0.3 * k * dt * a.v[p, 1]
    bsc = a.copy()
    y = a.x[:, 1] + b
    wrap0 = y >= Lb
    bsc.x[:, 1] = np.where(wrap0, y - Lb, y)
    bsc.x[:, 0] = np.where(wrap0, np.mod(a.x[:, 0] - D(t0), Lb), a.x[:, 0])
    bsc.v[:, 0] = a.v[:, 0] + shear * b - np.where(wrap0, shear * Lb, 0.0)
    assert 0 < wrap0.sum() < a.n
    sa.time = t0
    sb = oracle.Sim(bsc, dt=dt, mode=0)
    sb.time = t0
    crossed, across, total = 0, 0, 0
    for _ in range(k):
        yb = sb.x[:, 1].copy()
        sa.step()
        sb.step()
        crossed += int(np.sum(np.abs(sb.x[:, 1] - yb) > 0.5 * Lb))
        assert len(sa.hist) == len(sb.hist)
        total += len(sb.hist)
        hi_, hj_ = sb.hist.i.astype(np.int64), sb.hist.j.astype(np.int64)
        across += int(np.sum(np.abs(yb[hi_] - yb[hj_]) > 0.5 * Lb))
    # particles wrapped during the run, and many contacts acted through the
    # sheared image
    assert crossed >= 1 and across > 0.05 * total and total > 20 * k
    assert np.all(np.abs(sa.x[:, 1] - a.x[:, 1]) < 0.25 * Lb)  # the reference never wraps
    # bring the shifted copy back: w = number of wraps relative to the shift
    w = np.rint((sa.x[:, 1] + b - sb.x[:, 1]) / Lb)
    t1 = sa.time
    # the boosted copy also drifts along x with the flow speed at b
    xb = np.mod(sb.x[:, 0] + w * D(t1) - shear * b * (t1 - t0), Lb)
    dx = xb - sa.x[:, 0]
    dx -= Lb * np.rint(dx / Lb)
    move = np.linalg.norm(sa.x - a.x, axis=1).max()
    assert np.abs(dx).max() <= 1e-6 * move
    assert np.abs(sb.x[:, 1] + w * Lb - b - sa.x[:, 1]).max() <= 1e-6 * move
    assert np.abs(sb.x[:, 2] - sa.x[:, 2]).max() <= 1e-6 * move
    dv = sa.v - a.v
    vscale = np.abs(dv).max()
    assert np.abs(sb.v[:, 0] + w * shear * Lb - shear * b - sa.v[:, 0]).max() <= 1e-6 * vscale
    assert np.abs(sb.v[:, 1:] - sa.v[:, 1:]).max() <= 1e-6 * vscale
    assert np.abs(sb.w - sa.w).max() <= 1e-6 * np.abs(sa.w).max()
