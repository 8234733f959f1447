"""Pins of the oracle's mover (eq. 9, leapfrog) and grain/boundary treatment."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import geometry as geo
from oracle import mover
from oracle.pic import Config, Simulation, Species


def _sim(alpha, wce, q, m, phi_kind="linear", kappa=1.0, dt=0.05, x1_out=-0.05):
    cfg = Config(alpha=alpha, n1=32, n2=32, x1_out=x1_out, wce=wce, kappa=kappa, dt=dt,
                 species=[Species(q=q, m=m, weight=1.0)])
    sim = Simulation(cfg)
    X1, X2 = sim.grid.mesh()
    if phi_kind == "linear":
        sim.set_phi(-2.5 + 2.5 * (X1 + 1.0) / (1.0 + x1_out))
    else:
        sim.set_phi(np.zeros(sim.grid.shape))
    sim.frozen = True
    sim.inject_enabled = False
    return sim


def _state(sim):
    p = sim.particles(0)
    R, Z = geo.cyl_of(p["x1"], p["x2"], sim.cfg.alpha)
    return R, Z, p["vR"], p["vZ"], p["vT"]


def _eq9_rhs(alpha, qm, kappa, wce, b):
    """eq. (9) in normalised units with E = -b grad x1 (the field of the potential
    linear in x1), state (R, Z, VR, VZ, VT, azimuth)."""
    def f(t, y):
        R, Z, VR, VZ, VT, _ = y
        x1, x2 = geo.conforming_of(R, Z, alpha)
        x1R, x1Z, _, _ = geo.metric(x1, x2, alpha)
        ER, EZ = -b * x1R, -b * x1Z
        return [kappa * VR, kappa * VZ,
                qm * (kappa * ER - wce * VT) + kappa * VT * VT / R,
                qm * kappa * EZ,
                qm * wce * VR - kappa * VR * VT / R,
                kappa * VT / R]
    return f


@pytest.mark.parametrize("alpha,wce,q", [(0.0, 0.0, 1.0), (0.2, 0.0, 1.0), (0.2, 0.7, 1.0), (0.15, 1.3, -1.0)])
def test_leapfrog_converges_to_eq9_at_second_order(alpha, wce, q):
    """Positions after a fixed time converge to an accurate ODE integration of
    eq. (9) (centrifugal, Coriolis and axial-field terms as printed) with error
    ratio ~4 per halving of dt.  v^{-1/2} is taken from the ODE and rotated into
    the meridional frame of x^0, as leapfrog requires."""
    T, m = 1.6, 1.0
    R0_, Z0_, VR0, VZ0, VT0 = 4.0, 1.0, -0.4, 0.3, 0.5
    b = 2.5 / 0.95
    f = _eq9_rhs(alpha, q / m, 1.0, wce, b)
    ref = solve_ivp(f, (0, T), [R0_, Z0_, VR0, VZ0, VT0, 0.0], rtol=1e-12, atol=1e-12).y[:, -1]
    errs = []
    for dt in (0.04, 0.02, 0.01):
        back = solve_ivp(f, (0, -dt / 2), [R0_, Z0_, VR0, VZ0, VT0, 0.0], rtol=1e-13, atol=1e-13).y[:, -1]
        dphi = 0.0 - back[5]
        c, s = np.cos(dphi), np.sin(dphi)
        vR = c * back[2] + s * back[4]
        vT = -s * back[2] + c * back[4]
        sim = _sim(alpha, wce, q, m, dt=dt)
        x1, x2 = geo.conforming_of(R0_, Z0_, alpha)
        sim.set_particles(0, [x1], [x2], [vR], [back[3]], [vT])
        sim.run(int(round(T / dt)))
        R, Z, *_ = _state(sim)
        errs.append(np.hypot(R[0] - ref[0], Z[0] - ref[1]))
    assert errs[2] < 2e-3
    assert 3.3 < errs[0] / errs[1] < 4.8 and 3.3 < errs[1] / errs[2] < 4.8, errs


def _cartesian_boris(p, v, qm, kappa, wce, dt, nsteps, alpha, b):
    """Textbook 3D Cartesian Boris (Birdsall & Langdon) in the field -b grad x1 and
    the axial field of eq. (9), which is B_z = -B in a right-handed (R, Theta, Z)
    frame.  Independent of the oracle's meridional-plane formulation."""
    p = np.array(p, dtype=float)
    v = np.array(v, dtype=float)
    tvec = np.array([0.0, 0.0, -qm * wce * dt / 2])
    svec = 2 * tvec / (1 + tvec @ tvec)
    out = []
    for _ in range(nsteps):
        R = np.hypot(p[0], p[1])
        x1, x2 = geo.conforming_of(R, p[2], alpha)
        x1R, x1Z, _, _ = geo.metric(x1, x2, alpha)
        ER, EZ = -b * x1R, -b * x1Z
        E = np.array([ER * p[0] / R, ER * p[1] / R, EZ])
        vm = v + 0.5 * qm * kappa * dt * E
        vp = vm + np.cross(vm + np.cross(vm, tvec), svec)
        v = vp + 0.5 * qm * kappa * dt * E
        p = p + kappa * dt * v
        out.append((p.copy(), v.copy()))
    return out


@pytest.mark.parametrize("alpha,wce,q,start", [(0.2, 0.9, 1.0, (3.0, 0.5, -0.3, 0.2, 0.6)),
                                               (0.1, 0.0, 1.0, (0.02, 4.0, -0.5, 0.1, 0.01)),
                                               (0.0, 1.5, -1.0, (0.3, -3.0, -0.2, 0.3, 0.05))])
def test_equals_cartesian_boris(alpha, wce, q, start):
    """The meridional-plane leapfrog is the 3D Cartesian Boris scheme restricted
    by symmetry: (R, Z, |v|, L_z) agree to round-off every step, also on orbits
    that pass next to or across the axis."""
    R0_, Z0_, vR, vZ, vT = start
    b = 2.5 / 0.95
    m, dt, n = 1.0, 0.05, 60
    ref = _cartesian_boris([R0_, 0, Z0_], [vR, vT, vZ], q / m, 1.0, wce, dt, n, alpha, b)
    sim = _sim(alpha, wce, q, m, dt=dt)
    x1, x2 = geo.conforming_of(R0_, Z0_, alpha)
    sim.set_particles(0, [x1], [x2], [vR], [vZ], [vT])
    for k in range(n):
        sim.step()
        if sim.resident(0) == 0:
            pytest.fail("particle left the domain")
        R, Z, VR, VZ, VT = _state(sim)
        p, v = ref[k]
        assert abs(R[0] - np.hypot(p[0], p[1])) < 1e-11
        assert abs(Z[0] - p[2]) < 1e-11
        assert abs(VZ[0] - v[2]) < 1e-11
        assert abs(np.hypot(VR[0], VT[0]) - np.hypot(v[0], v[1])) < 1e-11
        assert abs(R[0] * VT[0] - (p[0] * v[1] - p[1] * v[0])) < 1e-11


def test_pure_magnetic_field_exact_gyration_and_energy():
    """E = 0: the discrete orbit is the exact Boris gyration -- velocity turns by
    2 atan(omega dt / 2) per step, so x^n = x^0 + kappa dt u (e^{i n th} - 1) /
    (e^{i th} - 1) in the transverse plane (closed form), |v| is conserved to
    round-off, Z advances uniformly."""
    q, m, wce, dt = -1.0, 1.0, 2.0, 0.05
    sim = _sim(0.0, wce, q, m, phi_kind="zero", dt=dt)
    R0_, Z0_, vR, vZ, vT = 5.0, 0.3, 0.3, 0.05, -0.2
    x1, x2 = geo.conforming_of(R0_, Z0_, 0.0)
    sim.set_particles(0, [x1], [x2], [vR], [vZ], [vT])
    th = 2 * np.arctan(q / m * wce * dt / 2)
    u = np.exp(1j * th) * (vR + 1j * vT)        # v^{1/2} in the Cartesian frame of x^0
    speed0 = np.sqrt(vR ** 2 + vZ ** 2 + vT ** 2)
    for n in range(1, 201):
        sim.step()
        R, Z, VR, VZ, VT = _state(sim)
        xn = R0_ + dt * u * (np.exp(1j * n * th) - 1) / (np.exp(1j * th) - 1)
        assert abs(R[0] - abs(xn)) < 1e-12
        assert abs(Z[0] - (Z0_ + n * dt * vZ)) < 1e-12
        assert abs(np.sqrt(VR[0] ** 2 + VZ[0] ** 2 + VT[0] ** 2) - speed0) < 1e-14


def test_chord_through_sphere_is_absorbed_at_first_crossing():
    """alpha = 0: a step whose straight chord cuts through the unit sphere is an
    absorption even though its endpoint is outside; the impact point is the
    first root of |P0 + t d| = 1 (closed form)."""
    R, Z = np.array([1.2]), np.array([0.05])
    vR, vZ, vT = np.array([-10.0]), np.array([0.3]), np.array([0.2])
    step = 0.25                                   # chord length 2.5 > diameter
    Rn, Zn, *_ = mover.drift(R, Z, vR, vZ, vT, step)
    x1n, _ = geo.conforming_of(Rn, Zn, 0.0)
    assert x1n[0] > -1.0                          # endpoint outside the grain
    hit, t_in = mover.grain_hits(R, Z, vR, vZ, vT, step, x1n, 0.0)
    assert hit[0]
    X, Y, Zi = mover.impact(R, Z, vR, vZ, vT, step, t_in, 0.0)
    p0 = np.array([R[0], 0.0, Z[0]])
    d = step * np.array([vR[0], vT[0], vZ[0]])
    a, bq, c = d @ d, 2 * p0 @ d, p0 @ p0 - 1
    t1 = (-bq - np.sqrt(bq * bq - 4 * a * c)) / (2 * a)
    assert np.allclose([X[0], Y[0], Zi[0]], p0 + t1 * d, atol=1e-12)
    # a chord passing outside the sphere is not absorbed
    vZ2 = np.array([10.0])
    Rn, Zn, *_ = mover.drift(np.array([1.2]), np.array([1.2]), np.array([-1.0]), vZ2, vT, 0.05)
    x1n, _ = geo.conforming_of(Rn, Zn, 0.0)
    hit, _ = mover.grain_hits(np.array([1.2]), np.array([1.2]), np.array([-1.0]), vZ2, vT, 0.05, x1n, 0.0)
    assert not hit[0]


def test_impact_tallies_frame():
    """The impact tally rotates the velocity into the meridional plane of the
    impact point: angular momentum equals the Cartesian x v_y - y v_x."""
    X, Y, Zi = np.array([0.6]), np.array([0.8]), np.array([0.0])
    vR, vZ, vT = np.array([-1.0]), np.array([0.5]), np.array([0.25])
    b, vRi, vZi, L = mover.impact_tallies(X, Y, Zi, vR, vZ, vT, 8)
    assert b[0] == 4
    assert np.isclose(L[0], X[0] * vT[0] - Y[0] * vR[0])
    assert np.isclose(vRi[0], 0.6 * -1.0 + 0.8 * 0.25)
    assert vZi[0] == 0.5


def test_escape_and_bookkeeping():
    """A particle driven past x1_out escapes; counts add up exactly."""
    sim = _sim(0.1, 0.0, -1.0, 1.0, phi_kind="zero", dt=0.5)
    x1, x2 = geo.conforming_of(np.array([15.0, 3.0]), np.array([0.0, 0.0]), 0.1)
    sim.set_particles(0, x1, x2, [5.0, -3.0], [0.0, 0.0], [0.0, 0.0])
    sim.run(3)
    assert sim.escaped[0] == 1 and sim.absorbed[0] == 1 and sim.resident(0) == 0


def _inside_brute(P, alpha):
    """Inside the grain: r <= rho(x2), the grain radius of eq. (3) at x1 = -1."""
    r = np.linalg.norm(P, axis=-1)
    with np.errstate(invalid="ignore", divide="ignore"):
        x2 = np.where(r > 0, P[..., 2] / np.where(r > 0, r, 1.0), 0.0)
    return r <= geo.r_of(-1.0, x2, alpha)


@pytest.mark.parametrize("alpha", [0.0, 0.1, 0.2, -0.2, 0.24, -0.2499])
def test_chord_impact_matches_dense_sampling(alpha):
    """Any |alpha| < 1/4: the chord test's outcome and first crossing against a
    brute-force scan of 8001 points per chord with the grain's definition
    r <= rho(x2) (cases within 1e-7 of grazing, where the scan itself is unsure,
    are left out)."""
    rng = np.random.default_rng(7)
    n = 2000
    # start points just outside the grain, any direction and chord length
    x2 = rng.uniform(-1, 1, n)
    rg = geo.r_of(-1.0, x2, alpha)
    r0 = rg * (1.0 + rng.uniform(1e-4, 0.6, n))
    s = np.sqrt(1 - x2 * x2)
    R, Z = r0 * s, r0 * x2
    d = rng.normal(size=(n, 3))
    d *= (rng.uniform(0.01, 2.5, n) / np.linalg.norm(d, axis=1))[:, None]
    # half of the chords pass the origin at a distance r* between the smallest
    # grain radius and r_c = 2/3 (there G is concave around the closest point),
    # tangentially, near the end of the grain that is closest to the origin
    m = n // 2
    rmin = geo.r_of(-1.0, -np.sign(alpha) if alpha else 1.0, alpha)
    rs = rng.uniform(rmin, max(rmin, 2.0 / 3.0) + 0.05, m)
    th = rng.uniform(0.0, 0.5, m)
    zs = -np.sign(alpha) if alpha else 1.0
    Pc = np.stack([rs * np.sin(th), np.zeros(m), zs * rs * np.cos(th)], axis=1)
    u = np.cross(Pc, rng.normal(size=(m, 3)))
    u /= np.linalg.norm(u, axis=1)[:, None]
    L = rng.uniform(0.05, 1.5, m)
    f = rng.uniform(0.2, 0.8, m)
    P0 = Pc - (f * L)[:, None] * u
    R[:m] = np.hypot(P0[:, 0], P0[:, 1])
    Z[:m] = P0[:, 2]
    # rotate the chord so that its start is in the meridional plane Y = 0
    c, s = P0[:, 0] / R[:m], P0[:, 1] / R[:m]
    dd = L[:, None] * u
    d[:m] = np.stack([c * dd[:, 0] + s * dd[:, 1], -s * dd[:, 0] + c * dd[:, 1], dd[:, 2]], axis=1)
    keep = ~_inside_brute(np.stack([R, 0 * R, Z], axis=1), alpha)
    R, Z, d = R[keep], Z[keep], d[keep]
    hit, t = mover.chord_impact(R, Z, d[:, 0], d[:, 1], d[:, 2], alpha)
    ts = np.linspace(0.0, 1.0, 8001)
    P = np.stack([R[:, None] + ts * d[:, 0:1], ts * d[:, 1:2], Z[:, None] + ts * d[:, 2:3]], axis=-1)
    ins = _inside_brute(P, alpha)
    any_in = ins.any(axis=1)
    # margin: distance of the chord's samples from the surface, relative
    r = np.linalg.norm(P, axis=-1)
    with np.errstate(invalid="ignore", divide="ignore"):
        margin = np.min(np.abs(r - geo.r_of(-1.0, P[..., 2] / r, alpha)), axis=1)
    sure = margin > 1e-7
    assert np.array_equal(hit[sure], any_in[sure])
    assert hit.sum() > 100 and (~hit).sum() > 100
    # the first crossing lies within one sample of the scan's first inside point
    k = np.argmax(ins, axis=1)
    h = hit & any_in
    assert np.all(t[h] <= ts[k[h]] + 1e-12)
    assert np.all(t[h] >= ts[np.maximum(k[h] - 1, 0)] - 1e-12)
    # and it is on the surface: r = rho(x2) there
    Pi = np.stack([R + t * d[:, 0], t * d[:, 1], Z + t * d[:, 2]], axis=-1)[h]
    ri = np.linalg.norm(Pi, axis=-1)
    assert np.allclose(ri, geo.r_of(-1.0, Pi[:, 2] / ri, alpha), rtol=1e-12)


def test_grazing_chord_on_a_dipole_grain_is_absorbed():
    """alpha = 0.2: a chord whose end points and whose closest approach to the
    origin are all outside the grain, but which clips it between them, is an
    absorption (the earlier closest-approach test missed it)."""
    alpha = 0.2
    R = np.array([1.01])
    Z = np.array([-0.1])
    d = np.array([0.0, 0.0, 0.45])
    for t in (0.0, 1.0):
        x1, _ = geo.conforming_of(R + t * d[0], Z + t * d[2], alpha)
        assert x1[0] > -1.0
    tc = -(Z[0] * d[2]) / (d[2] ** 2)
    x1c, _ = geo.conforming_of(R, Z + tc * d[2], alpha)
    assert x1c[0] > -1.0
    hit, t = mover.chord_impact(R, Z, d[0:1], d[1:2], d[2:3], alpha)
    assert hit[0]
    x1i, _ = geo.conforming_of(R, Z + t * d[2], alpha)
    assert abs(x1i[0] + 1.0) < 1e-12
    # a chord that passes the origin deep inside the grain (where x1 from eq. 2
    # is not below -1 any more) is absorbed at its first crossing
    P0, d = np.array([1.2, 0.0, -0.6]), np.array([-2.4, 0.0, 1.2])
    hit, t = mover.chord_impact(P0[0:1], P0[2:3], d[0:1], d[1:2], d[2:3], alpha)
    assert hit[0] and 0.1 < t[0] < 0.25
    Pi = P0 + t[0] * d
    x1i, _ = geo.conforming_of(np.hypot(Pi[0], Pi[1]), Pi[2], alpha)
    assert abs(x1i + 1.0) < 1e-12
