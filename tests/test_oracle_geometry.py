"""Pins of the oracle's geometry (eqs. 2-5, 7, 8, 10) against closed forms and
independent numerical constructions (not against a retyped copy of the formula)."""
import numpy as np
import pytest
from scipy import integrate

from oracle import geometry as geo
from oracle import grid as gridmod

ALPHAS = [0.0, 0.1, -0.15, 0.2, 0.24]


@pytest.mark.parametrize("alpha", ALPHAS)
def test_inverse_map_round_trip(alpha):
    """eq. (3) inverts eq. (2): r -> x1 -> r and x1 -> r -> x1 to a few ulp."""
    r = np.linspace(1.0, 60.0, 301)[:, None] * np.ones((1, 41))
    x2 = np.linspace(-1.0, 1.0, 41)[None, :] * np.ones((301, 1))
    # only points outside the grain (x1 >= -1) are in the domain
    x1 = geo.x1_of(r, x2, alpha)
    ok = x1 >= -1.0
    r_back = geo.r_of(x1, x2, alpha)
    assert np.max(np.abs(r_back - r)[ok] / r[ok]) < 8e-16 * 8
    x1s = np.linspace(-1.0, -0.01, 200)[:, None]
    x2s = np.linspace(-1.0, 1.0, 57)[None, :]
    back = geo.x1_of(geo.r_of(x1s, x2s, alpha), x2s, alpha)
    assert np.max(np.abs(back - x1s)) < 1e-15 * 8


@pytest.mark.parametrize("alpha", ALPHAS)
def test_inverse_is_the_outer_root(alpha):
    """r(x1, x2) is the positive root of x1 r^2 + r + alpha x2 = 0 (from eq. 2)
    that lies outside the grain; numpy's polynomial root finder is the check."""
    rng = np.random.default_rng(1)
    for _ in range(50):
        x1 = -rng.uniform(0.02, 1.0)
        x2 = rng.uniform(-1.0, 1.0)
        roots = np.roots([x1, 1.0, alpha * x2])
        roots = roots[np.isreal(roots)].real
        assert np.isclose(geo.r_of(x1, x2, alpha), roots.max(), rtol=1e-12)


def test_sphere_special_case():
    """alpha = 0: x1 = -1/r; the grain x1 = -1 is the unit sphere."""
    x1 = np.linspace(-1.0, -0.05, 20)
    assert np.allclose(geo.r_of(x1, 0.3, 0.0), -1.0 / x1, rtol=1e-15)
    assert np.allclose(geo.r_of(-1.0, np.linspace(-1, 1, 9), 0.0), 1.0)


@pytest.mark.parametrize("alpha", ALPHAS)
def test_metric_matches_finite_differences(alpha):
    """Analytic dx1/dR, dx1/dZ, dx2/dR, dx2/dZ against central differences of the
    composed map (R, Z) -> (x1, x2)."""
    rng = np.random.default_rng(2)
    x1 = rng.uniform(-1.0, -0.05, 200)
    x2 = rng.uniform(-0.98, 0.98, 200)
    R, Z = geo.cyl_of(x1, x2, alpha)
    h = 1e-6
    a1, a2 = geo.conforming_of(R + h, Z, alpha)
    b1, b2 = geo.conforming_of(R - h, Z, alpha)
    c1, c2 = geo.conforming_of(R, Z + h, alpha)
    d1, d2 = geo.conforming_of(R, Z - h, alpha)
    fd = [(a1 - b1) / (2 * h), (c1 - d1) / (2 * h), (a2 - b2) / (2 * h), (c2 - d2) / (2 * h)]
    an = geo.metric(x1, x2, alpha)
    for f, a in zip(fd, an):
        assert np.max(np.abs(f - a)) < 1e-7


@pytest.mark.parametrize("alpha", ALPHAS)
def test_laplace_coefficients_are_the_metric_tensor(alpha):
    """eq. (7): the d2/dx1^2, d2/dx2^2 and mixed coefficients are |grad x1|^2,
    |grad x2|^2 and 2 grad x1 . grad x2 built from the (finite-difference-pinned)
    analytic metric."""
    x1, x2 = np.meshgrid(np.linspace(-1, -0.05, 30), np.linspace(-1, 1, 31))
    x1R, x1Z, x2R, x2Z = geo.metric(x1, x2, alpha)
    c11, c22, c12, _ = geo.laplace_coeffs(x1, x2, alpha)
    assert np.allclose(c11, x1R ** 2 + x1Z ** 2, rtol=1e-13, atol=0)
    assert np.allclose(c22, x2R ** 2 + x2Z ** 2, rtol=1e-13, atol=1e-300)
    assert np.allclose(c12, 2 * (x1R * x2R + x1Z * x2Z), rtol=1e-12, atol=1e-15)


def test_laplacian_of_coordinates_by_finite_differences():
    """First-order coefficient of eq. (7): Lap(x2) = -2 x2 / r^2, and x1 is
    harmonic; checked with a 3D Cartesian finite-difference Laplacian."""
    alpha = 0.2
    rng = np.random.default_rng(3)
    h = 1e-3
    for _ in range(20):
        p = rng.normal(size=3)
        p *= rng.uniform(1.5, 8.0) / np.linalg.norm(p)

        def coords(q):
            R = np.hypot(q[0], q[1])
            return geo.conforming_of(R, q[2], alpha)

        lap1 = lap2 = 0.0
        c0 = coords(p)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            cp, cm = coords(p + e), coords(p - e)
            lap1 += (cp[0] - 2 * c0[0] + cm[0]) / h ** 2
            lap2 += (cp[1] - 2 * c0[1] + cm[1]) / h ** 2
        r = np.linalg.norm(p)
        _, _, _, c2 = geo.laplace_coeffs(c0[0], c0[1], alpha)
        assert abs(lap1) < 1e-5
        assert abs(lap2 - c2) < 1e-5 * max(1.0, abs(c2))
        assert np.isclose(c2, -2 * c0[1] / r ** 2)


def test_sphere_area_and_volume():
    """alpha = 0: integral of eq. (4) is 4 pi r^2; node volumes (eq. 5) sum to the
    spherical-shell volume 4 pi (r_out^3 - 1) / 3."""
    for x1 in (-1.0, -0.5, -0.1):
        area, _ = integrate.quad(lambda t: geo.dA_dx2(x1, t, 0.0), -1, 1)
        assert np.isclose(area, 4 * np.pi / x1 ** 2, rtol=1e-13)
    g = gridmod.Grid(32, 16, -0.1, 0.0)
    assert np.isclose(gridmod.domain_volume(g), 4 * np.pi / 3 * (1000.0 - 1.0), rtol=1e-12)
    g = gridmod.Grid(64, 32, -0.02, 0.0)
    assert np.isclose(gridmod.domain_volume(g), 4 * np.pi / 3 * (50.0 ** 3 - 1.0), rtol=1e-12)


@pytest.mark.parametrize("alpha", [0.1, 0.2, -0.24])
def test_volume_any_alpha_by_shells(alpha):
    """Node volumes sum to the volume of revolution between the grain and the
    outer surface, (2 pi / 3) int (r_out^3 - r_in^3) dx2 -- spherical-coordinate
    construction, independent of eq. (5)."""
    g = gridmod.Grid(48, 40, -0.1, alpha)
    ref, _ = integrate.quad(lambda t: geo.r_of(-0.1, t, alpha) ** 3 - geo.r_of(-1.0, t, alpha) ** 3,
                            -1, 1, epsabs=0, epsrel=1e-13, limit=200)
    assert np.isclose(gridmod.domain_volume(g), 2 * np.pi / 3 * ref, rtol=1e-11)


@pytest.mark.parametrize("alpha", [0.1, 0.2, -0.24])
def test_area_any_alpha_by_arc_length(alpha):
    """eq. (4) integrates to the area of the surface of revolution computed from
    the meridional curve (R(theta), Z(theta)) by 2 pi int R ds (Pappus), with ds
    from numerical differentiation of the curve."""
    for x1 in (-1.0, -0.3):
        th = np.linspace(0, np.pi, 200001)
        x2 = np.cos(th)
        R, Z = geo.cyl_of(x1, x2, alpha)
        ds = np.hypot(np.diff(R), np.diff(Z))
        area_curve = 2 * np.pi * np.sum(0.5 * (R[1:] + R[:-1]) * ds)
        area_eq4, _ = integrate.quad(lambda t: geo.dA_dx2(x1, t, alpha), -1, 1, epsrel=1e-13)
        assert np.isclose(area_eq4, area_curve, rtol=1e-8)


@pytest.mark.parametrize("alpha", [0.0, 0.15, -0.2, 0.24])
def test_gauss_flux_of_grad_x1(alpha):
    """-x1 is the potential of a unit point charge plus a dipole, so the flux of
    grad x1 through any surface x1 = const is 4 pi (Gauss's law)."""
    for x1 in (-1.0, -0.4, -0.1):
        def f(t):
            a, b, _, _ = geo.metric(x1, t, alpha)
            return np.hypot(a, b) * geo.dA_dx2(x1, t, alpha)
        flux, _ = integrate.quad(f, -1, 1, epsrel=1e-13)
        assert np.isclose(flux, 4 * np.pi, rtol=1e-11)


@pytest.mark.parametrize("alpha", [0.15, 0.24])
def test_vacuum_conductor_has_no_net_force(alpha):
    """A conductor in vacuum feels no net force: the integral of |grad x1| x1_Z dA
    (the Maxwell stress of the vacuum field, up to a constant) vanishes."""
    def f(t):
        a, b, _, _ = geo.metric(-1.0, t, alpha)
        return np.hypot(a, b) * b * geo.dA_dx2(-1.0, t, alpha)
    val, _ = integrate.quad(f, -1, 1, epsabs=1e-14, limit=200)
    scale, _ = integrate.quad(lambda t: abs(f(t)), -1, 1, limit=200)
    assert abs(val) < 1e-11 * scale


def test_alpha_range():
    assert geo.check_alpha(0.2499, -0.1)
    assert not geo.check_alpha(0.25, -0.1)
    assert not geo.check_alpha(-0.3, -0.1)
    assert not geo.check_alpha(0.1, 0.0)
    assert not geo.check_alpha(0.1, -1.0)
