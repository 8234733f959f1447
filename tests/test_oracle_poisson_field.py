"""Pins of the oracle's Poisson solve (eqs. 6-7) and field (eq. 10)."""
import numpy as np
import pytest

from oracle import field
from oracle import geometry as geo
from oracle.grid import Grid
from oracle.philox import philox4x32_10
from oracle.poisson import PoissonSolver


def _kat():
    import os
    p = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    for line in open(p):
        if line.startswith("#") or not line.strip():
            continue
        yield [int(t, 16) for t in line.split()]


def test_philox_known_answers():
    """The oracle's Philox4x32-10 reproduces the published known-answer vectors."""
    for v in _kat():
        out = philox4x32_10(*v[:4], *v[4:6])
        assert [int(x) for x in out] == v[6:]


@pytest.mark.parametrize("alpha", [0.0, 0.2, -0.24])
def test_vacuum_solution_is_linear_in_x1(alpha):
    """x1 is harmonic (charge + dipole potential), so with rho = 0 and fixed
    potentials on x1 = -1 and x1 = x1_out the discrete solution is exactly
    linear in x1: every difference in the stencil is exact on it."""
    g = Grid(48, 40, -0.1, alpha)
    S = PoissonSolver(g)
    phi = S.solve(np.zeros(g.shape), -2.5, 0.0)
    X1, _ = g.mesh()
    lin = -2.5 + 2.5 * (X1 + 1.0) / 0.9
    assert np.max(np.abs(phi - lin)) < 1e-13


def _manufactured(g, which):
    X1, X2 = g.mesh()
    r = geo.r_of(X1, X2, g.alpha)
    R, Z = geo.cyl_of(X1, X2, g.alpha)
    return {"r2": (r * r, 6.0), "Z": (Z, 0.0), "R2": (R * R, 4.0), "Z2": (Z * Z, 2.0),
            "Zr": (Z * r * r, 10.0 * Z)}[which]


@pytest.mark.parametrize("alpha", [0.0, 0.2])
@pytest.mark.parametrize("which", ["r2", "Z", "R2", "Z2", "Zr"])
def test_manufactured_solutions_second_order(alpha, which):
    """Cartesian Laplacians of r^2, Z, R^2, Z^2 and Z r^2 are 6, 0, 4, 2 and 10 Z;
    the discrete solution with those sources converges to the function at
    second order -- every coefficient of eq. (7), its sign and the axis rows
    enter (a dropped or mis-signed term leaves an O(1) error)."""
    errs = []
    for n in (16, 32, 64):
        g = Grid(n, n, -0.1, alpha)
        f, lap = _manufactured(g, which)
        b = np.broadcast_to(lap, g.shape).copy()
        b[:, 0] = f[:, 0]
        b[:, -1] = f[:, -1]
        phi = PoissonSolver(g).solve_rhs(b)
        errs.append(np.max(np.abs(phi - f)) / np.max(np.abs(f)))
    order = np.log2(errs[1] / errs[2])
    assert 1.8 < order < 2.3, errs
    assert errs[2] < 2e-2


def test_spherical_source_symmetric_solution():
    """alpha = 0 and a source depending on r only: the solution does not depend
    on x2 (to round-off) and matches the radial ODE solution to O(h^2):
    Lap(phi) = -k  ->  phi = -k r^2 / 6 + A + B / r."""
    g = Grid(64, 32, -0.1, 0.0)
    k = 3.0
    S = PoissonSolver(g)
    phi = S.solve(np.full(g.shape, -k), -2.5, 0.0)
    assert np.max(np.abs(phi - phi[0:1, :])) < 1e-11
    r = -1.0 / g.x1_nodes()
    ro = r[-1]
    # phi(1) = -2.5, phi(ro) = 0
    Bc = (-2.5 + k / 6 - (k * ro * ro / 6)) / (1.0 - 1.0 / ro)
    Ac = k * ro * ro / 6 - Bc / ro
    exact = -k * r * r / 6 + Ac + Bc / r
    assert np.max(np.abs(phi[5] - exact)) < 2e-2 * np.max(np.abs(exact))


def test_mirror_symmetry_at_alpha_zero():
    """alpha = 0: a source mirrored in x2 gives a mirrored potential."""
    g = Grid(32, 32, -0.1, 0.0)
    rng = np.random.default_rng(4)
    src = rng.normal(size=g.shape)
    src = src + src[::-1, :]
    phi = PoissonSolver(g).solve(src, -2.5, 0.0)
    assert np.max(np.abs(phi - phi[::-1, :])) < 1e-12


@pytest.mark.parametrize("alpha", [0.0, 0.2])
def test_gradient_and_gather_exact_on_linear_potential(alpha):
    """phi = a + b x1 + c x2: central and one-sided differences are exact, the
    bilinear interpolation of constants is exact, so the gathered field equals
    -(b grad x1 + c grad x2) with the analytic metric, at any particle position."""
    g = Grid(24, 20, -0.2, alpha)
    X1, X2 = g.mesh()
    b, c = 2.7, -0.4
    phi = 0.3 + b * X1 + c * X2
    p1, p2 = field.nodal_gradient(phi, g)
    assert np.allclose(p1, b, atol=1e-12) and np.allclose(p2, c, atol=1e-12)
    rng = np.random.default_rng(5)
    x1 = rng.uniform(-1.0, -0.2, 500)
    x2 = rng.uniform(-1.0, 1.0, 500)
    ER, EZ = field.electric_field(p1, p2, x1, x2, g)
    # independent construction: finite differences of the potential in (R, Z)
    R, Z = geo.cyl_of(x1, x2, alpha)
    h = 1e-6

    def pot(RR, ZZ):
        a1, a2 = geo.conforming_of(RR, ZZ, alpha)
        return 0.3 + b * a1 + c * a2

    ER_fd = -(pot(R + h, Z) - pot(R - h, Z)) / (2 * h)
    EZ_fd = -(pot(R, Z + h) - pot(R, Z - h)) / (2 * h)
    inside = R > 1e-3
    assert np.max(np.abs(ER - ER_fd)[inside]) < 1e-6
    assert np.max(np.abs(EZ - EZ_fd)[inside]) < 1e-6


def test_gradient_second_order_on_smooth_potential():
    """Nodal derivatives of a smooth function converge at second order,
    including the one-sided edge formulas."""
    errs = []
    for n in (16, 32, 64):
        g = Grid(n, n, -0.1, 0.1)
        X1, X2 = g.mesh()
        phi = np.sin(3 * X1) * np.cos(2 * X2)
        p1, p2 = field.nodal_gradient(phi, g)
        e1 = np.max(np.abs(p1 - 3 * np.cos(3 * X1) * np.cos(2 * X2)))
        e2 = np.max(np.abs(p2 + 2 * np.sin(3 * X1) * np.sin(2 * X2)))
        errs.append(max(e1, e2))
    assert 1.8 < np.log2(errs[1] / errs[2]) < 2.3
