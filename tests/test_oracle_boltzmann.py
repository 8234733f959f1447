"""Pins of the oracle's Boltzmann-electron field solve (Section 2: electrons not
moved, n_e = n0 exp(e phi / Te), eq. 6 then nonlinear in phi)."""
import numpy as np
import pytest

from oracle import geometry as geo
from oracle.grid import Grid
from oracle.poisson import assemble, solve_boltzmann


def _debye_huckel(r, kappa, phi_g, r_out):
    """Spherical Debye-Hueckel potential: phi'' + (2/r) phi' = phi / kappa^2 with
    phi(1) = phi_g, phi(r_out) = 0, i.e. (C1 exp(-r/kappa) + C2 exp(r/kappa)) / r."""
    M = np.array([[np.exp(-1.0 / kappa), np.exp(1.0 / kappa)],
                  [np.exp(-r_out / kappa), np.exp(r_out / kappa)]])
    c = np.linalg.solve(M, np.array([phi_g, 0.0]))
    return (c[0] * np.exp(-r / kappa) + c[1] * np.exp(r / kappa)) / r


@pytest.mark.parametrize("kappa", [0.5, 1.0, 3.0])
def test_small_potential_is_debye_screened(kappa):
    """Uniform unit ion density and a grain potential of 1e-6 Te/e around a
    sphere: exp(phi) = 1 + phi to 5e-7, so the solution is the Debye-Hueckel
    closed form, reached at second order in the grid (the screening term's
    sign and its 1/kappa^2 enter: a wrong sign gives an oscillating solution, a
    wrong power a different decay length)."""
    phi_g = 1e-6
    errs = []
    for n in (64, 128):
        g = Grid(n, 8, -0.1, 0.0)
        phi, _ = solve_boltzmann(g, assemble(g), np.ones(g.shape), kappa, phi_g, 0.0)
        X1, X2 = g.mesh()
        ex = _debye_huckel(geo.r_of(X1, X2, 0.0), kappa, phi_g, 10.0)
        errs.append(np.max(np.abs(phi - ex)) / phi_g)
    assert errs[1] < 2e-5
    assert errs[0] / errs[1] > 3.5


def test_neutral_plasma_has_zero_potential():
    """n_i = n_e = n0 everywhere is a solution with phi = 0 on both boundaries."""
    g = Grid(32, 24, -0.2, 0.15)
    phi, _ = solve_boltzmann(g, assemble(g), np.ones(g.shape), 1.0, 0.0, 0.0)
    assert np.max(np.abs(phi)) < 1e-14


@pytest.mark.parametrize("alpha", [0.0, 0.2])
def test_newton_reaches_a_large_amplitude_solution(alpha):
    """A manufactured potential of O(1) amplitude (electron density varying by
    e^2.5 across the domain): with rho_p chosen so that it solves the discrete
    equations, Newton returns it to round-off, with quadratic convergence (a few
    steps from the linear start, ten here)."""
    g = Grid(40, 32, -0.1, alpha)
    A = assemble(g)
    X1, X2 = g.mesh()
    s = (X1 + 1.0) / 0.9
    phi_m = -2.5 + 2.5 * s + 0.5 * np.sin(np.pi * s) * (1.0 + 0.3 * X2)
    kappa = 0.7
    # A phi = -(rho_p - exp(phi)) / kappa^2 on the unknown nodes
    rho_p = np.exp(phi_m) - kappa ** 2 * (A @ phi_m.ravel()).reshape(g.shape)
    phi, it = solve_boltzmann(g, A, rho_p, kappa, -2.5, 0.0)
    assert np.max(np.abs(phi - phi_m)) < 1e-12
    assert it <= 12
