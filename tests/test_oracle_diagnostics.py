"""Pins of the oracle's grain diagnostics (Section 2, the sentences after eq. 10:
the normal field on the conducting grain gives its surface charge, and the
electric force on the grain follows from the surface field).

Each test calls Simulation.surface_field / grain_charge / electric_force on a
potential written in closed form here, and compares with a value fixed by the
mathematics, not by a retyped copy of the oracle's formula:
  * a potential linear in x1 between the two fixed boundary potentials is the
    vacuum solution (x1 is harmonic); its normal field has flux
    -phi_1 * (flux of grad x1) = -4 pi phi_1 through the grain for any alpha
    (Gauss's law for the point charge plus dipole whose potential is -x1), so
    the grain charge is 4 pi (phi_grain - phi_out) / (1 + x1_out);
  * for a sphere (alpha = 0) and phi = phi_grain + (x1 + 1)(a + b x2), the
    one-sided derivative is exact, |grad x1| = 1 and n_Z = x2 on the grain, so
    E_n = -(a + b x2) at the nodes; the Maxwell stress integral
    2 pi int (a + b x2)^2 / 2 x2 dx2 is (4 pi / 3) a b, and the trapezoid rule
    over nodes spaced h adds exactly (4 pi / 3) a b h^2 / 2 (the rule integrates
    the odd powers exactly and x2^2 with error h^2 / 3);
  * a conductor in vacuum feels no net force for any alpha: the trapezoid sum
    tends to zero at second order.
"""
import numpy as np
import pytest

from oracle import geometry as geo
from oracle.pic import Config, Simulation

PHI_G, PHI_OUT = -2.5, 0.0


def _sim(alpha, n1, n2, x1_out=-0.1):
    return Simulation(Config(alpha=alpha, n1=n1, n2=n2, x1_out=x1_out), vacuum_field=False)


def _vacuum_phi(sim):
    X1, _ = sim.grid.mesh()
    return PHI_G + (PHI_OUT - PHI_G) * (X1 + 1.0) / (1.0 + sim.cfg.x1_out)


@pytest.mark.parametrize("alpha", [0.0, 0.1, -0.15, 0.2, 0.24])
@pytest.mark.parametrize("x1_out", [-0.1, -0.5])
def test_vacuum_grain_charge(alpha, x1_out):
    exact = 4.0 * np.pi * (PHI_G - PHI_OUT) / (1.0 + x1_out)
    errs = []
    for n2 in (32, 64, 128, 256):
        sim = _sim(alpha, 16, n2, x1_out)
        sim.set_phi(_vacuum_phi(sim))
        errs.append(abs(sim.grain_charge() - exact) / abs(exact))
    errs = np.array(errs)
    assert errs[-1] < 2e-5
    if errs[0] > 1e-12:
        order = np.log2(errs[:-1] / errs[1:])
        assert np.all((order > 1.8) & (order < 2.2)), order
    else:
        # alpha = 0: the integrand |grad x1| dA/dx2 = 2 pi is constant
        assert np.all(errs < 1e-13)


@pytest.mark.parametrize("a,b", [(0.7, -1.3), (-2.0, 0.4), (1.0, 1.0)])
def test_sphere_surface_field_and_force_closed_form(a, b):
    for n2 in (16, 64, 200):
        sim = _sim(0.0, 12, n2)
        X1, X2 = sim.grid.mesh()
        sim.set_phi(PHI_G + (X1 + 1.0) * (a + b * X2))
        En, nZ = sim.surface_field()
        x2 = sim.grid.x2_nodes()
        assert np.allclose(En, -(a + b * x2), rtol=0, atol=1e-12 * (abs(a) + abs(b)))
        assert np.allclose(nZ, x2, rtol=0, atol=1e-15)
        h = 2.0 / n2
        exact = 4.0 * np.pi / 3.0 * a * b * (1.0 + 0.5 * h * h)
        assert np.isclose(sim.electric_force(), exact, rtol=1e-12, atol=0)
        # the charge: -2 pi int (a + b x2) dx2 = -4 pi a (the trapezoid is exact on linears)
        assert np.isclose(sim.grain_charge(), -4.0 * np.pi * a, rtol=1e-12)


@pytest.mark.parametrize("alpha", [0.15, -0.2, 0.24])
def test_vacuum_force_vanishes_at_second_order(alpha):
    errs = []
    for n2 in (32, 64, 128, 256):
        sim = _sim(alpha, 16, n2)
        sim.set_phi(_vacuum_phi(sim))
        En, nZ = sim.surface_field()
        # gross stress (same integrand without the sign of n_Z) as the scale
        x2 = sim.grid.x2_nodes()
        g = 0.5 * En * En * np.abs(nZ) * geo.dA_dx2(-1.0, x2, alpha)
        gross = np.sum(0.5 * (g[1:] + g[:-1])) * sim.grid.h2
        errs.append(abs(sim.electric_force()) / gross)
    errs = np.array(errs)
    assert errs[-1] < 1e-4
    order = np.log2(errs[:-1] / errs[1:])
    assert np.all(order > 1.8), order
