"""Conversion of physical inputs to the normalised parameters of the oracle.

Oracle module (test infrastructure only; the product path never imports it).

eq. (1): Phi0 = Q / (4 pi eps0 R0), alpha = p / (Q R0).  The normalisation
(lengths in R0, potential in Te/e, time in 1/omega_pe) makes the screening
parameter kappa = lambda_De / R0 with lambda_De = sqrt(eps0 Te / (n0 e^2)).
"""
import math

E_CHARGE = 1.602176634e-19      # C (exact, SI 2019)
EPS0 = 8.8541878128e-12         # F/m (CODATA 2018)


def normalise(R0_m, Q_e, p_e_m, n0_m3, me_over_mi, Te_eV, Ti_eV):
    """Dimensionless parameters of a grain/plasma given in physical units."""
    Q = Q_e * E_CHARGE
    lam = math.sqrt(EPS0 * Te_eV * E_CHARGE / (n0_m3 * E_CHARGE ** 2))
    phi0 = Q / (4 * math.pi * EPS0 * R0_m)          # volts
    return {
        "alpha": (p_e_m * E_CHARGE) / (Q * R0_m),
        "kappa": lam / R0_m,
        "phi0_over_Te": phi0 / Te_eV,
        "mi_over_me": 1.0 / me_over_mi,
        "Ti_over_Te": Ti_eV / Te_eV,
    }
