"""Shape-conforming coordinates of the charge+dipole grain, in plain FP64.

Oracle module (test infrastructure only; the product path never imports it).

All lengths are in units of the grain radius R0 (the paper's normalised r).
Paper passages followed (Section 2, "Model implementation"):
  * eq. (1): grain surfaces are equipotentials of a point charge plus a dipole,
    alpha = p / (Q R0);
  * eq. (2): x1 = -(1/r) (1 + alpha cos(theta) / r),  x2 = cos(theta);
  * eq. (3): analytic inverse r(x1, x2) (the root that is positive for x1 < 0);
  * eq. (4): surface element dA on a surface of constant x1;
  * eq. (5): volume element dOmega;
  * eq. (7): coefficients of the Laplace operator in (x1, x2);
  * eq. (8): cylindrical embedding R = r sqrt(1 - x2^2), Z = r x2;
  * eq. (10): the coordinate derivatives dx1/dR, dx1/dZ, dx2/dR, dx2/dZ, found
    analytically (the paper states they are analytic; the closed forms below are
    derived from eqs. (2) and (8) by the chain rule and pinned against finite
    differences in the tests).
"""
import numpy as np

TWO_PI = 2.0 * np.pi


def x1_of(r, x2, alpha):
    """eq. (2): x1 = -(1/r)(1 + alpha x2 / r)."""
    r = np.asarray(r, dtype=np.float64)
    return -(1.0 / r) * (1.0 + alpha * np.asarray(x2, dtype=np.float64) / r)


def r_of(x1, x2, alpha):
    """eq. (3): r = -(1 + sqrt(1 - 4 alpha x1 x2)) / (2 x1)."""
    x1 = np.asarray(x1, dtype=np.float64)
    x2 = np.asarray(x2, dtype=np.float64)
    return -(1.0 + np.sqrt(1.0 - 4.0 * alpha * x1 * x2)) / (2.0 * x1)


def cyl_of(x1, x2, alpha):
    """eq. (8) (lengths in R0): R = r sqrt(1 - x2^2), Z = r x2."""
    r = r_of(x1, x2, alpha)
    x2 = np.asarray(x2, dtype=np.float64)
    return r * np.sqrt(np.maximum(1.0 - x2 * x2, 0.0)), r * x2


def conforming_of(R, Z, alpha):
    """Inverse of eq. (8) followed by eq. (2): (R, Z) -> (x1, x2)."""
    R = np.asarray(R, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):   # the origin maps to NaN
        r = np.hypot(R, Z)
        x2 = Z / r
        return x1_of(r, x2, alpha), x2


def dA_dx2(x1, x2, alpha):
    """eq. (4) divided by dx2 (R0 = 1):
    2 pi r^2 sqrt(1 + (1 - x2^2) (alpha / (r + 2 alpha x2))^2)."""
    r = r_of(x1, x2, alpha)
    x2 = np.asarray(x2, dtype=np.float64)
    t = alpha / (r + 2.0 * alpha * x2)
    return TWO_PI * r * r * np.sqrt(1.0 + (1.0 - x2 * x2) * t * t)


def dOmega_dx1dx2(x1, x2, alpha):
    """eq. (5) divided by dx1 dx2 (R0 = 1): 2 pi r^4 / (1 + 2 alpha x2 / r)."""
    r = r_of(x1, x2, alpha)
    x2 = np.asarray(x2, dtype=np.float64)
    return TWO_PI * r ** 4 / (1.0 + 2.0 * alpha * x2 / r)


def laplace_coeffs(x1, x2, alpha):
    """eq. (7): coefficients (c11, c22, c12, c2) of
    c11 d2/dx1^2 + c22 d2/dx2^2 + c12 d2/dx1dx2 + c2 d/dx2."""
    r = r_of(x1, x2, alpha)
    x2 = np.asarray(x2, dtype=np.float64)
    s2 = 1.0 - x2 * x2
    c11 = ((r + 2.0 * alpha * x2) ** 2 + alpha * alpha * s2) / r ** 6
    c22 = s2 / r ** 2
    c12 = -2.0 * alpha * s2 / r ** 4
    c2 = -2.0 * x2 / r ** 2
    return c11, c22, c12, c2


def metric(x1, x2, alpha):
    """Coordinate derivatives used in eq. (10), analytic in (r, x2):
    dx1/dR = s (r + 3 alpha x2) / r^3,  dx1/dZ = (x2 r + alpha (3 x2^2 - 1)) / r^3,
    dx2/dR = -x2 s / r,                 dx2/dZ = s^2 / r,   s = sqrt(1 - x2^2)."""
    r = r_of(x1, x2, alpha)
    x2 = np.asarray(x2, dtype=np.float64)
    s = np.sqrt(np.maximum(1.0 - x2 * x2, 0.0))
    r3 = r ** 3
    x1R = s * (r + 3.0 * alpha * x2) / r3
    x1Z = (x2 * r + alpha * (3.0 * x2 * x2 - 1.0)) / r3
    x2R = -x2 * s / r
    x2Z = s * s / r
    return x1R, x1Z, x2R, x2Z


def check_alpha(alpha, x1_out):
    """Range of validity of eqs. (3) and (5) over the domain x1 in [-1, x1_out]:
    1 - 4 alpha x1 x2 >= 0 and r + 2 alpha x2 > 0 everywhere, which holds iff
    |alpha| < 1/4 (at |alpha| = 1/4 one pole of the grain becomes a cusp)."""
    return abs(alpha) < 0.25 and -1.0 < x1_out < 0.0
