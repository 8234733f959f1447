"""Electric field: nodal potential derivatives, interpolation, eq. (10).

Oracle module (test infrastructure only; the product path never imports it).

Paper passages: Section 2, eq. (10) and the sentence after it -- dphi/dx1 and
dphi/dx2 are found numerically at the grid nodes and then interpolated to the
particle position, while the coordinate derivatives are analytic at the particle;
Section 1 -- field values at the nodes are spatially interpolated to particles;
Section 2 -- finite differences are second order.

Readings: central differences at interior nodes, second-order one-sided
differences at the four edges (x1 = -1, x1_out and the axis x2 = +-1); the
interpolation is bilinear in the logical coordinates (the same cloud-in-cell
shape as the charge weighting).
"""
import numpy as np

from . import geometry as geo


def _d_axis(phi, h, axis):
    """Second-order derivative along `axis`: central inside, one-sided at ends."""
    phi = np.moveaxis(np.asarray(phi, dtype=np.float64), axis, 0)
    d = np.empty_like(phi)
    d[1:-1] = (phi[2:] - phi[:-2]) / (2.0 * h)
    d[0] = (-3.0 * phi[0] + 4.0 * phi[1] - phi[2]) / (2.0 * h)
    d[-1] = (3.0 * phi[-1] - 4.0 * phi[-2] + phi[-3]) / (2.0 * h)
    return np.moveaxis(d, 0, axis)


def nodal_gradient(phi, grid):
    """(dphi/dx1, dphi/dx2) at every node; arrays indexed [i2, i1]."""
    return _d_axis(phi, grid.h1, axis=1), _d_axis(phi, grid.h2, axis=0)


def locate(x1, x2, grid):
    """Cell indices and fractional offsets of positions (x1, x2)."""
    t1 = (np.asarray(x1) + 1.0) / grid.h1
    t2 = (np.asarray(x2) + 1.0) / grid.h2
    i1 = np.clip(np.floor(t1).astype(np.int64), 0, grid.n1 - 1)
    i2 = np.clip(np.floor(t2).astype(np.int64), 0, grid.n2 - 1)
    return i1, i2, t1 - i1, t2 - i2


def interpolate(values, x1, x2, grid):
    """Bilinear interpolation of nodal values ([i2, i1]) to positions."""
    i1, i2, f1, f2 = locate(x1, x2, grid)
    v = np.asarray(values)
    return ((1 - f1) * (1 - f2) * v[i2, i1] + f1 * (1 - f2) * v[i2, i1 + 1]
            + (1 - f1) * f2 * v[i2 + 1, i1] + f1 * f2 * v[i2 + 1, i1 + 1])


def electric_field(phi1_nodes, phi2_nodes, x1, x2, grid):
    """eq. (10): E_R = -(x1_R phi_1 + x2_R phi_2), E_Z = -(x1_Z phi_1 + x2_Z phi_2),
    with (phi_1, phi_2) interpolated and the metric analytic at the particle.
    Units: Te / (e R0)."""
    p1 = interpolate(phi1_nodes, x1, x2, grid)
    p2 = interpolate(phi2_nodes, x1, x2, grid)
    x1R, x1Z, x2R, x2Z = geo.metric(x1, x2, grid.alpha)
    return -(x1R * p1 + x2R * p2), -(x1Z * p1 + x2Z * p2)
