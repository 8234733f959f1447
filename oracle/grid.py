"""Uniform (x1, x2) grid and the node volumes used for charge weighting.

Oracle module (test infrastructure only; the product path never imports it).

Paper passages: Section 2 states that the grid is uniform in (x1, x2), that the
grain is x1 = -1 and the outer boundary a constant x1 in (-1, 0), and that the
volume element dOmega (eq. 5) is used for charge weighting.

Readings (the paper is silent on these):
  * "an N1 x N2 grid" counts cells; x1 is the first index.  Nodes are
    i1 = 0..N1 (x1 = -1 + i1 h1, h1 = (1 + x1_out)/N1) and i2 = 0..N2
    (x2 = -1 + i2 h2, h2 = 2/N2).  Node (i1, i2) is stored at i2 (N1 + 1) + i1.
  * the particle shape is bilinear (cloud-in-cell) in the logical coordinates;
    the volume that a node's density refers to is V_ij = integral of the node's
    bilinear hat function times dOmega over its (up to four) cells, so that a
    macro-particle load uniform in physical volume gives an expected density of
    exactly n0 at every node.  The integral is done with 12 x 12 Gauss-Legendre
    points per cell.
"""
from dataclasses import dataclass

import numpy as np

from . import geometry as geo


@dataclass(frozen=True)
class Grid:
    n1: int
    n2: int
    x1_out: float
    alpha: float

    @property
    def h1(self):
        return (1.0 + self.x1_out) / self.n1

    @property
    def h2(self):
        return 2.0 / self.n2

    @property
    def shape(self):
        """(nodes along x2, nodes along x1): arrays are indexed [i2, i1]."""
        return (self.n2 + 1, self.n1 + 1)

    def x1_nodes(self):
        return -1.0 + self.h1 * np.arange(self.n1 + 1)

    def x2_nodes(self):
        return -1.0 + self.h2 * np.arange(self.n2 + 1)

    def mesh(self):
        """Node coordinates as [i2, i1] arrays (X1, X2)."""
        return np.meshgrid(self.x1_nodes(), self.x2_nodes(), indexing="xy")


def node_volumes(grid, order=12):
    """V_ij = integral over the support of hat_ij of dOmega (eq. 5), [i2, i1]."""
    gx, gw = np.polynomial.legendre.leggauss(order)
    u = 0.5 * (gx + 1.0)            # quadrature nodes on [0, 1]
    w = 0.5 * gw
    h1, h2 = grid.h1, grid.h2
    i = np.arange(grid.n1)
    # [cell i1, point along x1, point along x2]
    U = u[None, :, None]
    Vv = u[None, None, :]
    W = (w[:, None] * w[None, :])[None, :, :] * h1 * h2
    x1 = -1.0 + (i[:, None, None] + U) * h1
    vol = np.zeros(grid.shape)
    for j in range(grid.n2):
        x2 = -1.0 + (j + Vv) * h2
        f = geo.dOmega_dx1dx2(x1, x2, grid.alpha) * W
        vol[j, :-1] += np.sum(f * (1 - U) * (1 - Vv), axis=(1, 2))
        vol[j, 1:] += np.sum(f * U * (1 - Vv), axis=(1, 2))
        vol[j + 1, :-1] += np.sum(f * (1 - U) * Vv, axis=(1, 2))
        vol[j + 1, 1:] += np.sum(f * U * Vv, axis=(1, 2))
    return vol


def node_loads(grid, fun, order=8):
    """integral over the support of hat_ij of fun(x1, x2) dOmega, [i2, i1]
    (Gauss-Legendre, order^2 points per cell)."""
    gx, gw = np.polynomial.legendre.leggauss(order)
    u = 0.5 * (gx + 1.0)
    w = 0.5 * gw
    h1, h2 = grid.h1, grid.h2
    i = np.arange(grid.n1)
    U = u[None, :, None]
    Vv = u[None, None, :]
    W = (w[:, None] * w[None, :])[None, :, :] * h1 * h2
    x1 = -1.0 + (i[:, None, None] + U) * h1
    out = np.zeros(grid.shape)
    for j in range(grid.n2):
        x2 = -1.0 + (j + Vv) * h2 + 0.0 * x1
        f = geo.dOmega_dx1dx2(x1, x2, grid.alpha) * fun(x1 + 0.0 * x2, x2) * W
        out[j, :-1] += np.sum(f * (1 - U) * (1 - Vv), axis=(1, 2))
        out[j, 1:] += np.sum(f * U * (1 - Vv), axis=(1, 2))
        out[j + 1, :-1] += np.sum(f * (1 - U) * Vv, axis=(1, 2))
        out[j + 1, 1:] += np.sum(f * U * Vv, axis=(1, 2))
    return out


def domain_volume(grid, order=12):
    """Integral of dOmega over the whole domain (sum of the node volumes)."""
    return float(np.sum(node_volumes(grid, order)))


def outer_area(grid):
    """Area of the outer boundary x1 = x1_out: integral of eq. (4) over x2,
    by composite Gauss-Legendre on 64 panels."""
    gx, gw = np.polynomial.legendre.leggauss(16)
    edges = np.linspace(-1.0, 1.0, 65)
    total = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        x2 = 0.5 * (a + b) + 0.5 * (b - a) * gx
        total += 0.5 * (b - a) * np.sum(gw * geo.dA_dx2(grid.x1_out, x2, grid.alpha))
    return float(total)
