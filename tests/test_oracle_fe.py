"""Pins of the oracle's conservative (finite-element) form of the Laplacian in
the curvilinear coordinates (an alternative to eq. 7's expanded operator)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import geometry as geo
from oracle.grid import Grid, node_loads, node_volumes
from oracle.poisson import assemble_fe, solve_fe


@pytest.mark.parametrize("alpha", [0.0, 0.2, -0.24])
def test_symmetric_and_rows_sum_to_zero(alpha):
    """S = S^T, and every full row sums to zero (the hats sum to one, so a
    constant has no gradient): the node fluxes balance exactly -- Gauss's law."""
    g = Grid(24, 20, -0.15, alpha)
    S = assemble_fe(g, full=True)
    scale = abs(S).max()
    assert abs(S - S.T).max() <= 1e-14 * scale
    assert np.abs(np.asarray(S.sum(axis=1))).max() <= 1e-13 * scale


def test_gauss_law_between_plasma_and_boundaries():
    """With the solution of a given node charge Q, the residuals of the
    Dirichlet rows (the boundaries' induced charges) plus the plasma charge sum
    to zero to round-off: sum_a (S_full phi)_a = 0."""
    g = Grid(32, 24, -0.1, 0.2)
    rng = np.random.default_rng(1)
    Q = rng.uniform(0.0, 1.0, g.shape) * node_volumes(g)
    Q[:, 0] = Q[:, -1] = 0.0
    phi = solve_fe(g, assemble_fe(g), Q, 1.0, -2.5, 0.0)
    r = assemble_fe(g, full=True) @ phi.ravel()
    nx = g.n1 + 1
    boundary = r[0::nx].sum() + r[g.n1::nx].sum()
    interior = -Q.sum()                      # S phi = -Q on the unknown rows (kappa = 1)
    assert abs(boundary + interior) <= 1e-10 * np.abs(Q).sum()


def _manufactured(X1, X2, alpha, which):
    r = geo.r_of(X1, X2, alpha)
    R, Z = geo.cyl_of(X1, X2, alpha)
    return {"r2": (r * r, lambda a, b: 6.0 + 0.0 * a), "Z": (Z, lambda a, b: 0.0 * a),
            "Zr": (Z * r * r, lambda a, b: 10.0 * geo.cyl_of(a, b, alpha)[1])}[which]


@pytest.mark.parametrize("alpha", [0.0, 0.2])
@pytest.mark.parametrize("which", ["r2", "Z", "Zr"])
def test_manufactured_solutions_second_order(alpha, which):
    """Cartesian Laplacians of r^2, Z and Z r^2 are 6, 0 and 10 Z: the
    finite-element solution with the loads of those sources converges to the
    function at second order (every metric term and the volume element enter)."""
    errs = []
    for n in (16, 32, 64):
        g = Grid(n, n, -0.1, alpha)
        X1, X2 = g.mesh()
        ex, lap = _manufactured(X1, X2, alpha, which)
        load = node_loads(g, lap)
        S = assemble_fe(g)
        nx = n + 1
        b = load.ravel().copy()
        b[0::nx] = ex[:, 0]
        b[n::nx] = ex[:, -1]
        phi = spla.spsolve(S.tocsc(), b).reshape(g.shape)
        errs.append(np.max(np.abs(phi - ex)) / np.max(np.abs(ex)))
    assert errs[2] < 1e-3
    # second order, or exact: at alpha = 0, r^2 depends on x1 alone and the
    # one-dimensional radial problem is reproduced to round-off
    assert errs[1] / errs[2] > 3.3 or errs[2] < 1e-11
