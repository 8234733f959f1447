"""Curvilinear Poisson solve, eqs. (6)-(7), second-order finite differences, FP64.

Oracle module (test infrastructure only; the product path never imports it).

Paper passages: Section 2, eq. (6) (Poisson's equation in (x1, x2)), eq. (7)
(the Laplace operator, including the mixed d2/dx1dx2 term and the first-order
d/dx2 term), the statement that finite-difference derivatives on the uniform
grid are second order and that the linear system is solved by LU decomposition,
and Section 1 (both boundaries held at fixed potentials).

Readings (the paper does not spell these out):
  * normalised units: lengths in R0, potential in Te/e, density in n0, so eq. (6)
    reads  Lap(phi) = -(R0/lambda_D)^2 * sum_s q_s n_s  (q_s in units of e);
  * Dirichlet rows at the grain x1 = -1 (phi_grain) and at x1 = x1_out (phi_out);
  * interior nodes use the 9-point central stencil: second differences for
    d2/dx1^2 and d2/dx2^2, the four-corner central formula for d2/dx1dx2, central
    first difference for d/dx2;
  * on the symmetry axis (x2 = +-1) the coefficients of d2/dx2^2 and d2/dx1dx2
    vanish (they carry 1 - x2^2), so the row keeps the d2/dx1^2 term and the
    d/dx2 term, the latter by the second-order one-sided difference
    (+-3 phi_j -+ 4 phi_{j-+1} +- phi_{j-+2}) / (2 h2).
Conservative form (an alternative to eq. 7's expanded operator, selected by
the caller): the Laplacian written as a divergence in (x1, x2), discretised by
bilinear finite elements -- S_ab = -integral of grad N_a . grad N_b dOmega with
the metric g^ij = grad x_i . grad x_j of eqs. (2), (7) and the volume element
of eq. (5), 2 x 2 Gauss points per cell (assemble_fe).  S is symmetric, its
full rows sum to zero (the bilinear hats sum to one), and its right-hand side
is the charge of the node, -(1/kappa^2) integral of rho N_a dOmega: Gauss's law
holds exactly between the plasma's node charges and the boundary rows.

Boltzmann electrons (Section 2, last paragraph: the electrons are not moved,
their density follows the Boltzmann relation instead): with n_e = n0 exp(phi)
in these units (phi in Te/e, n0 = 1; the physical sign, electrons gather where
phi is high), eq. (6) becomes Lap(phi) = -(1/kappa^2) (rho_p - exp(phi)), rho_p
the charge density of the moved species, solved by Newton's method on the same
discrete operator (solve_boltzmann).
The linear system is factorised by sparse LU (SuperLU through scipy), the
library routine standing in for the LAPACK LU the paper names, and each solve is
followed by two steps of FP64 iterative refinement (as LAPACK's expert drivers
do): the operator's rows differ in scale by ~r^4, and without refinement the
LU round-off alone reaches ~1e-9 of |phi| on a 512 x 512 grid.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import geometry as geo


def assemble(grid):
    """Sparse matrix of the discrete operator over all nodes (Dirichlet rows are
    identity rows).  Unknown ordering: node (i1, i2) -> i2 (N1 + 1) + i1.
    The entries are formed for all rows of a kind at once (numpy arrays); a
    node's coefficient from two terms (the centre) is their sum."""
    n1, n2 = grid.n1, grid.n2
    h1, h2 = grid.h1, grid.h2
    nx = n1 + 1
    X1, X2 = grid.mesh()
    c11, c22, c12, c2 = geo.laplace_coeffs(X1, X2, grid.alpha)
    rows, cols, vals = [], [], []

    def put(j, i, dj, di, v):
        rows.append((j * nx + i).ravel())
        cols.append(((j + dj) * nx + (i + di)).ravel())
        vals.append(np.broadcast_to(v, j.shape).ravel())

    # Dirichlet columns: identity rows
    jd, idd = np.meshgrid(np.arange(n2 + 1), np.array([0, n1]), indexing="ij")
    put(jd, idd, 0, 0, np.ones(jd.shape))
    # every unknown row: d2/dx1^2
    ju, iu = np.meshgrid(np.arange(n2 + 1), np.arange(1, n1), indexing="ij")
    a11 = c11[ju, iu] / (h1 * h1)
    put(ju, iu, 0, -1, a11)
    put(ju, iu, 0, 1, a11)
    put(ju, iu, 0, 0, -2.0 * a11)
    # axis rows: one-sided d/dx2; d2/dx2^2 and mixed terms vanish
    #   forward (j=0):  (-3 p0 + 4 p1 - p2) / (2 h2)
    #   backward (j=N): ( 3 pN - 4 pN-1 + pN-2) / (2 h2)
    for jj, sgn in ((0, 1), (n2, -1)):
        ja, ia = np.meshgrid(np.array([jj]), np.arange(1, n1), indexing="ij")
        b = c2[ja, ia] / (2.0 * h2)
        put(ja, ia, 0, 0, -3.0 * sgn * b)
        put(ja, ia, sgn, 0, 4.0 * sgn * b)
        put(ja, ia, 2 * sgn, 0, -1.0 * sgn * b)
    # interior rows
    ji, ii = np.meshgrid(np.arange(1, n2), np.arange(1, n1), indexing="ij")
    a22 = c22[ji, ii] / (h2 * h2)
    b2 = c2[ji, ii] / (2.0 * h2)
    a12 = c12[ji, ii] / (4.0 * h1 * h2)
    put(ji, ii, -1, 0, a22 - b2)
    put(ji, ii, 1, 0, a22 + b2)
    put(ji, ii, 0, 0, -2.0 * a22)
    put(ji, ii, 1, 1, a12)
    put(ji, ii, -1, -1, a12)
    put(ji, ii, 1, -1, -a12)
    put(ji, ii, -1, 1, -a12)
    nn = (n1 + 1) * (n2 + 1)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nn, nn))


class PoissonSolver:
    """Factorises the operator once; solve() maps a right-hand side to phi."""

    def __init__(self, grid):
        self.grid = grid
        self.A = assemble(grid)
        self.lu = spla.splu(self.A.tocsc())

    def rhs(self, source, phi_grain, phi_out):
        """Right-hand side: `source` (values of Lap(phi) at the nodes, [i2, i1])
        on the unknown nodes, boundary potentials on the Dirichlet rows."""
        b = np.array(source, dtype=np.float64, copy=True)
        b[:, 0] = phi_grain
        b[:, -1] = phi_out
        return b

    def solve(self, source, phi_grain, phi_out):
        return self.solve_rhs(self.rhs(source, phi_grain, phi_out))

    def solve_rhs(self, b, refine=2):
        """Solve with a full right-hand side already holding the boundary rows."""
        b = np.asarray(b, dtype=np.float64).ravel()
        x = self.lu.solve(b)
        for _ in range(refine):
            x = x + self.lu.solve(b - self.A @ x)
        return x.reshape(self.grid.shape)


def source_from_density(charge_density, lambdaD_over_R0):
    """eq. (6) in normalised units: Lap(phi) = -(R0/lambda_D)^2 * rho,
    rho = sum_s q_s n_s (units of e n0)."""
    return -np.asarray(charge_density, dtype=np.float64) / (lambdaD_over_R0 ** 2)


def solve_boltzmann(grid, A, rho_p, kappa, phi_grain, phi_out, phi0=None, tol=1e-12, max_newton=60):
    """Newton's method for A phi = -(rho_p - exp(phi)) / kappa^2 on the unknown
    nodes, phi = phi_grain / phi_out on the Dirichlet columns (A from assemble).
    Each step solves J dphi = -F with J = A - diag(exp(phi)) / kappa^2 (unknown
    rows) by sparse LU with two steps of iterative refinement (as in
    PoissonSolver); stops when the update falls below tol * max|phi| and
    returns (phi, newton steps)."""
    nx = grid.n1 + 1
    n = A.shape[0]
    unknown = np.ones(n, dtype=bool)
    unknown[0::nx] = False
    unknown[grid.n1::nx] = False
    bnd = np.zeros(n)
    bnd[0::nx] = phi_grain
    bnd[grid.n1::nx] = phi_out
    src_p = source_from_density(np.asarray(rho_p, dtype=np.float64).ravel(), kappa)
    if phi0 is None:
        # linear start: the electron density held at n0
        b = np.where(unknown, src_p + 1.0 / kappa ** 2, bnd)
        phi = spla.spsolve(A.tocsc(), b)
    else:
        phi = np.array(phi0, dtype=np.float64).ravel().copy()
        phi[~unknown] = bnd[~unknown]
    for it in range(1, max_newton + 1):
        e = np.where(unknown, np.exp(phi) / kappa ** 2, 0.0)
        F = A @ phi - np.where(unknown, src_p + e, bnd)
        J = (A - sp.diags(e)).tocsc()
        lu = spla.splu(J)
        d = lu.solve(-F)
        for _ in range(2):
            d = d + lu.solve(-F - J @ d)
        phi = phi + d
        if np.max(np.abs(d)) <= tol * max(np.max(np.abs(phi)), 1.0):
            return phi.reshape(grid.shape), it
    raise RuntimeError("Newton did not converge")


def assemble_fe(grid, full=False):
    """Bilinear finite-element matrix of the conservative form (module doc):
    S_ab = -sum over cells of sum over 2 x 2 Gauss points w J g^ij dN_a/dx_i
    dN_b/dx_j, J = dOmega/dx1dx2 (eq. 5), g11 = c11, g22 = c22, g12 = c12 / 2 of
    eq. (7).  With full=False the Dirichlet rows (i1 = 0, n1) are identity rows,
    as in assemble; with full=True every row is the element sum."""
    n1, n2 = grid.n1, grid.n2
    h1, h2 = grid.h1, grid.h2
    nx = n1 + 1
    g = 0.5 / np.sqrt(3.0)
    pts = (0.5 - g, 0.5 + g)
    I, J = np.meshgrid(np.arange(n1), np.arange(n2), indexing="xy")   # [j, i] cells
    K = {}
    for u in pts:
        for v in pts:
            x1 = -1.0 + (I + u) * h1
            x2 = -1.0 + (J + v) * h2
            jac = geo.dOmega_dx1dx2(x1, x2, grid.alpha) * 0.25 * h1 * h2
            c11, c22, c12, _ = geo.laplace_coeffs(x1, x2, grid.alpha)
            # local corners (di, dj): N = (u or 1-u)(v or 1-v)
            grads = {}
            for di in (0, 1):
                for dj in (0, 1):
                    fu = u if di else 1.0 - u
                    fv = v if dj else 1.0 - v
                    grads[(di, dj)] = ((1.0 if di else -1.0) * fv / h1, fu * (1.0 if dj else -1.0) / h2)
            for a, (a1, a2) in grads.items():
                for b, (b1, b2) in grads.items():
                    val = jac * (c11 * a1 * b1 + 0.5 * c12 * (a1 * b2 + a2 * b1) + c22 * a2 * b2)
                    K[(a, b)] = K.get((a, b), 0.0) - val
    rows, cols, vals = [], [], []
    for (a, b), val in K.items():
        ra = (J + a[1]) * nx + (I + a[0])
        cb = (J + b[1]) * nx + (I + b[0])
        rows.append(ra.ravel())
        cols.append(cb.ravel())
        vals.append(val.ravel())
    nn = nx * (n2 + 1)
    S = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nn, nn))
    if full:
        return S
    dirichlet = np.zeros(nn, dtype=bool)
    dirichlet[0::nx] = True
    dirichlet[n1::nx] = True
    keep = sp.diags((~dirichlet).astype(np.float64))
    return (keep @ S + sp.diags(dirichlet.astype(np.float64))).tocsr()


def solve_fe(grid, S, charge, kappa, phi_grain, phi_out):
    """Solve of the conservative form: S phi = -(1/kappa^2) charge on the
    unknown nodes (charge = integral of rho N_a dOmega, [i2, i1]), the boundary
    potentials on the Dirichlet rows; sparse LU with two refinement steps."""
    nx = grid.n1 + 1
    b = -np.asarray(charge, dtype=np.float64).ravel() / kappa ** 2
    b[0::nx] = phi_grain
    b[grid.n1::nx] = phi_out
    lu = spla.splu(S.tocsc())
    x = lu.solve(b)
    for _ in range(2):
        x = x + lu.solve(b - S @ x)
    return x.reshape(grid.shape)
