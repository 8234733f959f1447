// Host-side set-up of a grain, all in FP64: node volumes (eq. 5 integrated
// against the bilinear hats), the outer-boundary area (eq. 4), rejection bounds
// for loading and injection, the 9-point stencil of eq. (7) with its axis rows,
// the Galerkin coarse operators of the multigrid hierarchy and the dense
// inverse of the coarsest one.
#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <thread>
#include <vector>

#include "host_setup.h"

namespace apic {

namespace {

double r_at(double x1, double x2, double a) { return -(1.0 + std::sqrt(1.0 - 4.0 * a * x1 * x2)) / (2.0 * x1); }

// eq. (5) per unit dx1 dx2
double dOmega(double x1, double x2, double a) {
    const double r = r_at(x1, x2, a);
    return 2.0 * M_PI * r * r * r * r / (1.0 + 2.0 * a * x2 / r);
}

// eq. (4) per unit dx2
double dA(double x1, double x2, double a) {
    const double r = r_at(x1, x2, a);
    const double t = a / (r + 2.0 * a * x2);
    return 2.0 * M_PI * r * r * std::sqrt(1.0 + (1.0 - x2 * x2) * t * t);
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                double q0 = 1.0, q1 = z;
                for (int k = 2; k <= n; ++k) {
                    const double q2 = ((2.0 * k - 1.0) * z * q1 - (k - 1.0) * q0) / k;
                    q0 = q1;
                    q1 = q2;
                }
                const double dq = n * (z * q1 - q0) / (z * z - 1.0);
                x[i] = z;
                w[i] = 2.0 / ((1.0 - z * z) * dq * dq);
                break;
            }
        }
    }
}

}  // namespace

void node_volumes(int n1, int n2, double x1_out, double a, std::vector<double>& vol) {
    const int nx = n1 + 1;
    const double h1 = (1.0 + x1_out) / n1, h2 = 2.0 / n2;
    vol.assign((size_t)nx * (n2 + 1), 0.0);
    std::vector<double> gx, gw;
    gauss_legendre(12, gx, gw);
    const int q = (int)gx.size();
    for (int j = 0; j < n2; ++j) {
        for (int i = 0; i < n1; ++i) {
            double s00 = 0, s10 = 0, s01 = 0, s11 = 0;
            for (int p = 0; p < q; ++p) {
                const double u = 0.5 * (gx[p] + 1.0), wu = 0.5 * gw[p];
                const double x1 = -1.0 + (i + u) * h1;
                for (int k = 0; k < q; ++k) {
                    const double v = 0.5 * (gx[k] + 1.0), wv = 0.5 * gw[k];
                    const double x2 = -1.0 + (j + v) * h2;
                    const double f = dOmega(x1, x2, a) * wu * wv * h1 * h2;
                    s00 += f * (1 - u) * (1 - v);
                    s10 += f * u * (1 - v);
                    s01 += f * (1 - u) * v;
                    s11 += f * u * v;
                }
            }
            vol[(size_t)j * nx + i] += s00;
            vol[(size_t)j * nx + i + 1] += s10;
            vol[(size_t)(j + 1) * nx + i] += s01;
            vol[(size_t)(j + 1) * nx + i + 1] += s11;
        }
    }
}

double outer_area(double x1_out, double a) {
    std::vector<double> gx, gw;
    gauss_legendre(16, gx, gw);
    double total = 0.0;
    const int panels = 64;
    for (int p = 0; p < panels; ++p) {
        const double lo = -1.0 + 2.0 * p / panels, hi = -1.0 + 2.0 * (p + 1) / panels;
        for (size_t k = 0; k < gx.size(); ++k)
            total += 0.5 * (hi - lo) * gw[k] * dA(x1_out, 0.5 * (lo + hi) + 0.5 * (hi - lo) * gx[k], a);
    }
    return total;
}

double bound_volume_marginal(double x1_out, double a) {
    double m = 0.0;
    for (int k = 0; k <= 4096; ++k) {
        const double x2 = -1.0 + 2.0 * k / 4096.0;
        const double ro = r_at(x1_out, x2, a), ri = r_at(-1.0, x2, a);
        m = std::max(m, ro * ro * ro - ri * ri * ri);
    }
    return 1.0001 * m;
}

double bound_outer_area_density(double x1_out, double a) {
    double m = 0.0;
    for (int k = 0; k <= 4096; ++k) m = std::max(m, dA(x1_out, -1.0 + 2.0 * k / 4096.0, a));
    return 1.0001 * m;
}

double grain_max_radius(double a) {
    // r(-1, x2) = (1 + sqrt(1 + 4 a x2)) / 2 is largest at x2 = sign(a)
    return 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * std::fabs(a))) * (1.0 + 1e-6);
}

// ------------------------------------------------------------------ stencils
void fine_stencil(int n1, int n2, double x1_out, double a, Stencil& s) {
    const int nx = n1 + 1;
    const size_t nodes = (size_t)nx * (n2 + 1);
    s.n1 = n1;
    s.n2 = n2;
    for (auto& v : s.c) v.assign(nodes, 0.0);
    s.nn.assign(nx, 0.0);
    s.ss.assign(nx, 0.0);
    const double h1 = (1.0 + x1_out) / n1, h2 = 2.0 / n2;
    for (int j = 0; j <= n2; ++j) {
        const double x2 = -1.0 + j * h2;
        for (int i = 1; i < n1; ++i) {
            const double x1 = -1.0 + i * h1;
            const double r = r_at(x1, x2, a);
            const double s2 = (j == 0 || j == n2) ? 0.0 : 1.0 - x2 * x2;
            const double c11 = ((r + 2.0 * a * x2) * (r + 2.0 * a * x2) + a * a * s2) / std::pow(r, 6);
            const double c22 = s2 / (r * r);
            const double c12 = -2.0 * a * s2 / std::pow(r, 4);
            const double c2 = -2.0 * x2 / (r * r);
            const size_t o = (size_t)j * nx + i;
            const double a11 = c11 / (h1 * h1);
            s.c[ST_W][o] = a11;
            s.c[ST_E][o] = a11;
            s.c[ST_C][o] = -2.0 * a11;
            if (j == 0) {
                // d/dx2 one-sided forward: (-3 p0 + 4 p1 - p2) / (2 h2)
                const double b = c2 / (2.0 * h2);
                s.c[ST_C][o] += -3.0 * b;
                s.c[ST_N][o] = 4.0 * b;
                s.nn[i] = -b;
            } else if (j == n2) {
                // one-sided backward: (3 pN - 4 pN-1 + pN-2) / (2 h2)
                const double b = c2 / (2.0 * h2);
                s.c[ST_C][o] += 3.0 * b;
                s.c[ST_S][o] = -4.0 * b;
                s.ss[i] = b;
            } else {
                const double a22 = c22 / (h2 * h2);
                const double b2 = c2 / (2.0 * h2);
                const double a12 = c12 / (4.0 * h1 * h2);
                s.c[ST_S][o] = a22 - b2;
                s.c[ST_N][o] = a22 + b2;
                s.c[ST_C][o] += -2.0 * a22;
                s.c[ST_NE][o] = a12;
                s.c[ST_SW][o] = a12;
                s.c[ST_NW][o] = -a12;
                s.c[ST_SE][o] = -a12;
            }
        }
    }
}

// A_c = (P^T / 4) A_f P on the unknowns; P bilinear, zero on Dirichlet columns.
// Conservative form: bilinear finite elements, S_ab = -integral of grad N_a .
// grad N_b dOmega with the metric of eqs. (2), (7) and the volume element of
// eq. (5), 2 x 2 Gauss points per cell.  Symmetric; the rows of the unknown
// nodes (1 <= i1 <= n1 - 1) are filled, as for the expanded operator.
void fine_stencil_fe(int n1, int n2, double x1_out, double a, Stencil& s) {
    const int nx = n1 + 1;
    const size_t nodes = (size_t)nx * (n2 + 1);
    s.n1 = n1;
    s.n2 = n2;
    for (auto& v : s.c) v.assign(nodes, 0.0);
    s.nn.clear();
    s.ss.clear();
    const double h1 = (1.0 + x1_out) / n1, h2 = 2.0 / n2;
    const double g = 0.5 / std::sqrt(3.0);
    const double pts[2] = {0.5 - g, 0.5 + g};
    // stencil index of the offset (di, dj) of a column node from its row node
    auto idx = [](int di, int dj) {
        static const int T[3][3] = {{ST_SW, ST_S, ST_SE}, {ST_W, ST_C, ST_E}, {ST_NW, ST_N, ST_NE}};
        return T[dj + 1][di + 1];
    };
    for (int j = 0; j < n2; ++j)
        for (int i = 0; i < n1; ++i)
            for (double u : pts)
                for (double v : pts) {
                    const double x1 = -1.0 + (i + u) * h1, x2 = -1.0 + (j + v) * h2;
                    const double r = r_at(x1, x2, a);
                    const double s2 = 1.0 - x2 * x2;
                    const double c11 = ((r + 2.0 * a * x2) * (r + 2.0 * a * x2) + a * a * s2) / std::pow(r, 6);
                    const double c22 = s2 / (r * r);
                    const double g12 = -a * s2 / std::pow(r, 4);
                    const double jac = dOmega(x1, x2, a) * 0.25 * h1 * h2;
                    double d1[4], d2[4];
                    for (int k = 0; k < 4; ++k) {
                        const int di = k & 1, dj = k >> 1;
                        const double fu = di ? u : 1.0 - u, fv = dj ? v : 1.0 - v;
                        d1[k] = (di ? 1.0 : -1.0) * fv / h1;
                        d2[k] = fu * (dj ? 1.0 : -1.0) / h2;
                    }
                    for (int ka = 0; ka < 4; ++ka) {
                        const int ia = i + (ka & 1), ja = j + (ka >> 1);
                        if (ia == 0 || ia == n1) continue;
                        const size_t o = (size_t)ja * nx + ia;
                        for (int kb = 0; kb < 4; ++kb) {
                            const double val = jac * (c11 * d1[ka] * d1[kb] + g12 * (d1[ka] * d2[kb] + d2[ka] * d1[kb]) +
                                                      c22 * d2[ka] * d2[kb]);
                            s.c[idx((kb & 1) - (ka & 1), (kb >> 1) - (ka >> 1))][o] -= val;
                        }
                    }
                }
}

void galerkin_coarse(const Stencil& f, Stencil& c) {
    const int n1f = f.n1, n2f = f.n2, nxf = n1f + 1;
    const int n1c = n1f / 2, n2c = n2f / 2, nxc = n1c + 1;
    c.n1 = n1c;
    c.n2 = n2c;
    const size_t nodes_c = (size_t)nxc * (n2c + 1);
    for (auto& v : c.c) v.assign(nodes_c, 0.0);
    c.nn.clear();
    c.ss.clear();
    static const int DJ[ST_COUNT] = {0, 0, 0, -1, 1, -1, -1, 1, 1};
    static const int DI[ST_COUNT] = {0, -1, 1, 0, 0, -1, 1, -1, 1};
    const bool has_axis = !f.nn.empty();
    for (int J = 0; J <= n2c; ++J) {
        for (int I = 1; I < n1c; ++I) {
            double acc[3][3] = {{0}};
            for (int dj = -1; dj <= 1; ++dj) {
                const int j = 2 * J + dj;
                if (j < 0 || j > n2f) continue;
                for (int di = -1; di <= 1; ++di) {
                    const int i = 2 * I + di;
                    if (i <= 0 || i >= n1f) continue;
                    const double wr = 0.25 * (dj == 0 ? 1.0 : 0.5) * (di == 0 ? 1.0 : 0.5);
                    const size_t o = (size_t)j * nxf + i;
                    // fine stencil entries of row (j, i)
                    int nent = ST_COUNT;
                    int ej[ST_COUNT + 1], ei[ST_COUNT + 1];
                    double ev[ST_COUNT + 1];
                    for (int k = 0; k < ST_COUNT; ++k) {
                        ej[k] = DJ[k];
                        ei[k] = DI[k];
                        ev[k] = f.c[k][o];
                    }
                    if (has_axis && j == 0) { ej[nent] = 2; ei[nent] = 0; ev[nent] = f.nn[i]; ++nent; }
                    if (has_axis && j == n2f) { ej[nent] = -2; ei[nent] = 0; ev[nent] = f.ss[i]; ++nent; }
                    for (int k = 0; k < nent; ++k) {
                        if (ev[k] == 0.0) continue;
                        const int mj = j + ej[k], mi = i + ei[k];
                        if (mj < 0 || mj > n2f || mi <= 0 || mi >= n1f) continue;
                        // coarse nodes interpolating to (mj, mi)
                        const int J0 = mj >> 1, I0 = mi >> 1;
                        const int nJ = (mj & 1) ? 2 : 1, nI = (mi & 1) ? 2 : 1;
                        const double pj = (mj & 1) ? 0.5 : 1.0, pi = (mi & 1) ? 0.5 : 1.0;
                        for (int a = 0; a < nJ; ++a) {
                            const int Jc = J0 + a;
                            for (int b = 0; b < nI; ++b) {
                                const int Ic = I0 + b;
                                if (Ic <= 0 || Ic >= n1c) continue;
                                const int dJ = Jc - J, dI = Ic - I;
                                if (dJ < -1 || dJ > 1 || dI < -1 || dI > 1)
                                    throw std::runtime_error("galerkin stencil wider than 3x3");
                                acc[dJ + 1][dI + 1] += wr * ev[k] * pj * pi;
                            }
                        }
                    }
                }
            }
            const size_t oc = (size_t)J * nxc + I;
            for (int k = 0; k < ST_COUNT; ++k) c.c[k][oc] = acc[DJ[k] + 1][DI[k] + 1];
        }
    }
}

// Dense matrix of a (coarse) stencil with identity rows on the Dirichlet columns.
void dense_matrix(const Stencil& s, std::vector<double>& A) {
    const int nx = s.n1 + 1;
    const int m = nx * (s.n2 + 1);
    A.assign((size_t)m * m, 0.0);
    static const int DJ[ST_COUNT] = {0, 0, 0, -1, 1, -1, -1, 1, 1};
    static const int DI[ST_COUNT] = {0, -1, 1, 0, 0, -1, 1, -1, 1};
    for (int j = 0; j <= s.n2; ++j)
        for (int i = 0; i < nx; ++i) {
            const int row = j * nx + i;
            if (i == 0 || i == s.n1) {
                A[(size_t)row * m + row] = 1.0;
                continue;
            }
            for (int k = 0; k < ST_COUNT; ++k) {
                const double v = s.c[k][row];
                if (v == 0.0) continue;
                const int jj = j + DJ[k], ii = i + DI[k];
                if (jj < 0 || jj > s.n2) continue;
                A[(size_t)row * m + jj * nx + ii] += v;
            }
            if (!s.nn.empty() && j == 0) A[(size_t)row * m + 2 * nx + i] += s.nn[i];
            if (!s.ss.empty() && j == s.n2) A[(size_t)row * m + (s.n2 - 2) * nx + i] += s.ss[i];
        }
}

// Inverse of a banded m x m matrix (row-major; zero outside |r - c| <= w, w
// found from the entries): Gaussian elimination with partial pivoting inside
// the band (the rows of U then reach at most 2w past the diagonal, the row
// interchanges are applied as they occur, as in banded LINPACK), then one
// solve per column of the identity, the columns split over `threads`.
// Returns false on a zero pivot.
bool invert(std::vector<double> A, int m, std::vector<double>& inv, int threads) {
    int w = 0;
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c)
            if (A[(size_t)r * m + c] != 0.0) w = std::max(w, std::abs(r - c));
    std::vector<int> piv(m);
    for (int col = 0; col < m; ++col) {
        const int rend = std::min(m, col + w + 1), cend = std::min(m, col + 2 * w + 1);
        int p = col;
        for (int r = col + 1; r < rend; ++r)
            if (std::fabs(A[(size_t)r * m + col]) > std::fabs(A[(size_t)p * m + col])) p = r;
        if (A[(size_t)p * m + col] == 0.0) return false;
        piv[col] = p;
        if (p != col)
            for (int k = col; k < cend; ++k) std::swap(A[(size_t)p * m + k], A[(size_t)col * m + k]);
        const double d = 1.0 / A[(size_t)col * m + col];
        for (int r = col + 1; r < rend; ++r) {
            double& l = A[(size_t)r * m + col];
            if (l == 0.0) continue;
            l *= d;
            for (int k = col + 1; k < cend; ++k) A[(size_t)r * m + k] -= l * A[(size_t)col * m + k];
        }
    }
    inv.assign((size_t)m * m, 0.0);
    auto columns = [&](int first, int step) {
        std::vector<double> b(m);
        for (int k = first; k < m; k += step) {
            std::fill(b.begin(), b.end(), 0.0);
            b[k] = 1.0;
            // forward: the interchanges and multipliers of the elimination
            // (nothing happens before column k - w)
            for (int col = std::max(0, k - w); col < m; ++col) {
                if (piv[col] != col) std::swap(b[piv[col]], b[col]);
                const double t = b[col];
                if (t == 0.0) continue;
                const int rend = std::min(m, col + w + 1);
                for (int r = col + 1; r < rend; ++r) b[r] -= A[(size_t)r * m + col] * t;
            }
            for (int r = m - 1; r >= 0; --r) {
                double v = b[r];
                const int cend = std::min(m, r + 2 * w + 1);
                for (int c = r + 1; c < cend; ++c) v -= A[(size_t)r * m + c] * b[c];
                b[r] = v / A[(size_t)r * m + r];
            }
            for (int r = 0; r < m; ++r) inv[(size_t)r * m + k] = b[r];
        }
    };
    threads = std::max(1, std::min(threads, m));
    std::vector<std::thread> pool;
    for (int t = 1; t < threads; ++t) pool.emplace_back(columns, t, threads);
    columns(0, threads);
    for (auto& t : pool) t.join();
    return true;
}

// |D^-1 A_{unknown, Dirichlet} u_Dirichlet|^2 for the boundary potentials
// (D = diagonal of A, the row scaling of the multigrid residual norms).
double boundary_coupling_norm2(const Stencil& s, double pg, double po) {
    const int nx = s.n1 + 1;
    double sum = 0.0;
    for (int j = 0; j <= s.n2; ++j) {
        double v1 = 0.0, v2 = 0.0;
        const size_t o1 = (size_t)j * nx + 1, o2 = (size_t)j * nx + s.n1 - 1;
        v1 += s.c[ST_W][o1] * pg;
        if (j > 0) v1 += s.c[ST_SW][o1] * pg;
        if (j < s.n2) v1 += s.c[ST_NW][o1] * pg;
        v2 += s.c[ST_E][o2] * po;
        if (j > 0) v2 += s.c[ST_SE][o2] * po;
        if (j < s.n2) v2 += s.c[ST_NE][o2] * po;
        v1 /= s.c[ST_C][o1];
        v2 /= s.c[ST_C][o2];
        if (o1 == o2) sum += (v1 + v2) * (v1 + v2);
        else sum += v1 * v1 + v2 * v2;
    }
    return sum;
}

}  // namespace apic
