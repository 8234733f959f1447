// FP64 geometric multigrid for the curvilinear Poisson problem, eqs. (6)-(7).
//
// The paper solves the finite-difference system by LU (Section 2).  On the GPU
// the same discrete system is solved by multigrid V-cycles: Galerkin coarse
// operators (R A P, bilinear P, R = P^T / 4, built on the host), alternating
// zebra line Gauss-Seidel smoothing (x1-, x2-, then x1-lines; each line is a
// tridiagonal system solved in LDS by parallel cyclic reduction, or, for the
// many long lines of a large ensemble, by the partition method), and a dense
// inverse on the coarsest grid (a few hundred to a few thousand nodes).  The operator's
// anisotropy changes direction across the domain (the x1 coefficient falls like
// r^-4), which is why both line directions are relaxed.
//
// Every kernel works on one level of all grains of the ensemble at once
// (blockIdx.y = grain, level arrays from the MGDesc table); grains whose
// hierarchy is shallower, or whose solve has converged, leave at once.  A
// V-cycle ends with the row-scaled residual norm and a convergence check on
// the device, so cycles can be replayed from a graph without host reads.
#include <type_traits>

#include "apic_internal.h"
#include "device_common.h"

namespace apic {

constexpr int MG_BLOCK = 256;

// FP64 reciprocal: hardware estimate refined by two Newton steps (correct to
// about 1 ulp); replaces the much longer division sequence in the line solves.
__device__ inline double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}

// Parallel cyclic reduction on a set of tridiagonal systems held in LDS (a:
// sub, b: diagonal, c: super, d: rhs).  Equation e belongs to system e / L and
// couples only inside its system; a[first] = c[last] = 0.  Each thread owns up
// to K equations and keeps their diagonals in registers; the LDS array b holds
// the reciprocals of the diagonals (Newton-refined, one per equation and step,
// read by both neighbours).  On return d[e] * b[e] is the solution.
template <int K, int NT>
__device__ __forceinline__ void pcr_solve(double* a, double* b, double* c, double* d, int L, int total) {
    int jj[K];
    double bb[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = threadIdx.x + k * NT;
        jj[k] = e % L;
        bb[k] = 1.0;
        if (e < total) {
            bb[k] = b[e];
            b[e] = rcp64(bb[k]);
        }
    }
    __syncthreads();
    for (int s = 1; s < L; s <<= 1) {
        double na[K], nb[K], nc[K], nd[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e = threadIdx.x + k * NT;
            if (e < total) {
                const int j = jj[k];
                double ai = a[e], bi = bb[k], ci = c[e], di = d[e];
                double an = 0.0, cn = 0.0;
                if (j - s >= 0) {
                    const double m = ai * b[e - s];
                    bi -= m * c[e - s];
                    di -= m * d[e - s];
                    an = -m * a[e - s];
                }
                if (j + s < L) {
                    const double m = ci * b[e + s];
                    bi -= m * a[e + s];
                    di -= m * d[e + s];
                    cn = -m * c[e + s];
                }
                na[k] = an;
                nb[k] = bi;
                nc[k] = cn;
                nd[k] = di;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e = threadIdx.x + k * NT;
            if (e < total) {
                a[e] = na[k];
                bb[k] = nb[k];
                b[e] = rcp64(nb[k]);
                c[e] = nc[k];
                d[e] = nd[k];
            }
        }
        __syncthreads();
    }
}

// Tridiagonal systems held in LDS (a: sub, b: diagonal, c: super, d: rhs;
// equations 0..total-1, systems concatenated with a[first] = c[last] = 0),
// solved by the partition method.  Thread t takes the chunk of P consecutive
// equations starting at t P into registers; a forward and a backward
// elimination pass inside the chunk express each of its unknowns through the
// chunk's first and last unknowns.  Those 2 NT unknowns satisfy a tridiagonal
// system of their own (the chunk's first equation couples the previous
// chunk's last unknown, its last equation the next chunk's first), solved by
// cyclic reduction in LDS; every thread then recovers its chunk.  Without
// pivoting, as the line systems of the discrete operator are diagonally
// dominant.  Needs P >= 2, NT P >= total and LDS arrays of max(total, 2 NT)
// entries; on return d[e] holds the solution.
template <int P, int NT>
__device__ __forceinline__ void tri_solve(double* a, double* b, double* c, double* d, int total) {
    static_assert(P >= 2, "a chunk needs a first and a last equation");
    const int e0 = threadIdx.x * P;
    double A[P], B[P], C[P], D[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int e = e0 + p;
        const bool in = e < total;
        A[p] = in ? a[e] : 0.0;
        B[p] = in ? b[e] : 1.0;
        C[p] = in ? c[e] : 0.0;
        D[p] = in ? d[e] : 0.0;
    }
    __syncthreads();
    // forward pass: equation p >= 1 becomes A[p] y_0 + y_p + C[p] y_{p+1} = D[p]
    double pa = -1.0, pc = 0.0, pd = 0.0;
#pragma unroll
    for (int p = 1; p < P; ++p) {
        const double r = rcp64(B[p] - A[p] * pc);
        pa = -A[p] * pa * r;
        pd = (D[p] - A[p] * pd) * r;
        pc = C[p] * r;
        A[p] = pa;
        C[p] = pc;
        D[p] = pd;
    }
    const double la = A[P - 1], lc = C[P - 1], ld = D[P - 1];
    // backward pass: equation P-2 .. 1 becomes A[p] y_0 + y_p + C[p] y_{P-1} = D[p]
    double xa = 0.0, xc = -1.0, xd = 0.0;
#pragma unroll
    for (int p = P - 2; p >= 1; --p) {
        const double cp = C[p];
        A[p] -= cp * xa;
        D[p] -= cp * xd;
        C[p] = -cp * xc;
        xa = A[p];
        xc = C[p];
        xd = D[p];
    }
    const int r0 = 2 * threadIdx.x;
    a[r0] = A[0];
    b[r0] = B[0] - C[0] * xa;
    c[r0] = -C[0] * xc;
    d[r0] = D[0] - C[0] * xd;
    a[r0 + 1] = la;
    b[r0 + 1] = 1.0;
    c[r0 + 1] = lc;
    d[r0 + 1] = ld;
    __syncthreads();
    pcr_solve<2, NT>(a, b, c, d, 2 * NT, 2 * NT);
    const double y0 = d[r0] * b[r0];
    const double yl = d[r0 + 1] * b[r0 + 1];
    __syncthreads();
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int e = e0 + p;
        if (e < total) d[e] = p == 0 ? y0 : p == P - 1 ? yl : D[p] - A[p] * y0 - C[p] * yl;
    }
    __syncthreads();
}

// Coefficients of the 9-point operator at one unknown node (nn / ss: the
// second-neighbour couplings of the axis rows of the finest level).
struct Coef {
    double C, W, E, S, N, SW, SE, NW, NE, nn, ss;
};

// Coarse levels: the Galerkin stencil arrays.
// With Boltzmann electrons every level's diagonal carries the Newton term
// (`shift`, subtracted from the centre coefficient).
struct StoredStencil {
    const double* st;
    const double* sh;
    int n2;
    __device__ explicit StoredStencil(const MGDesc& D) : st(D.st), sh(D.shift), n2(D.n2) {}
    __device__ Coef at(int, int, size_t o) const {
        // node-major: the nine coefficients of a node in five 16-byte loads
        using d2 = double __attribute__((ext_vector_type(2)));
        const gptr<const d2> p = gbl(reinterpret_cast<const d2*>(st + ST_STRIDE * o));
        const d2 v0 = p[0], v1 = p[1], v2 = p[2], v3 = p[3], v4 = p[4];
        Coef c;
        c.C = v0.x;
        if (sh) c.C -= gbl(sh)[o];
        c.W = v0.y;
        c.E = v1.x;
        c.S = v1.y;
        c.N = v2.x;
        c.SW = v2.y;
        c.SE = v3.x;
        c.NW = v3.y;
        c.NE = v4.x;
        c.nn = 0.0;
        c.ss = 0.0;
        return c;
    }
    __device__ double diag(int, int, size_t o) const {
        return gbl(st)[ST_STRIDE * o + ST_C] - (sh ? gbl(sh)[o] : 0.0);
    }
};

// Finest level: the central differences of eq. (7) evaluated at the node
// (r from eq. 3, second-order one-sided d/dx2 on the axis rows), the
// expressions the host uses to build the hierarchy.  Nothing is read from
// memory, which removes 72 bytes per node from every sweep of the largest
// level.  The reciprocals of the grid spacings come from the level's
// descriptor and the two per-node divisions are Newton-refined reciprocals
// (within an ulp of the host's quotients; the FP64 divisions were a large
// part of these kernels' instructions on many-grain ensembles).
struct FineStencil {
    double a, h1, h2, ih1sq, ih2sq, i2h2, i4h1h2;
    const double* sh;
    int n2;
    __device__ explicit FineStencil(const MGDesc& D)
        : a(D.alpha), h1(D.h1), h2(D.h2), ih1sq(D.ih1sq), ih2sq(D.ih2sq), i2h2(D.i2h2), i4h1h2(D.i4h1h2),
          sh(D.shift), n2(D.n2) {}
    __device__ Coef at(int j, int i, size_t o) const {
        const double x1 = -1.0 + i * h1, x2 = -1.0 + j * h2;
        const double r = (1.0 + sqrt(1.0 - 4.0 * a * x1 * x2)) * rcp64(-2.0 * x1);
        const bool edge = (j == 0 || j == n2);
        const double s2 = edge ? 0.0 : 1.0 - x2 * x2;
        const double ir2 = rcp64(r * r);
        const double t = r + 2.0 * a * x2;
        const double a11 = (t * t + a * a * s2) * (ir2 * ir2 * ir2) * ih1sq;
        const double c2 = -2.0 * x2 * ir2;
        Coef c;
        c.W = a11;
        c.E = a11;
        c.C = -2.0 * a11;
        c.S = c.N = c.SW = c.SE = c.NW = c.NE = c.nn = c.ss = 0.0;
        if (j == 0) {
            const double b = c2 * i2h2;
            c.C += -3.0 * b;
            c.N = 4.0 * b;
            c.nn = -b;
        } else if (j == n2) {
            const double b = c2 * i2h2;
            c.C += 3.0 * b;
            c.S = -4.0 * b;
            c.ss = b;
        } else {
            const double a22 = s2 * ir2 * ih2sq;
            const double b2 = c2 * i2h2;
            const double a12 = -2.0 * a * s2 * (ir2 * ir2) * i4h1h2;
            c.S = a22 - b2;
            c.N = a22 + b2;
            c.C += -2.0 * a22;
            c.NE = a12;
            c.SW = a12;
            c.NW = -a12;
            c.SE = -a12;
        }
        if (sh) c.C -= gbl(sh)[o];
        return c;
    }
    __device__ double diag(int j, int i, size_t o) const { return at(j, i, o).C; }
};

// (A u) at an unknown node (j, i) of a level.
template <class ST>
__device__ inline double apply_A(const ST& st, gptr<const double> u, int n2, int nx, int j, int i) {
    const size_t o = (size_t)j * nx + i;
    const Coef k = st.at(j, i, o);
    double au = k.C * u[o] + k.W * u[o - 1] + k.E * u[o + 1];
    if (j > 0) au += k.S * u[o - nx] + k.SW * u[o - nx - 1] + k.SE * u[o - nx + 1];
    if (j < n2) au += k.N * u[o + nx] + k.NW * u[o + nx - 1] + k.NE * u[o + nx + 1];
    if (j == 0) au += k.nn * u[o + 2 * nx];
    if (j == n2) au += k.ss * u[o - 2 * nx];
    return au;
}

__device__ inline bool level_active(const MGDesc& D, const MGState* ms) {
    return D.n1 != 0 && !D.coarsest && !ms[blockIdx.y].done;
}

// Index of this workgroup's line among the `lines` lines (or line blocks) of
// its grain: they are dealt out in eight contiguous ranges, one per XCD
// (blockIdx.x mod 8; gridDim.x is a multiple of 8 and at least the grain's
// count rounded up to 8), so neighbouring lines, which read each other's
// values, share an L2, and a grain with fewer lines than the largest one still
// spreads them over all eight XCDs.  Workgroups left over get `lines` or more.
__device__ inline int xcd_line(int lines) {
    const int per = (lines + 7) >> 3;
    const int k = (int)(blockIdx.x >> 3);
    return k < per ? (int)(blockIdx.x & 7) * per + k : lines;
}

// Relaxation of the lines i2 = j (j = color, color + 2, ...): unknowns i1 = 1..n1-1.
// On the finest level the axis rows j = 0 and j = n2 also couple to the rows
// two away (one-sided d/dx2), which have their colour: an axis row is relaxed
// after both colours, by the workgroup of the odd row next to it, once that row
// is solved (its other neighbours are even rows, already final), so that no line
// reads a line that another workgroup of the same launch is rewriting.
// With cl (the next coarser level) the sweep also applies the coarse-grid
// correction u += P uc: a line's solution does not depend on its own old
// value, only on its neighbour lines, so the first colour of the first sweep
// after the correction reads its two neighbour rows prolonged (bilinear P) and
// the other rows never need the correction added before they are solved.
// With TP > 0 each line is solved by the partition method (TP equations per
// thread) instead of cyclic reduction over all of it.
template <int K, int NT, class ST, int TP = 0>
__global__ void __launch_bounds__(NT)
k_relax_x1(const MGDesc* __restrict__ lv, const MGState* __restrict__ ms, int color,
           const MGDesc* __restrict__ cl) {
    extern __shared__ double lds[];
    const MGDesc& D = lv[blockIdx.y];
    if (!level_active(D, ms)) return;
    const int n1 = D.n1, n2 = D.n2;
    int j;
    int j_axis = -1;     // finest level (n2 >= 8), odd colour: the axis row solved after row j
    if constexpr (std::is_same<ST, FineStencil>::value) {
        const int line = xcd_line((n2 + 2 - color) / 2);
        j = color + 2 * line;
        if (color == 1 && j == 1) j_axis = 0;
        if (color == 1 && j == ((n2 & 1) ? n2 - 2 : n2 - 1)) j_axis = n2;
        if (j == 0 || j >= n2) {
            // the axis rows are solved after the odd rows, which read them: a
            // prolonging launch applies their correction here (no line of the
            // even colour reads them)
            if (color == 0 && line == 0 && cl != nullptr && cl[blockIdx.y].n1 != 0) {
                const MGDesc& C = cl[blockIdx.y];
                const int nx = n1 + 1, ncx = C.n1 + 1, n2c = C.n2;
                const gptr<double> u = gbl(D.u);
                const gptr<const double> uc = gbl(static_cast<const double*>(C.u));
                for (int t = threadIdx.x; t < 2 * nx; t += NT) {
                    const int top = t >= nx, i = top ? t - nx : t;
                    const int r = top ? n2 : 0, J = top ? n2c : 0;
                    const int I0 = i >> 1, I1 = I0 + (i & 1);
                    u[(size_t)r * nx + i] += 0.5 * (uc[(size_t)J * ncx + I0] + uc[(size_t)J * ncx + I1]);
                }
            }
            return;
        }
    } else {
        j = color + 2 * xcd_line((n2 + 2 - color) / 2);
        if (j > n2) return;
    }
    const int L = n1 - 1;
    const int cap = TP > 0 && L < 2 * NT ? 2 * NT : L;
    double* a = lds;
    double* b = a + cap;
    double* c = b + cap;
    double* d = c + cap;
    double* nb = d + cap;     // rows j - 1 and j + 1 with the correction, [2][nx]
    const int nx = n1 + 1;
    const ST st(D);
    const gptr<double> u = gbl(D.u);
    const gptr<const double> f = gbl(static_cast<const double*>(D.f));
    for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
        if (j_axis < 0) break;
        // the axis row reads row j, just written by this workgroup
        __syncthreads();
        j = j_axis;
    }
    const bool pro = pass == 0 && cl != nullptr && cl[blockIdx.y].n1 != 0;
    if (pro) {
        const MGDesc& C = cl[blockIdx.y];
        const int ncx = C.n1 + 1;
        const gptr<const double> uc = gbl(static_cast<const double*>(C.u));
        for (int t = threadIdx.x; t < 2 * nx; t += NT) {
            const int r = t < nx ? j - 1 : j + 1, i = t < nx ? t : t - nx;
            double v = 0.0;
            if (r >= 0 && r <= n2) {
                const int J0 = r >> 1, J1 = J0 + (r & 1), I0 = i >> 1, I1 = I0 + (i & 1);
                v = u[(size_t)r * nx + i] + 0.25 * (uc[(size_t)J0 * ncx + I0] + uc[(size_t)J0 * ncx + I1] +
                                                    uc[(size_t)J1 * ncx + I0] + uc[(size_t)J1 * ncx + I1]);
            }
            nb[t] = v;
        }
        __syncthreads();
    }
    for (int k = threadIdx.x; k < L; k += NT) {
        const int i = k + 1;
        const size_t o = (size_t)j * nx + i;
        const Coef q = st.at(j, i, o);
        double rhs = f[o];
        if (pro) {
            if (j > 0) rhs -= q.S * nb[i] + q.SW * nb[i - 1] + q.SE * nb[i + 1];
            if (j < n2) rhs -= q.N * nb[nx + i] + q.NW * nb[nx + i - 1] + q.NE * nb[nx + i + 1];
        } else {
            if (j > 0) rhs -= q.S * u[o - nx] + q.SW * u[o - nx - 1] + q.SE * u[o - nx + 1];
            if (j < n2) rhs -= q.N * u[o + nx] + q.NW * u[o + nx - 1] + q.NE * u[o + nx + 1];
        }
        if (j == 0) rhs -= q.nn * u[o + 2 * nx];
        if (j == n2) rhs -= q.ss * u[o - 2 * nx];
        double aa = q.W, cc = q.E;
        if (i == 1) { rhs -= aa * u[o - 1]; aa = 0.0; }
        if (i == n1 - 1) { rhs -= cc * u[o + 1]; cc = 0.0; }
        a[k] = aa;
        b[k] = q.C;
        c[k] = cc;
        d[k] = rhs;
    }
    __syncthreads();
    if constexpr (TP > 0) {
        tri_solve<TP, NT>(a, b, c, d, L);
        for (int k = threadIdx.x; k < L; k += NT) u[(size_t)j * nx + k + 1] = d[k];
    } else {
        pcr_solve<K, NT>(a, b, c, d, L, L);
        for (int k = threadIdx.x; k < L; k += NT) u[(size_t)j * nx + k + 1] = d[k] * b[k];
    }
    }
}

// Relaxation of LPB lines i1 = i (i = 1 + color, 3 + color, ...) per workgroup:
// unknowns i2 = 0..n2.  Neighbouring lines of one colour are read together so
// that the row-wise loads stay within a cache line.  On the finest level the
// axis rows carry a second-neighbour coupling (one-sided d/dx2); it is
// eliminated with the adjacent row so each line stays tridiagonal.
template <int K, int LPB, int NT, class ST>
__global__ void __launch_bounds__(NT)
k_relax_x2(const MGDesc* __restrict__ lv, const MGState* __restrict__ ms, int color) {
    extern __shared__ double lds[];
    __shared__ double axis_nn[LPB], axis_ss[LPB];
    const MGDesc& D = lv[blockIdx.y];
    if (!level_active(D, ms)) return;
    const int n1 = D.n1, n2 = D.n2;
    const int i0 = 1 + color + 2 * LPB * xcd_line(((n1 - color) / 2 + LPB - 1) / LPB);
    if (i0 > n1 - 1) return;
    const int L = n2 + 1;
    const int total = LPB * L;
    double* a = lds;
    double* b = a + total;
    double* c = b + total;
    double* d = c + total;
    const int nx = n1 + 1;
    const ST st(D);
    const gptr<double> u = gbl(D.u);
    const gptr<const double> f = gbl(static_cast<const double*>(D.f));
    for (int q = threadIdx.x; q < total; q += NT) {
        const int m = q % LPB, j = q / LPB;
        const int i = i0 + 2 * m;
        const int e = m * L + j;
        if (i > n1 - 1) {
            a[e] = 0.0;
            b[e] = 1.0;
            c[e] = 0.0;
            d[e] = 0.0;
            continue;
        }
        const size_t o = (size_t)j * nx + i;
        const Coef k = st.at(j, i, o);
        double rhs = f[o] - k.W * u[o - 1] - k.E * u[o + 1];
        if (j > 0) rhs -= k.SW * u[o - nx - 1] + k.SE * u[o - nx + 1];
        if (j < n2) rhs -= k.NW * u[o + nx - 1] + k.NE * u[o + nx + 1];
        a[e] = j > 0 ? k.S : 0.0;
        b[e] = k.C;
        c[e] = j < n2 ? k.N : 0.0;
        d[e] = rhs;
        if (j == 0) axis_nn[m] = k.nn;
        if (j == n2) axis_ss[m] = k.ss;
    }
    __syncthreads();
    if (threadIdx.x < LPB) {
        const int m = threadIdx.x, i = i0 + 2 * m;
        const double g = axis_nn[m];
        if (i <= n1 - 1 && g != 0.0) {
            const int e = m * L;
            const double mm = g / c[e + 1];
            b[e] -= mm * a[e + 1];
            c[e] -= mm * b[e + 1];
            d[e] -= mm * d[e + 1];
        }
    }
    if (threadIdx.x >= 64 && threadIdx.x < 64 + LPB) {
        const int m = threadIdx.x - 64, i = i0 + 2 * m;
        const double g = axis_ss[m];
        if (i <= n1 - 1 && g != 0.0) {
            const int e = m * L + n2;
            const double mm = g / a[e - 1];
            a[e] -= mm * b[e - 1];
            b[e] -= mm * c[e - 1];
            d[e] -= mm * d[e - 1];
        }
    }
    __syncthreads();
    pcr_solve<K, NT>(a, b, c, d, L, total);
    for (int q = threadIdx.x; q < total; q += NT) {
        const int m = q % LPB, j = q / LPB;
        const int i = i0 + 2 * m;
        if (i > n1 - 1) continue;
        const int e = m * L + j;
        u[(size_t)j * nx + i] = d[e] * b[e];
    }
}

// ------------------------------------------------------------------ finest x2 lines
// On the finest level the x2 sweeps run on transposed copies uT, fT (x2
// fastest): an x2 line is then contiguous and its loads coalesce, instead of
// every load of a wave touching 64 different rows.  u is transposed before
// the x2 sweeps of a smoothing step and back after them; fT once per solve.
// This pays when the finest levels of the ensemble do not fit in the L2
// caches; small grids sweep the columns in place.
constexpr int TR_TILE = 32;

// which = 0: u -> uT, 1: uT -> u, 2: f -> fT
template <int WHICH>
__global__ void __launch_bounds__(256)
k_transpose(const MGDesc* __restrict__ lv, const MGState* __restrict__ ms) {
    __shared__ double t[TR_TILE][TR_TILE + 1];
    const MGDesc& D = lv[blockIdx.y];
    if (!level_active(D, ms)) return;
    const int cols = D.n1 + 1, rows = D.n2 + 1;   // normal layout [row][col]
    const int tiles_x = (cols + TR_TILE - 1) / TR_TILE;
    const int tiles_y = (rows + TR_TILE - 1) / TR_TILE;
    if ((int)blockIdx.x >= tiles_x * tiles_y) return;
    const int ty = blockIdx.x / tiles_x, tx = blockIdx.x - ty * tiles_x;
    const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;   // 32 x 8 threads
    if (WHICH == 1) {
        // transposed [col][row] -> normal
        for (int k = ly; k < TR_TILE; k += 8) {
            const int i = tx * TR_TILE + k, j = ty * TR_TILE + lx;
            if (i < cols && j < rows) t[k][lx] = gbl(D.uT)[(size_t)i * rows + j];
        }
        __syncthreads();
        for (int k = ly; k < TR_TILE; k += 8) {
            const int j = ty * TR_TILE + k, i = tx * TR_TILE + lx;
            if (i < cols && j < rows) gbl(D.u)[(size_t)j * cols + i] = t[lx][k];
        }
    } else {
        const gptr<const double> src = gbl(static_cast<const double*>(WHICH == 0 ? D.u : D.f));
        const gptr<double> dst = gbl(WHICH == 0 ? D.uT : D.fT);
        for (int k = ly; k < TR_TILE; k += 8) {
            const int j = ty * TR_TILE + k, i = tx * TR_TILE + lx;
            if (i < cols && j < rows) t[k][lx] = src[(size_t)j * cols + i];
        }
        __syncthreads();
        for (int k = ly; k < TR_TILE; k += 8) {
            const int i = tx * TR_TILE + k, j = ty * TR_TILE + lx;
            if (i < cols && j < rows) dst[(size_t)i * rows + j] = t[lx][k];
        }
    }
}

// x2 lines i = 1 + color, 3 + color, ... of the finest level on uT / fT; the
// axis rows' second-neighbour coupling is eliminated with the adjacent row.
template <int P, int NT>
__global__ void __launch_bounds__(NT)
k_relax_x2t(const MGDesc* __restrict__ lv, const MGState* __restrict__ ms, int color) {
    extern __shared__ double lds[];
    __shared__ double axis_nn, axis_ss;
    const MGDesc& D = lv[blockIdx.y];
    if (!level_active(D, ms)) return;
    const int n1 = D.n1, n2 = D.n2;
    const int i = 1 + color + 2 * xcd_line((n1 - color) / 2);
    if (i > n1 - 1) return;
    const int L = n2 + 1;
    const int cap = L > 2 * NT ? L : 2 * NT;
    double* a = lds;
    double* b = a + cap;
    double* c = b + cap;
    double* d = c + cap;
    const FineStencil st(D);
    const gptr<double> ut = gbl(D.uT);
    const gptr<const double> ft = gbl(static_cast<const double*>(D.fT));
    const size_t base = (size_t)i * L;
    for (int j = threadIdx.x; j < L; j += NT) {
        const size_t o = base + j;
        const Coef k = st.at(j, i, (size_t)j * (n1 + 1) + i);
        double rhs = ft[o] - k.W * ut[o - L] - k.E * ut[o + L];
        if (j > 0) rhs -= k.SW * ut[o - L - 1] + k.SE * ut[o + L - 1];
        if (j < n2) rhs -= k.NW * ut[o - L + 1] + k.NE * ut[o + L + 1];
        a[j] = j > 0 ? k.S : 0.0;
        b[j] = k.C;
        c[j] = j < n2 ? k.N : 0.0;
        d[j] = rhs;
        if (j == 0) axis_nn = k.nn;
        if (j == n2) axis_ss = k.ss;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double mm = axis_nn / c[1];
        b[0] -= mm * a[1];
        c[0] -= mm * b[1];
        d[0] -= mm * d[1];
        const double m2 = axis_ss / a[n2 - 1];
        a[n2] -= m2 * b[n2 - 1];
        b[n2] -= m2 * c[n2 - 1];
        d[n2] -= m2 * d[n2 - 1];
    }
    __syncthreads();
    tri_solve<P, NT>(a, b, c, d, L);
    for (int j = threadIdx.x; j < L; j += NT) ut[base + j] = d[j];
}

// Block sum of a per-thread value (fixed order), written by thread 0.
__device__ inline double block_sum(double v) {
    __shared__ double red[MG_BLOCK / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < MG_BLOCK / 64; ++w) t += red[w];
    __syncthreads();
    return t;
}

// Sum of nb partial sums in a fixed order (one workgroup).
__device__ inline double sum_parts(const double* __restrict__ p, int nb) {
    double v = 0.0;
    for (int k = threadIdx.x; k < nb; k += MG_BLOCK) v += p[k];
    return block_sum(v);
}

// |D^-1 (f - A u)|^2 over the unknown nodes of the finest level (D = diagonal
// of A, lv = the finest level): the operator's rows differ in scale by ~r^4,
// and the row-scaled norm weighs every node alike.  One partial sum per
// workgroup, part[grain][block]; the batch counters of the check that follows
// are cleared here.
template <class ST>
__global__ void __launch_bounds__(MG_BLOCK)
k_residual_norm(const MGDesc* __restrict__ lv, const MGState* __restrict__ ms, double* __restrict__ part,
                MGBatch* __restrict__ mb) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        mb->pending_prev = mb->pending;
        mb->pending = 0;
        mb->max_cycles = 0;
    }
    const MGDesc& D = lv[blockIdx.y];
    double rr = 0.0;
    const int idx = blockIdx.x * MG_BLOCK + threadIdx.x;
    if (D.n1 != 0 && !ms[blockIdx.y].done && idx < D.nodes) {
        const int n1 = D.n1, n2 = D.n2, nx = n1 + 1;
        const int j = idx / nx, i = idx - j * nx;
        if (i > 0 && i < n1) {
            const ST st(D);
            const Coef k = st.at(j, i, idx);
            const gptr<const double> u = gbl(static_cast<const double*>(D.u));
            double au = k.C * u[idx] + k.W * u[idx - 1] + k.E * u[idx + 1];
            if (j > 0) au += k.S * u[idx - nx] + k.SW * u[idx - nx - 1] + k.SE * u[idx - nx + 1];
            if (j < n2) au += k.N * u[idx + nx] + k.NW * u[idx + nx - 1] + k.NE * u[idx + nx + 1];
            if (j == 0) au += k.nn * u[idx + 2 * nx];
            if (j == n2) au += k.ss * u[idx - 2 * nx];
            const double q = (gbl(D.f)[idx] - au) / k.C;
            rr = q * q;
        }
    }
    const double t = block_sum(rr);
    if (threadIdx.x == 0) gbl(part)[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

// Per grain (blockIdx.x): its partial norms added in a fixed order (so a solve
// is reproducible bit for bit), then the convergence check: the grain is done
// once |D^-1 r| <= tol |D^-1 b| (b with the boundary coupling) or when its
// residual is not finite.  part_b (the right-hand side's partials, at the start
// of a solve) is summed into b2 when given; count_cycle marks the check that
// ends a V-cycle.  The batch counters (grains pending, largest cycle count, a
// non-finite residual) gather the grains' states by atomics.
__global__ void __launch_bounds__(MG_BLOCK)
k_mg_sum_check(MGState* __restrict__ ms, const GrainDesc* __restrict__ gd, int nb, const double* __restrict__ part,
               const double* __restrict__ part_b, double tol2, int count_cycle, MGBatch* __restrict__ mb) {
    const int g = blockIdx.x;
    MGState& m = ms[g];
    if (!m.done) {
        const double r2 = sum_parts(part + (size_t)g * nb, nb);
        const double b2 = part_b ? sum_parts(part_b + (size_t)g * nb, nb) : 0.0;
        if (threadIdx.x == 0) {
            if (part_b) m.b2 = b2;
            m.r2 = r2;
            m.last_r2 = r2;
            if (count_cycle) m.cycles += 1;
            if (!(r2 == r2) || !(m.b2 == m.b2)) {
                atomicOr(&mb->nan, 1);
                m.done = 1;
            } else if (r2 <= tol2 * (m.b2 + gd[g].bnd2)) {
                m.done = 1;
            }
        }
    }
    if (threadIdx.x == 0) {
        if (!m.done) atomicAdd(&mb->pending, 1);
        atomicMax(&mb->max_cycles, m.cycles);
    }
}
// |D^-1 f|^2 over the unknown nodes, partial sums as above
template <class ST>
__global__ void __launch_bounds__(MG_BLOCK)
k_rhs_norm(const MGDesc* __restrict__ lv, const MGState* __restrict__ ms, double* __restrict__ part) {
    const MGDesc& D = lv[blockIdx.y];
    double* out = part + (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (D.n1 == 0 || ms[blockIdx.y].done || (int)(blockIdx.x * MG_BLOCK) >= D.nodes) {
        if (threadIdx.x == 0) *out = 0.0;
        return;
    }
    const int nx = D.n1 + 1;
    const int idx = blockIdx.x * MG_BLOCK + threadIdx.x;
    double v = 0.0;
    if (idx < D.nodes) {
        const int i = idx % nx;
        if (i > 0 && i < D.n1) {
            const ST st(D);
            const double q = gbl(D.f)[idx] / st.diag(idx / nx, i, idx);
            v = q * q;
        }
    }
    const double t = block_sum(v);
    if (threadIdx.x == 0) *out = t;
}

// Start of a solve: grains other than `only` (if >= 0) are excluded from it.
__global__ void __launch_bounds__(MG_BLOCK)
k_mg_reset(MGState* __restrict__ ms, int ngrains, int only, int in_step) {
    for (int g = threadIdx.x; g < ngrains; g += MG_BLOCK) {
        const bool solved = only < 0 || g == only;
        ms[g].r2 = 0.0;
        ms[g].b2 = 0.0;
        ms[g].cycles = 0;
        ms[g].done = solved ? 0 : 1;
        // an in-step solve leaves a history to extrapolate from; a standalone
        // solve (a new density or new particles) starts a new one
        if (in_step) ms[g].extrap = 1;
        else if (solved) ms[g].extrap = 0;
    }
}

// Initial guess of an in-step solve, linear extrapolation in time from the
// last two solutions: u <- 2 u - uprev, uprev <- u (the time step is fixed).
// Without a history (first in-step solve after a standalone one) the guess is
// the last solution and the history starts.  Dirichlet nodes are set again
// afterwards.
__global__ void __launch_bounds__(MG_BLOCK)
k_extrapolate(const MGDesc* __restrict__ lv, const MGState* __restrict__ ms) {
    const MGDesc& D = lv[blockIdx.y];
    const int o = blockIdx.x * MG_BLOCK + threadIdx.x;
    if (D.n1 == 0 || o >= D.nodes) return;
    const gptr<double> u = gbl(D.u);
    const gptr<double> up = gbl(D.uprev);
    const double t = u[o];
    if (ms[blockIdx.y].extrap) u[o] = 2.0 * t - up[o];
    up[o] = t;
}


// Coarse right-hand side fc = P^T (f - A u) / 4 on the coarse unknowns, the
// fine residuals formed on the fly (full weighting without rows outside the
// grid); fc = 0 on the coarse Dirichlet columns; the coarse correction uc is
// cleared.
template <class ST>
__global__ void __launch_bounds__(MG_BLOCK)
k_restrict_residual(const MGDesc* __restrict__ fine, const MGDesc* __restrict__ coarse,
                    const MGState* __restrict__ ms) {
    const MGDesc& F = fine[blockIdx.y];
    const MGDesc& C = coarse[blockIdx.y];
    if (C.n1 == 0 || !level_active(F, ms)) return;
    const int n1c = C.n1, nxc = n1c + 1;
    const int n2f = F.n2, nxf = F.n1 + 1;
    const int idx = blockIdx.x * MG_BLOCK + threadIdx.x;
    if (idx >= C.nodes) return;
    gbl(C.u)[idx] = 0.0;
    const int J = idx / nxc, I = idx - J * nxc;
    if (I == 0 || I == n1c) {
        gbl(C.f)[idx] = 0.0;
        return;
    }
    const ST st(F);
    double acc = 0.0;
    for (int dj = -1; dj <= 1; ++dj) {
        const int j = 2 * J + dj;
        if (j < 0 || j > n2f) continue;
        const double wj = dj == 0 ? 1.0 : 0.5;
        for (int di = -1; di <= 1; ++di) {
            const int i = 2 * I + di;      // 1 <= i <= n1f - 1
            const double wi = di == 0 ? 1.0 : 0.5;
            const double r = gbl(F.f)[(size_t)j * nxf + i] - apply_A(st, gbl(static_cast<const double*>(F.u)), n2f, nxf, j, i);
            acc += wj * wi * r;
        }
    }
    gbl(C.f)[idx] = 0.25 * acc;
}

// The same restriction from the finest level, by tiles of RT x RT coarse
// nodes: the workgroup first forms the fine residuals under its tile once
// each ((2 RT + 1)^2 nodes, into LDS), then every coarse node adds up its nine
// weighted ones in the order above.  The per-node
// form evaluates the finest operator at every fine node for each of the up to
// four coarse nodes that use it.
constexpr int RT = 16;
constexpr int RF = 2 * RT + 1;
static_assert(RT * RT == MG_BLOCK, "one coarse node per thread");

__global__ void __launch_bounds__(MG_BLOCK)
k_restrict_residual_fine(const MGDesc* __restrict__ fine, const MGDesc* __restrict__ coarse,
                         const MGState* __restrict__ ms) {
    __shared__ double res[RF * RF];
    const MGDesc& F = fine[blockIdx.y];
    const MGDesc& C = coarse[blockIdx.y];
    if (C.n1 == 0 || !level_active(F, ms)) return;
    const int n1c = C.n1, n2c = C.n2, nxc = n1c + 1;
    const int n1f = F.n1, n2f = F.n2, nxf = n1f + 1;
    const int tx = (nxc + RT - 1) / RT, ty = (n2c + RT) / RT;
    if ((int)blockIdx.x >= tx * ty) return;
    const int I0 = ((int)blockIdx.x % tx) * RT, J0 = ((int)blockIdx.x / tx) * RT;
    const FineStencil st(F);
    const gptr<const double> u = gbl(static_cast<const double*>(F.u));
    const gptr<const double> f = gbl(static_cast<const double*>(F.f));
    // fine node (2 J0 - 1 + b, 2 I0 - 1 + a) -> res[b RF + a]; 0 outside the unknowns
    for (int t = threadIdx.x; t < RF * RF; t += MG_BLOCK) {
        const int b = t / RF, a = t - b * RF;
        const int i = 2 * I0 - 1 + a, j = 2 * J0 - 1 + b;
        double r = 0.0;
        if (i >= 1 && i <= n1f - 1 && j >= 0 && j <= n2f) r = f[(size_t)j * nxf + i] - apply_A(st, u, n2f, nxf, j, i);
        res[t] = r;
    }
    __syncthreads();
    const int I = I0 + (int)threadIdx.x % RT, J = J0 + (int)threadIdx.x / RT;
    if (I > n1c || J > n2c) return;
    const int idx = J * nxc + I;
    gbl(C.u)[idx] = 0.0;
    if (I == 0 || I == n1c) {
        gbl(C.f)[idx] = 0.0;
        return;
    }
    double acc = 0.0;
    for (int dj = -1; dj <= 1; ++dj) {
        const int j = 2 * J + dj;
        if (j < 0 || j > n2f) continue;
        const double wj = dj == 0 ? 1.0 : 0.5;
        for (int di = -1; di <= 1; ++di) {
            const double wi = di == 0 ? 1.0 : 0.5;
            acc += wj * wi * res[(2 * (J - J0) + dj + 1) * RF + 2 * (I - I0) + di + 1];
        }
    }
    gbl(C.f)[idx] = 0.25 * acc;
}

// The same restriction from a level whose u is zero (every level below the
// finest in a sawtooth cycle: the restriction into it cleared it), where the
// residual is f itself: C.f = R F.f, C.u = 0.
__global__ void __launch_bounds__(MG_BLOCK)
k_restrict_rhs(const MGDesc* __restrict__ fine, const MGDesc* __restrict__ coarse,
               const MGState* __restrict__ ms) {
    const MGDesc& F = fine[blockIdx.y];
    const MGDesc& C = coarse[blockIdx.y];
    if (C.n1 == 0 || !level_active(F, ms)) return;
    const int n1c = C.n1, nxc = n1c + 1;
    const int n2f = F.n2, nxf = F.n1 + 1;
    const int idx = blockIdx.x * MG_BLOCK + threadIdx.x;
    if (idx >= C.nodes) return;
    gbl(C.u)[idx] = 0.0;
    const int J = idx / nxc, I = idx - J * nxc;
    if (I == 0 || I == n1c) {
        gbl(C.f)[idx] = 0.0;
        return;
    }
    const gptr<const double> f = gbl(static_cast<const double*>(F.f));
    double acc = 0.0;
    for (int dj = -1; dj <= 1; ++dj) {
        const int j = 2 * J + dj;
        if (j < 0 || j > n2f) continue;
        const double wj = dj == 0 ? 1.0 : 0.5;
        for (int di = -1; di <= 1; ++di) {
            const int i = 2 * I + di;
            const double wi = di == 0 ? 1.0 : 0.5;
            acc += wj * wi * f[(size_t)j * nxf + i];
        }
    }
    gbl(C.f)[idx] = 0.25 * acc;
}

// fine u += P uc (bilinear) on the fine unknowns
__global__ void __launch_bounds__(MG_BLOCK)
k_prolong_add(const MGDesc* __restrict__ fine, const MGDesc* __restrict__ coarse,
              const MGState* __restrict__ ms) {
    const MGDesc& F = fine[blockIdx.y];
    const MGDesc& C = coarse[blockIdx.y];
    if (C.n1 == 0 || !level_active(F, ms)) return;
    const int nxc = C.n1 + 1, n1f = F.n1, nxf = n1f + 1;
    const int idx = blockIdx.x * MG_BLOCK + threadIdx.x;
    if (idx >= F.nodes) return;
    const int j = idx / nxf, i = idx - j * nxf;
    if (i == 0 || i == n1f) return;
    const int J0 = j >> 1, I0 = i >> 1;
    const int J1 = (j & 1) ? J0 + 1 : J0;
    const int I1 = (i & 1) ? I0 + 1 : I0;
    const gptr<const double> uc = gbl(static_cast<const double*>(C.u));
    const double v = 0.25 * (uc[(size_t)J0 * nxc + I0] + uc[(size_t)J0 * nxc + I1] +
                             uc[(size_t)J1 * nxc + I0] + uc[(size_t)J1 * nxc + I1]);
    gbl(F.u)[idx] += v;
}

// Dense solve on a grain's coarsest level: u = A^-1 rhs with rhs = f on the
// unknowns and rhs = u on the Dirichlet columns (identity rows of A), so the
// same kernel serves a correction level (u = 0 there) and a grid that is
// itself small enough.  The workgroup stages rhs in LDS once; each wave then
// streams CS_RW rows of the inverse together (rows padded to an even length,
// two entries per lane and load), so every rhs pair read from LDS serves
// CS_RW rows and CS_RW loads are in flight per step.  The kernel writes u only
// on unknown rows and reads it only on Dirichlet columns.
constexpr int CS_RW = 4;                          // rows per wave
constexpr int CS_ROWS = CS_RW * (MG_BLOCK / 64);  // rows per workgroup
constexpr int CS_STAGE = 8;

__global__ void __launch_bounds__(MG_BLOCK)
k_coarse_solve(const MGDesc* __restrict__ lv, const MGState* __restrict__ ms) {
    extern __shared__ double rhs[];
    typedef double dbl2 __attribute__((ext_vector_type(2)));
    const MGDesc& D = lv[blockIdx.y];
    if (D.n1 == 0 || !D.coarsest || ms[blockIdx.y].done) return;
    const int m = D.m, mp = (m + 1) & ~1, nx = D.n1 + 1;
    const int row0 = blockIdx.x * CS_ROWS;
    if (row0 >= m) return;
    const gptr<double> u = gbl(D.u);
    const gptr<const double> f = gbl(static_cast<const double*>(D.f));
    // staged in batches of CS_STAGE independent loads per thread (a loop of
    // one load and one LDS store per trip would wait out every load in turn)
    for (int k0 = threadIdx.x; k0 < mp; k0 += CS_STAGE * MG_BLOCK) {
        double v[CS_STAGE];
#pragma unroll
        for (int j = 0; j < CS_STAGE; ++j) {
            const int k = k0 + j * MG_BLOCK;
            v[j] = 0.0;
            if (k < m) {
                const int i = k % nx;
                v[j] = (i == 0 || i == D.n1) ? u[k] : f[k];
            }
        }
#pragma unroll
        for (int j = 0; j < CS_STAGE; ++j)
            if (k0 + j * MG_BLOCK < mp) rhs[k0 + j * MG_BLOCK] = v[j];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int rw = row0 + (threadIdx.x >> 6) * CS_RW;
    if (rw >= m) return;
    // rows past the end repeat the last row (loaded, never stored)
    gptr<const dbl2> a[CS_RW];
#pragma unroll
    for (int r = 0; r < CS_RW; ++r) a[r] = (gptr<const dbl2>)gbl(D.inv + (size_t)min(rw + r, m - 1) * mp);
    const dbl2* x = reinterpret_cast<const dbl2*>(rhs);
    double acc[CS_RW];
#pragma unroll
    for (int r = 0; r < CS_RW; ++r) acc[r] = 0.0;
#pragma unroll 2
    for (int k = lane; k < mp / 2; k += 64) {
        const dbl2 xv = x[k];
#pragma unroll
        for (int r = 0; r < CS_RW; ++r) {
            const dbl2 v = a[r][k];
            acc[r] += v.x * xv.x + v.y * xv.y;
        }
    }
#pragma unroll
    for (int r = 0; r < CS_RW; ++r) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc[r] += __shfl_xor(acc[r], o);
    }
    if (lane == 0) {
#pragma unroll
        for (int r = 0; r < CS_RW; ++r) {
            const int row = rw + r;
            const int ri = row % nx;
            if (row < m && ri != 0 && ri != D.n1) u[row] = acc[r];
        }
    }
}

// ------------------------------------------------------------------ launches
// Line-solve launches.  An x1 line of more than 1024 unknowns is solved by the
// partition method (512 threads of five equations), one of 513 to 1024 by
// cyclic reduction with 1024 threads, else 256; an x2 line gets 512 threads
// beyond 256 unknowns, else 256 (fewer equations per thread, a
// shorter PCR critical path).  Where a sweep has fewer than four lines per
// compute unit, a line of 257 to 512 unknowns (x1) or more than 512 (x2) gets
// one thread per unknown: with about one workgroup per compute unit the extra
// waves cover the LDS round trips; with many lines they only add idle lanes.
// The x2 sweeps group LPB neighbouring lines of one colour per workgroup while
// that still leaves at least two workgroups per compute unit.
static int round8(int x) { return (x + 7) / 8 * 8; }

static bool few_lines(const apic_ctx* ctx, int lines) { return lines < 4 * ctx->num_cus; }

static int pcr_k(int total, int nt) {
    const int k = (total + nt - 1) / nt;
    return k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : 8;
}

// LDS of an x1-line workgroup: the tridiagonal system, plus the two prolonged
// neighbour rows when it applies the coarse-grid correction
static size_t x1_lds(int mn1, bool prolong) {
    return sizeof(double) * (4 * (size_t)(mn1 - 1) + (prolong ? 2 * (size_t)(mn1 + 1) : 0));
}

// x1 lines by the partition method (TP equations per thread, NT threads).
template <int TP, int NT, class ST>
static void relax_x1_tri(apic_ctx* ctx, int l, int color, bool prolong) {
    const int mn1 = ctx->lvl_max_n1[l], mn2 = ctx->lvl_max_n2[l];
    const size_t L = (size_t)std::max(mn1 - 1, 2 * NT);
    const size_t lds = sizeof(double) * (4 * L + (prolong ? 2 * (size_t)(mn1 + 1) : 0));
    const int lines = (mn2 + 1 - color + 1) / 2;
    const int G = (int)ctx->grains.size();
    hipLaunchKernelGGL((k_relax_x1<1, NT, ST, TP>), dim3(round8(lines), G), dim3(NT), lds, ctx->stream,
                       ctx->mgdesc + (size_t)l * G, ctx->mgs, color,
                       prolong ? ctx->mgdesc + (size_t)(l + 1) * G : (const MGDesc*)nullptr);
}

template <int K, int NT, class ST>
static void relax_x1_launch(apic_ctx* ctx, int l, int color, bool prolong) {
    const int mn1 = ctx->lvl_max_n1[l], mn2 = ctx->lvl_max_n2[l];
    const size_t lds = x1_lds(mn1, prolong);
    const int lines = (mn2 + 1 - color + 1) / 2;
    const int G = (int)ctx->grains.size();
    hipLaunchKernelGGL((k_relax_x1<K, NT, ST>), dim3(round8(lines), G), dim3(NT), lds, ctx->stream,
                       ctx->mgdesc + (size_t)l * G, ctx->mgs, color,
                       prolong ? ctx->mgdesc + (size_t)(l + 1) * G : (const MGDesc*)nullptr);
}

template <int K, int LPB, int NT, class ST>
static void relax_x2_launch(apic_ctx* ctx, int l, int color) {
    const int mn1 = ctx->lvl_max_n1[l], mn2 = ctx->lvl_max_n2[l];
    const size_t lds = 4 * sizeof(double) * (size_t)LPB * (mn2 + 1);
    const int lines = (mn1 - 1 - color + 1) / 2;
    if (lines <= 0) return;
    const int blocks = (lines + LPB - 1) / LPB;
    const int G = (int)ctx->grains.size();
    hipLaunchKernelGGL((k_relax_x2<K, LPB, NT, ST>), dim3(round8(blocks), G), dim3(NT), lds, ctx->stream,
                       ctx->mgdesc + (size_t)l * G, ctx->mgs, color);
}

template <int NT, class ST>
static void relax_x1_k(apic_ctx* ctx, int l, int color, bool prolong) {
    switch (pcr_k(ctx->lvl_max_n1[l] - 1, NT)) {
        case 1: relax_x1_launch<1, NT, ST>(ctx, l, color, prolong); break;
        case 2: relax_x1_launch<2, NT, ST>(ctx, l, color, prolong); break;
        case 4: relax_x1_launch<4, NT, ST>(ctx, l, color, prolong); break;
        default: relax_x1_launch<8, NT, ST>(ctx, l, color, prolong); break;
    }
}

template <int LPB, int NT, class ST>
static void relax_x2_k(apic_ctx* ctx, int l, int color) {
    switch (pcr_k(LPB * (ctx->lvl_max_n2[l] + 1), NT)) {
        case 1: relax_x2_launch<1, LPB, NT, ST>(ctx, l, color); break;
        case 2: relax_x2_launch<2, LPB, NT, ST>(ctx, l, color); break;
        case 4: relax_x2_launch<4, LPB, NT, ST>(ctx, l, color); break;
        default: relax_x2_launch<8, LPB, NT, ST>(ctx, l, color); break;
    }
}

// Both colours of the x1-line sweep of level l (on the finest level the odd
// colour also solves the two axis rows); with prolong, the first colour also applies the coarse-grid
// correction from level l + 1.
template <class ST>
static void sweep_x1(apic_ctx* ctx, int l, bool prolong) {
    const int colors = 2;
    if (prolong && x1_lds(ctx->lvl_max_n1[l], true) > 65536) {
        // rows too long to stage two more of them: the correction separately
        const int G = (int)ctx->grains.size();
        const int fn = ctx->lvl_max_nodes[l];
        hipLaunchKernelGGL(k_prolong_add, dim3((fn + MG_BLOCK - 1) / MG_BLOCK, G), dim3(MG_BLOCK), 0,
                           ctx->stream, ctx->mgdesc + (size_t)l * G, ctx->mgdesc + (size_t)(l + 1) * G,
                           ctx->mgs);
        prolong = false;
    }
    for (int color = 0; color < colors; ++color) {
        const bool pro = prolong && color == 0;
        // lines beyond 1024 unknowns (grids up to 2048 cells wide: at most 2047 <= 5 x 512):
        // the partition method, whose chunk eliminations need no barrier and whose
        // cyclic reduction runs on the 1024 chunk ends (c5 field 3.77 -> 3.42 ms against
        // cyclic reduction over the whole line with 1024 threads)
        if (ctx->lvl_max_n1[l] - 1 > 1024) relax_x1_tri<5, 512, ST>(ctx, l, color, pro);
        else if (ctx->lvl_max_n1[l] - 1 > 512) relax_x1_k<1024, ST>(ctx, l, color, pro);
        else if (ctx->lvl_max_n1[l] - 1 > 256 && few_lines(ctx, ctx->lvl_lines_x1[l]))
            relax_x1_k<512, ST>(ctx, l, color, pro);
        else relax_x1_k<256, ST>(ctx, l, color, pro);
    }
}

// Both colours of the x2-line sweep of level l (lines read in place).
template <class ST>
static void sweep_x2(apic_ctx* ctx, int l) {
    const int Lx2 = ctx->lvl_max_n2[l] + 1;
    const int lines = ctx->lvl_lines_x2[l];   // x2 lines of one colour, summed over grains
    int lpb = 4;
    while (lpb > 1 && (4 * sizeof(double) * (size_t)lpb * Lx2 > 61440 || lpb * Lx2 > 8 * 256 ||
                       lines / lpb < 2 * ctx->num_cus))
        lpb >>= 1;
    for (int color = 0; color < 2; ++color) {
        if (lpb == 4) relax_x2_k<4, 256, ST>(ctx, l, color);
        else if (lpb == 2) relax_x2_k<2, 256, ST>(ctx, l, color);
        else if (Lx2 > 512 && few_lines(ctx, lines)) relax_x2_k<1, 1024, ST>(ctx, l, color);
        else if (Lx2 > 256) relax_x2_k<1, 512, ST>(ctx, l, color);
        else relax_x2_k<1, 256, ST>(ctx, l, color);
    }
}

template <int WHICH>
static void transpose(apic_ctx* ctx) {
    const int G = (int)ctx->grains.size();
    const int tiles = ((ctx->max_n1 + TR_TILE) / TR_TILE) * ((ctx->max_n2 + TR_TILE) / TR_TILE);
    hipLaunchKernelGGL(k_transpose<WHICH>, dim3(tiles, G), dim3(256), 0, ctx->stream, ctx->mgdesc, ctx->mgs);
}

// Shape of the partition solver for `total` equations per workgroup: NT
// threads of P equations each (line lengths are bounded by the grid limits,
// at most 2048 equations).
template <template <int, int> class Launch, class... Args>
static void with_tri_shape(int total, Args... args) {
    if (total <= 64 * 3) Launch<3, 64>::run(args...);
    else if (total <= 64 * 5) Launch<5, 64>::run(args...);
    else if (total <= 64 * 9) Launch<9, 64>::run(args...);
    else if (total <= 128 * 9) Launch<9, 128>::run(args...);
    else Launch<17, 128>::run(args...);
}

template <int P, int NT>
struct RelaxX2T {
    static void run(apic_ctx* ctx, int color) {
        const int G = (int)ctx->grains.size();
        const int lines = (ctx->lvl_max_n1[0] - 1 - color + 1) / 2;
        const int L = ctx->lvl_max_n2[0] + 1;
        const size_t lds = 4 * sizeof(double) * (size_t)std::max(L, 2 * NT);
        hipLaunchKernelGGL((k_relax_x2t<P, NT>), dim3(round8(lines), G), dim3(NT), lds, ctx->stream, ctx->mgdesc,
                           ctx->mgs, color);
    }
};

// Smoothing of level l after its coarse-grid correction: x1 lines, x2 lines,
// x1 lines (each sweep both colours).  No smoothing precedes the restriction
// (a sawtooth cycle): on these operators that converges per cycle about as
// fast as one alternating sweep before and after the correction, with six
// sweep launches per level instead of eight.  The finest level's operator is
// evaluated at the nodes (its x2 sweeps on the transposed copies when the
// level is large), the coarse ones are stored.
template <class ST>
static void smooth_st(apic_ctx* ctx, int l) {
    sweep_x1<ST>(ctx, l, true);
    sweep_x2<ST>(ctx, l);
    sweep_x1<ST>(ctx, l, false);
}

static void smooth(apic_ctx* ctx, int l) {
    if (l > 0 || ctx->opts.conservative_poisson) {   // stored operator
        smooth_st<StoredStencil>(ctx, l);
        return;
    }
    if (!ctx->x2_transposed) {
        smooth_st<FineStencil>(ctx, 0);
        return;
    }
    sweep_x1<FineStencil>(ctx, 0, true);
    transpose<0>(ctx);
    for (int color = 0; color < 2; ++color) with_tri_shape<RelaxX2T>(ctx->lvl_max_n2[0] + 1, ctx, color);
    transpose<1>(ctx);
    sweep_x1<FineStencil>(ctx, 0, false);
}

// The dense solves of every grain's coarsest level (whatever level that is) in
// one launch.
static void coarse_solve(apic_ctx* ctx) {
    const int G = (int)ctx->grains.size();
    const int m = ctx->max_coarse_m;
    if (m <= 0) return;
    const size_t lds = sizeof(double) * (size_t)((m + 1) & ~1);
    hipLaunchKernelGGL(k_coarse_solve, dim3((m + CS_ROWS - 1) / CS_ROWS, G), dim3(MG_BLOCK), lds, ctx->stream,
                       ctx->mgdesc_coarse, ctx->mgs);
}

static int norm_blocks(apic_ctx* ctx) { return (ctx->lvl_max_nodes[0] + MG_BLOCK - 1) / MG_BLOCK; }

// Residual norm of the finest level, then its per-grain sums and the
// convergence check (the right-hand side's partials are summed too at the start
// of a solve).
static void residual_check(apic_ctx* ctx, double tol, int count_cycle, bool with_b) {
    const int G = (int)ctx->grains.size();
    const int nb = norm_blocks(ctx);
    if (ctx->opts.conservative_poisson)
        hipLaunchKernelGGL(k_residual_norm<StoredStencil>, dim3(nb, G), dim3(MG_BLOCK), 0, ctx->stream, ctx->mgdesc,
                           ctx->mgs, ctx->norm_part, ctx->mgb);
    else
        hipLaunchKernelGGL(k_residual_norm<FineStencil>, dim3(nb, G), dim3(MG_BLOCK), 0, ctx->stream, ctx->mgdesc,
                           ctx->mgs, ctx->norm_part, ctx->mgb);
    hipLaunchKernelGGL(k_mg_sum_check, dim3(G), dim3(MG_BLOCK), 0, ctx->stream, ctx->mgs, ctx->gdesc, nb,
                       ctx->norm_part, with_b ? ctx->norm_part + (size_t)G * nb : nullptr, tol * tol, count_cycle,
                       ctx->mgb);
}

// Start of a solve on the current right-hand side (Dirichlet values already
// set): |D^-1 b|^2, the initial residual, and the check (grains that already
// meet the tolerance are done).
hipError_t mg_begin(apic_ctx* ctx, double tol, int only_grain, bool in_step) {
    const int G = (int)ctx->grains.size();
    hipLaunchKernelGGL(k_mg_reset, dim3(1), dim3(MG_BLOCK), 0, ctx->stream, ctx->mgs, G, only_grain, (int)in_step);
    if (ctx->opts.conservative_poisson)
        hipLaunchKernelGGL(k_rhs_norm<StoredStencil>, dim3(norm_blocks(ctx), G), dim3(MG_BLOCK), 0, ctx->stream,
                           ctx->mgdesc, ctx->mgs, ctx->norm_part + (size_t)G * norm_blocks(ctx));
    else
        hipLaunchKernelGGL(k_rhs_norm<FineStencil>, dim3(norm_blocks(ctx), G), dim3(MG_BLOCK), 0, ctx->stream,
                           ctx->mgdesc, ctx->mgs, ctx->norm_part + (size_t)G * norm_blocks(ctx));
    residual_check(ctx, tol, 0, true);
    if (ctx->x2_transposed) transpose<2>(ctx);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Boltzmann electrons
// With n_e = exp(phi) (units n0, Te/e), eq. (6) reads A phi = s rho_p - s exp(phi),
// s = -1/kappa^2 (rhs_scale).  A Newton step linearises exp about the current
// phi: (A - E) phi' = s rho_p + E (1 - phi) with E = -s exp(phi) on the unknown
// nodes.  The multigrid solves it with E subtracted from every level's diagonal:
// on the finest level E itself, on each coarser one the full-weighting average
// of the level above (the row sums of the Galerkin product R E P, as P carries
// a constant to a constant), and the coarsest level's dense inverse is formed
// again on the device.
__global__ void __launch_bounds__(MG_BLOCK)
k_newton_prepare(const GrainDesc* __restrict__ gd, const MGDesc* __restrict__ lv, int only) {
    const GrainDesc& G = gd[blockIdx.y];
    const MGDesc& D = lv[blockIdx.y];
    if (only >= 0 && (int)blockIdx.y != only) return;
    const int idx = blockIdx.x * MG_BLOCK + threadIdx.x;
    if (idx >= D.nodes) return;
    const int i = idx % D.nx;
    double* sh = const_cast<double*>(D.shift);
    if (i == 0 || i == D.n1) {
        gbl(sh)[idx] = 0.0;
        return;
    }
    const double u = gbl(static_cast<const double*>(D.u))[idx];
    const double e = -G.rhs_scale * exp(u);
    gbl(D.uold)[idx] = u;
    gbl(sh)[idx] = e;
    gbl(D.f)[idx] = G.rhs_scale * gbl(static_cast<const double*>(G.rho))[idx] + e * (1.0 - u);
}

__global__ void __launch_bounds__(MG_BLOCK)
k_restrict_shift(const MGDesc* __restrict__ fine, const MGDesc* __restrict__ coarse, int only) {
    const MGDesc& F = fine[blockIdx.y];
    const MGDesc& C = coarse[blockIdx.y];
    if (C.n1 == 0 || (only >= 0 && (int)blockIdx.y != only)) return;
    const int n1c = C.n1, nxc = n1c + 1;
    const int n2f = F.n2, nxf = F.n1 + 1;
    const int idx = blockIdx.x * MG_BLOCK + threadIdx.x;
    if (idx >= C.nodes) return;
    const int J = idx / nxc, I = idx - J * nxc;
    double* out = const_cast<double*>(C.shift);
    if (I == 0 || I == n1c) {
        gbl(out)[idx] = 0.0;
        return;
    }
    const gptr<const double> e = gbl(F.shift);
    double acc = 0.0;
    for (int dj = -1; dj <= 1; ++dj) {
        const int j = 2 * J + dj;
        if (j < 0 || j > n2f) continue;
        const double wj = dj == 0 ? 1.0 : 0.5;
        for (int di = -1; di <= 1; ++di) {
            const double wi = di == 0 ? 1.0 : 0.5;
            acc += wj * wi * e[(size_t)j * nxf + 2 * I + di];
        }
    }
    gbl(out)[idx] = 0.25 * acc;
}

// Dense inverse of a grain's coarsest operator (with its Newton term) in one
// workgroup: the m x m matrix (identity rows on the Dirichlet columns) is
// assembled in LDS and inverted in place by Gauss-Jordan elimination with
// partial pivoting (the row interchanges are undone on the columns of the
// inverse at the end), then written with rows padded to an even length.
constexpr int INV_BLOCK = 1024;   // sixteen waves, each taking whole rows

template <class ST>
__global__ void __launch_bounds__(INV_BLOCK)
k_coarse_invert(const MGDesc* __restrict__ lv, int only) {
    extern __shared__ double M[];
    __shared__ double colk[BOLTZ_INV_MAX];
    __shared__ int piv[BOLTZ_INV_MAX];
    __shared__ int prow;
    const MGDesc& D = lv[blockIdx.y];
    if (D.n1 == 0 || !D.coarsest || (only >= 0 && (int)blockIdx.y != only)) return;
    const int m = D.m, nx = D.n1 + 1, n2 = D.n2;
    if (m > BOLTZ_INV_MAX) return;   // the host never builds such a level
    for (int t = threadIdx.x; t < m * m; t += INV_BLOCK) M[t] = 0.0;
    __syncthreads();
    const ST st(D);
    for (int o = threadIdx.x; o < m; o += INV_BLOCK) {
        const int j = o / nx, i = o - j * nx;
        double* row = M + (size_t)o * m;
        if (i == 0 || i == D.n1) {
            row[o] = 1.0;
            continue;
        }
        const Coef k = st.at(j, i, o);
        row[o] = k.C;
        row[o - 1] = k.W;
        row[o + 1] = k.E;
        if (j > 0) {
            row[o - nx] = k.S;
            row[o - nx - 1] = k.SW;
            row[o - nx + 1] = k.SE;
        }
        if (j < n2) {
            row[o + nx] = k.N;
            row[o + nx - 1] = k.NW;
            row[o + nx + 1] = k.NE;
        }
        if (j == 0) row[o + 2 * nx] += k.nn;
        if (j == n2) row[o - 2 * nx] += k.ss;
    }
    __syncthreads();
    for (int k = 0; k < m; ++k) {
        if (threadIdx.x < 64) {
            // pivot: largest |M[r][k]|, r >= k (first of equal ones)
            double best = -1.0;
            int br = k;
            for (int r = k + (int)threadIdx.x; r < m; r += 64) {
                const double v = fabs(M[(size_t)r * m + k]);
                if (v > best) {
                    best = v;
                    br = r;
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(best, off);
                const int orow = __shfl_xor(br, off);
                if (ov > best || (ov == best && orow < br)) {
                    best = ov;
                    br = orow;
                }
            }
            if (threadIdx.x == 0) {
                prow = br;
                piv[k] = br;
            }
        }
        __syncthreads();
        const int p = prow;
        if (p != k)
            for (int c = threadIdx.x; c < m; c += INV_BLOCK) {
                const double t = M[(size_t)k * m + c];
                M[(size_t)k * m + c] = M[(size_t)p * m + c];
                M[(size_t)p * m + c] = t;
            }
        __syncthreads();
        const double pinv = 1.0 / M[(size_t)k * m + k];
        for (int r = threadIdx.x; r < m; r += INV_BLOCK) colk[r] = M[(size_t)r * m + k];
        __syncthreads();
        for (int c = threadIdx.x; c < m; c += INV_BLOCK)
            M[(size_t)k * m + c] = (c == k ? 1.0 : M[(size_t)k * m + c]) * pinv;
        __syncthreads();
        for (int r = (int)threadIdx.x >> 6; r < m; r += INV_BLOCK / 64) {
            if (r == k) continue;
            const double fr = colk[r];
            double* row = M + (size_t)r * m;
            for (int c = threadIdx.x & 63; c < m; c += 64) row[c] = (c == k ? 0.0 : row[c]) - M[(size_t)k * m + c] * fr;
        }
        __syncthreads();
    }
    // undo the row interchanges on the columns, last first
    for (int k = m - 1; k >= 0; --k) {
        const int p = piv[k];
        if (p != k)
            for (int r = threadIdx.x; r < m; r += INV_BLOCK) {
                const double t = M[(size_t)r * m + k];
                M[(size_t)r * m + k] = M[(size_t)r * m + p];
                M[(size_t)r * m + p] = t;
            }
        __syncthreads();
    }
    const int mp = (m + 1) & ~1;
    double* inv = const_cast<double*>(D.inv);
    for (int r = (int)threadIdx.x >> 6; r < m; r += INV_BLOCK / 64)
        for (int c = threadIdx.x & 63; c < mp; c += 64) gbl(inv)[(size_t)r * mp + c] = c < m ? M[(size_t)r * m + c] : 0.0;
}

// Damped Newton: a step changes phi by at most NEWTON_MAX_STEP (Te/e) at any
// node.  Far from the solution (a new density, a first solve) the linearised
// exp(phi) badly underestimates the growth of the electron density where phi
// rises, and a full step overshoots; near it the limit never acts.
constexpr double NEWTON_MAX_STEP = 1.0;

__global__ void __launch_bounds__(MG_BLOCK)
k_newton_limit(const MGDesc* __restrict__ lv, int only) {
    const MGDesc& D = lv[blockIdx.y];
    if (only >= 0 && (int)blockIdx.y != only) return;
    const int idx = blockIdx.x * MG_BLOCK + threadIdx.x;
    if (idx >= D.nodes) return;
    const int i = idx % D.nx;
    if (i == 0 || i == D.n1) return;
    const double u0 = gbl(D.uold)[idx];
    const double d = gbl(D.u)[idx] - u0;
    if (d > NEWTON_MAX_STEP) gbl(D.u)[idx] = u0 + NEWTON_MAX_STEP;
    else if (d < -NEWTON_MAX_STEP) gbl(D.u)[idx] = u0 - NEWTON_MAX_STEP;
}

hipError_t newton_limit(apic_ctx* ctx, int only) {
    const int G = (int)ctx->grains.size();
    hipLaunchKernelGGL(k_newton_limit, dim3(norm_blocks(ctx), G), dim3(MG_BLOCK), 0, ctx->stream, ctx->mgdesc, only);
    return hipGetLastError();
}

// The Newton linearisation about the current phi on every level, and (invert)
// the coarsest inverses.  A solve forms them on its first Newton step only:
// later steps change E little, and an inexact coarsest operator only slows the
// cycles' convergence to the same fine-level solution.
hipError_t newton_prepare(apic_ctx* ctx, int only, bool invert) {
    const int G = (int)ctx->grains.size();
    const int nl = ctx->n_levels;
    hipLaunchKernelGGL(k_newton_prepare, dim3(norm_blocks(ctx), G), dim3(MG_BLOCK), 0, ctx->stream, ctx->gdesc,
                       ctx->mgdesc, only);
    for (int l = 0; l + 1 < nl; ++l) {
        const int cn = ctx->lvl_max_nodes[l + 1];
        hipLaunchKernelGGL(k_restrict_shift, dim3((cn + MG_BLOCK - 1) / MG_BLOCK, G), dim3(MG_BLOCK), 0,
                           ctx->stream, ctx->mgdesc + (size_t)l * G, ctx->mgdesc + (size_t)(l + 1) * G, only);
    }
    for (int l = 0; l < nl && invert; ++l) {
        const int m = ctx->lvl_max_m[l];
        if (m <= 0) continue;
        const size_t lds = sizeof(double) * (size_t)m * m;
        if (l == 0)
            hipLaunchKernelGGL(k_coarse_invert<FineStencil>, dim3(1, G), dim3(INV_BLOCK), lds, ctx->stream,
                               ctx->mgdesc, only);
        else
            hipLaunchKernelGGL(k_coarse_invert<StoredStencil>, dim3(1, G), dim3(INV_BLOCK), lds, ctx->stream,
                               ctx->mgdesc + (size_t)l * G, only);
    }
    return hipGetLastError();
}

hipError_t mg_extrapolate(apic_ctx* ctx) {
    const int G = (int)ctx->grains.size();
    hipLaunchKernelGGL(k_extrapolate, dim3(norm_blocks(ctx), G), dim3(MG_BLOCK), 0, ctx->stream, ctx->mgdesc, ctx->mgs);
    return hipGetLastError();
}

// workgroups of the finest level's tiled restriction: the most coarse tiles of any grain
static int restrict_tiles(const apic_ctx* ctx) {
    const int G = (int)ctx->grains.size();
    int tiles = 1;
    for (int g = 0; g < G; ++g) {
        const MGDesc& c = ctx->mgdesc_h[(size_t)G + g];
        if (c.n1 == 0) continue;
        tiles = std::max(tiles, ((c.n1 + RT) / RT) * ((c.n2 + RT) / RT));
    }
    return tiles;
}

// One V-cycle (sawtooth: restriction of the current residual down to the
// coarsest level, then correction and smoothing on the way up) of every grain
// not yet done, then (check) the residual norm and the convergence check.
hipError_t mg_vcycle_launches(apic_ctx* ctx, double tol, bool check) {
    const int G = (int)ctx->grains.size();
    const int nl = ctx->n_levels;
    for (int l = 0; l + 1 < nl; ++l) {
        const int cn = ctx->lvl_max_nodes[l + 1];
        if (l == 0 && ctx->opts.conservative_poisson)
            hipLaunchKernelGGL(k_restrict_residual<StoredStencil>, dim3((cn + MG_BLOCK - 1) / MG_BLOCK, G),
                               dim3(MG_BLOCK), 0, ctx->stream, ctx->mgdesc, ctx->mgdesc + (size_t)G, ctx->mgs);
        else if (l == 0)
            hipLaunchKernelGGL(k_restrict_residual_fine, dim3(restrict_tiles(ctx), G), dim3(MG_BLOCK), 0,
                               ctx->stream, ctx->mgdesc, ctx->mgdesc + (size_t)G, ctx->mgs);
        else  // level l's u was cleared by the restriction into it
            hipLaunchKernelGGL(k_restrict_rhs, dim3((cn + MG_BLOCK - 1) / MG_BLOCK, G),
                               dim3(MG_BLOCK), 0, ctx->stream, ctx->mgdesc + (size_t)l * G,
                               ctx->mgdesc + (size_t)(l + 1) * G, ctx->mgs);
    }
    coarse_solve(ctx);   // each grain's restriction chain ends at its coarsest level
    for (int l = nl - 2; l >= 0; --l) smooth(ctx, l);   // correction applied by the first sweep
    if (check) residual_check(ctx, tol, 1, false);
    return hipGetLastError();
}


}  // namespace apic
