// FP64 geometric multigrid for the curvilinear Poisson problem, eqs. (6)-(7).
//
// The paper solves the finite-difference system by LU (Section 2).  On the GPU
// the same discrete system is solved by multigrid V-cycles: Galerkin coarse
// operators (R A P, bilinear P, R = P^T / 4, built on the host), alternating
// zebra line Gauss-Seidel smoothing (x1-lines, then x2-lines; each line is a
// tridiagonal system solved in LDS by parallel cyclic reduction, one workgroup
// per line), and a dense inverse on the coarsest grid.  The operator's
// anisotropy changes direction across the domain (the x1 coefficient falls
// like r^-4), which is why both line directions are relaxed.
#include "apic_internal.h"

namespace apic {

constexpr int MG_BLOCK = 256;

// Parallel cyclic reduction on a tridiagonal system held in LDS (a: sub, b:
// diagonal, c: super, d: rhs; a[0] = c[n-1] = 0).  Each thread owns up to K
// equations.  On return d[i] / b[i] is the solution.
template <int K>
__device__ void pcr_solve(double* a, double* b, double* c, double* d, int n) {
    for (int s = 1; s < n; s <<= 1) {
        double na[K], nb[K], nc[K], nd[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = threadIdx.x + k * MG_BLOCK;
            if (i < n) {
                double ai = a[i], bi = b[i], ci = c[i], di = d[i];
                double an = 0.0, cn = 0.0;
                if (i - s >= 0) {
                    const double m = ai / b[i - s];
                    bi -= m * c[i - s];
                    di -= m * d[i - s];
                    an = -m * a[i - s];
                }
                if (i + s < n) {
                    const double m = ci / b[i + s];
                    bi -= m * a[i + s];
                    di -= m * d[i + s];
                    cn = -m * c[i + s];
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
            const int i = threadIdx.x + k * MG_BLOCK;
            if (i < n) {
                a[i] = na[k];
                b[i] = nb[k];
                c[i] = nc[k];
                d[i] = nd[k];
            }
        }
        __syncthreads();
    }
}

struct StencilPtrs {
    const double *C, *W, *E, *S, *N, *SW, *SE, *NW, *NE;
};

__host__ __device__ inline StencilPtrs stencil_ptrs(const double* st, int nodes) {
    StencilPtrs p;
    p.C = st + ST_C * (size_t)nodes;
    p.W = st + ST_W * (size_t)nodes;
    p.E = st + ST_E * (size_t)nodes;
    p.S = st + ST_S * (size_t)nodes;
    p.N = st + ST_N * (size_t)nodes;
    p.SW = st + ST_SW * (size_t)nodes;
    p.SE = st + ST_SE * (size_t)nodes;
    p.NW = st + ST_NW * (size_t)nodes;
    p.NE = st + ST_NE * (size_t)nodes;
    return p;
}

// Relaxation of the lines i2 = j (j = color, color + 2, ...): unknowns i1 = 1..n1-1.
template <int K>
__global__ void __launch_bounds__(MG_BLOCK)
k_relax_x1(int n1, int n2, int color, const double* __restrict__ st, int nodes,
           const double* __restrict__ nn, const double* __restrict__ ss, double* __restrict__ u,
           const double* __restrict__ f) {
    extern __shared__ double lds[];
    const int L = n1 - 1;
    double* a = lds;
    double* b = a + L;
    double* c = b + L;
    double* d = c + L;
    const int j = color + 2 * blockIdx.x;
    if (j > n2) return;
    const int nx = n1 + 1;
    const StencilPtrs p = stencil_ptrs(st, nodes);
    for (int k = threadIdx.x; k < L; k += MG_BLOCK) {
        const int i = k + 1;
        const size_t o = (size_t)j * nx + i;
        double rhs = f[o];
        if (j > 0) rhs -= p.S[o] * u[o - nx] + p.SW[o] * u[o - nx - 1] + p.SE[o] * u[o - nx + 1];
        if (j < n2) rhs -= p.N[o] * u[o + nx] + p.NW[o] * u[o + nx - 1] + p.NE[o] * u[o + nx + 1];
        if (nn && j == 0) rhs -= nn[i] * u[o + 2 * nx];
        if (ss && j == n2) rhs -= ss[i] * u[o - 2 * nx];
        double aa = p.W[o], cc = p.E[o];
        if (i == 1) { rhs -= aa * u[o - 1]; aa = 0.0; }
        if (i == n1 - 1) { rhs -= cc * u[o + 1]; cc = 0.0; }
        a[k] = aa;
        b[k] = p.C[o];
        c[k] = cc;
        d[k] = rhs;
    }
    __syncthreads();
    pcr_solve<K>(a, b, c, d, L);
    for (int k = threadIdx.x; k < L; k += MG_BLOCK) u[(size_t)j * nx + k + 1] = d[k] / b[k];
}

// Relaxation of the lines i1 = i (i = 1 + color, 3 + color, ...): unknowns
// i2 = 0..n2.  On the finest level the axis rows carry a second-neighbour
// coupling (one-sided d/dx2); it is eliminated with the adjacent row so the
// line stays tridiagonal.
template <int K>
__global__ void __launch_bounds__(MG_BLOCK)
k_relax_x2(int n1, int n2, int color, const double* __restrict__ st, int nodes,
           const double* __restrict__ nn, const double* __restrict__ ss, double* __restrict__ u,
           const double* __restrict__ f) {
    extern __shared__ double lds[];
    const int L = n2 + 1;
    double* a = lds;
    double* b = a + L;
    double* c = b + L;
    double* d = c + L;
    const int i = 1 + color + 2 * blockIdx.x;
    if (i > n1 - 1) return;
    const int nx = n1 + 1;
    const StencilPtrs p = stencil_ptrs(st, nodes);
    for (int j = threadIdx.x; j < L; j += MG_BLOCK) {
        const size_t o = (size_t)j * nx + i;
        double rhs = f[o] - p.W[o] * u[o - 1] - p.E[o] * u[o + 1];
        if (j > 0) rhs -= p.SW[o] * u[o - nx - 1] + p.SE[o] * u[o - nx + 1];
        if (j < n2) rhs -= p.NW[o] * u[o + nx - 1] + p.NE[o] * u[o + nx + 1];
        a[j] = j > 0 ? p.S[o] : 0.0;
        b[j] = p.C[o];
        c[j] = j < n2 ? p.N[o] : 0.0;
        d[j] = rhs;
    }
    __syncthreads();
    if (nn && threadIdx.x == 0) {
        const double m = nn[i] / c[1];
        b[0] -= m * a[1];
        c[0] -= m * b[1];
        d[0] -= m * d[1];
    }
    if (ss && threadIdx.x == 1) {
        const double m = ss[i] / a[n2 - 1];
        a[n2] -= m * b[n2 - 1];
        b[n2] -= m * c[n2 - 1];
        d[n2] -= m * d[n2 - 1];
    }
    __syncthreads();
    pcr_solve<K>(a, b, c, d, L);
    for (int j = threadIdx.x; j < L; j += MG_BLOCK) u[(size_t)j * nx + i] = d[j] / b[j];
}

// r = f - A u on the unknown nodes, 0 on the Dirichlet columns; optionally
// accumulates |D^-1 r|^2 (D = diagonal of A): the operator's rows differ in
// scale by ~r^4, and the row-scaled norm weighs every node alike.
__global__ void __launch_bounds__(MG_BLOCK)
k_residual(int n1, int n2, const double* __restrict__ st, int nodes, const double* __restrict__ nn,
           const double* __restrict__ ss, const double* __restrict__ u,
           const double* __restrict__ f, double* __restrict__ r, double* norm2) {
    __shared__ double red[MG_BLOCK / 64];
    const int nx = n1 + 1;
    const int idx = blockIdx.x * MG_BLOCK + threadIdx.x;
    double rr = 0.0;
    if (idx < nodes) {
        const int j = idx / nx, i = idx - j * nx;
        double v = 0.0;
        if (i > 0 && i < n1) {
            const StencilPtrs p = stencil_ptrs(st, nodes);
            const size_t o = idx;
            double au = p.C[o] * u[o] + p.W[o] * u[o - 1] + p.E[o] * u[o + 1];
            if (j > 0) au += p.S[o] * u[o - nx] + p.SW[o] * u[o - nx - 1] + p.SE[o] * u[o - nx + 1];
            if (j < n2) au += p.N[o] * u[o + nx] + p.NW[o] * u[o + nx - 1] + p.NE[o] * u[o + nx + 1];
            if (nn && j == 0) au += nn[i] * u[o + 2 * nx];
            if (ss && j == n2) au += ss[i] * u[o - 2 * nx];
            v = f[o] - au;
        }
        if (r) r[idx] = v;
        if (i > 0 && i < n1) {
            const double q = v / st[ST_C * (size_t)nodes + idx];
            rr = q * q;
        }
    }
    if (norm2) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) rr += __shfl_xor(rr, o);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rr;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < MG_BLOCK / 64; ++w) t += red[w];
            atomicAdd(norm2, t);
        }
    }
}

// |D^-1 f|^2 over the unknown nodes
__global__ void __launch_bounds__(MG_BLOCK)
k_rhs_norm(int n1, int nodes, const double* __restrict__ diag, const double* __restrict__ f,
           double* norm2) {
    __shared__ double red[MG_BLOCK / 64];
    const int nx = n1 + 1;
    const int idx = blockIdx.x * MG_BLOCK + threadIdx.x;
    double v = 0.0;
    if (idx < nodes) {
        const int i = idx % nx;
        if (i > 0 && i < n1) {
            const double q = f[idx] / diag[idx];
            v = q * q;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < MG_BLOCK / 64; ++w) t += red[w];
        atomicAdd(norm2, t);
    }
}

// coarse f = P^T r / 4 on the coarse unknowns (full weighting without the
// rows outside the grid), 0 on the coarse Dirichlet columns
__global__ void __launch_bounds__(MG_BLOCK)
k_restrict(int n1f, int n2f, int n1c, int n2c, const double* __restrict__ rf,
           double* __restrict__ fc) {
    const int nxc = n1c + 1, nxf = n1f + 1;
    const int idx = blockIdx.x * MG_BLOCK + threadIdx.x;
    if (idx >= nxc * (n2c + 1)) return;
    const int J = idx / nxc, I = idx - J * nxc;
    if (I == 0 || I == n1c) { fc[idx] = 0.0; return; }
    double acc = 0.0;
    for (int dj = -1; dj <= 1; ++dj) {
        const int j = 2 * J + dj;
        if (j < 0 || j > n2f) continue;
        const double wj = dj == 0 ? 1.0 : 0.5;
        const double* row = rf + (size_t)j * nxf + 2 * I;
        acc += wj * (0.5 * row[-1] + row[0] + 0.5 * row[1]);
    }
    fc[idx] = 0.25 * acc;
}

// fine u += P uc (bilinear) on the fine unknowns
__global__ void __launch_bounds__(MG_BLOCK)
k_prolong_add(int n1f, int n2f, int n1c, const double* __restrict__ uc, double* __restrict__ uf) {
    const int nxc = n1c + 1, nxf = n1f + 1;
    const int idx = blockIdx.x * MG_BLOCK + threadIdx.x;
    if (idx >= nxf * (n2f + 1)) return;
    const int j = idx / nxf, i = idx - j * nxf;
    if (i == 0 || i == n1f) return;
    const int J0 = j >> 1, I0 = i >> 1;
    const int J1 = (j & 1) ? J0 + 1 : J0;
    const int I1 = (i & 1) ? I0 + 1 : I0;
    const double v = 0.25 * (uc[(size_t)J0 * nxc + I0] + uc[(size_t)J0 * nxc + I1] +
                             uc[(size_t)J1 * nxc + I0] + uc[(size_t)J1 * nxc + I1]);
    uf[idx] += v;
}

// coarsest grid: u = A^-1 f (dense inverse with identity Dirichlet rows)
__global__ void __launch_bounds__(MG_BLOCK)
k_coarse_solve(int m, const double* __restrict__ inv, const double* __restrict__ f,
               double* __restrict__ u) {
    const int row = blockIdx.x * MG_BLOCK + threadIdx.x;
    if (row >= m) return;
    const double* a = inv + (size_t)row * m;
    double acc = 0.0;
    for (int k = 0; k < m; ++k) acc += a[k] * f[k];
    u[row] = acc;
}

template <int K>
static void relax_level(apic_ctx* ctx, Grain& g, int l) {
    MGLevel& L = g.mg[l];
    const double* nn = l == 0 ? g.axis_nn : nullptr;
    const double* ss = l == 0 ? g.axis_ss : nullptr;
    const size_t lds1 = 4 * sizeof(double) * (size_t)(L.n1 - 1);
    const size_t lds2 = 4 * sizeof(double) * (size_t)(L.n2 + 1);
    for (int color = 0; color < 2; ++color) {
        const int lines = (L.n2 + 1 - color + 1) / 2;
        hipLaunchKernelGGL(k_relax_x1<K>, dim3(lines), dim3(MG_BLOCK), lds1, ctx->stream, L.n1,
                           L.n2, color, L.st, L.nodes, nn, ss, L.u, L.f);
    }
    for (int color = 0; color < 2; ++color) {
        const int lines = (L.n1 - 1 - color + 1) / 2;
        if (lines <= 0) continue;
        hipLaunchKernelGGL(k_relax_x2<K>, dim3(lines), dim3(MG_BLOCK), lds2, ctx->stream, L.n1,
                           L.n2, color, L.st, L.nodes, nn, ss, L.u, L.f);
    }
}

static void relax(apic_ctx* ctx, Grain& g, int l) {
    const MGLevel& L = g.mg[l];
    const int longest = std::max(L.n1 - 1, L.n2 + 1);
    const int K = (longest + MG_BLOCK - 1) / MG_BLOCK;
    if (K <= 1) relax_level<1>(ctx, g, l);
    else if (K <= 2) relax_level<2>(ctx, g, l);
    else if (K <= 4) relax_level<4>(ctx, g, l);
    else relax_level<8>(ctx, g, l);
}

hipError_t mg_vcycle(apic_ctx* ctx, Grain& g) {
    const int nl = (int)g.mg.size();
    for (int l = 0; l + 1 < nl; ++l) {
        MGLevel& F = g.mg[l];
        MGLevel& C = g.mg[l + 1];
        relax(ctx, g, l);
        hipLaunchKernelGGL(k_residual, dim3((F.nodes + MG_BLOCK - 1) / MG_BLOCK), dim3(MG_BLOCK), 0,
                           ctx->stream, F.n1, F.n2, F.st, F.nodes, l == 0 ? g.axis_nn : nullptr,
                           l == 0 ? g.axis_ss : nullptr, F.u, F.f, F.r, nullptr);
        hipLaunchKernelGGL(k_restrict, dim3((C.nodes + MG_BLOCK - 1) / MG_BLOCK), dim3(MG_BLOCK), 0,
                           ctx->stream, F.n1, F.n2, C.n1, C.n2, F.r, C.f);
        hipError_t e = launch_fill(ctx, C.u, sizeof(double) * (size_t)C.nodes);
        if (e != hipSuccess) return e;
    }
    MGLevel& B = g.mg[nl - 1];
    hipLaunchKernelGGL(k_coarse_solve, dim3((B.nodes + MG_BLOCK - 1) / MG_BLOCK), dim3(MG_BLOCK), 0,
                       ctx->stream, B.nodes, g.coarse_inv, B.f, B.u);
    for (int l = nl - 2; l >= 0; --l) {
        MGLevel& F = g.mg[l];
        MGLevel& C = g.mg[l + 1];
        hipLaunchKernelGGL(k_prolong_add, dim3((F.nodes + MG_BLOCK - 1) / MG_BLOCK), dim3(MG_BLOCK),
                           0, ctx->stream, F.n1, F.n2, C.n1, C.u, F.u);
        relax(ctx, g, l);
    }
    return hipGetLastError();
}

hipError_t mg_residual_norm(apic_ctx* ctx, Grain& g, double* norm2_dev) {
    MGLevel& F = g.mg[0];
    hipError_t e = launch_fill(ctx, norm2_dev, sizeof(double));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_residual, dim3((F.nodes + MG_BLOCK - 1) / MG_BLOCK), dim3(MG_BLOCK), 0,
                       ctx->stream, F.n1, F.n2, F.st, F.nodes, g.axis_nn, g.axis_ss, F.u, F.f,
                       nullptr, norm2_dev);
    return hipGetLastError();
}

hipError_t mg_rhs_norm(apic_ctx* ctx, Grain& g, double* norm2_dev) {
    MGLevel& F = g.mg[0];
    hipError_t e = launch_fill(ctx, norm2_dev, sizeof(double));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rhs_norm, dim3((F.nodes + MG_BLOCK - 1) / MG_BLOCK), dim3(MG_BLOCK), 0,
                       ctx->stream, F.n1, F.nodes, F.st + ST_C * (size_t)F.nodes, F.f, norm2_dev);
    return hipGetLastError();
}

}  // namespace apic
