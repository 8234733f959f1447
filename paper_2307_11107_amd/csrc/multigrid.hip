// FP64 geometric multigrid for the curvilinear Poisson problem, eqs. (6)-(7).
//
// The paper solves the finite-difference system by LU (Section 2).  On the GPU
// the same discrete system is solved by multigrid V-cycles: Galerkin coarse
// operators (R A P, bilinear P, R = P^T / 4, built on the host), alternating
// zebra line Gauss-Seidel smoothing (x1-lines, then x2-lines; each line is a
// tridiagonal system solved in LDS by parallel cyclic reduction), and a dense
// inverse on the coarsest grid (at most a few hundred nodes).  The operator's
// anisotropy changes direction across the domain (the x1 coefficient falls like
// r^-4), which is why both line directions are relaxed.  One V-cycle is
// captured once into a HIP graph and replayed.
#include "apic_internal.h"

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
// to K equations.  On return d[e] / b[e] is the solution.
template <int K, int NT>
__device__ void pcr_solve(double* a, double* b, double* c, double* d, int L, int total) {
    int jj[K];
#pragma unroll
    for (int k = 0; k < K; ++k) jj[k] = (threadIdx.x + k * NT) % L;
    for (int s = 1; s < L; s <<= 1) {
        double na[K], nb[K], nc[K], nd[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e = threadIdx.x + k * NT;
            if (e < total) {
                const int j = jj[k];
                double ai = a[e], bi = b[e], ci = c[e], di = d[e];
                double an = 0.0, cn = 0.0;
                if (j - s >= 0) {
                    const double m = ai * rcp64(b[e - s]);
                    bi -= m * c[e - s];
                    di -= m * d[e - s];
                    an = -m * a[e - s];
                }
                if (j + s < L) {
                    const double m = ci * rcp64(b[e + s]);
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
                b[e] = nb[k];
                c[e] = nc[k];
                d[e] = nd[k];
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

// (A u) at an unknown node (j, i) of a level; nn / ss carry the finest level's
// second-neighbour axis couplings (null on coarse levels).
__device__ inline double apply_A(const StencilPtrs& p, const double* __restrict__ nn,
                                 const double* __restrict__ ss, const double* __restrict__ u, int n2,
                                 int nx, int j, int i) {
    const size_t o = (size_t)j * nx + i;
    double au = p.C[o] * u[o] + p.W[o] * u[o - 1] + p.E[o] * u[o + 1];
    if (j > 0) au += p.S[o] * u[o - nx] + p.SW[o] * u[o - nx - 1] + p.SE[o] * u[o - nx + 1];
    if (j < n2) au += p.N[o] * u[o + nx] + p.NW[o] * u[o + nx - 1] + p.NE[o] * u[o + nx + 1];
    if (nn && j == 0) au += nn[i] * u[o + 2 * nx];
    if (ss && j == n2) au += ss[i] * u[o - 2 * nx];
    return au;
}

// Relaxation of the lines i2 = j (j = color, color + 2, ...): unknowns i1 = 1..n1-1.
template <int K, int NT>
__global__ void __launch_bounds__(NT)
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
    for (int k = threadIdx.x; k < L; k += NT) {
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
    pcr_solve<K, NT>(a, b, c, d, L, L);
    for (int k = threadIdx.x; k < L; k += NT) u[(size_t)j * nx + k + 1] = d[k] * rcp64(b[k]);
}

// Relaxation of LPB lines i1 = i (i = 1 + color, 3 + color, ...) per workgroup:
// unknowns i2 = 0..n2.  Neighbouring lines of one colour are read together so
// that the row-wise loads stay within a cache line.  On the finest level the
// axis rows carry a second-neighbour coupling (one-sided d/dx2); it is
// eliminated with the adjacent row so each line stays tridiagonal.
template <int K, int LPB, int NT>
__global__ void __launch_bounds__(NT)
k_relax_x2(int n1, int n2, int color, const double* __restrict__ st, int nodes,
           const double* __restrict__ nn, const double* __restrict__ ss, double* __restrict__ u,
           const double* __restrict__ f) {
    extern __shared__ double lds[];
    const int L = n2 + 1;
    const int total = LPB * L;
    double* a = lds;
    double* b = a + total;
    double* c = b + total;
    double* d = c + total;
    const int i0 = 1 + color + 2 * LPB * blockIdx.x;
    if (i0 > n1 - 1) return;
    const int nx = n1 + 1;
    const StencilPtrs p = stencil_ptrs(st, nodes);
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
        double rhs = f[o] - p.W[o] * u[o - 1] - p.E[o] * u[o + 1];
        if (j > 0) rhs -= p.SW[o] * u[o - nx - 1] + p.SE[o] * u[o - nx + 1];
        if (j < n2) rhs -= p.NW[o] * u[o + nx - 1] + p.NE[o] * u[o + nx + 1];
        a[e] = j > 0 ? p.S[o] : 0.0;
        b[e] = p.C[o];
        c[e] = j < n2 ? p.N[o] : 0.0;
        d[e] = rhs;
    }
    __syncthreads();
    if (threadIdx.x < LPB && nn) {
        const int m = threadIdx.x, i = i0 + 2 * m;
        if (i <= n1 - 1) {
            const int e = m * L;
            const double mm = nn[i] / c[e + 1];
            b[e] -= mm * a[e + 1];
            c[e] -= mm * b[e + 1];
            d[e] -= mm * d[e + 1];
        }
    }
    if (threadIdx.x >= 64 && threadIdx.x < 64 + LPB && ss) {
        const int m = threadIdx.x - 64, i = i0 + 2 * m;
        if (i <= n1 - 1) {
            const int e = m * L + n2;
            const double mm = ss[i] / a[e - 1];
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
        u[(size_t)j * nx + i] = d[e] * rcp64(b[e]);
    }
}

// Block sum of a per-thread value, one atomic per block.
__device__ inline void block_sum_add(double v, double* dst) {
    __shared__ double red[MG_BLOCK / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < MG_BLOCK / 64; ++w) t += red[w];
        atomicAdd(dst, t);
    }
}

// |D^-1 (f - A u)|^2 over the unknown nodes of the finest level (D = diagonal
// of A): the operator's rows differ in scale by ~r^4, and the row-scaled norm
// weighs every node alike.
__global__ void __launch_bounds__(MG_BLOCK)
k_residual_norm(int n1, int n2, const double* __restrict__ st, int nodes,
                const double* __restrict__ nn, const double* __restrict__ ss,
                const double* __restrict__ u, const double* __restrict__ f, double* norm2) {
    const int nx = n1 + 1;
    const int idx = blockIdx.x * MG_BLOCK + threadIdx.x;
    double rr = 0.0;
    if (idx < nodes) {
        const int j = idx / nx, i = idx - j * nx;
        if (i > 0 && i < n1) {
            const StencilPtrs p = stencil_ptrs(st, nodes);
            const double q = (f[idx] - apply_A(p, nn, ss, u, n2, nx, j, i)) / p.C[idx];
            rr = q * q;
        }
    }
    block_sum_add(rr, norm2);
}

// |D^-1 f|^2 over the unknown nodes
__global__ void __launch_bounds__(MG_BLOCK)
k_rhs_norm(int n1, int nodes, const double* __restrict__ diag, const double* __restrict__ f,
           double* norm2) {
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
    block_sum_add(v, norm2);
}

// Coarse right-hand side fc = P^T (f - A u) / 4 on the coarse unknowns, the
// fine residuals formed on the fly (full weighting without rows outside the
// grid); fc = 0 on the coarse Dirichlet columns; the coarse correction uc is
// cleared.
__global__ void __launch_bounds__(MG_BLOCK)
k_restrict_residual(int n1f, int n2f, const double* __restrict__ st, int nodes_f,
                    const double* __restrict__ nn, const double* __restrict__ ss,
                    const double* __restrict__ u, const double* __restrict__ f, int n1c, int n2c,
                    double* __restrict__ fc, double* __restrict__ uc) {
    const int nxc = n1c + 1, nxf = n1f + 1;
    const int idx = blockIdx.x * MG_BLOCK + threadIdx.x;
    if (idx >= nxc * (n2c + 1)) return;
    uc[idx] = 0.0;
    const int J = idx / nxc, I = idx - J * nxc;
    if (I == 0 || I == n1c) {
        fc[idx] = 0.0;
        return;
    }
    const StencilPtrs p = stencil_ptrs(st, nodes_f);
    double acc = 0.0;
    for (int dj = -1; dj <= 1; ++dj) {
        const int j = 2 * J + dj;
        if (j < 0 || j > n2f) continue;
        const double wj = dj == 0 ? 1.0 : 0.5;
        for (int di = -1; di <= 1; ++di) {
            const int i = 2 * I + di;      // 1 <= i <= n1f - 1
            const double wi = di == 0 ? 1.0 : 0.5;
            const double r = f[(size_t)j * nxf + i] - apply_A(p, nn, ss, u, n2f, nxf, j, i);
            acc += wj * wi * r;
        }
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

// coarsest grid: u = A^-1 f (dense inverse with identity Dirichlet rows), one
// wave per row
__global__ void __launch_bounds__(MG_BLOCK)
k_coarse_solve(int m, const double* __restrict__ inv, const double* __restrict__ f,
               double* __restrict__ u) {
    const int row = blockIdx.x * (MG_BLOCK / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= m) return;
    const double* a = inv + (size_t)row * m;
    double acc = 0.0;
    for (int k = lane; k < m; k += 64) acc += a[k] * f[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) u[row] = acc;
}

// Line-solve launches.  A line of L unknowns gets NT = 512 threads when it is
// long (fewer equations per thread, shorter PCR critical path), else 256; the
// x2 sweeps group LPB neighbouring lines of one colour per workgroup while
// that still leaves at least two workgroups per compute unit.
template <int K, int NT>
static void relax_x1_launch(apic_ctx* ctx, const MGLevel& L, const double* nn, const double* ss, int color) {
    const size_t lds = 4 * sizeof(double) * (size_t)(L.n1 - 1);
    const int lines = (L.n2 + 1 - color + 1) / 2;
    hipLaunchKernelGGL((k_relax_x1<K, NT>), dim3(lines), dim3(NT), lds, ctx->stream, L.n1, L.n2,
                       color, L.st, L.nodes, nn, ss, L.u, L.f);
}

template <int K, int LPB, int NT>
static void relax_x2_launch(apic_ctx* ctx, const MGLevel& L, const double* nn, const double* ss, int color) {
    const size_t lds = 4 * sizeof(double) * (size_t)LPB * (L.n2 + 1);
    const int lines = (L.n1 - 1 - color + 1) / 2;
    if (lines <= 0) return;
    const int blocks = (lines + LPB - 1) / LPB;
    hipLaunchKernelGGL((k_relax_x2<K, LPB, NT>), dim3(blocks), dim3(NT), lds, ctx->stream, L.n1,
                       L.n2, color, L.st, L.nodes, nn, ss, L.u, L.f);
}

static int pcr_k(int total, int nt) {
    const int k = (total + nt - 1) / nt;
    return k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : 8;
}

template <int NT>
static void relax_x1_k(apic_ctx* ctx, const MGLevel& L, const double* nn, const double* ss, int color) {
    switch (pcr_k(L.n1 - 1, NT)) {
        case 1: relax_x1_launch<1, NT>(ctx, L, nn, ss, color); break;
        case 2: relax_x1_launch<2, NT>(ctx, L, nn, ss, color); break;
        case 4: relax_x1_launch<4, NT>(ctx, L, nn, ss, color); break;
        default: relax_x1_launch<8, NT>(ctx, L, nn, ss, color); break;
    }
}

template <int LPB, int NT>
static void relax_x2_k(apic_ctx* ctx, const MGLevel& L, const double* nn, const double* ss, int color) {
    switch (pcr_k(LPB * (L.n2 + 1), NT)) {
        case 1: relax_x2_launch<1, LPB, NT>(ctx, L, nn, ss, color); break;
        case 2: relax_x2_launch<2, LPB, NT>(ctx, L, nn, ss, color); break;
        case 4: relax_x2_launch<4, LPB, NT>(ctx, L, nn, ss, color); break;
        default: relax_x2_launch<8, LPB, NT>(ctx, L, nn, ss, color); break;
    }
}

static void relax(apic_ctx* ctx, Grain& g, int l) {
    const MGLevel& L = g.mg[l];
    const double* nn = l == 0 ? g.axis_nn : nullptr;
    const double* ss = l == 0 ? g.axis_ss : nullptr;
    for (int color = 0; color < 2; ++color) {
        if (L.n1 - 1 > 512) relax_x1_k<512>(ctx, L, nn, ss, color);
        else relax_x1_k<256>(ctx, L, nn, ss, color);
    }
    const int Lx2 = L.n2 + 1;
    const int lines = (L.n1 - 1 + 1) / 2;
    int lpb = 4;
    while (lpb > 1 && (4 * sizeof(double) * (size_t)lpb * Lx2 > 65536 || lpb * Lx2 > 8 * 256 ||
                       (lines + lpb - 1) / lpb < 2 * ctx->num_cus))
        lpb >>= 1;
    for (int color = 0; color < 2; ++color) {
        if (lpb == 4) relax_x2_k<4, 256>(ctx, L, nn, ss, color);
        else if (lpb == 2) relax_x2_k<2, 256>(ctx, L, nn, ss, color);
        else if (Lx2 > 512) relax_x2_k<1, 512>(ctx, L, nn, ss, color);
        else relax_x2_k<1, 256>(ctx, L, nn, ss, color);
    }
}

static void vcycle_launches(apic_ctx* ctx, Grain& g) {
    const int nl = (int)g.mg.size();
    for (int l = 0; l + 1 < nl; ++l) {
        MGLevel& F = g.mg[l];
        MGLevel& C = g.mg[l + 1];
        relax(ctx, g, l);
        hipLaunchKernelGGL(k_restrict_residual, dim3((C.nodes + MG_BLOCK - 1) / MG_BLOCK),
                           dim3(MG_BLOCK), 0, ctx->stream, F.n1, F.n2, F.st, F.nodes,
                           l == 0 ? g.axis_nn : nullptr, l == 0 ? g.axis_ss : nullptr, F.u, F.f,
                           C.n1, C.n2, C.f, C.u);
    }
    MGLevel& B = g.mg[nl - 1];
    hipLaunchKernelGGL(k_coarse_solve, dim3((B.nodes + MG_BLOCK / 64 - 1) / (MG_BLOCK / 64)),
                       dim3(MG_BLOCK), 0, ctx->stream, B.nodes, g.coarse_inv, B.f, B.u);
    for (int l = nl - 2; l >= 0; --l) {
        MGLevel& F = g.mg[l];
        MGLevel& C = g.mg[l + 1];
        hipLaunchKernelGGL(k_prolong_add, dim3((F.nodes + MG_BLOCK - 1) / MG_BLOCK), dim3(MG_BLOCK),
                           0, ctx->stream, F.n1, F.n2, C.n1, C.u, F.u);
        relax(ctx, g, l);
    }
    // row-scaled residual norm of the result
    MGLevel& F = g.mg[0];
    (void)launch_fill(ctx, &g.ctr->norm2, sizeof(double));
    hipLaunchKernelGGL(k_residual_norm, dim3((F.nodes + MG_BLOCK - 1) / MG_BLOCK), dim3(MG_BLOCK), 0,
                       ctx->stream, F.n1, F.n2, F.st, F.nodes, g.axis_nn, g.axis_ss, F.u, F.f,
                       &g.ctr->norm2);
}

// One V-cycle followed by the residual norm into ctr->norm2.  The launch
// sequence is captured once into a graph (when the stream can be captured)
// and replayed afterwards.
hipError_t mg_vcycle(apic_ctx* ctx, Grain& g) {
    if (!g.vcycle_exec && ctx->graphs) {
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            vcycle_launches(ctx, g);
            e = hipStreamEndCapture(ctx->stream, &graph);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&g.vcycle_exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            g.vcycle_exec = nullptr;
            ctx->graphs = false;
        }
    }
    if (g.vcycle_exec) return hipGraphLaunch(g.vcycle_exec, ctx->stream);
    vcycle_launches(ctx, g);
    return hipGetLastError();
}

hipError_t mg_residual_norm(apic_ctx* ctx, Grain& g, double* norm2_dev) {
    MGLevel& F = g.mg[0];
    hipError_t e = launch_fill(ctx, norm2_dev, sizeof(double));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_residual_norm, dim3((F.nodes + MG_BLOCK - 1) / MG_BLOCK), dim3(MG_BLOCK), 0,
                       ctx->stream, F.n1, F.n2, F.st, F.nodes, g.axis_nn, g.axis_ss, F.u, F.f,
                       norm2_dev);
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
