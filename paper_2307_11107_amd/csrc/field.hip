// Grid kernels beside the particle loop: charge density from the deposits
// (weighting with the node volumes of eq. 5), the right-hand side of eq. (6),
// the nodal derivatives of phi (second-order differences, used by eq. 10), and
// the electric force on the grain from the surface field (Section 2: the field
// on the conducting surface gives the surface charge and the electric force).
#include "apic_internal.h"
#include "device_common.h"

namespace apic {

__global__ void k_fill_u32(uint32_t* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_fill(apic_ctx* ctx, void* p, size_t bytes) {
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    size_t grid = (n + 255) / 256;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)grid), dim3(256), 0, ctx->stream,
                       static_cast<uint32_t*>(p), n);
    return hipGetLastError();
}

// rho = sum_s q_s w_s dep_s / V_node  (units e n0)
template <typename D>
__global__ void k_rho(int nodes, int ns, const D* __restrict__ dep0, const D* __restrict__ dep1,
                      double c0, double c1, const double* __restrict__ vol, double* __restrict__ rho) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nodes) return;
    double q = c0 * (double)dep0[i];
    if (ns > 1) q += c1 * (double)dep1[i];
    rho[i] = q / vol[i];
}

hipError_t launch_rho(apic_ctx* ctx, Grain& g) {
    const int grid = (g.nodes + 255) / 256;
    const double c0 = g.sp[0].q * g.sp[0].w;
    const double c1 = g.ns > 1 ? g.sp[1].q * g.sp[1].w : 0.0;
    if (ctx->opts.precision == APIC_FP32_SPLIT)
        hipLaunchKernelGGL(k_rho<float>, dim3(grid), dim3(256), 0, ctx->stream, g.nodes, g.ns,
                           static_cast<const float*>(g.dep[0]),
                           static_cast<const float*>(g.dep[g.ns > 1 ? 1 : 0]), c0, c1, g.vol, g.rho);
    else
        hipLaunchKernelGGL(k_rho<double>, dim3(grid), dim3(256), 0, ctx->stream, g.nodes, g.ns,
                           static_cast<const double*>(g.dep[0]),
                           static_cast<const double*>(g.dep[g.ns > 1 ? 1 : 0]), c0, c1, g.vol,
                           g.rho);
    return hipGetLastError();
}

// f = -(1/kappa^2) rho at the unknown nodes (eq. 6 normalised); 0 on Dirichlet columns
__global__ void k_rhs(int n1, int nx, int nodes, double scale, const double* __restrict__ rho,
                      double* __restrict__ f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nodes) return;
    const int i1 = i % nx;
    f[i] = (i1 == 0 || i1 == n1) ? 0.0 : scale * rho[i];
}

hipError_t launch_rhs_from_rho(apic_ctx* ctx, Grain& g) {
    const int grid = (g.nodes + 255) / 256;
    hipLaunchKernelGGL(k_rhs, dim3(grid), dim3(256), 0, ctx->stream, g.gp.n1, g.gp.nx, g.nodes,
                       -1.0 / (g.gp.kappa * g.gp.kappa), g.rho, g.mg[0].f);
    return hipGetLastError();
}

// Dirichlet values: phi = phi_grain on x1 = -1, phi_out on x1 = x1_out
__global__ void k_set_boundary(int n1, int nx, int n2, double pg, double po, double* __restrict__ u) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > n2) return;
    u[j * nx] = pg;
    u[j * nx + n1] = po;
}

hipError_t launch_set_boundary(apic_ctx* ctx, Grain& g) {
    hipLaunchKernelGGL(k_set_boundary, dim3((g.gp.n2 + 256) / 256), dim3(256), 0, ctx->stream,
                       g.gp.n1, g.gp.nx, g.gp.n2, g.cfg.phi_grain, g.cfg.phi_out, g.mg[0].u);
    return hipGetLastError();
}

// Initial guess for the next solve: u <- 2 u - prev, prev <- old u (linear
// extrapolation in time from the two previous potentials).
__global__ void k_extrapolate(int nodes, double* __restrict__ u, double* __restrict__ prev) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nodes) return;
    const double now = u[i];
    u[i] = 2.0 * now - prev[i];
    prev[i] = now;
}

hipError_t launch_extrapolate(apic_ctx* ctx, Grain& g) {
    hipLaunchKernelGGL(k_extrapolate, dim3((g.nodes + 255) / 256), dim3(256), 0, ctx->stream, g.nodes,
                       g.mg[0].u, g.phi_prev);
    return hipGetLastError();
}

__global__ void k_copy(int n, double* __restrict__ dst, const double* __restrict__ src) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

hipError_t launch_copy(apic_ctx* ctx, double* dst, const double* src, int n) {
    hipLaunchKernelGGL(k_copy, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, n, dst, src);
    return hipGetLastError();
}

// Nodal (dphi/dx1, dphi/dx2): central inside, second-order one-sided on the edges.
template <typename V>
__global__ void k_gradient(int n1, int n2, double ih1, double ih2, const double* __restrict__ phi,
                           V* __restrict__ grad) {
    const int i1 = blockIdx.x * blockDim.x + threadIdx.x;
    const int i2 = blockIdx.y;
    if (i1 > n1) return;
    const int nx = n1 + 1;
    const double* row = phi + (size_t)i2 * nx;
    double d1, d2;
    if (i1 == 0) d1 = (-3.0 * row[0] + 4.0 * row[1] - row[2]) * 0.5 * ih1;
    else if (i1 == n1) d1 = (3.0 * row[n1] - 4.0 * row[n1 - 1] + row[n1 - 2]) * 0.5 * ih1;
    else d1 = (row[i1 + 1] - row[i1 - 1]) * 0.5 * ih1;
    if (i2 == 0) d2 = (-3.0 * row[i1] + 4.0 * row[i1 + nx] - row[i1 + 2 * nx]) * 0.5 * ih2;
    else if (i2 == n2) d2 = (3.0 * row[i1] - 4.0 * row[i1 - nx] + row[i1 - 2 * nx]) * 0.5 * ih2;
    else d2 = (row[i1 + nx] - row[i1 - nx]) * 0.5 * ih2;
    V v;
    v.x = d1;
    v.y = d2;
    grad[(size_t)i2 * nx + i1] = v;
}

hipError_t launch_gradient(apic_ctx* ctx, Grain& g) {
    dim3 grid((g.gp.n1 + 256) / 256, g.gp.n2 + 1);
    if (ctx->opts.precision == APIC_FP32_SPLIT)
        hipLaunchKernelGGL(k_gradient<float2>, grid, dim3(256), 0, ctx->stream, g.gp.n1, g.gp.n2,
                           g.gp.inv_h1, g.gp.inv_h2, g.mg[0].u, static_cast<float2*>(g.grad));
    else
        hipLaunchKernelGGL(k_gradient<double2>, grid, dim3(256), 0, ctx->stream, g.gp.n1, g.gp.n2,
                           g.gp.inv_h1, g.gp.inv_h2, g.mg[0].u, static_cast<double2*>(g.grad));
    return hipGetLastError();
}

// Electric force on the grain, F_Z = integral over x1 = -1 of E_n^2 / 2 * n_Z dA
// (Maxwell stress on a conductor), E_n = -|grad x1| dphi/dx1, trapezoid in x2.
__global__ void k_grain_force(int n1, int n2, double alpha, double h2, double ih1,
                              const double* __restrict__ phi, double* __restrict__ acc) {
    __shared__ double red[256];
    const int nx = n1 + 1;
    double sum = 0.0;
    for (int j = threadIdx.x; j <= n2; j += blockDim.x) {
        const double x2 = -1.0 + j * h2;
        const double r = r_of(-1.0, x2, alpha);
        const double s = sqrt(fmax(1.0 - x2 * x2, 0.0));
        const Metric<double> m = metric_at(r, x2, s, alpha);
        const double gn = sqrt(m.x1R * m.x1R + m.x1Z * m.x1Z);
        const double* row = phi + (size_t)j * nx;
        const double p1 = (-3.0 * row[0] + 4.0 * row[1] - row[2]) * 0.5 * ih1;
        const double En = -gn * p1;
        const double t = alpha / (r + 2.0 * alpha * x2);
        const double dA = 6.283185307179586 * r * r * sqrt(1.0 + (1.0 - x2 * x2) * t * t);
        const double w = (j == 0 || j == n2) ? 0.5 : 1.0;
        sum += w * 0.5 * En * En * (m.x1Z / gn) * dA;
    }
    red[threadIdx.x] = sum;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *acc += red[0] * h2;
}

hipError_t launch_grain_force(apic_ctx* ctx, Grain& g) {
    hipLaunchKernelGGL(k_grain_force, dim3(1), dim3(256), 0, ctx->stream, g.gp.n1, g.gp.n2,
                       g.gp.alpha, g.gp.h2, g.gp.inv_h1, g.mg[0].u, &g.ctr->F_el_sum);
    return hipGetLastError();
}

}  // namespace apic
