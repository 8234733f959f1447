// Grid kernels beside the particle loop, run for every grain of the ensemble at
// once (blockIdx.y = grain): charge density from the deposits (weighting with
// the node volumes of eq. 5), the right-hand side of eq. (6), the Dirichlet
// values, the nodal derivatives of phi (second-order differences, used by
// eq. 10), and the electric force on the grain from the surface field
// (Section 2: the field on the conducting surface gives the surface charge and
// the electric force).
#include "apic_internal.h"
#include "device_common.h"

namespace apic {

constexpr int FB = 256;

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

static dim3 node_grid(apic_ctx* ctx) {
    return dim3((ctx->max_nodes + FB - 1) / FB, (unsigned)ctx->grains.size());
}

// deposit sums of every species to zero
__global__ void __launch_bounds__(FB)
k_clear_deposits(const GrainDesc* __restrict__ gd, int word_bytes) {
    const GrainDesc& G = gd[blockIdx.y];
    const int i = blockIdx.x * FB + threadIdx.x;
    if (i >= G.nodes) return;
    for (int s = 0; s < G.ns; ++s) {
        if (word_bytes == 4) gbl(static_cast<float*>(const_cast<void*>(G.dep[s])))[i] = 0.f;
        else gbl(static_cast<double*>(const_cast<void*>(G.dep[s])))[i] = 0.0;
    }
}

hipError_t launch_clear_deposits(apic_ctx* ctx) {
    hipLaunchKernelGGL(k_clear_deposits, node_grid(ctx), dim3(FB), 0, ctx->stream, ctx->gdesc,
                       ctx->opts.precision == APIC_FP32_SPLIT ? 4 : 8);
    return hipGetLastError();
}

// rho = sum_s q_s w_s dep_s / V_node (units e n0); f = -(1/kappa^2) rho at the
// unknown nodes (eq. 6 normalised), 0 on the Dirichlet columns; in the
// conservative form f = -(1/kappa^2) times the node's charge (rho V_node)
template <typename D>
__global__ void __launch_bounds__(FB)
k_rho_rhs(const GrainDesc* __restrict__ gd) {
    const GrainDesc& G = gd[blockIdx.y];
    const int i = blockIdx.x * FB + threadIdx.x;
    if (i >= G.nodes) return;
    double q = G.cw[0] * (double)gbl(static_cast<const D*>(G.dep[0]))[i];
    if (G.ns > 1) q += G.cw[1] * (double)gbl(static_cast<const D*>(G.dep[1]))[i];
    const double rho = q / gbl(G.vol)[i];
    gbl(G.rho)[i] = rho;
    const int i1 = i % G.nx;
    gbl(G.f)[i] = (i1 == 0 || i1 == G.n1) ? 0.0 : G.rhs_scale * (G.fe ? q : rho);
}

hipError_t launch_rho_rhs(apic_ctx* ctx) {
    if (ctx->opts.precision == APIC_FP32_SPLIT)
        hipLaunchKernelGGL(k_rho_rhs<float>, node_grid(ctx), dim3(FB), 0, ctx->stream, ctx->gdesc);
    else
        hipLaunchKernelGGL(k_rho_rhs<double>, node_grid(ctx), dim3(FB), 0, ctx->stream, ctx->gdesc);
    return hipGetLastError();
}

// f from a given rho of one grain
__global__ void __launch_bounds__(FB)
k_rhs(const GrainDesc* __restrict__ gd, int grain) {
    const GrainDesc& G = gd[grain];
    const int i = blockIdx.x * FB + threadIdx.x;
    if (i >= G.nodes) return;
    const int i1 = i % G.nx;
    const double rho = gbl(G.rho)[i];
    gbl(G.f)[i] = (i1 == 0 || i1 == G.n1) ? 0.0 : G.rhs_scale * (G.fe ? rho * gbl(G.vol)[i] : rho);
}

hipError_t launch_rhs_from_rho(apic_ctx* ctx, int grain) {
    const int nodes = ctx->grains[grain].nodes;
    hipLaunchKernelGGL(k_rhs, dim3((nodes + FB - 1) / FB), dim3(FB), 0, ctx->stream, ctx->gdesc, grain);
    return hipGetLastError();
}

// Dirichlet values: phi = phi_grain on x1 = -1, phi_out on x1 = x1_out
__global__ void __launch_bounds__(FB)
k_set_boundary(const GrainDesc* __restrict__ gd) {
    const GrainDesc& G = gd[blockIdx.y];
    const int j = blockIdx.x * FB + threadIdx.x;
    if (j > G.n2) return;
    gbl(G.u)[j * G.nx] = G.phi_grain;
    gbl(G.u)[j * G.nx + G.n1] = G.phi_out;
}

hipError_t launch_set_boundary(apic_ctx* ctx) {
    hipLaunchKernelGGL(k_set_boundary, dim3((ctx->max_n2 + FB) / FB, (unsigned)ctx->grains.size()),
                       dim3(FB), 0, ctx->stream, ctx->gdesc);
    return hipGetLastError();
}

// Nodal (dphi/dx1, dphi/dx2): central inside, second-order one-sided on the edges.
template <typename V>
__global__ void __launch_bounds__(FB)
k_gradient(const GrainDesc* __restrict__ gd) {
    const GrainDesc& G = gd[blockIdx.y];
    const int idx = blockIdx.x * FB + threadIdx.x;
    if (idx >= G.nodes) return;
    const int n1 = G.n1, n2 = G.n2, nx = G.nx;
    const int i2 = idx / nx, i1 = idx - i2 * nx;
    const double ih1 = G.inv_h1, ih2 = G.inv_h2;
    const gptr<const double> row = gbl(static_cast<const double*>(G.u) + (size_t)i2 * nx);
    double d1, d2;
    if (i1 == 0) d1 = (-3.0 * row[0] + 4.0 * row[1] - row[2]) * 0.5 * ih1;
    else if (i1 == n1) d1 = (3.0 * row[n1] - 4.0 * row[n1 - 1] + row[n1 - 2]) * 0.5 * ih1;
    else d1 = (row[i1 + 1] - row[i1 - 1]) * 0.5 * ih1;
    if (i2 == 0) d2 = (-3.0 * row[i1] + 4.0 * row[i1 + nx] - row[i1 + 2 * nx]) * 0.5 * ih2;
    else if (i2 == n2) d2 = (3.0 * row[i1] - 4.0 * row[i1 - nx] + row[i1 - 2 * nx]) * 0.5 * ih2;
    else d2 = (row[i1 + nx] - row[i1 - nx]) * 0.5 * ih2;
    using E = decltype(V().x);
    const gptr<E> g = gbl(static_cast<E*>(G.grad));
    g[2 * (size_t)idx] = (E)d1;
    g[2 * (size_t)idx + 1] = (E)d2;
}

hipError_t launch_gradient(apic_ctx* ctx) {
    if (ctx->opts.precision == APIC_FP32_SPLIT)
        hipLaunchKernelGGL(k_gradient<float2>, node_grid(ctx), dim3(FB), 0, ctx->stream, ctx->gdesc);
    else
        hipLaunchKernelGGL(k_gradient<double2>, node_grid(ctx), dim3(FB), 0, ctx->stream, ctx->gdesc);
    return hipGetLastError();
}

// Normal field on the grain at node i2 = j, E_n = -|grad x1| dphi/dx1 (the
// one-sided nodal derivative on x1 = -1); |grad x1|, n_Z = x1_Z / |grad x1| and
// r of the node are returned too.  The surface charge density is eps0 E_n.
__device__ inline double surface_En(const GrainDesc& G, int j, double& gn, double& nZ, double& r) {
    const double alpha = G.alpha;
    const double x2 = -1.0 + j * G.h2;
    r = r_of(-1.0, x2, alpha);
    const double s = sqrt(fmax(1.0 - x2 * x2, 0.0));
    const Metric<double> m = metric_at(r, x2, s, alpha);
    gn = sqrt(m.x1R * m.x1R + m.x1Z * m.x1Z);
    nZ = m.x1Z / gn;
    const gptr<const double> row = gbl(static_cast<const double*>(G.u) + (size_t)j * G.nx);
    const double p1 = (-3.0 * row[0] + 4.0 * row[1] - row[2]) * 0.5 * G.inv_h1;
    return -gn * p1;
}

// Electric force on the grain, F_Z = integral over x1 = -1 of E_n^2 / 2 * n_Z dA
// (Maxwell stress on a conductor), trapezoid in x2; one workgroup per grain.
__global__ void __launch_bounds__(FB)
k_grain_force(const GrainDesc* __restrict__ gd) {
    __shared__ double red[FB];
    const GrainDesc& G = gd[blockIdx.x];
    const int n2 = G.n2;
    const double alpha = G.alpha, h2 = G.h2;
    double sum = 0.0;
    for (int j = threadIdx.x; j <= n2; j += blockDim.x) {
        const double x2 = -1.0 + j * h2;
        double gn, nZ, r;
        const double En = surface_En(G, j, gn, nZ, r);
        const double t = alpha / (r + 2.0 * alpha * x2);
        const double dA = 6.283185307179586 * r * r * sqrt(1.0 + (1.0 - x2 * x2) * t * t);
        const double w = (j == 0 || j == n2) ? 0.5 : 1.0;
        sum += w * 0.5 * En * En * nZ * dA;
    }
    red[threadIdx.x] = sum;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) gbl(&G.ctr->F_el_sum)[0] += red[0] * h2;
}

// E_n at the grain nodes of one grain (out: n2 + 1 values, device)
__global__ void __launch_bounds__(FB)
k_surface_field(const GrainDesc* __restrict__ gd, int grain, double* __restrict__ out) {
    const GrainDesc& G = gd[grain];
    const int j = blockIdx.x * FB + threadIdx.x;
    if (j > G.n2) return;
    double gn, nZ, r;
    gbl(out)[j] = surface_En(G, j, gn, nZ, r);
}

hipError_t launch_surface_field(apic_ctx* ctx, int grain, double* out) {
    const int n2 = ctx->grains[grain].gp.n2;
    hipLaunchKernelGGL(k_surface_field, dim3((n2 + FB) / FB), dim3(FB), 0, ctx->stream, ctx->gdesc, grain, out);
    return hipGetLastError();
}

hipError_t launch_grain_force(apic_ctx* ctx) {
    hipLaunchKernelGGL(k_grain_force, dim3((unsigned)ctx->grains.size()), dim3(FB), 0, ctx->stream,
                       ctx->gdesc);
    return hipGetLastError();
}

}  // namespace apic
