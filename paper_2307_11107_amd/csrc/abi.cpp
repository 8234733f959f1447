// C ABI of the aspherical PIC particle loop (declared in include/apic.h):
// context set-up, particle loading, the time step, the Poisson solve, tallies
// and read-back.  All arithmetic of the loop runs in the HIP kernels; this file
// validates arguments, builds the FP64 geometry tables once, orders the
// kernel launches on the context's stream and moves data across the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "apic_internal.h"
#include "device_common.h"
#include "host_setup.h"

using namespace apic;

namespace {

std::string g_init_error;

int fail(apic_ctx* ctx, int code, const std::string& msg) {
    if (ctx) ctx->err = msg;
    else g_init_error = msg;
    return code;
}

#define HIPCHK(ctx, call)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ctx, e_ == hipErrorOutOfMemory ? APIC_ENOMEM : APIC_EDEVICE,        \
                        std::string(#call) + ": " + hipGetErrorString(e_));                 \
    } while (0)

int dev_alloc(apic_ctx* ctx, void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return APIC_OK;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(ctx, APIC_ENOMEM, "hipMalloc(" + std::to_string(bytes) + " bytes) failed: " +
                                          hipGetErrorString(e));
    }
    return APIC_OK;
}

template <typename T>
int alloc_t(apic_ctx* ctx, T** p, size_t count) {
    void* v = nullptr;
    int rc = dev_alloc(ctx, &v, sizeof(T) * count);
    *p = static_cast<T*>(v);
    return rc;
}

#define TRY(x)                   \
    do {                         \
        int rc_ = (x);           \
        if (rc_ != APIC_OK) return rc_; \
    } while (0)


struct Timer {
    apic_ctx* ctx;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    Timer(apic_ctx* c, int k) : ctx(c), kind(k) {
        if (!ctx->profiling) return;
        if (ctx->event_pool.size() < 2) {
            hipEvent_t e;
            for (int i = 0; i < 64; ++i)
                if (hipEventCreate(&e) == hipSuccess) ctx->event_pool.push_back(e);
        }
        if (ctx->event_pool.size() < 2) return;
        a = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        b = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        (void)hipEventRecord(a, ctx->stream);
    }
    ~Timer() {
        if (!a) return;
        (void)hipEventRecord(b, ctx->stream);
        ctx->timers.push_back(TimerPair{a, b, kind});
        if (ctx->timers.size() > 4096) {
            // harvest to bound the number of live events
            (void)hipEventSynchronize(b);
            for (auto& t : ctx->timers) {
                float ms = 0;
                if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) ctx->t_ms[t.kind] += ms;
                ctx->event_pool.push_back(t.a);
                ctx->event_pool.push_back(t.b);
            }
            ctx->timers.clear();
        }
    }
};

// ---------------------------------------------------------------- Poisson driver
int read_norms(apic_ctx* ctx, Grain& g, double* r2, double* b2, double* e2 = nullptr) {
    double h[3];
    HIPCHK(ctx, hipMemcpyAsync(h, &g.ctr->norm2, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    *r2 = h[0];
    if (b2) *b2 = h[1];
    if (e2) *e2 = h[2];
    return APIC_OK;
}

// Multigrid cycles on the current right-hand side (mg[0].f) with phi's
// boundary values set; stops at |D^-1 r| <= tol |D^-1 b| (b includes the
// boundary coupling, D is the diagonal of the operator), at stagnation
// (standalone solves), or after max_cycles.
int solve_field(apic_ctx* ctx, Grain& g, double tol, int max_cycles, bool to_floor, int* cycles,
                bool extrapolate = false) {
    HIPCHK(ctx, launch_set_boundary(ctx, g));
    HIPCHK(ctx, mg_rhs_norm(ctx, g, &g.ctr->norm2_b));
    HIPCHK(ctx, mg_residual_norm(ctx, g, &g.ctr->norm2));
    // in the time loop the starting guess is the previous potential, or its
    // linear extrapolation from the two previous steps when that has the
    // smaller residual (a smooth evolution favours it, noise does not)
    const bool try_ex = extrapolate && g.have_prev;
    if (try_ex) {
        HIPCHK(ctx, launch_extrapolate(ctx, g));
        HIPCHK(ctx, mg_residual_norm(ctx, g, &g.ctr->norm2_e));
    } else if (extrapolate) {
        HIPCHK(ctx, launch_copy(ctx, g.phi_prev, g.mg[0].u, g.nodes));
    }
    double r2 = 0, b2 = 0, e2 = 0;
    TRY(read_norms(ctx, g, &r2, &b2, &e2));
    if (try_ex) {
        if (e2 < r2) r2 = e2;
        else HIPCHK(ctx, launch_copy(ctx, g.mg[0].u, g.phi_prev, g.nodes));
    }
    if (extrapolate) g.have_prev = true;
    const double bnorm = std::sqrt(b2 + g.bnd_norm2);
    double r = std::sqrt(r2), prev = r;
    int c = 0;
    while (c < max_cycles && r > tol * bnorm) {
        HIPCHK(ctx, mg_vcycle(ctx, g));   // also leaves the new residual norm in ctr->norm2
        TRY(read_norms(ctx, g, &r2, nullptr));
        r = std::sqrt(r2);
        ++c;
        if (to_floor && c >= 4 && r > 0.6 * prev) break;
        prev = r;
    }
    if (!(r == r)) return fail(ctx, APIC_EDEVICE, "Poisson solve produced NaN");
    if (cycles) *cycles = c;
    return APIC_OK;
}

// Deposit the current particles and solve for phi.
int rebuild_field(apic_ctx* ctx, Grain& g, double tol, int max_cycles, bool to_floor) {
    const size_t dbytes = (ctx->opts.precision == APIC_FP32_SPLIT ? 4 : 8) * (size_t)g.nodes;
    for (int s = 0; s < g.ns; ++s) {
        HIPCHK(ctx, launch_fill(ctx, g.dep[s], dbytes));
        HIPCHK(ctx, launch_deposit_all(ctx, g, s));
    }
    HIPCHK(ctx, launch_rho(ctx, g));
    HIPCHK(ctx, launch_rhs_from_rho(ctx, g));
    int cyc = 0;
    TRY(solve_field(ctx, g, tol, max_cycles, to_floor, &cyc));
    ctx->timed_mg_cycles += ctx->profiling ? cyc : 0;
    HIPCHK(ctx, launch_gradient(ctx, g));
    g.field_stale = false;
    g.have_prev = false;
    return APIC_OK;
}

int check_grain(apic_ctx* ctx, int32_t grain) {
    if (!ctx) return fail(nullptr, APIC_EINVAL, "null context");
    if (grain < 0 || grain >= (int)ctx->grains.size())
        return fail(ctx, APIC_EINVAL, "grain index out of range");
    return APIC_OK;
}

void free_grain(Grain& g) {
    auto F = [](void* p) {
        if (p) (void)hipFree(p);
    };
    for (int s = 0; s < APIC_MAX_SPECIES; ++s) {
        for (int k = 0; k < 2; ++k) {
            PBuf& b = g.buf[s][k];
            F(b.pos0);
            F(b.pos1);
            F(b.pos2);
            F(b.vR);
            F(b.vZ);
            F(b.vT);
            F(b.id);
            b = PBuf();
        }
        F(g.dep[s]);
        g.dep[s] = nullptr;
    }
    F(g.ctr);
    F(g.vol);
    F(g.grad);
    F(g.rho);
    F(g.phi_prev);
    F(g.tally);
    F(g.tally_count);
    F(g.axis_nn);
    F(g.axis_ss);
    F(g.coarse_inv);
    F(g.sort_count);
    F(g.sort_offset);
    F(g.scan_tmp);
    if (g.vcycle_exec) (void)hipGraphExecDestroy(g.vcycle_exec);
    g.vcycle_exec = nullptr;
    for (auto& L : g.mg) {
        F(L.st);
        F(L.u);
        F(L.f);
        F(L.r);
    }
    g.mg.clear();
    g.ctr = nullptr;
}

int validate_cfg(const apic_grain_cfg& c) {
    if (!(std::fabs(c.alpha) < 0.25)) return APIC_ERANGE;
    if (!(c.x1_out > -1.0 && c.x1_out < 0.0)) return APIC_ERANGE;
    if (c.n1 < 8 || c.n2 < 8 || c.n1 > 2048 || c.n2 > 2046) return APIC_ERANGE;
    if (c.n_species < 1 || c.n_species > APIC_MAX_SPECIES) return APIC_EINVAL;
    if (!(c.dt > 0.0) || !(c.kappa > 0.0) || c.n_bins < 0) return APIC_EINVAL;
    for (int s = 0; s < c.n_species; ++s) {
        const apic_species& sp = c.sp[s];
        if (!(sp.m > 0.0) || !(sp.T >= 0.0) || !(sp.n >= 0.0) || sp.n_macro < 0 || sp.capacity < 0 ||
            !(sp.weight >= 0.0))
            return APIC_EINVAL;
        if (sp.n_macro > (int64_t)2000000000) return APIC_ERANGE;
    }
    return APIC_OK;
}

int setup_grain(apic_ctx* ctx, Grain& g, const apic_grain_cfg& c, int gi) {
    g.cfg = c;
    g.ns = c.n_species;
    const int n1 = c.n1, n2 = c.n2, nx = n1 + 1;
    g.nodes = nx * (n2 + 1);
    g.ncells = n1 * n2;
    GrainParams& gp = g.gp;
    gp.n1 = n1;
    gp.n2 = n2;
    gp.nx = nx;
    gp.n_bins = c.n_bins > 0 ? c.n_bins : n2;
    gp.alpha = c.alpha;
    gp.x1_out = c.x1_out;
    gp.h1 = (1.0 + c.x1_out) / n1;
    gp.h2 = 2.0 / n2;
    gp.inv_h1 = n1 / (1.0 + c.x1_out);
    gp.inv_h2 = n2 / 2.0;
    gp.kappa = c.kappa;
    gp.dt = c.dt;
    gp.step = c.kappa * c.dt;
    gp.r_grain_max = grain_max_radius(c.alpha);
    gp.M_vol = bound_volume_marginal(c.x1_out, c.alpha);
    gp.M_area = bound_outer_area_density(c.x1_out, c.alpha);
    gp.key0 = (uint32_t)(c.seed & 0xFFFFFFFFull);
    gp.key1 = (uint32_t)((c.seed >> 32) + (uint64_t)gi);

    node_volumes(n1, n2, c.x1_out, c.alpha, g.vol_host);
    g.V = 0.0;
    for (double v : g.vol_host) g.V += v;
    g.A_out = outer_area(c.x1_out, c.alpha);

    for (int s = 0; s < g.ns; ++s) {
        const apic_species& a = c.sp[s];
        SpeciesParams& p = g.sp[s];
        p.q = a.q;
        p.m = a.m;
        p.T = a.T;
        p.e_bind = a.e_bind;
        p.w = a.weight > 0 ? a.weight : (a.n_macro > 0 ? a.n * g.V / (double)a.n_macro : 0.0);
        const double qm = a.q / a.m;
        p.qm_half = 0.5 * qm * c.kappa * c.dt;
        const double t = 0.5 * qm * c.wce * c.dt;
        p.rot_c = (1.0 - t * t) / (1.0 + t * t);
        p.rot_s = 2.0 * t / (1.0 + t * t);
        p.rot_cm1 = -2.0 * t * t / (1.0 + t * t);
        p.sigma = std::sqrt(a.T / a.m);
        const double flux = a.n * std::sqrt(a.T / (2.0 * M_PI * a.m));
        const double n_real = p.w > 0 ? flux * g.A_out * c.kappa * c.dt / p.w : 0.0;
        if (n_real > 1e12) return fail(ctx, APIC_ERANGE, "injection rate too large");
        g.inj_inc[s] = (uint64_t)std::llround(n_real * 4294967296.0);
        g.inj_acc[s] = 0;
        int64_t cap = a.capacity;
        if (cap == 0) cap = (int64_t)(1.5 * (double)a.n_macro) + 64 * (int64_t)std::ceil(n_real) + 4096;
        if (cap > (int64_t)2000000000) return fail(ctx, APIC_ERANGE, "particle capacity above 2^31");
        g.capacity[s] = cap;
        g.host_slots[s] = 0;
    }

    // ---- device allocations
    const bool split = ctx->opts.precision == APIC_FP32_SPLIT;
    const size_t fsz = split ? 4 : 8;
    for (int s = 0; s < g.ns; ++s) {
        const size_t cap = (size_t)g.capacity[s];
        for (int k = 0; k < 2; ++k) {
            PBuf& b = g.buf[s][k];
            if (split) TRY(dev_alloc(ctx, &b.pos0, 4 * cap));
            TRY(dev_alloc(ctx, &b.pos1, fsz * cap));
            TRY(dev_alloc(ctx, &b.pos2, fsz * cap));
            TRY(dev_alloc(ctx, &b.vR, fsz * cap));
            TRY(dev_alloc(ctx, &b.vZ, fsz * cap));
            TRY(dev_alloc(ctx, &b.vT, fsz * cap));
            TRY(alloc_t(ctx, &b.id, cap));
        }
        TRY(dev_alloc(ctx, &g.dep[s], fsz * (size_t)g.nodes));
    }
    TRY(alloc_t(ctx, &g.ctr, 1));
    TRY(alloc_t(ctx, &g.vol, (size_t)g.nodes));
    TRY(dev_alloc(ctx, &g.grad, 2 * fsz * (size_t)g.nodes));
    TRY(alloc_t(ctx, &g.rho, (size_t)g.nodes));
    TRY(alloc_t(ctx, &g.phi_prev, (size_t)g.nodes));
    TRY(alloc_t(ctx, &g.tally, (size_t)5 * g.ns * gp.n_bins));
    TRY(alloc_t(ctx, &g.tally_count, (size_t)g.ns * gp.n_bins));
    // sort tiles: the smallest square power-of-two tile giving at most 8192 tiles
    gp.tile_log2 = 3;
    while (((n1 + (1 << gp.tile_log2) - 1) >> gp.tile_log2) * ((n2 + (1 << gp.tile_log2) - 1) >> gp.tile_log2) > 8192)
        ++gp.tile_log2;
    gp.ntx = (n1 + (1 << gp.tile_log2) - 1) >> gp.tile_log2;
    gp.ntiles = gp.ntx * ((n2 + (1 << gp.tile_log2) - 1) >> gp.tile_log2);
    const size_t hist_len = (size_t)gp.ntiles * sort_blocks() + 1;
    TRY(alloc_t(ctx, &g.sort_count, hist_len));
    TRY(alloc_t(ctx, &g.sort_offset, hist_len));
    HIPCHK(ctx, launch_fill(ctx, g.sort_count, sizeof(int) * hist_len));
    g.scan_tmp_bytes = scan_temp_bytes((int)hist_len);
    TRY(dev_alloc(ctx, &g.scan_tmp, g.scan_tmp_bytes));
    HIPCHK(ctx, launch_fill(ctx, g.ctr, sizeof(DevCounters)));
    HIPCHK(ctx, launch_fill(ctx, g.tally, sizeof(double) * 5 * g.ns * gp.n_bins));
    HIPCHK(ctx, launch_fill(ctx, g.tally_count, sizeof(unsigned long long) * g.ns * gp.n_bins));
    HIPCHK(ctx, launch_fill(ctx, g.rho, sizeof(double) * g.nodes));
    HIPCHK(ctx, hipMemcpyAsync(g.vol, g.vol_host.data(), sizeof(double) * g.nodes,
                               hipMemcpyHostToDevice, ctx->stream));

    // ---- multigrid hierarchy
    // coarsen by two while both cell counts are even and at least 8, and stop
    // at the first level with at most 600 nodes (solved by a dense inverse)
    std::vector<Stencil> levels(1);
    fine_stencil(n1, n2, c.x1_out, c.alpha, levels[0]);
    while ((levels.back().n1 + 1) * (levels.back().n2 + 1) > 600 && levels.back().n1 % 2 == 0 &&
           levels.back().n2 % 2 == 0 && std::min(levels.back().n1, levels.back().n2) / 2 >= 4) {
        Stencil cs;
        galerkin_coarse(levels.back(), cs);
        levels.push_back(std::move(cs));
    }
    const Stencil& last = levels.back();
    const int m = (last.n1 + 1) * (last.n2 + 1);
    if (m > 4096) return fail(ctx, APIC_ERANGE, "grid does not coarsen far enough for multigrid");
    std::vector<double> A, inv;
    dense_matrix(last, A);
    if (!invert(A, m, inv)) return fail(ctx, APIC_EDEVICE, "coarsest multigrid operator is singular");
    g.coarse_nodes = m;
    TRY(alloc_t(ctx, &g.coarse_inv, (size_t)m * m));
    std::vector<double> stage;
    g.mg.resize(levels.size());
    for (size_t l = 0; l < levels.size(); ++l) {
        MGLevel& L = g.mg[l];
        L.n1 = levels[l].n1;
        L.n2 = levels[l].n2;
        L.nx = L.n1 + 1;
        L.nodes = L.nx * (L.n2 + 1);
        TRY(alloc_t(ctx, &L.st, (size_t)ST_COUNT * L.nodes));
        TRY(alloc_t(ctx, &L.u, (size_t)L.nodes));
        TRY(alloc_t(ctx, &L.f, (size_t)L.nodes));
        TRY(alloc_t(ctx, &L.r, (size_t)L.nodes));
        HIPCHK(ctx, launch_fill(ctx, L.u, sizeof(double) * L.nodes));
        HIPCHK(ctx, launch_fill(ctx, L.f, sizeof(double) * L.nodes));
        HIPCHK(ctx, launch_fill(ctx, L.r, sizeof(double) * L.nodes));
        stage.resize((size_t)ST_COUNT * L.nodes);
        for (int k = 0; k < ST_COUNT; ++k)
            std::copy(levels[l].c[k].begin(), levels[l].c[k].end(), stage.begin() + (size_t)k * L.nodes);
        HIPCHK(ctx, hipMemcpy(L.st, stage.data(), sizeof(double) * stage.size(), hipMemcpyHostToDevice));
    }
    TRY(alloc_t(ctx, &g.axis_nn, (size_t)nx));
    TRY(alloc_t(ctx, &g.axis_ss, (size_t)nx));
    HIPCHK(ctx, hipMemcpy(g.axis_nn, levels[0].nn.data(), sizeof(double) * nx, hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMemcpy(g.axis_ss, levels[0].ss.data(), sizeof(double) * nx, hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMemcpy(g.coarse_inv, inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice));
    g.bnd_norm2 = boundary_coupling_norm2(levels[0], c.phi_grain, c.phi_out);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));

    // vacuum field until particles are loaded
    HIPCHK(ctx, launch_fill(ctx, g.rho, sizeof(double) * g.nodes));
    HIPCHK(ctx, launch_rhs_from_rho(ctx, g));
    TRY(solve_field(ctx, g, 1e-15, 100, true, nullptr));
    HIPCHK(ctx, launch_gradient(ctx, g));
    g.field_stale = true;
    return APIC_OK;
}

int do_step(apic_ctx* ctx, Grain& g) {
    const bool frozen = ctx->opts.frozen_field != 0;
    const double tol = ctx->opts.poisson_tol > 0 ? ctx->opts.poisson_tol : 1e-10;
    const int maxc = ctx->opts.poisson_max_cycles > 0 ? ctx->opts.poisson_max_cycles : 40;
    if (g.field_stale && !frozen) TRY(rebuild_field(ctx, g, tol, maxc, false));
    g.field_stale = false;
    const size_t dbytes = (ctx->opts.precision == APIC_FP32_SPLIT ? 4 : 8) * (size_t)g.nodes;
    for (int s = 0; s < g.ns; ++s) {
        if (!frozen) HIPCHK(ctx, launch_fill(ctx, g.dep[s], dbytes));
        Timer t(ctx, 0);
        HIPCHK(ctx, launch_push(ctx, g, s));
        if (ctx->profiling) ++ctx->push_launches;
    }
    if (ctx->opts.inject) {
        Timer t(ctx, 1);
        for (int s = 0; s < g.ns; ++s) {
            g.inj_acc[s] += g.inj_inc[s];
            const int64_t n_new = (int64_t)(g.inj_acc[s] >> 32);
            g.inj_acc[s] &= 0xFFFFFFFFull;
            if (n_new > 0)
                HIPCHK(ctx, launch_inject(ctx, g, s, n_new, (uint32_t)(g.step_index & 0xFFFFFFFFull)));
        }
    }
    {
        Timer t(ctx, 3);
        if (!frozen) {
            HIPCHK(ctx, launch_rho(ctx, g));
            HIPCHK(ctx, launch_rhs_from_rho(ctx, g));
            int cyc = 0;
            TRY(solve_field(ctx, g, tol, maxc, false, &cyc, true));
            if (ctx->profiling) ctx->timed_mg_cycles += cyc;
            HIPCHK(ctx, launch_gradient(ctx, g));
        }
        HIPCHK(ctx, launch_grain_force(ctx, g));
    }
    g.step_index++;
    const int k = ctx->opts.sort_every > 0 ? ctx->opts.sort_every : 8;
    if (g.step_index % (uint64_t)k == 0) {
        Timer t(ctx, 2);
        for (int s = 0; s < g.ns; ++s) HIPCHK(ctx, launch_sort(ctx, g, s));
    }
    if (ctx->profiling) ++ctx->timed_steps;
    return APIC_OK;
}

}  // namespace

// ======================================================================== ABI
extern "C" {

int apic_init(const apic_grain_cfg* cfgs, int32_t n_grains, const apic_opts* opts, apic_ctx** out) {
    if (!out) return fail(nullptr, APIC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfgs || n_grains < 1 || n_grains > 4096)
        return fail(nullptr, APIC_EINVAL, "need 1 <= n_grains <= 4096 and a config array");
    for (int i = 0; i < n_grains; ++i) {
        const int v = validate_cfg(cfgs[i]);
        if (v == APIC_ERANGE)
            return fail(nullptr, v, "grain " + std::to_string(i) +
                                        ": need |alpha| < 1/4, -1 < x1_out < 0, 8 <= n1 <= 2048, "
                                        "8 <= n2 <= 2046");
        if (v != APIC_OK) return fail(nullptr, v, "grain " + std::to_string(i) + ": invalid configuration");
    }
    apic_ctx* ctx = new apic_ctx();
    std::memset(&ctx->opts, 0, sizeof(apic_opts));
    if (opts) ctx->opts = *opts;
    if (ctx->opts.precision != APIC_FP32_SPLIT && ctx->opts.precision != APIC_FP64) {
        delete ctx;
        return fail(nullptr, APIC_EINVAL, "precision must be APIC_FP32_SPLIT or APIC_FP64");
    }
    int rc = APIC_OK;
    hipError_t e = hipGetDevice(&ctx->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ctx->num_cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
    if (e != hipSuccess) {
        g_init_error = std::string("no HIP device: ") + hipGetErrorString(e);
        delete ctx;
        return APIC_EDEVICE;
    }
    ctx->stream = static_cast<hipStream_t>(ctx->opts.stream);
    if (!ctx->stream) {
        // the legacy default stream cannot be captured into graphs: use our own
        e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            g_init_error = std::string("hipStreamCreate: ") + hipGetErrorString(e);
            delete ctx;
            return APIC_EDEVICE;
        }
        ctx->own_stream = true;
    }
    ctx->grains.resize(n_grains);
    for (int i = 0; i < n_grains && rc == APIC_OK; ++i) rc = setup_grain(ctx, ctx->grains[i], cfgs[i], i);
    if (rc != APIC_OK) {
        g_init_error = ctx->err;
        for (auto& g : ctx->grains) free_grain(g);
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
        delete ctx;
        return rc;
    }
    *out = ctx;
    return APIC_OK;
}

int apic_inject(apic_ctx* ctx, int32_t grain, int32_t species, int64_t n, const double* x1,
                const double* x2, const double* vR, const double* vZ, const double* vTheta) {
    TRY(check_grain(ctx, grain));
    Grain& g = ctx->grains[grain];
    if (species < 0 || species >= g.ns) return fail(ctx, APIC_EINVAL, "species index out of range");
    const bool load = n < 0;
    if (load && (x1 || x2 || vR || vZ || vTheta))
        return fail(ctx, APIC_EINVAL, "n < 0 requests a volume load: arrays must be NULL");
    if (!load && n > 0 && !(x1 && x2 && vR && vZ && vTheta))
        return fail(ctx, APIC_EINVAL, "particle arrays must be non-NULL");
    const int64_t count = load ? g.cfg.sp[species].n_macro : n;
    if (count > g.capacity[species])
        return fail(ctx, APIC_ENOMEM, "particle count exceeds the species capacity");
    const int s = species;
    g.cur[s] = 0;
    if (load) {
        if (count > 0) HIPCHK(ctx, launch_load(ctx, g, s, count));
    } else if (count > 0) {
        double* tmp = nullptr;
        int* bad = nullptr;
        TRY(alloc_t(ctx, &tmp, (size_t)5 * count));
        if (alloc_t(ctx, &bad, 1) != APIC_OK) {
            (void)hipFree(tmp);
            return APIC_ENOMEM;
        }
        const double* src[5] = {x1, x2, vR, vZ, vTheta};
        hipError_t e = hipSuccess;
        for (int k = 0; k < 5 && e == hipSuccess; ++k)
            e = hipMemcpyAsync(tmp + (size_t)k * count, src[k], sizeof(double) * count,
                               hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess) e = launch_fill(ctx, bad, sizeof(int));
        if (e == hipSuccess)
            e = launch_set_particles(ctx, g, s, count, tmp, tmp + count, tmp + 2 * count,
                                     tmp + 3 * count, tmp + 4 * count, bad);
        int hbad = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        (void)hipFree(tmp);
        (void)hipFree(bad);
        if (e != hipSuccess) return fail(ctx, APIC_EDEVICE, std::string("apic_inject: ") + hipGetErrorString(e));
        if (hbad) return fail(ctx, APIC_EINVAL, "particle outside the domain (-1 < x1 < x1_out, |x2| <= 1)");
    }
    // counters of this species restart with the new population
    DevCounters h;
    HIPCHK(ctx, hipMemcpyAsync(&h, g.ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    h.n[s] = count;
    h.injected[s] = (uint64_t)count;
    h.absorbed[s] = 0;
    h.escaped[s] = 0;
    h.pushed[s] = 0;
    h.next_id[s] = (uint32_t)count;
    HIPCHK(ctx, hipMemcpyAsync(g.ctr, &h, sizeof(DevCounters), hipMemcpyHostToDevice, ctx->stream));
    for (int k = 0; k < 5; ++k)
        HIPCHK(ctx, launch_fill(ctx, g.tally + ((size_t)k * g.ns + s) * g.gp.n_bins,
                                sizeof(double) * g.gp.n_bins));
    HIPCHK(ctx, launch_fill(ctx, g.tally_count + (size_t)s * g.gp.n_bins,
                            sizeof(unsigned long long) * g.gp.n_bins));
    g.host_slots[s] = count;
    HIPCHK(ctx, launch_sort(ctx, g, s));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    g.field_stale = true;
    return APIC_OK;
}

int apic_step(apic_ctx* ctx, int64_t n_steps) {
    if (!ctx) return fail(nullptr, APIC_EINVAL, "null context");
    if (n_steps < 0) return fail(ctx, APIC_EINVAL, "n_steps < 0");
    for (int64_t k = 0; k < n_steps; ++k)
        for (auto& g : ctx->grains) TRY(do_step(ctx, g));
    return APIC_OK;
}

int apic_solve_poisson(apic_ctx* ctx, int32_t grain, const double* rho, double* phi_out) {
    TRY(check_grain(ctx, grain));
    Grain& g = ctx->grains[grain];
    if (rho) {
        HIPCHK(ctx, hipMemcpyAsync(g.rho, rho, sizeof(double) * g.nodes, hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(ctx, launch_rhs_from_rho(ctx, g));
        TRY(solve_field(ctx, g, 1e-15, 100, true, nullptr));
        HIPCHK(ctx, launch_gradient(ctx, g));
        g.field_stale = false;
        g.have_prev = false;
    } else {
        TRY(rebuild_field(ctx, g, 1e-15, 100, true));
    }
    if (phi_out)
        HIPCHK(ctx, hipMemcpyAsync(phi_out, g.mg[0].u, sizeof(double) * g.nodes, hipMemcpyDeviceToHost,
                                   ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return APIC_OK;
}

int apic_tallies(apic_ctx* ctx, int32_t grain, apic_tally* out) {
    TRY(check_grain(ctx, grain));
    if (!out) return fail(ctx, APIC_EINVAL, "out is NULL");
    Grain& g = ctx->grains[grain];
    DevCounters h;
    HIPCHK(ctx, hipMemcpyAsync(&h, g.ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, ctx->stream));
    unsigned long long* live = nullptr;
    TRY(alloc_t(ctx, &live, APIC_MAX_SPECIES));
    unsigned long long hl[APIC_MAX_SPECIES] = {0, 0};
    hipError_t e = hipSuccess;
    for (int s = 0; s < g.ns && e == hipSuccess; ++s) e = launch_count_live(ctx, g, s, live + s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hl, live, sizeof(hl), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    (void)hipFree(live);
    if (e != hipSuccess) return fail(ctx, APIC_EDEVICE, std::string("apic_tallies: ") + hipGetErrorString(e));
    if (h.overflow) return fail(ctx, APIC_ENOMEM, "particle capacity exceeded during injection");
    out->n_species = g.ns;
    out->n_bins = g.gp.n_bins;
    out->steps = g.step_index;
    for (int s = 0; s < APIC_MAX_SPECIES; ++s) {
        const bool on = s < g.ns;
        out->injected[s] = on ? h.injected[s] : 0;
        out->absorbed[s] = on ? h.absorbed[s] : 0;
        out->escaped[s] = on ? h.escaped[s] : 0;
        out->resident[s] = on ? hl[s] : 0;
        out->particle_steps[s] = on ? h.pushed[s] : 0;
        out->weight[s] = on ? g.sp[s].w : 0.0;
    }
    out->F_el_sum = h.F_el_sum;
    const size_t nb = (size_t)g.ns * g.gp.n_bins;
    double* dst[5] = {out->charge, out->pR, out->pZ, out->L, out->energy};
    for (int k = 0; k < 5; ++k)
        if (dst[k])
            HIPCHK(ctx, hipMemcpyAsync(dst[k], g.tally + k * nb, sizeof(double) * nb,
                                       hipMemcpyDeviceToHost, ctx->stream));
    if (out->count)
        HIPCHK(ctx, hipMemcpyAsync(out->count, g.tally_count, sizeof(uint64_t) * nb,
                                   hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return APIC_OK;
}

int apic_particles(apic_ctx* ctx, int32_t grain, int32_t species, int64_t cap, double* x1,
                   double* x2, double* vR, double* vZ, double* vTheta, int64_t* id,
                   int64_t* n_out) {
    TRY(check_grain(ctx, grain));
    Grain& g = ctx->grains[grain];
    if (species < 0 || species >= g.ns) return fail(ctx, APIC_EINVAL, "species index out of range");
    if (!n_out || cap < 0 || (cap > 0 && !(x1 && x2 && vR && vZ && vTheta)))
        return fail(ctx, APIC_EINVAL, "bad output arrays");
    DevCounters h;
    HIPCHK(ctx, hipMemcpyAsync(&h, g.ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    const int64_t slots = h.n[species];
    double* tmp = nullptr;
    int64_t* tid = nullptr;
    const size_t m = (size_t)std::max<int64_t>(slots, 1);
    TRY(alloc_t(ctx, &tmp, 5 * m));
    if (alloc_t(ctx, &tid, m) != APIC_OK) {
        (void)hipFree(tmp);
        return APIC_ENOMEM;
    }
    std::vector<double> hx((size_t)5 * m);
    std::vector<int64_t> hid(m);
    unsigned long long found = 0;
    hipError_t e = launch_readback(ctx, g, species, slots, tmp, tmp + m, tmp + 2 * m, tmp + 3 * m,
                                   tmp + 4 * m, tid);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&found, &g.ctr->cursor, sizeof(found), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess && found > 0)
        e = hipMemcpy(hx.data(), tmp, sizeof(double) * 5 * m, hipMemcpyDeviceToHost);
    if (e == hipSuccess && found > 0) e = hipMemcpy(hid.data(), tid, sizeof(int64_t) * m, hipMemcpyDeviceToHost);
    (void)hipFree(tmp);
    (void)hipFree(tid);
    if (e != hipSuccess) return fail(ctx, APIC_EDEVICE, std::string("apic_particles: ") + hipGetErrorString(e));
    *n_out = (int64_t)found;
    if ((int64_t)found > cap) return fail(ctx, APIC_EINVAL, "cap smaller than the particle count");
    std::vector<size_t> order(found);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return hid[a] < hid[b]; });
    double* dst[5] = {x1, x2, vR, vZ, vTheta};
    for (size_t k = 0; k < found; ++k) {
        const size_t o = order[k];
        for (int c = 0; c < 5; ++c) dst[c][k] = hx[(size_t)c * m + o];
        if (id) id[k] = hid[o];
    }
    return APIC_OK;
}

int apic_fields(apic_ctx* ctx, int32_t grain, double* phi, double* rho) {
    TRY(check_grain(ctx, grain));
    Grain& g = ctx->grains[grain];
    if (phi)
        HIPCHK(ctx, hipMemcpyAsync(phi, g.mg[0].u, sizeof(double) * g.nodes, hipMemcpyDeviceToHost, ctx->stream));
    if (rho)
        HIPCHK(ctx, hipMemcpyAsync(rho, g.rho, sizeof(double) * g.nodes, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return APIC_OK;
}

int apic_set_profiling(apic_ctx* ctx, int32_t on) {
    if (!ctx) return fail(nullptr, APIC_EINVAL, "null context");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (auto& t : ctx->timers) {
        ctx->event_pool.push_back(t.a);
        ctx->event_pool.push_back(t.b);
    }
    ctx->timers.clear();
    for (double& v : ctx->t_ms) v = 0.0;
    ctx->push_launches = ctx->timed_steps = ctx->timed_particle_steps = ctx->timed_mg_cycles = 0;
    // particle-steps are taken from the device counters
    int64_t pushed = 0;
    for (auto& g : ctx->grains) {
        DevCounters h;
        HIPCHK(ctx, hipMemcpy(&h, g.ctr, sizeof(DevCounters), hipMemcpyDeviceToHost));
        for (int s = 0; s < g.ns; ++s) pushed += (int64_t)h.pushed[s];
    }
    ctx->timed_particle_steps = -pushed;
    ctx->profiling = on != 0;
    return APIC_OK;
}

int apic_timing(apic_ctx* ctx, apic_kernel_times* out) {
    if (!ctx || !out) return fail(ctx, APIC_EINVAL, "null argument");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (auto& t : ctx->timers) {
        float ms = 0;
        HIPCHK(ctx, hipEventElapsedTime(&ms, t.a, t.b));
        ctx->t_ms[t.kind] += ms;
        ctx->event_pool.push_back(t.a);
        ctx->event_pool.push_back(t.b);
    }
    ctx->timers.clear();
    int64_t pushed = 0;
    for (auto& g : ctx->grains) {
        DevCounters h;
        HIPCHK(ctx, hipMemcpy(&h, g.ctr, sizeof(DevCounters), hipMemcpyDeviceToHost));
        for (int s = 0; s < g.ns; ++s) pushed += (int64_t)h.pushed[s];
    }
    out->push_ms = ctx->t_ms[0];
    out->inject_ms = ctx->t_ms[1];
    out->sort_ms = ctx->t_ms[2];
    out->field_ms = ctx->t_ms[3];
    out->push_launches = ctx->push_launches;
    out->steps = ctx->timed_steps;
    out->particle_steps = ctx->timed_particle_steps + pushed;
    out->mg_cycles = ctx->timed_mg_cycles;
    return APIC_OK;
}

int apic_free(apic_ctx* ctx) {
    if (!ctx) return APIC_OK;
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& g : ctx->grains) free_grain(g);
    for (auto& t : ctx->timers) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return APIC_OK;
}

const char* apic_last_error(const apic_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

}  // extern "C"
