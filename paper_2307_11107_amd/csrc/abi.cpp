// C ABI of the aspherical PIC particle loop (declared in include/apic.h):
// context set-up, particle loading, the time step, the Poisson solve, tallies
// and read-back.  All arithmetic of the loop runs in the HIP kernels; this file
// validates arguments, builds the FP64 geometry tables once, builds the
// ensemble's descriptor tables, orders the kernel launches on the context's
// stream (captured into HIP graphs and replayed), runs the autotuner and moves
// data across the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
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

#define TRY(x)                   \
    do {                         \
        int rc_ = (x);           \
        if (rc_ != APIC_OK) return rc_; \
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

// HIP-event timer of one phase on the context's stream (profiling only).
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

bool split_mode(const apic_ctx* ctx) { return ctx->opts.precision == APIC_FP32_SPLIT; }
bool frozen_mode(const apic_ctx* ctx) { return ctx->opts.frozen_field != 0; }
double step_tol(const apic_ctx* ctx) { return ctx->opts.poisson_tol > 0 ? ctx->opts.poisson_tol : 1e-10; }
int step_max_cycles(const apic_ctx* ctx) {
    return ctx->opts.poisson_max_cycles > 0 ? ctx->opts.poisson_max_cycles : 40;
}

// ---------------------------------------------------------------- graphs
void drop_graphs(apic_ctx* ctx) {
    for (auto& g : ctx->graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

// Issues the launch sequence `fn` on the stream: captured into graph `id` the
// first time and replayed afterwards (eager if the stream cannot be captured).
template <typename F>
int run_phase(apic_ctx* ctx, int id, F fn) {
    if (!ctx->graph[id] && ctx->graphs && !ctx->tuning) {
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            fn();
            e = hipStreamEndCapture(ctx->stream, &graph);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&ctx->graph[id], graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            ctx->graph[id] = nullptr;
            ctx->graphs = false;
            drop_graphs(ctx);
        }
    }
    if (ctx->graph[id]) HIPCHK(ctx, hipGraphLaunch(ctx->graph[id], ctx->stream));
    else {
        fn();
        HIPCHK(ctx, hipGetLastError());
    }
    return APIC_OK;
}

// ---------------------------------------------------------------- Poisson driver
int read_batch(apic_ctx* ctx, MGBatch& b) {
    HIPCHK(ctx, hipMemcpyAsync(ctx->mgb_host, ctx->mgb, sizeof(MGBatch), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    b = *ctx->mgb_host;
    return APIC_OK;
}

// Multigrid solve of every grain (only >= 0: that grain alone) on the current
// right-hand sides.  A grain stops at |D^-1 r| <= tol |D^-1 b| (b with the
// boundary coupling, D the operator's diagonal); standalone solves (to_floor)
// also stop at stagnation.  In-step solves replay the captured V-cycle as many
// times as the previous solve needed before reading the convergence state once
// (cycles after convergence do nothing on the device).  Only the last two of
// those predicted cycles end with the residual norm and the check (two of the
// ~10 latency-bound launches of a cycle): the check before the last tells
// whether one cycle fewer would have done, and the prediction drops by one.
// Grains that converged earlier keep cycling until then, which only lowers
// their residual further.
int solve_linear(apic_ctx* ctx, double tol, int max_cycles, bool to_floor, int only, bool in_step, int* cycles) {
    MGBatch b;
    int launched = 0;
    if (in_step) {
        TRY(run_phase(ctx, G_PRE, [&] {
            (void)launch_rho_rhs(ctx);
            (void)mg_extrapolate(ctx);
            (void)launch_set_boundary(ctx);
            (void)mg_begin(ctx, tol, -1, true);
        }));
        const int pred = std::min(ctx->pred_cycles, max_cycles);
        for (; launched < pred; ++launched) {
            const bool check = launched + 2 >= pred;
            TRY(run_phase(ctx, check ? G_VC : G_VCN, [&] { (void)mg_vcycle_launches(ctx, tol, check); }));
        }
        TRY(read_batch(ctx, b));
        const bool one_fewer = pred >= 2 && b.pending == 0 && b.pending_prev == 0;
        while (b.pending > 0 && launched < max_cycles) {
            TRY(run_phase(ctx, G_VC, [&] { (void)mg_vcycle_launches(ctx, tol); }));
            ++launched;
            TRY(read_batch(ctx, b));
        }
        ctx->pred_cycles = one_fewer ? pred - 1 : launched;
        if (cycles) *cycles = launched;
        if (b.pending > 0) {
            // stopped at the cycle cap: counted per grain, reported in the tallies
            const int G = (int)ctx->grains.size();
            std::vector<MGState> m(G);
            HIPCHK(ctx, hipMemcpy(m.data(), ctx->mgs, sizeof(MGState) * G, hipMemcpyDeviceToHost));
            for (int g = 0; g < G; ++g)
                if (!m[g].done) ++ctx->grains[g].unconverged;
        }
    } else {
        HIPCHK(ctx, launch_set_boundary(ctx));
        HIPCHK(ctx, mg_begin(ctx, tol, only, false));
        TRY(read_batch(ctx, b));
        double prev = HUGE_VAL;
        while (b.pending > 0 && launched < max_cycles) {
            HIPCHK(ctx, mg_vcycle_launches(ctx, tol));
            ++launched;
            TRY(read_batch(ctx, b));
            if (to_floor) {
                // largest relative residual of the grains still iterating
                const int G = (int)ctx->grains.size();
                std::vector<MGState> m(G);
                HIPCHK(ctx, hipMemcpy(m.data(), ctx->mgs, sizeof(MGState) * G, hipMemcpyDeviceToHost));
                double r = 0.0;
                for (int g = 0; g < G; ++g)
                    if (only < 0 || g == only)
                        r = std::max(r, std::sqrt(m[g].last_r2 / (m[g].b2 + ctx->gdesc_h[g].bnd2 + 1e-300)));
                if (launched >= 4 && r > 0.6 * prev) break;
                prev = r;
            }
        }
    }
    if (b.nan) {
        HIPCHK(ctx, launch_fill(ctx, &ctx->mgb->nan, sizeof(int)));
        return fail(ctx, APIC_EDEVICE, "Poisson solve produced NaN");
    }
    if (cycles && !in_step) *cycles = b.max_cycles;
    return APIC_OK;
}

// Largest relative residual |D^-1 r| / |D^-1 b| of the grains solved, from the
// last convergence check.
int max_rel_residual(apic_ctx* ctx, int only, double& r) {
    const int G = (int)ctx->grains.size();
    std::vector<MGState> m(G);
    HIPCHK(ctx, hipMemcpy(m.data(), ctx->mgs, sizeof(MGState) * G, hipMemcpyDeviceToHost));
    r = 0.0;
    for (int g = 0; g < G; ++g)
        if (only < 0 || g == only) r = std::max(r, std::sqrt(m[g].last_r2 / (m[g].b2 + ctx->gdesc_h[g].bnd2 + 1e-300)));
    return APIC_OK;
}

// Boltzmann electrons: Newton's method on eq. (6) with n_e = exp(phi).  Each
// step linearises about the current phi (on every level, with the coarsest
// inverses formed again), runs V-cycles to the tolerance and limits the change
// of phi (damped Newton); the residual of a linearisation at its own starting
// point is the nonlinear residual, so the iteration ends when a step starts
// converged (or, solving to round-off, when that residual reaches round-off
// and stops falling).  In-step solves start from the extrapolated potential of
// the previous steps.
constexpr int MAX_NEWTON = 40;

int solve_newton(apic_ctx* ctx, double tol, int max_cycles, bool to_floor, int only, bool in_step, int* cycles) {
    if (in_step) {
        HIPCHK(ctx, launch_rho_rhs(ctx));
        HIPCHK(ctx, mg_extrapolate(ctx));
    }
    HIPCHK(ctx, launch_set_boundary(ctx));
    MGBatch b;
    int total = 0;
    double prev = HUGE_VAL;
    bool converged = false;
    for (int it = 0; it < MAX_NEWTON && !converged; ++it) {
        if (in_step) {
            // captured linearisation and start; then as many cycles as this
            // Newton step took in the previous solve before the state is read
            // (cycles of a converged grain do nothing on the device)
            TRY(run_phase(ctx, it == 0 ? G_NEWTON : G_NEWTON_NEXT, [&] {
                (void)newton_prepare(ctx, -1, it == 0);
                (void)mg_begin(ctx, tol, -1, true);
            }));
            const int pred = it < (int)ctx->newton_pred.size() ? std::min(ctx->newton_pred[it], max_cycles) : 0;
            for (int k = 0; k < pred; ++k) TRY(run_phase(ctx, G_VC, [&] { (void)mg_vcycle_launches(ctx, tol); }));
            TRY(read_batch(ctx, b));
            if (b.nan) break;
            if (b.pending == 0 && b.max_cycles == 0) {   // the step started converged
                converged = true;
                break;
            }
            while (b.pending > 0 && b.max_cycles < max_cycles) {
                TRY(run_phase(ctx, G_VC, [&] { (void)mg_vcycle_launches(ctx, tol); }));
                TRY(read_batch(ctx, b));
            }
            if ((int)ctx->newton_pred.size() <= it) ctx->newton_pred.resize(it + 1, 0);
            ctx->newton_pred[it] = b.max_cycles;
            HIPCHK(ctx, newton_limit(ctx, -1));
            total += b.max_cycles;
            continue;
        }
        HIPCHK(ctx, newton_prepare(ctx, only, it == 0));
        HIPCHK(ctx, mg_begin(ctx, tol, only, in_step));
        TRY(read_batch(ctx, b));
        if (b.nan) break;
        if (b.pending == 0) {
            converged = true;
            break;
        }
        double r0 = 0.0;
        TRY(max_rel_residual(ctx, only, r0));
        if (to_floor && (r0 <= 1e-13 || (it >= 3 && r0 < 1e-11 && r0 > 0.5 * prev))) {
            converged = true;
            break;
        }
        prev = r0;
        int launched = 0;
        double last = HUGE_VAL;
        while (b.pending > 0 && launched < max_cycles) {
            HIPCHK(ctx, mg_vcycle_launches(ctx, tol));
            ++launched;
            TRY(read_batch(ctx, b));
            if (to_floor) {
                double r = 0.0;
                TRY(max_rel_residual(ctx, only, r));
                if (launched >= 4 && r > 0.6 * last) break;
                last = r;
            }
        }
        HIPCHK(ctx, newton_limit(ctx, only));
        total += launched;
        if (b.nan) break;
    }
    if (b.nan) {
        HIPCHK(ctx, launch_fill(ctx, &ctx->mgb->nan, sizeof(int)));
        return fail(ctx, APIC_EDEVICE, "Poisson solve produced NaN");
    }
    if (!converged) return fail(ctx, APIC_EDEVICE, "Boltzmann-electron Newton iteration did not converge");
    if (cycles) *cycles = total;
    return APIC_OK;
}

int solve(apic_ctx* ctx, double tol, int max_cycles, bool to_floor, int only, bool in_step, int* cycles) {
    if (ctx->opts.boltzmann_electrons)
        return solve_newton(ctx, tol, max_cycles, to_floor, only, in_step, cycles);
    return solve_linear(ctx, tol, max_cycles, to_floor, only, in_step, cycles);
}

// Deposit the current particles of every grain and solve for phi.
int rebuild_fields(apic_ctx* ctx, double tol, int max_cycles, bool to_floor, int only) {
    HIPCHK(ctx, launch_clear_deposits(ctx));
    HIPCHK(ctx, launch_deposit(ctx));
    HIPCHK(ctx, launch_rho_rhs(ctx));
    int cyc = 0;
    TRY(solve(ctx, tol, max_cycles, to_floor, only, false, &cyc));
    HIPCHK(ctx, launch_gradient(ctx));
    for (size_t g = 0; g < ctx->grains.size(); ++g)
        if (only < 0 || (int)g == only) ctx->grains[g].field_stale = false;
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
        F(g.hist[s]);
        F(g.hist_off[s]);
        F(g.seg[s]);
        g.dep[s] = nullptr;
        g.hist[s] = g.hist_off[s] = g.seg[s] = nullptr;
    }
    F(g.ctr);
    F(g.vol);
    F(g.grad);
    F(g.rho);
    F(g.tally);
    F(g.tally_count);
    F(g.coarse_inv);
    for (auto& L : g.mg) {
        F(L.st);
        F(L.u);
        F(L.f);
        F(L.uT);
        F(L.fT);
        F(L.uprev);
        F(L.shift);
        F(L.uold);
    }
    g.mg.clear();
    g.ctr = nullptr;
}

void free_ctx(apic_ctx* ctx) {
    drop_graphs(ctx);
    for (auto& g : ctx->grains) free_grain(g);
    auto F = [](void* p) {
        if (p) (void)hipFree(p);
    };
    F(ctx->tasks);
    F(ctx->inj_block_task);
    F(ctx->chunk_prefix);
    F(ctx->gdesc);
    F(ctx->mgdesc);
    F(ctx->mgdesc_coarse);
    F(ctx->mgs);
    F(ctx->norm_part);
    F(ctx->mgb);
    if (ctx->mgb_host) (void)hipHostFree(ctx->mgb_host);
    for (auto& t : ctx->timers) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    if (ctx->side) (void)hipStreamSynchronize(ctx->side);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
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

// Smallest square power-of-two tile (at least 2^want cells) giving at most
// 8192 tiles on an n1 x n2 grid.
int tile_log2_for(int n1, int n2, int want) {
    int t = std::max(want, 2);
    while (((n1 + (1 << t) - 1) >> t) * ((n2 + (1 << t) - 1) >> t) > 8192) ++t;
    return t;
}

void set_tiles(GrainParams& gp, int t) {
    gp.tile_log2 = t;
    gp.ntx = (gp.n1 + (1 << t) - 1) >> t;
    gp.ntiles = gp.ntx * ((gp.n2 + (1 << t) - 1) >> t);
}

// Host part of a grain's set-up (no HIP calls; grains are set up in parallel).
struct HostSetup {
    std::vector<Stencil> levels;
    std::vector<double> inv;
    int max_dense = 600;        // largest level solved by the dense inverse
    int threads = 1;            // host threads for the inverse
    bool boltzmann = false;     // Newton term on every level: the coarsest inverse is formed on the device
    bool fe = false;            // conservative (finite-element) form on the finest level
    int rc = APIC_OK;
    std::string err;
};

// The coarsest level of a grain's hierarchy is solved by a dense inverse (one
// matrix-vector product per V-cycle, bandwidth-bound); every level above it
// costs ten latency-bound launches per cycle.  So the coarsest level is made as
// large as the ensemble's inverses allow: about 192 MB of them in total, at
// most 4400 nodes (65 x 65) and at least 600 per grain.
constexpr int DENSE_MAX_NODES = 4400;
// With Boltzmann electrons the coarsest operator changes with every Newton step
// and is inverted on the device, in one workgroup's LDS (BOLTZ_INV_MAX nodes).
int dense_limit(int n_grains) {
    const double per = 192.0 * (1 << 20) / (8.0 * n_grains);
    return std::max(600, std::min(DENSE_MAX_NODES, (int)std::sqrt(per)));
}

void host_setup(Grain& g, const apic_grain_cfg& c, int gi, HostSetup& hs) {
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
    set_tiles(gp, tile_log2_for(n1, n2, Schedule().tile_log2));

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
        if (n_real > 1e9) {
            hs.rc = APIC_ERANGE;
            hs.err = "injection rate too large";
            return;
        }
        g.inj_inc[s] = (uint64_t)std::llround(n_real * 4294967296.0);
        int64_t cap = a.capacity;
        if (cap == 0) cap = (int64_t)(1.5 * (double)a.n_macro) + 64 * (int64_t)std::ceil(n_real) + 4096;
        if (cap >= ((int64_t)1 << 30)) {   // the FP32 kernels address slots with 32-bit byte offsets
            hs.rc = APIC_ERANGE;
            hs.err = "particle capacity of 2^30 or more";
            return;
        }
        g.capacity[s] = cap;
        // sort workgroups: about 32k slots each, a power of two in [16, 1024]
        int sb = 16;
        while (sb < max_sort_blocks() && (int64_t)sb * 32768 < cap) sb <<= 1;
        g.sort_blocks[s] = sb;
    }

    // multigrid hierarchy: coarsen by two while both cell counts are even and
    // at least 8, and stop at the first level small enough for the dense
    // inverse.  The finest level itself is solved densely only when it is very
    // small: one product with a large inverse is less accurate than V-cycles
    // iterated on the FP64 residual, while on a correction level it is exact
    // enough.
    hs.levels.resize(1);
    if (hs.fe) fine_stencil_fe(n1, n2, c.x1_out, c.alpha, hs.levels[0]);
    else fine_stencil(n1, n2, c.x1_out, c.alpha, hs.levels[0]);
    const int fine_dense = std::min(600, hs.max_dense);
    while ((hs.levels.back().n1 + 1) * (hs.levels.back().n2 + 1) > (hs.levels.size() == 1 ? fine_dense : hs.max_dense) &&
           hs.levels.back().n1 % 2 == 0 &&
           hs.levels.back().n2 % 2 == 0 && std::min(hs.levels.back().n1, hs.levels.back().n2) / 2 >= 4) {
        Stencil cs;
        galerkin_coarse(hs.levels.back(), cs);
        hs.levels.push_back(std::move(cs));
    }
    const Stencil& last = hs.levels.back();
    const int m = (last.n1 + 1) * (last.n2 + 1);
    if (m > (hs.boltzmann ? BOLTZ_INV_MAX : DENSE_MAX_NODES)) {
        hs.rc = APIC_ERANGE;
        hs.err = hs.boltzmann ? "grid does not coarsen to 88 nodes for the Boltzmann-electron solve"
                              : "grid does not coarsen far enough for multigrid";
        return;
    }
    if (!hs.boltzmann) {
        std::vector<double> A;
        dense_matrix(last, A);
        if (!invert(A, m, hs.inv, hs.threads)) {
            hs.rc = APIC_EDEVICE;
            hs.err = "coarsest multigrid operator is singular";
            return;
        }
    }
    g.coarse_nodes = m;
    g.bnd_norm2 = boundary_coupling_norm2(hs.levels[0], c.phi_grain, c.phi_out);
}

// Device part of a grain's set-up.
int device_setup(apic_ctx* ctx, Grain& g, HostSetup& hs) {
    const bool split = split_mode(ctx);
    const size_t fsz = split ? 4 : 8;
    const int min_tile = tile_log2_for(g.gp.n1, g.gp.n2, 2);
    const int max_tiles = ((g.gp.n1 + (1 << min_tile) - 1) >> min_tile) * ((g.gp.n2 + (1 << min_tile) - 1) >> min_tile);
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
        const size_t hist_len = (size_t)max_tiles * g.sort_blocks[s];
        TRY(alloc_t(ctx, &g.hist[s], hist_len));
        TRY(alloc_t(ctx, &g.hist_off[s], hist_len + 1));
        TRY(alloc_t(ctx, &g.seg[s], hist_len / scan_seg_len() + 2));
        HIPCHK(ctx, launch_fill(ctx, g.dep[s], fsz * (size_t)g.nodes));
    }
    TRY(alloc_t(ctx, &g.ctr, 1));
    TRY(alloc_t(ctx, &g.vol, (size_t)g.nodes));
    TRY(dev_alloc(ctx, &g.grad, 2 * fsz * (size_t)g.nodes));
    TRY(alloc_t(ctx, &g.rho, (size_t)g.nodes));
    TRY(alloc_t(ctx, &g.tally, (size_t)5 * g.ns * g.gp.n_bins));
    TRY(alloc_t(ctx, &g.tally_count, (size_t)g.ns * g.gp.n_bins));
    HIPCHK(ctx, launch_fill(ctx, g.ctr, sizeof(DevCounters)));
    HIPCHK(ctx, launch_fill(ctx, g.tally, sizeof(double) * 5 * g.ns * g.gp.n_bins));
    HIPCHK(ctx, launch_fill(ctx, g.tally_count, sizeof(unsigned long long) * g.ns * g.gp.n_bins));
    HIPCHK(ctx, launch_fill(ctx, g.rho, sizeof(double) * g.nodes));
    HIPCHK(ctx, launch_fill(ctx, g.grad, 2 * fsz * (size_t)g.nodes));
    HIPCHK(ctx, hipMemcpyAsync(g.vol, g.vol_host.data(), sizeof(double) * g.nodes,
                               hipMemcpyHostToDevice, ctx->stream));
    // the dense inverse with rows padded to an even length (16-byte aligned rows)
    const size_t inv_pitch = (size_t)((g.coarse_nodes + 1) & ~1);
    TRY(alloc_t(ctx, &g.coarse_inv, (size_t)g.coarse_nodes * inv_pitch));
    HIPCHK(ctx, launch_fill(ctx, g.coarse_inv, sizeof(double) * g.coarse_nodes * inv_pitch));
    std::vector<double> stage;
    g.mg.resize(hs.levels.size());
    for (size_t l = 0; l < hs.levels.size(); ++l) {
        MGLevel& L = g.mg[l];
        L.n1 = hs.levels[l].n1;
        L.n2 = hs.levels[l].n2;
        L.nx = L.n1 + 1;
        L.nodes = L.nx * (L.n2 + 1);
        TRY(alloc_t(ctx, &L.u, (size_t)L.nodes));
        TRY(alloc_t(ctx, &L.f, (size_t)L.nodes));
        HIPCHK(ctx, launch_fill(ctx, L.u, sizeof(double) * L.nodes));
        HIPCHK(ctx, launch_fill(ctx, L.f, sizeof(double) * L.nodes));
        if (hs.boltzmann) {
            TRY(alloc_t(ctx, &L.shift, (size_t)L.nodes));
            HIPCHK(ctx, launch_fill(ctx, L.shift, sizeof(double) * L.nodes));
            if (l == 0) TRY(alloc_t(ctx, &L.uold, (size_t)L.nodes));
        }
        if (l == 0 && !hs.fe) {
            // the finest operator is evaluated at the nodes; its x2 sweeps may
            // use transposed copies of u and f
            TRY(alloc_t(ctx, &L.uT, (size_t)L.nodes));
            TRY(alloc_t(ctx, &L.fT, (size_t)L.nodes));
            TRY(alloc_t(ctx, &L.uprev, (size_t)L.nodes));
            continue;
        }
        if (l == 0) TRY(alloc_t(ctx, &L.uprev, (size_t)L.nodes));   // the stored finest level
        // node-major, ST_STRIDE doubles per node (the last one padding)
        TRY(alloc_t(ctx, &L.st, (size_t)ST_STRIDE * L.nodes));
        stage.assign((size_t)ST_STRIDE * L.nodes, 0.0);
        for (int k = 0; k < ST_COUNT; ++k)
            for (int o = 0; o < L.nodes; ++o) stage[(size_t)ST_STRIDE * o + k] = hs.levels[l].c[k][o];
        HIPCHK(ctx, hipMemcpy(L.st, stage.data(), sizeof(double) * stage.size(), hipMemcpyHostToDevice));
    }
    if (!hs.inv.empty())
        HIPCHK(ctx, hipMemcpy2DAsync(g.coarse_inv, sizeof(double) * inv_pitch, hs.inv.data(),
                                     sizeof(double) * g.coarse_nodes, sizeof(double) * g.coarse_nodes,
                                     g.coarse_nodes, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return APIC_OK;
}

// Per-task view of the ensemble for the particle kernels.
void fill_tasks(apic_ctx* ctx) {
    ctx->tasks_h.clear();
    ctx->inj_blocks = 0;
    ctx->max_ntiles = 0;
    ctx->max_sort_blocks = 0;
    ctx->max_segs = 1;
    for (size_t gi = 0; gi < ctx->grains.size(); ++gi) {
        Grain& g = ctx->grains[gi];
        double sig_max = 0.0;
        for (int s = 0; s < g.ns; ++s) sig_max = std::max(sig_max, g.sp[s].sigma);
        for (int s = 0; s < g.ns; ++s) {
            PushTask t;
            std::memset(&t, 0, sizeof(t));
            t.gp = g.gp;
            t.sp = g.sp[s];
            t.buf[0] = g.buf[s][0];
            t.buf[1] = g.buf[s][1];
            t.grad = g.grad;
            t.dep = g.dep[s];
            t.ctr = g.ctr;
            t.tally = g.tally;
            t.tally_count = g.tally_count;
            t.hist = g.hist[s];
            t.hist_off = g.hist_off[s];
            t.seg = g.seg[s];
            t.capacity = g.capacity[s];
            t.inj_inc = g.inj_inc[s];
            t.s = s;
            t.ns = g.ns;
            t.grain = (int)gi;
            t.sort_blocks = g.sort_blocks[s];
            // a species k times slower (thermal speed) than the grain's fastest
            // drifts out of its tiles k times later: sorted every
            // sort_every * 2^level steps, 2^level <= k, at most 16x apart
            t.sort_level = 0;
            while (t.sort_level + 1 < SORT_LEVELS && g.sp[s].sigma * (2 << t.sort_level) <= sig_max)
                ++t.sort_level;
            // a step injects at most floor(inj_inc / 2^32) + 1 particles; the
            // tasks' injection workgroups are laid end to end
            t.inj_block0 = ctx->inj_blocks;
            ctx->inj_blocks += (int)((((g.inj_inc[s] >> 32) + 1) + INJ_PER_BLOCK - 1) / INJ_PER_BLOCK);
            ctx->tasks_h.push_back(t);
            ctx->max_ntiles = std::max(ctx->max_ntiles, g.gp.ntiles);
            ctx->max_sort_blocks = std::max(ctx->max_sort_blocks, g.sort_blocks[s]);
            const int64_t len = (int64_t)g.gp.ntiles * g.sort_blocks[s];
            ctx->max_segs = std::max<int>(ctx->max_segs, (int)((len + scan_seg_len() - 1) / scan_seg_len()));
        }
    }
    ctx->ntasks = (int)ctx->tasks_h.size();
}

int upload_tasks(apic_ctx* ctx) {
    fill_tasks(ctx);
    HIPCHK(ctx, hipMemcpyAsync(ctx->tasks, ctx->tasks_h.data(), sizeof(PushTask) * ctx->ntasks,
                               hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return APIC_OK;
}

// Descriptor tables of the ensemble (after every grain is set up).
int build_tables(apic_ctx* ctx) {
    const int G = (int)ctx->grains.size();
    fill_tasks(ctx);
    TRY(alloc_t(ctx, &ctx->tasks, ctx->tasks_h.size()));
    TRY(alloc_t(ctx, &ctx->chunk_prefix, ctx->tasks_h.size() + 1));
    TRY(upload_tasks(ctx));
    {
        std::vector<int> bt(std::max(ctx->inj_blocks, 1), 0);
        for (int t = 0; t < ctx->ntasks; ++t) {
            const int end = t + 1 < ctx->ntasks ? ctx->tasks_h[t + 1].inj_block0 : ctx->inj_blocks;
            for (int b = ctx->tasks_h[t].inj_block0; b < end; ++b) bt[b] = t;
        }
        TRY(alloc_t(ctx, &ctx->inj_block_task, bt.size()));
        HIPCHK(ctx, hipMemcpy(ctx->inj_block_task, bt.data(), sizeof(int) * bt.size(), hipMemcpyHostToDevice));
    }

    ctx->gdesc_h.assign(G, GrainDesc());
    ctx->n_levels = 0;
    ctx->max_nodes = ctx->max_n1 = ctx->max_n2 = 0;
    for (int gi = 0; gi < G; ++gi) {
        Grain& g = ctx->grains[gi];
        GrainDesc& d = ctx->gdesc_h[gi];
        std::memset(&d, 0, sizeof(d));
        d.n1 = g.gp.n1;
        d.n2 = g.gp.n2;
        d.nx = g.gp.nx;
        d.nodes = g.nodes;
        d.ns = g.ns;
        d.inv_h1 = g.gp.inv_h1;
        d.inv_h2 = g.gp.inv_h2;
        d.h2 = g.gp.h2;
        d.alpha = g.gp.alpha;
        d.rhs_scale = -1.0 / (g.gp.kappa * g.gp.kappa);
        d.phi_grain = g.cfg.phi_grain;
        d.phi_out = g.cfg.phi_out;
        d.fe = ctx->opts.conservative_poisson != 0;
        for (int s = 0; s < g.ns; ++s) {
            d.cw[s] = g.sp[s].q * g.sp[s].w;
            d.dep[s] = g.dep[s];
        }
        d.bnd2 = g.bnd_norm2;
        d.vol = g.vol;
        d.rho = g.rho;
        d.u = g.mg[0].u;
        d.f = g.mg[0].f;
        d.grad = g.grad;
        d.ctr = g.ctr;
        ctx->n_levels = std::max(ctx->n_levels, (int)g.mg.size());
        ctx->max_nodes = std::max(ctx->max_nodes, g.nodes);
        ctx->max_n1 = std::max(ctx->max_n1, g.gp.n1);
        ctx->max_n2 = std::max(ctx->max_n2, g.gp.n2);
    }
    // the finest levels' u and f beyond half of the L2 caches (8 x 4 MB): x2
    // sweeps on transposed copies
    size_t fine_bytes = 0;
    for (auto& g : ctx->grains) fine_bytes += 16 * (size_t)g.nodes;
    // (the conservative form's finest level is stored: no transposed sweeps)
    ctx->x2_transposed = fine_bytes > ((size_t)16 << 20) && !ctx->opts.conservative_poisson;
    TRY(alloc_t(ctx, &ctx->gdesc, (size_t)G));
    HIPCHK(ctx, hipMemcpy(ctx->gdesc, ctx->gdesc_h.data(), sizeof(GrainDesc) * G, hipMemcpyHostToDevice));

    const int NL = ctx->n_levels;
    ctx->mgdesc_h.assign((size_t)NL * G, MGDesc());
    ctx->lvl_max_n1.assign(NL, 0);
    ctx->lvl_max_n2.assign(NL, 0);
    ctx->lvl_max_nodes.assign(NL, 0);
    ctx->lvl_lines_x2.assign(NL, 0);
    ctx->lvl_lines_x1.assign(NL, 0);
    ctx->lvl_max_m.assign(NL, 0);
    for (int l = 0; l < NL; ++l)
        for (int gi = 0; gi < G; ++gi) {
            MGDesc& d = ctx->mgdesc_h[(size_t)l * G + gi];
            std::memset(&d, 0, sizeof(d));
            Grain& g = ctx->grains[gi];
            if (l >= (int)g.mg.size()) continue;
            const MGLevel& L = g.mg[l];
            d.n1 = L.n1;
            d.n2 = L.n2;
            d.nx = L.nx;
            d.nodes = L.nodes;
            d.coarsest = l + 1 == (int)g.mg.size();
            d.m = d.coarsest ? g.coarse_nodes : 0;
            d.st = L.st;
            d.alpha = g.gp.alpha;
            d.h1 = g.gp.h1 * (double)(1 << l);
            d.h2 = g.gp.h2 * (double)(1 << l);
            d.ih1sq = 1.0 / (d.h1 * d.h1);
            d.ih2sq = 1.0 / (d.h2 * d.h2);
            d.i2h2 = 1.0 / (2.0 * d.h2);
            d.i4h1h2 = 1.0 / (4.0 * d.h1 * d.h2);
            d.u = L.u;
            d.f = L.f;
            d.uT = L.uT;
            d.fT = L.fT;
            d.uprev = L.uprev;
            d.inv = d.coarsest ? g.coarse_inv : nullptr;
            d.shift = L.shift;
            d.uold = L.uold;
            ctx->lvl_max_nodes[l] = std::max(ctx->lvl_max_nodes[l], L.nodes);
            if (!d.coarsest) {
                ctx->lvl_max_n1[l] = std::max(ctx->lvl_max_n1[l], L.n1);
                ctx->lvl_max_n2[l] = std::max(ctx->lvl_max_n2[l], L.n2);
                ctx->lvl_lines_x2[l] += L.n1 / 2;
                ctx->lvl_lines_x1[l] += L.n2 / 2;
            } else {
                ctx->lvl_max_m[l] = std::max(ctx->lvl_max_m[l], d.m);
            }
        }
    TRY(alloc_t(ctx, &ctx->mgdesc, ctx->mgdesc_h.size()));
    HIPCHK(ctx, hipMemcpy(ctx->mgdesc, ctx->mgdesc_h.data(), sizeof(MGDesc) * ctx->mgdesc_h.size(),
                          hipMemcpyHostToDevice));
    // each grain's coarsest level, so that one launch solves every grain's dense system
    std::vector<MGDesc> coarse_h(G);
    ctx->max_coarse_m = 0;
    for (int gi = 0; gi < G; ++gi) {
        const int l = (int)ctx->grains[gi].mg.size() - 1;
        coarse_h[gi] = ctx->mgdesc_h[(size_t)l * G + gi];
        ctx->max_coarse_m = std::max(ctx->max_coarse_m, coarse_h[gi].m);
    }
    TRY(alloc_t(ctx, &ctx->mgdesc_coarse, (size_t)G));
    HIPCHK(ctx, hipMemcpy(ctx->mgdesc_coarse, coarse_h.data(), sizeof(MGDesc) * G, hipMemcpyHostToDevice));
    TRY(alloc_t(ctx, &ctx->mgs, (size_t)G));
    TRY(alloc_t(ctx, &ctx->norm_part, (size_t)2 * G * ((ctx->lvl_max_nodes[0] + 255) / 256)));
    TRY(alloc_t(ctx, &ctx->mgb, 1));
    HIPCHK(ctx, launch_fill(ctx, ctx->mgs, sizeof(MGState) * G));
    HIPCHK(ctx, launch_fill(ctx, ctx->mgb, sizeof(MGBatch)));
    HIPCHK(ctx, hipHostMalloc((void**)&ctx->mgb_host, sizeof(MGBatch), hipHostMallocDefault));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return APIC_OK;
}

// Sort tiles of every grain for a preferred tile edge 2^t (each grain caps its
// tile count at 8192); the graphs depend on the tile counts and are rebuilt.
int apply_tiles(apic_ctx* ctx, int t) {
    for (auto& g : ctx->grains) set_tiles(g.gp, tile_log2_for(g.gp.n1, g.gp.n2, t));
    ctx->sched.tile_log2 = t;
    drop_graphs(ctx);
    return upload_tasks(ctx);
}

// Sort of the tasks whose sort level is at most `level` (all by default).
int sort_all(apic_ctx* ctx, int level = SORT_LEVELS - 1) {
    TRY(run_phase(ctx, G_SORT + level, [&] { (void)launch_sort(ctx, 0, ctx->ntasks, level); }));
    for (const PushTask& t : ctx->tasks_h)
        if (t.sort_level <= level) ctx->grains[t.grain].cur[t.s] ^= 1;
    return APIC_OK;
}

// sort of one (grain, species) task, outside the step graphs
int sort_one(apic_ctx* ctx, int grain, int s) {
    int t = 0;
    while (t < ctx->ntasks && !(ctx->tasks_h[t].grain == grain && ctx->tasks_h[t].s == s)) ++t;
    if (t == ctx->ntasks) return fail(ctx, APIC_EINVAL, "no such task");
    HIPCHK(ctx, launch_sort(ctx, t, 1));
    ctx->grains[grain].cur[s] = 1 - ctx->grains[grain].cur[s];
    return APIC_OK;
}

int push_phase(apic_ctx* ctx) {
    const bool frozen = frozen_mode(ctx);
    return run_phase(ctx, G_PUSH, [&] {
        if (!frozen) (void)launch_clear_deposits(ctx);
        (void)launch_push(ctx, !frozen);
    });
}

int sort_every(const apic_ctx* ctx) {
    if (ctx->opts.sort_every > 0 && !ctx->opts.autotune) return ctx->opts.sort_every;
    return ctx->sched.sort_every;
}

// One step of every grain: push (gather, kick, drift, boundaries, deposit),
// injection, charge density, FP64 solve, nodal gradient, grain force; a sort
// every sort_every steps.
// The sort of a step runs on the side stream, overlapped with the field solve
// of the same step (the solve needs only the deposit, the sort only the
// particles); the main stream waits for it at the end of the step.
int sort_all_async(apic_ctx* ctx, int level) {
    HIPCHK(ctx, hipEventRecord(ctx->ev_fork, ctx->stream));
    HIPCHK(ctx, hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0));
    hipStream_t main = ctx->stream;
    ctx->stream = ctx->side;
    int rc;
    {
        Timer t(ctx, 2);
        rc = sort_all(ctx, level);
    }
    ctx->stream = main;
    TRY(rc);
    HIPCHK(ctx, hipEventRecord(ctx->ev_join, ctx->side));
    return APIC_OK;
}

// One step of every grain: push (gather, kick, drift, boundaries, deposit),
// injection, charge density, FP64 solve, nodal gradient, grain force; a sort
// every sort_every steps.
int do_step(apic_ctx* ctx) {
    const bool frozen = frozen_mode(ctx);
    bool stale = false;
    for (auto& g : ctx->grains) stale |= g.field_stale;
    if (stale && !frozen) TRY(rebuild_fields(ctx, step_tol(ctx), step_max_cycles(ctx), false, -1));
    for (auto& g : ctx->grains) g.field_stale = false;
    {
        Timer t(ctx, 0);
        TRY(push_phase(ctx));
        if (ctx->profiling) ++ctx->push_launches;
    }
    if (ctx->opts.inject) {
        Timer t(ctx, 1);
        TRY(run_phase(ctx, G_INJ, [&] { (void)launch_inject(ctx, !frozen); }));
    }
    const uint64_t step = ctx->grains[0].step_index + 1;
    const uint64_t se = (uint64_t)sort_every(ctx);
    const bool sort_now = step % se == 0;
    if (sort_now) {
        // sort level: the tasks due at this multiple of sort_every
        int level = 0;
        for (uint64_t k = step / se; level + 1 < SORT_LEVELS && (k & 1) == 0; k >>= 1) ++level;
        TRY(sort_all_async(ctx, level));
    }
    {
        Timer t(ctx, 3);
        if (!frozen) {
            int cyc = 0;
            TRY(solve(ctx, step_tol(ctx), step_max_cycles(ctx), false, -1, true, &cyc));
            if (ctx->profiling) ctx->timed_mg_cycles += cyc;
        }
        TRY(run_phase(ctx, G_POST, [&] {
            if (!frozen) (void)launch_gradient(ctx);
            (void)launch_grain_force(ctx);
        }));
    }
    if (sort_now) HIPCHK(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0));
    for (auto& g : ctx->grains) g.step_index++;
    if (ctx->profiling) ++ctx->timed_steps;
    return APIC_OK;
}

// ---------------------------------------------------------------- autotuner
// Chooses the launch schedule on the first steps of the run, timing real steps
// with HIP events (every candidate gives the same particles up to the order of
// the deposit sums):
//   1. persistent push workgroups per CU: each candidate times one push;
//   2. sort tile edge: each candidate sorts, then times the next push;
//   3. sort interval: after a sort, the pushes of the following steps are
//      timed; the interval k minimises (sort + sum of the k pushes) / k.
struct TuneClock {
    hipEvent_t a = nullptr, b = nullptr;
    TuneClock() {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    ~TuneClock() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

template <typename F>
int timed(apic_ctx* ctx, TuneClock& c, F fn, float* ms) {
    HIPCHK(ctx, hipEventRecord(c.a, ctx->stream));
    TRY(fn());
    HIPCHK(ctx, hipEventRecord(c.b, ctx->stream));
    HIPCHK(ctx, hipEventSynchronize(c.b));
    HIPCHK(ctx, hipEventElapsedTime(ms, c.a, c.b));
    return APIC_OK;
}

// the rest of a step after the push (injection, field, force), untimed
int finish_step(apic_ctx* ctx) {
    const bool frozen = frozen_mode(ctx);
    if (ctx->opts.inject) TRY(run_phase(ctx, G_INJ, [&] { (void)launch_inject(ctx, !frozen); }));
    if (!frozen) TRY(solve(ctx, step_tol(ctx), step_max_cycles(ctx), false, -1, true, nullptr));
    TRY(run_phase(ctx, G_POST, [&] {
        if (!frozen) (void)launch_gradient(ctx);
        (void)launch_grain_force(ctx);
    }));
    for (auto& g : ctx->grains) g.step_index++;
    return APIC_OK;
}

// Runs tuning steps (each a real step) while *left > 0; returns when tuning is
// complete or the steps are used up (it resumes on the next call).
int autotune(apic_ctx* ctx, int64_t* left) {
    TuneState* st = &ctx->tune;
    const int resident = push_resident_per_cu(ctx);   // candidates 1 .. resident workgroups per CU
    const int tile_cand[] = {2, 3, 4};
    TuneClock clk;
    ctx->tuning = true;
    drop_graphs(ctx);
    bool stale = false;
    for (auto& g : ctx->grains) stale |= g.field_stale;
    if (stale && !frozen_mode(ctx)) TRY(rebuild_fields(ctx, step_tol(ctx), step_max_cycles(ctx), false, -1));
    for (auto& g : ctx->grains) g.field_stale = false;
    while (*left > 0 && !ctx->tuned) {
        float ms = 0;
        if (st->phase == 0) {
            ctx->sched.push_wg_per_cu = resident - st->idx;
            TRY(timed(ctx, clk, [&] { return push_phase(ctx); }, &ms));
            if (ms < st->best) {
                st->best = ms;
                st->best_val = resident - st->idx;
            }
            if (++st->idx == resident) {
                ctx->sched.push_wg_per_cu = st->best_val;
                drop_graphs(ctx);
                st->phase = 1;
                st->idx = 0;
                st->best = 1e30f;
            }
        } else if (st->phase == 1) {
            TRY(apply_tiles(ctx, tile_cand[st->idx]));
            float sms = 0;
            TRY(timed(ctx, clk, [&] { return sort_all(ctx); }, &sms));
            TRY(timed(ctx, clk, [&] { return push_phase(ctx); }, &ms));
            if (ms + sms / 8 < st->best) {
                st->best = ms + sms / 8;
                st->best_val = tile_cand[st->idx];
                st->sort_ms = sms;
            }
            if (++st->idx == 3) {
                TRY(apply_tiles(ctx, st->best_val));
                st->phase = 2;
                st->idx = 0;
            }
        } else {
            if (st->idx == 0) TRY(timed(ctx, clk, [&] { return sort_all(ctx); }, &st->sort_ms));
            TRY(timed(ctx, clk, [&] { return push_phase(ctx); }, &ms));
            st->push_after.push_back(ms);
            if (++st->idx == 16) {
                // the slower species are sorted 2^level times less often:
                // the sort's cost per interval is the share of the particles
                // sorted at every one of them
                double all = 0.0, due = 0.0;
                for (const PushTask& t : ctx->tasks_h) {
                    all += (double)t.capacity;
                    due += (double)t.capacity / (double)(1 << t.sort_level);
                }
                const double sort_share = all > 0.0 ? due / all : 1.0;
                double best = 1e30, sum = 0;
                int k_best = 8;
                for (int k = 1; k <= 16; ++k) {
                    sum += st->push_after[k - 1];
                    const double per = (st->sort_ms * sort_share + sum) / k;
                    if (per < best) {
                        best = per;
                        k_best = k;
                    }
                }
                ctx->sched.sort_every = k_best;
                ctx->tuned = true;
            }
        }
        TRY(finish_step(ctx));
        --*left;
        // the last phase left the particles 16 pushes out of order: the run
        // continues from a fresh sort of every task
        if (ctx->tuned) TRY(sort_all(ctx));
    }
    ctx->tuning = false;
    return APIC_OK;
}

int check_overflow(apic_ctx* ctx) {
    for (auto& g : ctx->grains) {
        uint32_t of = 0;
        HIPCHK(ctx, hipMemcpyAsync(&of, &g.ctr->overflow, sizeof(of), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        if (of) return fail(ctx, APIC_ENOMEM, "particle capacity exceeded during injection");
    }
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
    if (ctx->opts.boltzmann_electrons && ctx->opts.conservative_poisson) {
        delete ctx;
        return fail(nullptr, APIC_EINVAL, "conservative_poisson is not available with boltzmann_electrons");
    }
    if (ctx->opts.sort_every > 0) ctx->sched.sort_every = ctx->opts.sort_every;
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
    // side stream (default priority) for the sort overlapped with the solve
    e = hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming);
    if (e != hipSuccess) {
        g_init_error = std::string("hipStreamCreate: ") + hipGetErrorString(e);
        free_ctx(ctx);
        delete ctx;
        return APIC_EDEVICE;
    }
    ctx->grains.resize(n_grains);
    // host tables of all grains in parallel, then the device side in order
    std::vector<HostSetup> hs(n_grains);
    {
        const int hw = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
        const int nt = std::min(n_grains, hw);
        for (auto& h : hs) {
            h.boltzmann = ctx->opts.boltzmann_electrons != 0;
            h.fe = ctx->opts.conservative_poisson != 0;
            h.max_dense = h.boltzmann ? BOLTZ_INV_MAX : dense_limit(n_grains);
            h.threads = std::max(1, hw / nt);
        }
        std::vector<std::thread> pool;
        for (int w = 0; w < nt; ++w)
            pool.emplace_back([&, w] {
                for (int i = w; i < n_grains; i += nt) host_setup(ctx->grains[i], cfgs[i], i, hs[i]);
            });
        for (auto& t : pool) t.join();
    }
    int rc = APIC_OK;
    for (int i = 0; i < n_grains && rc == APIC_OK; ++i)
        if (hs[i].rc != APIC_OK) rc = fail(ctx, hs[i].rc, "grain " + std::to_string(i) + ": " + hs[i].err);
    for (int i = 0; i < n_grains && rc == APIC_OK; ++i) {
        rc = device_setup(ctx, ctx->grains[i], hs[i]);
        hs[i] = HostSetup();
    }
    if (rc == APIC_OK) rc = build_tables(ctx);
    if (rc == APIC_OK && noalloc_scratch(&ctx->scratch) != hipSuccess) {
        // only apic_inject_noalloc needs it; it reports the failure
        (void)hipGetLastError();
        ctx->scratch = nullptr;
    }
    if (rc == APIC_OK) {
        // vacuum field until particles are loaded
        rc = rebuild_fields(ctx, 1e-15, 100, true, -1);
        for (auto& g : ctx->grains) g.field_stale = true;
    }
    if (rc != APIC_OK) {
        g_init_error = ctx->err;
        free_ctx(ctx);
        delete ctx;
        return rc;
    }
    *out = ctx;
    return APIC_OK;
}

}  // extern "C"

namespace {

// Host-side check of explicit particles, before any device work.
int check_particles(apic_ctx* ctx, const Grain& g, int64_t count, const double* x1, const double* x2,
                    const double* vR, const double* vZ, const double* vTheta) {
    for (int64_t k = 0; k < count; ++k) {
        if (!(x1[k] > -1.0 && x1[k] < g.cfg.x1_out && x2[k] >= -1.0 && x2[k] <= 1.0))
            return fail(ctx, APIC_EINVAL, "particle " + std::to_string(k) +
                                              " outside the domain (-1 < x1 < x1_out, |x2| <= 1)");
        if (!(std::isfinite(vR[k]) && std::isfinite(vZ[k]) && std::isfinite(vTheta[k])))
            return fail(ctx, APIC_EINVAL, "particle " + std::to_string(k) + " has a non-finite velocity");
    }
    return APIC_OK;
}

// Explicit particles through a device staging area of 5 * count doubles
// (stage) and one flag word (bad): host -> staging copies, then k_set writes
// them into the species' current buffer in its storage form.
int upload_particles(apic_ctx* ctx, Grain& g, int s, int64_t count, const double* const src[5], double* stage,
                     int* bad) {
    hipError_t e = hipSuccess;
    for (int k = 0; k < 5 && e == hipSuccess; ++k)
        e = hipMemcpyAsync(stage + (size_t)k * count, src[k], sizeof(double) * count, hipMemcpyHostToDevice,
                           ctx->stream);
    if (e == hipSuccess) e = launch_fill(ctx, bad, sizeof(int));
    if (e == hipSuccess)
        e = launch_set_particles(ctx, g, s, count, stage, stage + count, stage + 2 * count, stage + 3 * count,
                                 stage + 4 * count, bad);
    int hbad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail(ctx, APIC_EDEVICE, std::string("apic_inject: ") + hipGetErrorString(e));
    if (hbad) return fail(ctx, APIC_EINVAL, "particle outside the domain (-1 < x1 < x1_out, |x2| <= 1)");
    return APIC_OK;
}

// After a species' particles are set: its counters restart with the new
// population, its tallies are cleared, it is sorted, and the field is due.
int finish_inject(apic_ctx* ctx, int grain, int s, int64_t count) {
    Grain& g = ctx->grains[grain];
    DevCounters h;
    HIPCHK(ctx, hipMemcpyAsync(&h, g.ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    h.n[s] = count;
    h.injected[s] = (uint64_t)count;
    h.absorbed[s] = 0;
    h.escaped[s] = 0;
    h.pushed[s] = 0;
    h.next_id[s] = (uint32_t)count;
    h.cur[s] = 0;
    HIPCHK(ctx, hipMemcpyAsync(g.ctr, &h, sizeof(DevCounters), hipMemcpyHostToDevice, ctx->stream));
    for (int k = 0; k < 5; ++k)
        HIPCHK(ctx, launch_fill(ctx, g.tally + ((size_t)k * g.ns + s) * g.gp.n_bins,
                                sizeof(double) * g.gp.n_bins));
    HIPCHK(ctx, launch_fill(ctx, g.tally_count + (size_t)s * g.gp.n_bins,
                            sizeof(unsigned long long) * g.gp.n_bins));
    TRY(sort_one(ctx, grain, s));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    g.field_stale = true;
    g.loaded[s] = true;
    return APIC_OK;
}

}  // namespace

extern "C" {

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
    if (!load) TRY(check_particles(ctx, g, count, x1, x2, vR, vZ, vTheta));
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
        const int rc = upload_particles(ctx, g, s, count, src, tmp, bad);
        (void)hipFree(tmp);
        (void)hipFree(bad);
        TRY(rc);
    }
    return finish_inject(ctx, grain, s, count);
}

int apic_inject_noalloc(apic_ctx* ctx, int32_t grain, int32_t species, int64_t n, const double* x1,
                        const double* x2, const double* vR, const double* vZ, const double* vTheta) {
    TRY(check_grain(ctx, grain));
    Grain& g = ctx->grains[grain];
    if (species < 0 || species >= g.ns) return fail(ctx, APIC_EINVAL, "species index out of range");
    if (n < 0 || n > NOALLOC_MAX_PARTICLES)
        return fail(ctx, APIC_EINVAL, "apic_inject_noalloc takes 0 to " + std::to_string(NOALLOC_MAX_PARTICLES) +
                                          " particles per call");
    if (n > 0 && !(x1 && x2 && vR && vZ && vTheta)) return fail(ctx, APIC_EINVAL, "particle arrays must be non-NULL");
    if (n > g.capacity[species]) return fail(ctx, APIC_ENOMEM, "particle count exceeds the species capacity");
    if (!ctx->scratch) return fail(ctx, APIC_EDEVICE, "the static staging array was not found on this device");
    TRY(check_particles(ctx, g, n, x1, x2, vR, vZ, vTheta));
    g.cur[species] = 0;
    if (n > 0) {
        const double* src[5] = {x1, x2, vR, vZ, vTheta};
        TRY(upload_particles(ctx, g, species, n, src, ctx->scratch,
                             reinterpret_cast<int*>(ctx->scratch + 5 * NOALLOC_MAX_PARTICLES)));
    }
    return finish_inject(ctx, grain, species, n);
}

int apic_step(apic_ctx* ctx, int64_t n_steps) {
    if (!ctx) return fail(nullptr, APIC_EINVAL, "null context");
    if (n_steps < 0) return fail(ctx, APIC_EINVAL, "n_steps < 0");
    int64_t left = n_steps;
    if (ctx->opts.inject && n_steps > 0)
        for (auto& g : ctx->grains)
            for (int s = 0; s < g.ns; ++s) g.loaded[s] = true;
    if (ctx->opts.autotune && !ctx->tuned && left > 0) TRY(autotune(ctx, &left));
    for (int64_t k = 0; k < left; ++k) TRY(do_step(ctx));
    if (n_steps > 0) TRY(check_overflow(ctx));
    return APIC_OK;
}

int apic_solve_poisson(apic_ctx* ctx, int32_t grain, const double* rho, double* phi_out) {
    TRY(check_grain(ctx, grain));
    Grain& g = ctx->grains[grain];
    if (rho) {
        HIPCHK(ctx, hipMemcpyAsync(g.rho, rho, sizeof(double) * g.nodes, hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(ctx, launch_rhs_from_rho(ctx, grain));
        TRY(solve(ctx, 1e-15, 100, true, grain, false, nullptr));
        HIPCHK(ctx, launch_gradient(ctx));
        g.field_stale = false;
    } else {
        TRY(rebuild_fields(ctx, 1e-15, 100, true, grain));
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
    out->unconverged_solves = g.unconverged;
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
    if (!g.loaded[species])
        return fail(ctx, APIC_ESTATE, "species " + std::to_string(species) +
                                          " holds no particles: load them with apic_inject (or step with injection) first");
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
    // order by id: ids are unique and dense (load indices, then the injection
    // counter), so a placement table over [min, max] sorts in linear time; a
    // sparse or repeated id range falls back to a comparison sort
    std::vector<int64_t> order;
    bool placed = false;
    if (found > 0) {
        const auto mm = std::minmax_element(hid.begin(), hid.begin() + (ptrdiff_t)found);
        const int64_t lo = *mm.first, span = *mm.second - lo + 1;
        if (span <= 4 * (int64_t)found + 1024) {
            std::vector<int64_t> at((size_t)span, -1);
            placed = true;
            for (size_t k = 0; k < found && placed; ++k) {
                int64_t& a = at[(size_t)(hid[k] - lo)];
                if (a >= 0) placed = false;
                a = (int64_t)k;
            }
            if (placed) {
                order.reserve(found);
                for (int64_t a : at)
                    if (a >= 0) order.push_back(a);
            }
        }
    }
    if (!placed) {
        order.resize(found);
        std::iota(order.begin(), order.end(), 0);
        std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return hid[a] < hid[b]; });
    }
    double* dst[5] = {x1, x2, vR, vZ, vTheta};
    for (size_t k = 0; k < found; ++k) {
        const size_t o = (size_t)order[k];
        for (int c = 0; c < 5; ++c) dst[c][k] = hx[(size_t)c * m + o];
        if (id) id[k] = hid[o];
    }
    return APIC_OK;
}

int apic_surface_field(apic_ctx* ctx, int32_t grain, double* E_n) {
    TRY(check_grain(ctx, grain));
    if (!E_n) return fail(ctx, APIC_EINVAL, "E_n is NULL");
    const int n = ctx->grains[grain].gp.n2 + 1;
    double* d = nullptr;
    TRY(alloc_t(ctx, &d, (size_t)n));
    hipError_t e = launch_surface_field(ctx, grain, d);
    if (e == hipSuccess) e = hipMemcpyAsync(E_n, d, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(ctx, APIC_EDEVICE, std::string("apic_surface_field: ") + hipGetErrorString(e));
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
    ctx->profiled |= ctx->profiling;
    return APIC_OK;
}

int apic_timing(apic_ctx* ctx, apic_kernel_times* out) {
    if (!ctx || !out) return fail(ctx, APIC_EINVAL, "null argument");
    if (!ctx->profiling && !ctx->profiled)
        return fail(ctx, APIC_ESTATE, "timing was never enabled: call apic_set_profiling(ctx, 1) first");
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

int apic_schedule(apic_ctx* ctx, apic_sched* out) {
    if (!ctx || !out) return fail(ctx, APIC_EINVAL, "null argument");
    out->push_wg_per_cu = std::min(ctx->sched.push_wg_per_cu, push_resident_per_cu(ctx));
    out->tile_log2 = ctx->sched.tile_log2;
    out->sort_every = sort_every(ctx);
    out->tuned = ctx->tuned ? 1 : 0;
    return APIC_OK;
}

int apic_free(apic_ctx* ctx) {
    if (!ctx) return APIC_OK;
    (void)hipStreamSynchronize(ctx->stream);
    free_ctx(ctx);
    delete ctx;
    return APIC_OK;
}

const char* apic_last_error(const apic_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

}  // extern "C"
