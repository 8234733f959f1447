// Internal structures of the APIC context and the launchers of its kernels.
//
// A context holds an ensemble of grains.  Every grain owns its grid, species,
// particle buffers, multigrid hierarchy and counters; the kernels of one step
// run over all grains at once from descriptor tables in device memory:
//   PushTask  -- one per (grain, species): particle buffers and parameters,
//                used by the push, deposit, injection and sort kernels;
//   GrainDesc -- one per grain: node arrays of the field kernels;
//   MGDesc    -- one per (level, grain): the multigrid level arrays.
// All per-step state (slot counts, current buffer, injection accumulator, step
// index, multigrid convergence) lives on the device, so a step is a fixed
// launch sequence that is captured into HIP graphs and replayed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "apic.h"
#include "host_setup.h"

namespace apic {

constexpr int INJ_BLOCK = 256;                  // threads per injection workgroup
constexpr int INJ_PER_BLOCK = 4 * INJ_BLOCK;    // particles per injection workgroup

// Per-species parameters seen by the kernels.
struct SpeciesParams {
    double q, m, T, w;          // charge (e), mass (me), temperature (Te), weight
    double e_bind;
    double qm_half;             // (q/m) kappa dt / 2        (electric half kick)
    double rot_c, rot_s;        // Boris rotation cos/sin of 2 atan(omega dt / 2)
    double rot_cm1;             // cos - 1 of that angle, without cancellation
    double sigma;               // thermal speed sqrt(T/m)
};

// Per-grain parameters seen by the kernels.
struct GrainParams {
    int n1, n2, nx, n_bins;     // nx = n1 + 1
    double alpha, x1_out, h1, h2, inv_h1, inv_h2;
    double step;                // kappa dt: displacement per unit velocity per step
    double kappa, dt;
    double r_grain_max;         // largest radius of the grain surface
    double M_vol, M_area;       // rejection bounds for loading / injection
    uint32_t key0, key1;        // Philox key
    int tile_log2, ntx, ntiles; // sort tiles: 2^tile_log2 cells square, ntx per row
};

// Device counters and per-step state of one grain (one allocation, zeroed at init).
struct DevCounters {
    int64_t n[APIC_MAX_SPECIES];              // particle slots in use (live + dead)
    uint64_t injected[APIC_MAX_SPECIES];
    uint64_t absorbed[APIC_MAX_SPECIES];
    uint64_t escaped[APIC_MAX_SPECIES];
    uint64_t pushed[APIC_MAX_SPECIES];        // sum over pushes of live particles
    int64_t n_sorted[APIC_MAX_SPECIES];       // live count found by the last sort
    unsigned long long cursor;                // scratch for compaction
    uint32_t next_id[APIC_MAX_SPECIES];
    uint32_t overflow;                        // capacity exceeded (sticky)
    int32_t cur[APIC_MAX_SPECIES];            // current particle buffer (0/1)
    uint32_t inj_id0[APIC_MAX_SPECIES];       // first id of this step's injection
    uint32_t inj_tag;                         // Philox stream of this step's injection
    uint64_t step;                            // injection steps taken
    uint64_t inj_acc[APIC_MAX_SPECIES];       // injection accumulator, 2^-32 particles
    int64_t inj_base[APIC_MAX_SPECIES];       // first slot of this step's injection
    int64_t inj_new[APIC_MAX_SPECIES];        // particles drawn this step
    double F_el_sum;                          // sum of per-step electric force
};

// Particle buffers of one species: SoA.  FP32 split: pos0 = int32 packed cell,
// pos1/pos2 = float offsets f1/f2 in [0,1); FP64: pos1/pos2 = double x1/x2.
struct PBuf {
    void* pos0 = nullptr;
    void* pos1 = nullptr;
    void* pos2 = nullptr;
    void* vR = nullptr;
    void* vZ = nullptr;
    void* vT = nullptr;
    uint32_t* id = nullptr;
};

// One (grain, species) of the ensemble, as the particle kernels see it.
struct PushTask {
    GrainParams gp;
    SpeciesParams sp;
    PBuf buf[2];                // double buffer; ctr->cur[s] selects the current one
    const void* grad;           // float2 / double2 nodal (dphi/dx1, dphi/dx2)
    void* dep;                  // float / double deposit sums of this species
    DevCounters* ctr;
    double* tally;              // [5][ns][n_bins]
    unsigned long long* tally_count;
    int* hist;                  // sort histograms, tile-major [ntiles][sort_blocks]
    int* hist_off;              // their exclusive scan, + 1 total
    int* seg;                   // scan partial sums
    int64_t capacity;
    uint64_t inj_inc;           // particles injected per step, 2^-32 units
    int s, ns, grain, sort_blocks;
    int inj_block0;             // first workgroup of this task in the injection launch
    int sort_level;             // sorted every (sort_every << sort_level) steps
};

// One grain, as the field kernels see it.
struct GrainDesc {
    int n1, n2, nx, nodes, ns;
    double inv_h1, inv_h2, h2, alpha, rhs_scale;    // rhs_scale = -1 / kappa^2
    double phi_grain, phi_out;
    int fe;                                         // conservative form: f from node charges
    double cw[APIC_MAX_SPECIES];                    // q w per species
    double bnd2;                                    // |A_ib u_b|^2 (row-scaled), constant
    const void* dep[APIC_MAX_SPECIES];
    const double* vol;
    double* rho;
    double* u;                  // phi (finest multigrid level)
    double* f;                  // right-hand side of the finest level
    void* grad;
    DevCounters* ctr;
};

// Doubles per node of a stored stencil: the nine coefficients and one of
// padding, so that a node's coefficients are five aligned 16-byte loads.
constexpr int ST_STRIDE = 10;

// One multigrid level of one grain.  n1 == 0: the grain has no such level.
struct MGDesc {
    int n1, n2, nx, nodes;
    int coarsest;               // this is the grain's last level (dense solve)
    int m;                      // nodes of the dense system (coarsest only)
    double alpha, h1, h2;       // finest level: geometry of its stencil (evaluated at the nodes)
    double ih1sq, ih2sq, i2h2, i4h1h2;   // 1/h1^2, 1/h2^2, 1/(2 h2), 1/(4 h1 h2)
    const double* st;           // stored levels: [node * ST_STRIDE + k], k = ST_C .. ST_NE
    double* u;
    double* f;
    double* uT;                 // finest level: u and f transposed (x2 fastest)
    double* fT;
    double* uprev;              // finest level: the potential of the previous step
    const double* inv;          // dense inverse (coarsest only)
    const double* shift;        // Boltzmann electrons: the Newton term subtracted from the
                                // operator's diagonal (nullptr: none)
    double* uold;               // Boltzmann electrons, finest level: phi before the Newton step
};

// Convergence state of the in-step multigrid solves, per grain.
struct MGState {
    double r2;                  // |D^-1 r|^2 of the last check
    double b2;                  // |D^-1 b|^2 of the current right-hand side
    double last_r2;             // r2 of the last check
    int done;                   // converged (or excluded from this solve)
    int cycles;                 // cycles run in this solve
    int extrap;                 // uprev holds the previous in-step solution
    int pad;
};

struct MGBatch {
    int pending;                // grains not yet converged
    int nan;                    // a residual was not finite
    int max_cycles;             // largest cycles count of this solve
    int pending_prev;           // `pending` of the check before the last one
};

struct MGLevel {
    int n1, n2, nx, nodes;
    double* st = nullptr;       // the nine coefficients C,W,E,S,N,SW,SE,NW,NE node-major,
                                // ST_STRIDE per node (stored levels; the default finest
                                // level's operator is evaluated at the nodes)
    double* u = nullptr;        // solution (level 0: phi) / correction
    double* f = nullptr;        // right-hand side
    double* uT = nullptr;       // finest level: u, f transposed for the x2 sweeps
    double* fT = nullptr;
    double* uprev = nullptr;    // finest level: previous step's potential
    double* shift = nullptr;    // Boltzmann electrons: diagonal Newton term of this level
    double* uold = nullptr;     // Boltzmann electrons, finest level: phi before the Newton step
};

struct Grain {
    apic_grain_cfg cfg;
    GrainParams gp;
    SpeciesParams sp[APIC_MAX_SPECIES];
    int ns = 0;
    int nodes = 0, ncells = 0;
    double V = 0, A_out = 0;
    std::vector<double> vol_host;
    uint64_t inj_inc[APIC_MAX_SPECIES] = {0, 0};    // injection per step, 2^-32 units
    uint64_t step_index = 0;
    uint64_t unconverged = 0;       // in-step solves stopped at the cycle cap
    bool loaded[APIC_MAX_SPECIES] = {false, false};  // particles set, loaded or injected
    bool field_stale = true;
    int64_t capacity[APIC_MAX_SPECIES] = {0, 0};
    PBuf buf[APIC_MAX_SPECIES][2];
    int cur[APIC_MAX_SPECIES] = {0, 0};             // host mirror of ctr->cur
    int sort_blocks[APIC_MAX_SPECIES] = {0, 0};
    // device arrays
    DevCounters* ctr = nullptr;
    double* vol = nullptr;          // node volumes
    void* grad = nullptr;           // float2 / double2 nodal (dphi/dx1, dphi/dx2)
    void* dep[APIC_MAX_SPECIES] = {nullptr, nullptr};  // float / double deposit sums
    double* rho = nullptr;          // charge density of the last deposit
    double* tally = nullptr;        // [5][ns][n_bins]: charge, pR, pZ, L, energy
    unsigned long long* tally_count = nullptr;   // [ns][n_bins]
    double* coarse_inv = nullptr;   // dense inverse of the coarsest operator
    int coarse_nodes = 0;
    double bnd_norm2 = 0;           // |A_interior,boundary u_boundary|^2 (host)
    std::vector<MGLevel> mg;
    int* hist[APIC_MAX_SPECIES] = {nullptr, nullptr};
    int* hist_off[APIC_MAX_SPECIES] = {nullptr, nullptr};
    int* seg[APIC_MAX_SPECIES] = {nullptr, nullptr};
};

// Launch schedule of the particle kernels (chosen by the autotuner or defaults).
struct Schedule {
    int push_wg_per_cu = 8;     // persistent push workgroups per compute unit (capped at
                                // what stays resident)
    int tile_log2 = 4;          // sort tile edge, log2 cells (capped per grain)
    int sort_every = 4;         // steps between sorts
};

// Progress of the autotuner across apic_step calls.
struct TuneState {
    int phase = 0, idx = 0;
    float best = 1e30f;
    int best_val = 0;
    float sort_ms = 0;
    std::vector<float> push_after;
};

struct TimerPair { hipEvent_t a, b; int kind; };

// Boltzmann electrons: largest coarsest level, inverted in one workgroup's LDS
// (88^2 doubles and the pivot scratch stay within 64 KiB)
constexpr int BOLTZ_INV_MAX = 88;
constexpr int SORT_LEVELS = 5;   // a slow species is sorted up to 16x less often
enum GraphId { G_PUSH = 0, G_INJ, G_PRE, G_VC, G_VCN, G_POST, G_NEWTON, G_NEWTON_NEXT, G_SORT,
               G_COUNT = G_SORT + SORT_LEVELS };

}  // namespace apic

struct apic_ctx {
    std::vector<apic::Grain> grains;
    apic_opts opts;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t side = nullptr;             // sort overlapped with the field solve
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool graphs = true;                     // capture repeated launch sequences
    int device = 0;
    int num_cus = 256;
    std::string err;
    // ensemble tables (device) and their host copies
    std::vector<apic::PushTask> tasks_h;
    apic::PushTask* tasks = nullptr;
    int ntasks = 0;
    int64_t* chunk_prefix = nullptr;        // [ntasks + 1] chunks of the current push
    std::vector<apic::GrainDesc> gdesc_h;
    apic::GrainDesc* gdesc = nullptr;
    int n_levels = 0;                       // deepest hierarchy of the ensemble
    std::vector<apic::MGDesc> mgdesc_h;     // [level][grain]
    apic::MGDesc* mgdesc = nullptr;
    apic::MGDesc* mgdesc_coarse = nullptr;  // [grains] each grain's coarsest level
    int max_coarse_m = 0;                   // largest dense system of the ensemble
    std::vector<int> lvl_max_n1, lvl_max_n2, lvl_max_nodes, lvl_lines_x1, lvl_lines_x2, lvl_max_m;
    apic::MGState* mgs = nullptr;           // [grains]
    double* norm_part = nullptr;            // [2][grains][blocks] partial norms (r, b)
    apic::MGBatch* mgb = nullptr;
    apic::MGBatch* mgb_host = nullptr;      // pinned
    int inj_blocks = 0;                     // workgroups of the injection launch (all tasks)
    int* inj_block_task = nullptr;          // [inj_blocks] task of each injection workgroup
    int max_ntiles = 0, max_sort_blocks = 0, max_segs = 0;
    int max_nodes = 0, max_n1 = 0, max_n2 = 0;
    bool x2_transposed = false;             // finest-level x2 sweeps on transposed copies
    int pred_cycles = 0;                    // cycles of the previous in-step solve
    std::vector<int> newton_pred;           // Boltzmann electrons: cycles of each Newton step
                                            // of the previous in-step solve
    // schedule and graphs
    apic::Schedule sched;
    bool tuned = false;
    bool tuning = false;                    // launches run eagerly while tuning
    apic::TuneState tune;
    hipGraphExec_t graph[apic::G_COUNT] = {};
    // profiling
    double* scratch = nullptr;              // static staging array of apic_inject_noalloc
    bool profiling = false;
    bool profiled = false;                  // timing was enabled at some point
    std::vector<apic::TimerPair> timers;   // recorded, not yet harvested
    std::vector<hipEvent_t> event_pool;
    double t_ms[4] = {0, 0, 0, 0};
    int64_t push_launches = 0, timed_steps = 0, timed_particle_steps = 0, timed_mg_cycles = 0;
};

namespace apic {

// ------------------------------------------------------------------ launchers
// particles.hip (ensemble-wide unless a grain is named)
hipError_t launch_push(apic_ctx* ctx, bool deposit);
hipError_t launch_deposit(apic_ctx* ctx);
hipError_t launch_inject(apic_ctx* ctx, bool deposit);
hipError_t launch_sort(apic_ctx* ctx, int first_task, int n_tasks, int max_level = SORT_LEVELS);
hipError_t launch_load(apic_ctx* ctx, Grain& g, int s, int64_t n);
hipError_t launch_set_particles(apic_ctx* ctx, Grain& g, int s, int64_t n, const double* dx1,
                                const double* dx2, const double* dvR, const double* dvZ,
                                const double* dvT, int* d_bad);
hipError_t launch_readback(apic_ctx* ctx, Grain& g, int s, int64_t n, double* dx1, double* dx2,
                           double* dvR, double* dvZ, double* dvT, int64_t* did);
hipError_t launch_count_live(apic_ctx* ctx, Grain& g, int s, unsigned long long* out);
// device address of the static staging array of apic_inject_noalloc on the
// current device (looked up once per device)
constexpr int64_t NOALLOC_MAX_PARTICLES = 262144;
hipError_t noalloc_scratch(double** out);
int max_sort_blocks();
int scan_seg_len();
int push_chunk(bool split);
int push_resident_per_cu(apic_ctx* ctx);

// field.hip
hipError_t launch_fill(apic_ctx* ctx, void* p, size_t bytes);
hipError_t launch_clear_deposits(apic_ctx* ctx);
hipError_t launch_rho_rhs(apic_ctx* ctx);
hipError_t launch_rhs_from_rho(apic_ctx* ctx, int grain);
hipError_t launch_gradient(apic_ctx* ctx);
hipError_t launch_surface_field(apic_ctx* ctx, int grain, double* out);
hipError_t launch_grain_force(apic_ctx* ctx);
hipError_t launch_set_boundary(apic_ctx* ctx);

// multigrid.hip
hipError_t mg_extrapolate(apic_ctx* ctx);
hipError_t newton_prepare(apic_ctx* ctx, int only, bool invert);
hipError_t newton_limit(apic_ctx* ctx, int only);
hipError_t mg_begin(apic_ctx* ctx, double tol, int only_grain, bool in_step);
hipError_t mg_vcycle_launches(apic_ctx* ctx, double tol, bool check = true);

}  // namespace apic
