// Internal structures of the APIC context and the launchers of its kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "apic.h"
#include "host_setup.h"

namespace apic {

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

// Device counters of one grain (one allocation, zeroed at init).
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
    uint32_t pad;
    double F_el_sum;                          // sum of per-step electric force
    double norm2;                             // scratch for residual norms
    double norm2_b;
    double norm2_e;
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

struct MGLevel {
    int n1, n2, nx, nodes;
    double* st = nullptr;       // 9 stencil arrays [k * nodes + node], k = C,W,E,S,N,SW,SE,NW,NE
    double* u = nullptr;        // solution (level 0: phi) / correction
    double* f = nullptr;        // right-hand side
    double* r = nullptr;        // residual
};

struct Grain {
    apic_grain_cfg cfg;
    GrainParams gp;
    SpeciesParams sp[APIC_MAX_SPECIES];
    int ns = 0;
    int nodes = 0, ncells = 0;
    double V = 0, A_out = 0;
    std::vector<double> vol_host;
    // injection fixed-point accumulators (units 2^-32 particles)
    uint64_t inj_inc[APIC_MAX_SPECIES] = {0, 0};
    uint64_t inj_acc[APIC_MAX_SPECIES] = {0, 0};
    uint64_t step_index = 0;
    bool field_stale = true;
    int64_t capacity[APIC_MAX_SPECIES] = {0, 0};
    int64_t host_slots[APIC_MAX_SPECIES] = {0, 0};  // upper bound of slots in use
    PBuf buf[APIC_MAX_SPECIES][2];
    int cur[APIC_MAX_SPECIES] = {0, 0};
    // device arrays
    DevCounters* ctr = nullptr;
    double* vol = nullptr;          // node volumes
    void* grad = nullptr;           // float2 / double2 nodal (dphi/dx1, dphi/dx2)
    void* dep[APIC_MAX_SPECIES] = {nullptr, nullptr};  // float / double deposit sums
    double* rho = nullptr;          // charge density of the last deposit
    double* phi_prev = nullptr;     // potential of the previous step (initial-guess extrapolation)
    bool have_prev = false;
    double* tally = nullptr;        // [5][ns][n_bins]: charge, pR, pZ, L, energy
    unsigned long long* tally_count = nullptr;   // [ns][n_bins]
    double* axis_nn = nullptr;      // level-0 second-neighbour coefficient on row i2 = 0
    double* axis_ss = nullptr;      // ... on row i2 = n2
    double* coarse_inv = nullptr;   // dense inverse of the coarsest operator
    int coarse_nodes = 0;
    double bnd_norm2 = 0;           // |A_interior,boundary u_boundary|^2 (host)
    std::vector<MGLevel> mg;
    hipGraphExec_t vcycle_exec = nullptr;   // captured V-cycle
    // sort scratch
    int* sort_count = nullptr;      // per-block tile histograms, ntiles * sort_blocks + 1
    int* sort_offset = nullptr;     // their exclusive scan
    void* scan_tmp = nullptr;
    size_t scan_tmp_bytes = 0;
};

struct TimerPair { hipEvent_t a, b; int kind; };

}  // namespace apic

struct apic_ctx {
    std::vector<apic::Grain> grains;
    apic_opts opts;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool graphs = true;                     // capture repeated launch sequences
    int device = 0;
    int num_cus = 256;
    std::string err;
    bool profiling = false;
    std::vector<apic::TimerPair> timers;   // recorded, not yet harvested
    std::vector<hipEvent_t> event_pool;
    double t_ms[4] = {0, 0, 0, 0};
    int64_t push_launches = 0, timed_steps = 0, timed_particle_steps = 0, timed_mg_cycles = 0;
};

namespace apic {

// ------------------------------------------------------------------ launchers
// particles.hip
hipError_t launch_push(apic_ctx* ctx, Grain& g, int s);
hipError_t launch_deposit_all(apic_ctx* ctx, Grain& g, int s);
hipError_t launch_inject(apic_ctx* ctx, Grain& g, int s, int64_t n_new, uint32_t stream_tag);
hipError_t launch_load(apic_ctx* ctx, Grain& g, int s, int64_t n);
hipError_t launch_set_particles(apic_ctx* ctx, Grain& g, int s, int64_t n, const double* dx1,
                                const double* dx2, const double* dvR, const double* dvZ,
                                const double* dvT, int* d_bad);
hipError_t launch_readback(apic_ctx* ctx, Grain& g, int s, int64_t n, double* dx1, double* dx2,
                           double* dvR, double* dvZ, double* dvT, int64_t* did);
hipError_t launch_sort(apic_ctx* ctx, Grain& g, int s);
hipError_t launch_add_slots(apic_ctx* ctx, Grain& g, int s, int64_t n_new);
hipError_t launch_count_live(apic_ctx* ctx, Grain& g, int s, unsigned long long* out);
size_t scan_temp_bytes(int n);
int sort_blocks();

// field.hip
hipError_t launch_fill(apic_ctx* ctx, void* p, size_t bytes);
hipError_t launch_rho(apic_ctx* ctx, Grain& g);
hipError_t launch_rhs_from_rho(apic_ctx* ctx, Grain& g);
hipError_t launch_gradient(apic_ctx* ctx, Grain& g);
hipError_t launch_grain_force(apic_ctx* ctx, Grain& g);
hipError_t launch_set_boundary(apic_ctx* ctx, Grain& g);
hipError_t launch_extrapolate(apic_ctx* ctx, Grain& g);
hipError_t launch_copy(apic_ctx* ctx, double* dst, const double* src, int n);

// multigrid.hip
hipError_t mg_vcycle(apic_ctx* ctx, Grain& g);
hipError_t mg_residual_norm(apic_ctx* ctx, Grain& g, double* norm2_dev);
hipError_t mg_rhs_norm(apic_ctx* ctx, Grain& g, double* norm2_dev);

}  // namespace apic
