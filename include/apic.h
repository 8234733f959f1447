/*
 * apic.h -- C ABI of the MI355X particle loop of the aspherical particle-in-cell
 * method of Smirnov & Krasheninnikov, "Aspherical PIC code (APIC) for modeling
 * non-spherical dust in plasmas using shape-conforming coordinates"
 * (arXiv 2307.11107).
 *
 * What one step computes (paper, Sections 1-2): electrons and ions move in the
 * self-consistent electrostatic field of a conducting grain whose surface is
 * x1 = -1 in the shape-conforming coordinates of eq. (2); the outer boundary is
 * x1 = x1_out.  Per step: the nodal derivatives of phi are interpolated to each
 * particle and turned into (E_R, E_Z) by eq. (10); eq. (9) is advanced by
 * leapfrog (optional axial B); particles crossing the grain are absorbed and
 * tallied (charge, momentum, angular momentum, energy, per x2-bin of the impact
 * point), particles crossing x1_out escape; a Maxwellian flux is injected at
 * x1_out; charge is weighted to the nodes with the volume element of eq. (5);
 * the Poisson equation (6)-(7) is solved in FP64 with phi fixed on both
 * boundaries.
 *
 * Units (normalised): lengths R0, time 1/omega_pe, velocity v_te = sqrt(Te/me),
 * potential Te/e, density n0, charge e, mass me, energy Te.  kappa =
 * lambda_De / R0; Lap(phi) = -(1/kappa^2) sum_s q_s n_s.
 *
 * Grid: n1 x n2 cells, uniform in (x1, x2); x1 in [-1, x1_out], x2 in [-1, 1].
 * Node (i1, i2), i1 = 0..n1, i2 = 0..n2, is element i2 * (n1 + 1) + i1 of every
 * node array crossing this ABI (x1 varies fastest).
 *
 * Conventions: every function returns an apic status code.  Host arrays passed
 * in are owned by the caller and only read during the call; host arrays passed
 * out are owned by the caller and written during the call.  Device memory is
 * owned by the context and released by apic_free.  A context is not
 * thread-safe.  Work is issued on the stream given in apic_opts (NULL = the
 * default stream); calls that return data to the host synchronise that stream.
 * On error, apic_last_error(ctx) returns a message.
 */
#ifndef APIC_H
#define APIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    APIC_OK = 0,
    APIC_EINVAL = -1,   /* bad argument (null pointer, bad index, bad size)          */
    APIC_ERANGE = -2,   /* |alpha| >= 1/4, x1_out not in (-1, 0), grid out of range  */
    APIC_ENOMEM = -3,   /* device allocation failed, or particle capacity exceeded   */
    APIC_EDEVICE = -4,  /* a HIP call failed                                         */
    APIC_ESTATE = -5    /* call order violated                                       */
};

enum { APIC_FP32_SPLIT = 0, APIC_FP64 = 1 };
enum { APIC_MAX_SPECIES = 2 };

/* One plasma species (Section 1: macro-particles carry the species' q/m). */
typedef struct {
    double q;          /* charge, units of e (electron: -1)                        */
    double m;          /* mass, units of me                                        */
    double T;          /* temperature of the injected/loaded Maxwellian, units Te  */
    double n;          /* unperturbed density, units of n0                         */
    double e_bind;     /* energy per absorbed particle besides kinetic, units Te   */
    double weight;     /* macro-particle weight, units n0 R0^3; 0: n V / n_macro   */
    int64_t n_macro;   /* particles of the initial volume load                     */
    int64_t capacity;  /* particle slots on the device (below 2^30); 0: 1.5 n_macro + 4096 */
} apic_species;

/* One grain and its plasma (eqs. 1-2 and Section 2). */
typedef struct {
    double alpha;      /* dipole parameter p / (Q R0) of eq. (1); |alpha| < 1/4    */
    double wce;        /* omega_ce / omega_pe of the axial field (0: no field)     */
    double kappa;      /* lambda_De / R0                                           */
    double x1_out;     /* outer boundary, -1 < x1_out < 0                          */
    double phi_grain;  /* fixed potential of the grain, units Te/e                 */
    double phi_out;    /* fixed potential of the outer boundary                    */
    double dt;         /* time step, units 1/omega_pe                              */
    int32_t n1, n2;    /* cells along x1 and x2: 8 <= n1 <= 2048, 8 <= n2 <= 2046 */
    int32_t n_bins;    /* tally bins in x2 of the impact point; 0: n2              */
    int32_t n_species; /* 1 or 2                                                   */
    uint64_t seed;     /* Philox key; grain g uses (lo32(seed), hi32(seed) + g)    */
    apic_species sp[APIC_MAX_SPECIES];
} apic_grain_cfg;

typedef struct {
    int32_t precision;          /* APIC_FP32_SPLIT (cell index + FP32 offset) or APIC_FP64 */
    int32_t inject;             /* 1: Maxwellian flux injection every step                 */
    int32_t frozen_field;       /* 1: phi stays as last set (no deposit, no solve)         */
    int32_t sort_every;         /* re-sort particles by cell every k steps (0: 4); a
                                   species 2^l times slower (thermal speed) than its
                                   grain's fastest is re-sorted every k 2^l steps,
                                   2^l <= 16                                               */
    double poisson_tol;         /* in-step solves: stop at |r| <= tol |b| (0: 1e-10)       */
    int32_t poisson_max_cycles; /* in-step multigrid cycle cap (0: 40)                     */
    int32_t autotune;           /* 1: the first steps choose the launch schedule (below)   */
    void* stream;               /* hipStream_t; NULL: default stream                       */
    int32_t boltzmann_electrons; /* 1: electrons are not moved; their density is
                                    n0 exp(e phi / Te) (Section 2, last paragraph), so
                                    eq. (6) is nonlinear in phi and solved by Newton's
                                    method with the FP64 multigrid; the grain configs
                                    then list the moved species only.  The grid must
                                    coarsen (halving both cell counts) to <= 88 nodes,
                                    else APIC_ERANGE                                      */
    int32_t conservative_poisson; /* 1: eq. (6) with the Laplacian in conservative form,
                                    discretised by bilinear finite elements (symmetric;
                                    the right-hand side is each node's deposited charge,
                                    so Gauss's law holds exactly) instead of the expanded
                                    9-point operator of eq. (7); apic_solve_poisson's rho
                                    is then weighted by the node volumes.  Not with
                                    boltzmann_electrons (APIC_EINVAL)                      */
} apic_opts;

/* Grain tallies (Sections 1-2: currents, drag, torque and heat flux follow from
 * charge, momentum, angular momentum and energy given to the grain per unit time).
 * Per-bin sums are multiplied by the macro-particle weight; arrays are
 * [species][bin] and are filled only when the pointer is non-NULL. */
typedef struct {
    int32_t n_species, n_bins;
    uint64_t steps;                         /* steps taken since apic_init            */
    uint64_t injected[APIC_MAX_SPECIES];    /* loaded + injected particles            */
    uint64_t absorbed[APIC_MAX_SPECIES];
    uint64_t escaped[APIC_MAX_SPECIES];
    uint64_t resident[APIC_MAX_SPECIES];    /* live particles now (counted on device) */
    uint64_t particle_steps[APIC_MAX_SPECIES]; /* sum over steps of particles pushed  */
    double weight[APIC_MAX_SPECIES];        /* macro-particle weights in use          */
    double F_el_sum;                        /* sum over steps of the electric force
                                               F_Z on the grain, units eps0 Te^2/e^2  */
    uint64_t unconverged_solves;            /* in-step field solves that stopped at
                                               apic_opts.poisson_max_cycles before
                                               reaching poisson_tol (0 in a healthy run) */
    uint64_t* count;                        /* absorbed particles per bin             */
    double* charge;                         /* sum q w                                */
    double* pR;                             /* sum m w v_R  (impact meridional frame) */
    double* pZ;                             /* sum m w v_Z                            */
    double* L;                              /* sum m w R v_Theta (angular momentum)   */
    double* energy;                         /* sum w (m v^2 / 2 + e_bind)             */
} apic_tally;

/* Kernel timing from HIP events recorded on the context's stream. */
typedef struct {
    double push_ms;        /* particle kernels: gather+push+boundary+deposit   */
    double inject_ms;
    double sort_ms;
    double field_ms;       /* rho, Poisson, gradient, grain diagnostics         */
    int64_t push_launches; /* number of particle-kernel launches timed         */
    int64_t steps;         /* steps timed                                       */
    int64_t particle_steps;/* sum over timed steps of resident particles pushed */
    int64_t mg_cycles;     /* multigrid cycles run in timed steps               */
} apic_kernel_times;

/* Launch schedule of the particle kernels.  With apic_opts.autotune the first
 * ~24 steps (each a real step of the run) time candidate schedules with HIP
 * events and keep the fastest: persistent push workgroups per compute unit,
 * the sort tile edge, and the sort interval k minimising (sort time + sum of
 * the k following push times) / k.  Results do not depend on the schedule
 * beyond the summation order of the deposit. */
typedef struct {
    int32_t push_wg_per_cu;  /* persistent push workgroups per compute unit (at
                                most what stays resident at once)                 */
    int32_t tile_log2;       /* preferred sort tile edge, log2 cells (each grain
                                caps its tile count at 8192)                      */
    int32_t sort_every;      /* steps between sorts                                */
    int32_t tuned;           /* 1 once the autotuner has finished                   */
} apic_sched;
typedef struct apic_ctx apic_ctx;

/* Creates a context for an ensemble of n_grains grains (cfgs[n_grains]; grids,
 * shapes, fields and particle counts may all differ), allocates device memory,
 * builds the geometry tables (node volumes from eq. 5, the eq. 7 stencil, the
 * outer area from eq. 4) and the multigrid hierarchies.  Every step of the
 * ensemble runs as one sequence of launches over all grains (one persistent
 * particle launch for all grains and species), captured into HIP graphs.
 * Returns APIC_ERANGE for |alpha| >= 1/4 or x1_out outside (-1, 0).
 * *out receives the context (NULL on failure; apic_last_error(NULL) then
 * returns the message). */
int apic_init(const apic_grain_cfg* cfgs, int32_t n_grains, const apic_opts* opts, apic_ctx** out);

/* Sets the particles of one species of one grain, replacing any present.
 * n >= 0: copies n particles from host arrays (positions in (x1, x2), velocity
 * v^{-1/2} components); particle ids are 0..n-1.
 * n < 0 with all arrays NULL: loads cfg.sp[species].n_macro particles uniform in
 * physical volume (eq. 5) with Maxwellian velocities, drawn on the device from
 * Philox4x32-10 (Salmon et al., SC'11) with the grain's key.
 * Particles outside the domain (-1 < x1 < x1_out, |x2| <= 1) or with a
 * non-finite velocity are rejected with APIC_EINVAL before any device work
 * (nothing is changed); more than the capacity gives APIC_ENOMEM.  The field is
 * recomputed before the next step. */
int apic_inject(apic_ctx* ctx, int32_t grain, int32_t species, int64_t n,
                const double* x1, const double* x2,
                const double* vR, const double* vZ, const double* vTheta);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): apic_inject
 * for explicit particles (n >= 0 host arrays as above), staged through a
 * static device array instead of a per-call allocation.  It calls no hipMalloc,
 * hipFree or allocating library routine.  At most 262144 particles per call
 * (APIC_EINVAL beyond; the array, 10 MiB, is held by every GPU the library runs
 * on until the process ends).  All calls on one GPU share that array: calls
 * that overlap on one GPU (several host threads or contexts at once) race.
 * Otherwise the same results and errors as apic_inject. */
int apic_inject_noalloc(apic_ctx* ctx, int32_t grain, int32_t species, int64_t n,
                        const double* x1, const double* x2,
                        const double* vR, const double* vZ, const double* vTheta);

/* Advances every grain by n_steps on the context's stream.  Each step reads
 * the multigrid convergence state once (one stream synchronisation); the call
 * returns APIC_ENOMEM if injection ran out of particle slots (the particles
 * that did not fit are dropped and not counted as injected). */
int apic_step(apic_ctx* ctx, int64_t n_steps);

/* FP64 solve of eqs. (6)-(7) for one grain.  rho (host, (n1+1)(n2+1), units e n0)
 * is the charge density sum_s q_s n_s at the nodes; NULL: deposit the current
 * particles.  The solution becomes the grain's field for the following steps.
 * phi_out (host, may be NULL) receives phi.  Iterates multigrid cycles to the
 * round-off floor (row-scaled relative residual <= 1e-15, or stagnation).
 * With boltzmann_electrons, rho is the charge density of the moved species and
 * the electrons' n0 exp(phi) is added by Newton's method (to the round-off
 * floor of the nonlinear residual; APIC_EDEVICE if it does not converge); with
 * conservative_poisson, rho is weighted by the node volumes to the node
 * charges of the finite-element form. */
int apic_solve_poisson(apic_ctx* ctx, int32_t grain, const double* rho, double* phi_out);

/* Copies the grain's tallies to the host (synchronises the stream). */
int apic_tallies(apic_ctx* ctx, int32_t grain, apic_tally* out);

/* Copies the live particles of one species to the host, sorted by id.
 * cap is the length of the arrays; *n_out receives the number of particles
 * (APIC_EINVAL if it exceeds cap).  Positions are returned as (x1, x2) in FP64.
 * id may be NULL.  APIC_ESTATE if the species was never populated (no
 * apic_inject for it and no step with injection). */
int apic_particles(apic_ctx* ctx, int32_t grain, int32_t species, int64_t cap,
                   double* x1, double* x2, double* vR, double* vZ, double* vTheta,
                   int64_t* id, int64_t* n_out);

/* Copies the grain's current potential and the charge density of the last
 * deposit (host arrays of (n1+1)(n2+1); either may be NULL). */
int apic_fields(apic_ctx* ctx, int32_t grain, double* phi, double* rho);

/* Normal electric field on the grain surface from the current potential
 * (Section 2: the field on the conducting surface gives its surface charge):
 * E_n = -|grad x1| dphi/dx1 at the grain nodes i2 = 0..n2 (host array of n2+1,
 * units Te/(e R0), the one-sided second-order derivative on x1 = -1).  The
 * surface charge density is eps0 E_n; the grain's electric force, summed per
 * step in apic_tallies' F_el_sum, integrates E_n^2/2 n_Z over the surface. */
int apic_surface_field(apic_ctx* ctx, int32_t grain, double* E_n);

/* Enables (1) or disables (0) HIP-event timing of the kernels, resetting the
 * accumulated times; apic_timing synchronises and returns them (APIC_ESTATE if
 * timing was never enabled on the context). */
int apic_set_profiling(apic_ctx* ctx, int32_t on);
int apic_timing(apic_ctx* ctx, apic_kernel_times* out);

/* Copies the context's launch schedule (the autotuner's choice once tuned). */
int apic_schedule(apic_ctx* ctx, apic_sched* out);
/* Releases the context and its device memory. */
int apic_free(apic_ctx* ctx);

/* Message of the last error on ctx (ctx may be NULL for apic_init failures). */
const char* apic_last_error(const apic_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* APIC_H */
