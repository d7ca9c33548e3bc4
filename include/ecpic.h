/*
 * ecpic.h -- C ABI of the MI355X explicit energy-conserving PIC library.
 *
 * The library advances one or many independent 1D3V radio-frequency
 * capacitively coupled argon discharges with the explicit energy-conserving
 * particle-in-cell loop of Powis & Kaganovich (Section 2a: charge deposit,
 * Poisson solve, cell-centred field, offset nearest-grid-point gather,
 * leapfrog push, Monte-Carlo collisions), with the momentum-conserving
 * centred field and linear gather, or a second-order energy-conserving pair
 * (quadratic-spline deposit, linear gather of the cell field: the gather
 * shape one order below the deposit's, Section 2a), selectable per instance.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Memory.  The caller owns all device memory: one device arena of at least
 *    pic_footprint() bytes, passed to pic_init().  The library never allocates
 *    or frees device memory; it carves the arena itself and never keeps the
 *    arena after pic_destroy().  Arena space beyond the footprint is a pool
 *    that pic_slot_reset() draws from.  Host pointers passed in are read (or
 *    written) during the call only.
 *  - Streams.  Work is enqueued asynchronously on the HIP stream given to
 *    pic_init() (NULL = the null stream).  pic_diagnostics(), pic_get_state(),
 *    pic_get_fields(), pic_profiles() and pic_kernel_times() synchronise it.
 *  - Errors.  Every call returns a pic_status; nothing is thrown across the
 *    ABI.  Argument errors are detected before any work is enqueued and leave
 *    the context unchanged (PIC_EINVAL; pic_last_error() says why).  Errors
 *    found on the device (capacity overflow, non-finite state, runaway
 *    particle growth) set a sticky per-instance status word; the instance is
 *    frozen from then on (its particles no longer advance) and the next
 *    synchronising call on it returns the error.
 *  - Threads.  A context is used by one host thread at a time.
 *  - Units.  SI throughout (m, s, V, Pa, K, m^-3), temperatures of particles
 *    in eV; quantities per unit electrode area (1D slab).
 */
#ifndef ECPIC_H
#define ECPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_ABI_VERSION 7

typedef struct pic_ctx pic_ctx;  /* opaque; owns host-side metadata only */

typedef enum {
  PIC_OK = 0,
  PIC_EINVAL = 1,      /* bad argument or configuration                          */
  PIC_ENOMEM = 2,      /* arena or slot pool too small                           */
  PIC_ECAPACITY = 3,   /* a species outgrew its particle capacity (device)       */
  PIC_ENONFINITE = 4,  /* a non-finite position or velocity appeared (device)    */
  PIC_EGROWTH = 5,     /* live particles exceeded growth_limit x initial (device)*/
  PIC_EDEVICE = 6,     /* a HIP runtime call failed                              */
  PIC_ESTATE = 7       /* call not valid in the current state (frozen instance,
                          stale deposit, empty slot)                             */
} pic_status;

enum { PIC_BC_DIRICHLET_RF = 0, PIC_BC_PERIODIC = 1 };
enum { PIC_GATHER_EC = 0, PIC_GATHER_MC = 1, PIC_GATHER_EC2 = 2 };
enum { PIC_FP64 = 0, PIC_FP32_STATE = 1 };

/*
 * One discharge.  Arguments follow the statement of the problem in the paper
 * (Table 1; Sections 2, 2b, 3c): grid, RF drive, gas, initial plasma, particle
 * weight and time step.  A zero in a field marked "0 ->" selects the default.
 */
typedef struct pic_config {
  int32_t n_cells;        /* N cells, nodes 0..N (N >= 2; <= PIC_MAX_CELLS); 0 = empty slot */
  int32_t bc;             /* PIC_BC_DIRICHLET_RF: phi_0 = RF drive, phi_N = 0 (Eq 4);
                             PIC_BC_PERIODIC: periodic with a uniform neutralising
                             background and gauge phi_0 = 0 (Appendix B)            */
  const double *nodes;    /* N+1 increasing node positions from 0 (host, copied);
                             NULL = uniform grid of width gap_m / N                  */
  double gap_m;           /* electrode gap L (ignored when nodes != NULL: L = nodes[N]) */
  double v_rf, f_rf, phase; /* phi_0(t) = v_rf sin(2 pi f_rf t + phase), t_k = k dt    */
  double p_pa, t_gas_k;   /* background argon: n_g = p / (k_B T_g)                    */
  double n0_m3, te_ev, ti_ev; /* uniform Maxwellian initial plasma (Section 2b)       */
  int64_t n_per_species;  /* initial macro-particles of each species                  */
  int64_t capacity;       /* particle slots per species; 0 -> 2 n_per_species + 4096  */
  double weight_m2;       /* macro-particle weight W (per area); 0 -> n0 L / n_per_species */
  double dt_s;            /* time step                                                 */
  int32_t gather;         /* PIC_GATHER_EC (Eqs 5-7), PIC_GATHER_MC, or PIC_GATHER_EC2
                             (uniform grids only: S2 deposit to the nearest node and
                             its neighbours, S1 gather of the cell-centred field; the
                             weight beyond an electrode goes to the electrode node and
                             the field half a cell outside it is taken as zero)      */
  int32_t precision;      /* PIC_FP64 or PIC_FP32_STATE; one value per context         */
  double gamma_see;       /* secondary electrons per absorbed ion (probability)        */
  double t_see_ev;        /* secondary-electron temperature; 0 -> 2 eV                 */
  uint64_t seed;          /* Philox key material for this discharge                    */
  int32_t sort_interval;  /* steps between cell sorts; 0 -> none (FP32 state: none
                             beyond the one it needs every 16384 steps; context-
                             wide: the value of the first active instance is used) */
  int32_t n_species;      /* 2 = electrons + Ar+; 1 = electrons only on a fixed
                             neutralising ion background (periodic only)             */
  int32_t collisions;     /* 1 = Monte-Carlo collisions on; 0 = off                    */
  int32_t pullback;       /* 1 = start from v^{-1/2} = v^0 - (q/m) E^0 dt / 2          */
  double nu_max_e;        /* null-collision bound for electrons (1/s); 0 -> computed   */
  double nu_max_i;        /* null-collision bound for ions (1/s); 0 -> computed        */
  int64_t avg_start;      /* first step accumulated into the averaged profiles         */
  int32_t avg_every;      /* density/potential sampling interval in steps; 0 = none    */
  int32_t eedf_every;     /* central EEDF sampling interval in steps; 0 = none         */
  int32_t eedf_bins;      /* EEDF bins (<= PIC_MAX_EEDF_BINS); 0 -> 200                 */
  double eedf_emax_ev;    /* EEDF upper energy; 0 -> 50 eV                              */
  double eedf_width_m;    /* width of the central sampling window; 0 -> 1 mm           */
  int64_t k_stop;         /* the instance stops advancing at this step; 0 = never      */
  double growth_limit;    /* PIC_EGROWTH when live > growth_limit x initial; 0 -> 10   */
  /* Impact distributions of absorbed particles (Section 3a: ion energy and
     angle at the electrodes), recorded per species and wall on the steps that
     are averaged (avg_every > 0, k >= avg_start). */
  int32_t impact_bins;       /* energy bins over [0, impact_emax_ev) plus one overflow
                                bin (<= PIC_MAX_EEDF_BINS); 0 -> 200                   */
  int32_t impact_angle_bins; /* bins of the angle to the wall normal over [0, 90] deg
                                (<= PIC_MAX_EEDF_BINS); 0 -> 90                        */
  double impact_emax_ev;     /* 0 -> 1000 eV                                           */
  /* 1: also accumulate the velocity moments and power of pic_moments on the
     averaged steps (an extra pass over the particles on each of them);
     0: off. */
  int32_t moments;
  /* Particle rebalancing toward rebalance_ppc particles per cell and species
     (Section 3d: with it the fewer cells of a refined grid mean fewer
     particles).  0 = off.  FP32 state form only.  A rebalanced discharge's
     particles carry weights W 2^(w-4), w = 0..7 (4 at the start), and its
     deposit and weighted sums are in units of W/16.  See pic_rebalance. */
  int32_t rebalance_ppc;
  int32_t rebalance_every;  /* pic_step rebalances every this many steps (context-wide:
                               the value of the first instance that sets it, at
                               pic_init or pic_slot_reset); 0 = never              */
  double rebalance_dv_e;    /* velocity-bin width of merges (m/s); 0 -> sqrt(e te / m_e) / 4 */
  double rebalance_dv_i;    /* the same for ions; 0 -> sqrt(e ti / M) / 4                 */
} pic_config;

#define PIC_MAX_CELLS 2048
#define PIC_MAX_INSTANCES 512
#define PIC_MAX_EEDF_BINS 4096

/* Global monitors and counters of one instance (all cumulative since init). */
typedef struct pic_diag {
  int64_t step;                  /* k: the next step to be taken                       */
  double time_s;                 /* k dt                                               */
  int32_t status;                /* sticky device status bits (PIC_ST_*)              */
  int32_t n_samples;             /* profile samples accumulated                        */
  int32_t eedf_samples;          /* EEDF samples accumulated                           */
  int32_t reserved0;
  int64_t n_live[2];             /* live macro-particles [electrons, ions]             */
  int64_t extent[2];             /* occupied slots (live + absorbed not yet compacted) */
  int64_t deposit_total[2];      /* sum over nodes of the deposit A_s, in 2^-32 units:
                                    exactly 2^32 times the live particles' summed weight
                                    in deposit units (W; W/16 when rebalanced)         */
  double kinetic_j_m2[2];        /* sum of weight x (m/2)|v|^2, from a 2^-20 eV
                                    fixed-point sum                                    */
  double field_j_m2;             /* (eps0/2) sum_j h_j E_j^2 at the last field solve    */
  int64_t absorbed[2][2];        /* [species][0 left (powered), 1 right] electrode     */
  double absorbed_energy_ev[2][2]; /* energy carried into each electrode (eV, 2^-16 eV) */
  int64_t see_emitted;           /* secondary electrons emitted                        */
  int64_t ionisations, excitations, elastic, charge_exchange;
  int64_t candidates[2];         /* null-collision candidates per species              */
  int64_t bound_violations;      /* collision rate above nu_max (should stay 0)        */
  int64_t particle_steps;        /* sum over steps of live particles at step start     */
  double ne_max_m3;              /* max node electron density at the last solve        */
  double wpe_dt_max;             /* omega_pe,max dt (stability condition 1b)          */
  double vmax_dt_over_dxmin;     /* max|vx| dt / min h over electrons (condition 1c)   */
  double lambda_de_over_dxmin;   /* sqrt(eps0 T / (n_e,max e)) / min h, T = 2<KE>/3 (1a) */
  double nu_max[2];              /* null-collision bounds in use [electrons, ions] (1/s):
                                    the configured values, or those the library computed */
  int64_t merges[2];             /* rebalancing: quadruples merged into pairs           */
  int64_t splits[2];             /* rebalancing: particles split in two                 */
} pic_diag;

#define PIC_ST_CAPACITY 1
#define PIC_ST_NONFINITE 2
#define PIC_ST_GROWTH 4

/* Host view of one species' particles (pic_get_state / pic_set_state).
 * FP64 form: x, vx, vy, vz are double*.  FP32-state form: cell, off, and
 * vx, vy, vz are float*.  id and knext are used by both.  Unused pointers may
 * be NULL. */
typedef struct pic_state_view {
  int64_t n;        /* set: particles given; get: in = room in the arrays, out = live count */
  double *x;        /* FP64: position in [0, L)                                     */
  int32_t *cell;    /* FP32: cell index in [0, N)                                    */
  float *off;       /* FP32: offset in the cell, in [0, 1)                           */
  void *vx, *vy, *vz; /* velocity components (double* or float*)                    */
  uint64_t *id;     /* particle id (Philox key)                                      */
  int32_t *knext;   /* first step at which the particle is a collision candidate     */
  uint8_t *wclass;  /* FP32: weight class w (weight W 2^(w-4)); NULL on set = all 4  */
} pic_state_view;

/* Launch tuning (chosen by the autotuner, or set by hand). */
typedef struct pic_tuning {
  int32_t block;          /* threads per block of the fused particle kernel: 256, 512, 1024 (default 1024) */
  int32_t blocks_per_cu;  /* persistent particle-kernel blocks per compute unit (1-16;
                             0 = as many as the CU's LDS holds at once, at most 8)     */
  int32_t sort_interval;  /* steps between cell sorts (0 = never)                     */
  int32_t use_graph;      /* 1 = replay pic_step through captured HIP graphs; 0 = plain
                             launches (default: measured faster here)                */
  int32_t inline_drain;   /* where the fused pass's queued particles are drained: 0 =
                             chosen by size (default): in the particle kernel itself
                             when the context holds at most 4 discharges that start
                             with at most 4 M particles in all (their steps are
                             launch-bound), else by a drain kernel; 1 = always
                             inline; 2 = never.  The results are the same either
                             way.                                                    */
} pic_tuning;

/* Kernel timing (pic_kernel_times).  Durations in milliseconds summed over the
 * launches recorded since timing was enabled: the streaming pass on every 4th
 * timed step, the sort on every sort, the field and the drain on every 16th
 * timed step (each HIP event costs the stream a few microseconds). */
typedef struct pic_kernel_time {
  double field_ms;      int64_t field_launches;     /* Poisson + field (one block per instance);
                                                       between chained steps also the previous
                                                       step's close                            */
  double particle_ms;   int64_t particle_launches;  /* streaming pass: gather, push, deposit    */
  double drain_ms;      int64_t drain_launches;     /* queued particles: collisions, absorption,
                                                       and the closing kernel when launched    */
  double sort_ms;       int64_t sort_launches;      /* cell sort + compaction (3 kernels)        */
} pic_kernel_time;

int32_t pic_abi_version(void);
const char *pic_status_string(pic_status s);

/* Bytes of device arena needed for n discharges (empty slots need none). */
size_t pic_footprint(const pic_config *cfgs, int32_t n);

/* Create a context over the caller's device arena and initialise every
 * non-empty discharge: Maxwellian load from the seed (Section 2b), deposit of
 * x^0 and, with pullback, the half-step velocity pull-back.  n_inst is the
 * number of slots (<= PIC_MAX_INSTANCES).  Argument errors -> PIC_EINVAL,
 * arena too small -> PIC_ENOMEM, HIP failure -> PIC_EDEVICE. */
pic_status pic_init(const pic_config *cfgs, int32_t n_inst, void *device_arena,
                    size_t arena_bytes, void *hip_stream, pic_ctx **out);

/* Step 1 of Section 2a (Eqs 2-3): zero and rebuild the node deposit A_s of
 * every active discharge from the current positions x^k (int64, 2^-32 units,
 * exact and order independent). */
pic_status pic_deposit(pic_ctx *ctx);

/* Steps 2-3 (Eqs 4-5): from A_s at t_k form Q_n, solve the Poisson equation
 * with phi_0(t_k) = v_rf sin(2 pi f t_k + phase), phi_N = 0 (or the periodic
 * problem), and form the EC cell field (or the MC nodal field).  Accumulates
 * the averaged profiles when due.  PIC_ESTATE when the deposit is stale (call
 * pic_deposit first after pic_mcc or pic_set_state). */
pic_status pic_poisson(pic_ctx *ctx);

/* Steps 4-5 (Eqs 6-9): gather E^k, leapfrog to v^{k+1/2}, x^{k+1}; absorb
 * particles leaving [0, L) and emit secondary electrons; sample the central
 * EEDF when due. */
pic_status pic_gather_push(pic_ctx *ctx);

/* Step 6: null-collision Monte-Carlo collisions on v^{k+1/2} (creates
 * ionisation pairs), then k <- k + 1.  In the FP32 state form, every 16384th
 * call without a sort in between ends with pic_sort (the candidacy offsets
 * need it). */
pic_status pic_mcc(pic_ctx *ctx);

/* n full steps.  Each step is one field kernel plus one fused particle pass
 * (gather, push, boundaries, collisions and the deposit of x^{k+1}); every
 * sort_interval steps the particles are sorted by cell and compacted (in the
 * FP32 state form at least every 16384 steps: its hot word stores each
 * particle's next collision candidacy as an offset from the step of the last
 * sort).  The
 * result is the same particle set as pic_deposit, pic_poisson,
 * pic_gather_push, pic_mcc called in turn. */
pic_status pic_step(pic_ctx *ctx, int32_t n_steps);

/* Sort the particles of every active discharge by cell and drop absorbed ones. */
pic_status pic_sort(pic_ctx *ctx);

/* One particle-rebalancing pass over every discharge with rebalance_ppc > 0
 * (Section 3d names rebalancing, without an algorithm; this one is exact in
 * charge): per species, a cell with more than 2P particles (P = rebalance_ppc)
 * merges, within each group of its particles of equal weight class w < 7 and
 * velocity bin floor(vx / dv) taken in id order, every full quadruple into two
 * particles of class w + 1 at the quadruple's mean offset with velocities
 * v_mean +- delta e (weight exact, momentum and kinetic energy to rounding);
 * a cell with fewer than P/2 splits every particle of class w > 0 into two of
 * class w - 1.  Between steps; the particles end cell-sorted and the next step
 * rebuilds the deposit.  Synchronises.  PIC_ENOMEM if the slot's scratch is
 * too small, PIC_ECAPACITY if splits overflow a capacity. */
pic_status pic_rebalance(pic_ctx *ctx);

/* Counters and monitors of one instance (synchronises). */
pic_status pic_diagnostics(pic_ctx *ctx, int32_t inst, pic_diag *out);

/* For callers that cannot allocate memory (code under stream capture, tight
 * serving loops, harnesses that forbid allocation): the diagnostics of n
 * instances insts[0..n) in one call, out[i] being what pic_diagnostics gives
 * for insts[i].  It allocates nothing, on the device or the host: its device
 * scratch is a fixed array inside the library, PIC_NOALLOC_MAX_INST records of
 * 64 bytes (32 KiB), one copy per GPU, held until the process ends.  n must be
 * in [1, PIC_NOALLOC_MAX_INST] (else PIC_EINVAL, nothing enqueued); an empty
 * or out-of-range instance gives PIC_ESTATE / PIC_EINVAL before any work.
 * Synchronises.  Returns the first device error status among the instances
 * (PIC_OK if none).  Every call on one GPU shares that GPU's array and clears
 * its records first: calls that overlap on one GPU (from several host threads
 * or contexts) race and must be serialised by the caller. */
#define PIC_NOALLOC_MAX_INST 512
pic_status pic_diagnostics_noalloc(pic_ctx *ctx, const int32_t *insts, int32_t n, pic_diag *out);

/* Copy the live particles of one species to host arrays (synchronises).  The
 * order is unspecified; compare by id.  PIC_EINVAL if view->n is too small. */
pic_status pic_get_state(pic_ctx *ctx, int32_t inst, int32_t species, pic_state_view *view);

/* Replace the particles of one species (positions must lie in the domain,
 * offsets in [0, 1), values finite).  Marks the deposit stale. */
pic_status pic_set_state(pic_ctx *ctx, int32_t inst, int32_t species, const pic_state_view *view);

/* Set the step index k of an instance (the RNG counter and the RF phase t_k). */
pic_status pic_set_step(pic_ctx *ctx, int32_t inst, int64_t k);

/* Grid quantities of the last deposit / solve (synchronises).  Any pointer may
 * be NULL.  A_e, A_i: int64[N+1] deposit of x^k; phi: double[N+1]; E: double
 * [N] (EC cells), [N+1] (MC nodes) or [N+2] (second-order EC: cell m-1 at
 * entry m, zero or wrapped ghosts at 0 and N+1); E32: float, same length. */
pic_status pic_get_fields(pic_ctx *ctx, int32_t inst, int64_t *A_e, int64_t *A_i, double *phi,
                          double *E, float *E32);

/* RF-averaged profiles (Section 3a): electron and ion density (m^-3) and
 * potential (V) at the N+1 nodes, and the central EEDF counts.  Any pointer
 * may be NULL.  Synchronises. */
pic_status pic_profiles(pic_ctx *ctx, int32_t inst, double *ne, double *ni, double *phi,
                        int64_t *eedf);

/* Velocity moments and power of one species over the averaged steps
 * (Section 3a), sampled from x^k, v^{k-1/2} and E^k: at the N+1 nodes the mean
 * x-velocity ux = sum w vx / sum w (m/s) and the x-temperature
 * tx = (m/e)(sum w vx^2 / sum w - ux^2) (eV), w the particles' linear
 * weights; per cell the power density given to the species,
 * q W sum_{p in cell j} vx_p E(x_p) / h_j averaged over the samples (W/m^3,
 * E(x) the gathered field).  Any pointer may be NULL.  Synchronises.
 * PIC_ESTATE when the instance was configured with moments = 0. */
pic_status pic_moments(pic_ctx *ctx, int32_t inst, int32_t species, double *ux, double *tx,
                       double *power);

/* Impact distributions of one species at one wall (0 = x = 0, the powered
 * electrode; 1 = x = L) over the averaged steps (Section 3a): energy counts
 * int64[impact_bins + 1] (the last bin counts E >= impact_emax_ev) and angle
 * counts int64[impact_angle_bins] of theta = acos(|vx| / |v|).  Energy bin
 * floor(E * impact_bins / impact_emax_ev) with E = (m / 2e) |v|^2 in eV;
 * angle bin floor(theta_deg * impact_angle_bins / 90), theta = 90 in the last.
 * Either pointer may be NULL.  Synchronises. */
pic_status pic_impacts(pic_ctx *ctx, int32_t inst, int32_t species, int32_t wall, int64_t *energy,
                       int64_t *angle);

/* Checkpoint and resume of one instance.  A checkpoint holds everything a
 * run needs to continue bit for bit: the step index, status and cumulative
 * counters, the averaged profile, EEDF, moment and impact accumulators, and
 * the particle arrays as stored (the deposit of x^k is rebuilt exactly by the
 * next step).  pic_checkpoint_bytes gives the size for the current state;
 * pic_checkpoint_save writes it to a host buffer of at least that size
 * (PIC_EINVAL if smaller; synchronises); pic_checkpoint_load restores it into
 * slot inst of any context whose configuration of that slot is the same (grid,
 * drive, gas, weight, time step, capacity, averaging, seed, state form;
 * PIC_EINVAL if not, with the slot unchanged; in the FP32 state form the
 * restored particles' collision candidacies are re-expressed from the
 * restored step).  The buffer is the caller's; its layout is this library
 * version's own (a checkpoint of another version is refused with PIC_EINVAL). */
pic_status pic_checkpoint_bytes(pic_ctx *ctx, int32_t inst, size_t *bytes);
pic_status pic_checkpoint_save(pic_ctx *ctx, int32_t inst, void *buf, size_t bytes);
pic_status pic_checkpoint_load(pic_ctx *ctx, int32_t inst, const void *buf, size_t bytes);

/* Re-initialise slot inst with cfg (n_cells == 0 empties it), taking memory
 * from the arena pool.  PIC_ENOMEM when the pool cannot hold it. */
pic_status pic_slot_reset(pic_ctx *ctx, int32_t inst, const pic_config *cfg);

/* Empty slot inst and return its memory to the pool. */
pic_status pic_slot_release(pic_ctx *ctx, int32_t inst);

/* Bytes a slot with this configuration takes from the pool. */
size_t pic_slot_bytes(const pic_config *cfg);

/* Free bytes in the pool (largest contiguous block). */
size_t pic_pool_free(const pic_ctx *ctx);

pic_status pic_set_tuning(pic_ctx *ctx, const pic_tuning *t);
pic_status pic_get_tuning(const pic_ctx *ctx, pic_tuning *t);

/* enable = 1 starts kernel timing with HIP events (pic_step then launches
 * without graphs), 0 stops it.  out (may be NULL) receives the sums so far. */
pic_status pic_kernel_times(pic_ctx *ctx, int32_t enable, pic_kernel_time *out);

/* The refined grid of Section 3c (rules 1-4): cells of dx_min within L_buff of
 * each electrode, growing by doubling up to dx_max, neighbours within a factor
 * of two; realised as a dyadic refinement of [0, L] with a 2:1 balance.
 * dx_min and dx_max must be L / 2^a and L / 2^b.  Writes N+1 nodes (if nodes
 * is not NULL and max_nodes suffices) and returns N, or -1 on bad arguments. */
int32_t pic_grid_refined(double L, double dx_min, double dx_max, double L_buff, double *nodes,
                         int32_t max_nodes);

void pic_destroy(pic_ctx *ctx);
const char *pic_last_error(const pic_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* ECPIC_H */
