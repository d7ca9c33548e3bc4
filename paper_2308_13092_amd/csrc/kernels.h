// kernels.h -- host-side launchers of the EC-PIC kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "device.h"

namespace ecpic {

enum Mode : int { M_DEPOSIT = 0, M_PUSH = 1, M_MCC = 2, M_FUSED = 3, M_PULLBACK = 4 };
// launch_particles only: the fused pass whose wavefronts drain their own
// queued particles (256-thread workgroups; no k_drain launch follows).
constexpr int M_FUSED_INLINE = 8;
// Contexts of at most kInlineDrainMaxDischarges discharges that start with
// at most kInlineDrainMaxSlots particles in all take the inline drain by
// default: their steps are bound by launch latency, not by HBM.  With more
// discharges every segment's end drains a few entries per wavefront, and the
// drain kernel wins (FP32, per step: one resolved discharge 42.5 us inline
// against 48.6, four 75 against 79, seven 99 against 72; sixteen small
// served requests 109 against 66).
constexpr int64_t kInlineDrainMaxSlots = 4 << 20;
constexpr int kInlineDrainMaxDischarges = 4;
// Contexts of more than four discharges that start with at least this many
// particles in all sort and drain with larger grids (measured: the batched
// sweep of 1.25e8 particles gains, a served trace of a few million loses).
constexpr int64_t kBatchGridSlots = 32 << 20;

// Particles per thread of a particle-kernel tile (a tile is block x this),
// and the tile of the drain and of the sort scatter, in particles or entries.
constexpr int kParticlesPerThread = 4;
constexpr int kDrainTile = 256;
constexpr int kSortTile = 1024;

// Dynamic LDS bytes of the particle kernels for grids of up to max_n cells.
size_t particle_lds_bytes(int prec, int max_n, int block);
size_t sort_lds_bytes(int max_n, int prec);

// Field solve of every instance; `classes` says which workgroup sizes the
// instances need (bit 0: field_class 1, bit 1: field_class 2).
int field_class(int n_cells);
void launch_field(const InstDev *insts, InstState *states, int n_inst, int classes, int mode,
                  hipStream_t s);
void launch_init(const InstDev *insts, InstState *states, int inst, int species, int prec,
                 double t_ev, int64_t n, hipStream_t s);
// Persistent pass over every particle of every active instance.
hipError_t launch_particles(const InstDev *insts, InstState *states, int n_inst, int prec,
                            int mode, int block, int grid, int max_n, hipStream_t s);
// Drain of the queued particles of a push / collision pass, then, when
// `close`, the pass's closing kernel (which ends the step in the collision and
// fused modes).  A fused step left open is closed by the next field launch
// (mode bit 2).
hipError_t launch_drain(const InstDev *insts, InstState *states, int n_inst, int prec, int mode,
                        int grid, bool close, hipStream_t s);
// Drain workgroups (of kDrainTile threads) resident on one CU at once, for the
// given state form and pass mode (M_PUSH, M_MCC or M_FUSED).
int drain_blocks_per_cu(int prec, int mode);
// The closing kernel of a fused pass alone (after an inline-drained pass).
void launch_finalize(const InstDev *insts, InstState *states, int n_inst, hipStream_t s);
// grid: workgroups of the scatter; count_grid: of the count.
hipError_t launch_sort(const InstDev *insts, InstState *states, int n_inst, int prec, int grid,
                       int count_grid, int max_n, hipStream_t s);
void launch_diag(const InstDev *insts, InstState *states, int inst, int prec, int64_t max_particles,
                 unsigned long long *out, hipStream_t s);
void launch_zero_deposit(const InstDev *insts, InstState *states, int n_inst, hipStream_t s);
// FP32 form: re-express instance inst's hot words, written with epoch E0,
// for a next pass at step k1 with epoch k1 (the caller then sets both).
void launch_reencode(const InstDev *insts, InstState *states, int inst, int64_t E0, int64_t k1,
                     hipStream_t s);
// Velocity moments and power of the discharges whose averaging is due.
void launch_moments(const InstDev *insts, InstState *states, int n_inst, int prec, int grid, int max_n,
                    hipStream_t s);

// Diagnostics reduction output layout (unsigned long long words): k_diag
// writes the live counts, kinetic-energy sums, the electrons' max |vx| and
// summed weight;
// k_deposit_total the two deposit totals.
enum : int { D_LIVE0 = 0, D_LIVE1 = 1, D_KE0 = 2, D_KE1 = 3, D_VMAX = 4, D_DEP0 = 5, D_DEP1 = 6,
             D_WE = 7, D_NWORDS = 8 };   // D_WE: the electrons' summed weight (deposit units)

// Rebalancing scratch of one slot (inside the slot's block): the candidate
// list's keys and values, double-buffered for the radix sorts, their scratch,
// and four counters.
struct RbScratch {
  unsigned long long *words = nullptr;   // [0] listed candidates, [2 + s] split children
  unsigned long long *k64[2] = {nullptr, nullptr};
  uint32_t *k32[2] = {nullptr, nullptr};
  uint32_t *val[2] = {nullptr, nullptr};
  void *temp = nullptr;
  size_t temp_bytes = 0;
  int64_t items = 0;                     // list capacity (both species' capacities)
};
// Scratch the two radix sorts need for `items` entries (0 if it cannot be
// queried); the launcher of one rebalancing pass over instance inst, whose
// state is cell-sorted (it synchronises the stream once, for the list length).
size_t rb_sort_temp_bytes(int64_t items);
hipError_t launch_rebalance(const InstDev *insts, InstState *states, int inst, int N, const RbScratch &sc,
                            hipStream_t st);

// The no-allocation diagnostics (noalloc.hip): a library-owned device array
// of kNoAllocMaxInst records of kNoAllocRecord words.
constexpr int kNoAllocMaxInst = 512;
constexpr int kNoAllocRecord = D_NWORDS;
// Look up the array's device address on `device` (which must be current),
// once per device; noalloc_scratch returns it (nullptr before the setup).
hipError_t noalloc_setup(int device);
unsigned long long *noalloc_scratch(int device);
void launch_fill_zero(unsigned long long *p, int n, hipStream_t s);
void launch_deposit_total(const InstDev *insts, const InstState *states, int inst,
                          unsigned long long *out, hipStream_t s);

}  // namespace ecpic
