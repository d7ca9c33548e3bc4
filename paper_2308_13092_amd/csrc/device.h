// device.h -- data layout and device helpers of the EC-PIC kernels (gfx950).
//
// Layout in HBM (all inside the caller's arena):
//   InstDev[n_inst]    read-only parameters and array pointers of every slot
//   InstState[n_inst]  step index, particle extents, sticky status, counters
//   per slot: a grid block (nodes, widths, walk tables, deposits, potential,
//             fields, averaging accumulators, sort counters) and, per species,
//             two particle buffers (the cell sort ping-pongs between them).
// Particles are stored as structure-of-arrays, each field a contiguous array
// of `cap` elements (cap is a multiple of 64, so every array is 256-B
// aligned):
//   FP32-state form: hw u32 | off f32 | vx f32 | knext i32 | {vy f32, vz f32, id u64}
//   FP64 form:       x f64  | vx f64  | vy f64 | vz f64 | knext i32 | id u64
// The FP32 form's hot word hw holds the cell and the particle's next collision
// candidacy as an offset from the slot's epoch step (see hw_encode), so the
// streaming pass reads 12 bytes per particle and writes at most 12 (the hot
// word only when the cell or the candidacy changed); the fields it never
// reads sit in one 16-B record per particle.
// A dead (absorbed) particle keeps its slot until the next sort with
// hw = kHwDead (FP32) or x = -1 (FP64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ecpic {

// CODATA 2018 (e and k_B exact in the 2019 SI).
constexpr double kQE = 1.602176634e-19;
constexpr double kME = 9.1093837015e-31;
constexpr double kAMU = 1.66053906660e-27;
constexpr double kEPS0 = 8.8541878128e-12;
constexpr double kKB = 1.380649e-23;
constexpr double kMAR = 39.948 * kAMU;
constexpr double kTWO_PI = 2.0 * 3.14159265358979323846;
constexpr double kEXC = 11.5;     // eV, excitation threshold
constexpr double kION = 15.76;    // eV, ionisation threshold
constexpr double kSIGMA_CX = 5.0e-19;
constexpr int32_t kINT32_MAX = 2147483647;

constexpr int kMaxInst = 512;
constexpr int kMaxCells = 2048;
constexpr int kNctr = 24;
// Counters updated by many workgroups are replicated: workgroup b adds into
// replica b % kRep, so no single address takes an atomic from every
// workgroup (same-address device atomics serialise); readers sum replicas.
constexpr int kRep = 32;

// Philox counter tags (counter word 1 = tag | species << 8).
enum : uint32_t {
  TAG_COLL = 0, TAG_EJECT = 1, TAG_GAS = 2, TAG_SEE = 3, TAG_CHILD = 4, TAG_SEE_POS = 5,
  TAG_SKIP = 7, TAG_INIT0 = 0xF0, TAG_INIT1 = 0xF1
};

// Cumulative counters in InstState::ctr.
enum : int {
  C_PSTEPS = 0, C_ABS = 1,            // C_ABS + 2*species + wall (wall 0 left, 1 right)
  C_EABS = 5,                         // absorbed energy, 2^-16 eV units, same indexing
  C_SEE = 9, C_IZ = 10, C_EX = 11, C_EL = 12, C_CX = 13, C_CAND = 14,   // C_CAND + species
  C_BOUND = 16, C_NONFINITE = 17, C_MERGE = 18, C_SPLIT = 19
};

enum : int { ST_CAPACITY = 1, ST_NONFINITE = 2, ST_GROWTH = 4 };

struct InstDev {
  int32_t active, N, bc, gather;
  int32_t nsp, uniform, collisions, eedf_bins;
  int32_t avg_every, eedf_every, int_path, pad0;
  int64_t avg_start, k_stop;
  int64_t cap[2];
  int64_t n_init[2];
  double L, dx, dt, hmin;
  double v_rf, w_rf, phase, growth_limit;
  double n_g, vti, vt_see, gamma_see;
  double nu_max[2], nudt[2], qmdt[2], qW[2], hq[2], mass[2];
  double W, cgauss;            // W: the unit weight of the deposit (class 4 weight x 2^-wunit)
  int32_t wunit, rb_ppc;       // wunit: 4 for a rebalanced discharge, else 0; rb_ppc: target per cell
  double rb_dv[2];             // velocity bin widths of the rebalancing merges (m/s)
  unsigned char *rb_flag[2];   // per cell: 1 merge, 2 split (rebalancing pass)
  double eedf_de, eedf_centre, eedf_half, pad1;
  float qmdt32[2], hq32[2];
  float dtoh32u, pad2[3];
  uint64_t seed;
  // grid block
  double *nodes, *h, *V;
  float *dtoh32, *rf32, *rb32;
  int *runs;                   // per cell: first | last << 16 of its run of equal widths
  int64_t *A[2][2];            // [k parity][species]
  double *phi, *E64;
  float *E32;
  double *accA[2], *acc_phi;
  unsigned long long *eedf;
  unsigned long long *impact;  // [species][wall][energy bins + 1 | angle bins]
  double *accM1[2], *accM2[2];  // averaged sum w vx, sum w vx^2 per node (CIC weights)
  double *accP[2];              // averaged sum vx E(x) per cell
  int32_t imp_bins, imp_abins;
  double imp_escale, imp_ascale;  // bins / emax (1/eV), angle bins / 90 (1/deg)
  int moments;                    // accumulate accM1, accM2, accP on the averaged steps
  unsigned long long *scount[2], *scursor[2];
  int4 *queue[2];              // per-species queue of particles for the drain kernel (QRec)
  // particles
  char *pbuf[2][2];            // [species][buffer]
};

// The instance table is written by the host between kernels and only read on
// the device.  Kernels read it through the constant address space, so the
// compiler may use scalar loads and keep its fields in registers across the
// kernels' stores to other memory (through a generic pointer every field
// would be reloaded after every store, since the store might alias it).
#define ECPIC_CONST __attribute__((address_space(4)))
typedef const ECPIC_CONST InstDev CInst;
__device__ __forceinline__ CInst *cinst(const InstDev *p) { return (CInst *)p; }

struct InstState {
  int64_t k;
  // FP32 form: the step the hot words' candidacy offsets count from (set by
  // every sort and re-encoding; k - epoch stays below kRebaseSteps + 1)
  int64_t epoch;
  int32_t status, parity;
  int32_t frozen, pad0;
  int64_t extent[2];
  unsigned long long step_live[2][kRep];
  unsigned long long step_absorbed[2][kRep];
  int64_t n_live[2];
  unsigned long long ctr[kNctr][kRep];
  double field_energy, ne_max;
  int32_t n_samples, eedf_samples;
  int64_t sort_live[2];
  unsigned long long qcount[2];   // queued particles of the current pass
  // Particles appended in this pass: electrons in bits 0-31, ions in bits
  // 32-63 (fewer than 2^31 each, capacity being at most 2^30), so one atomic
  // reserves the two products of an ionisation.  It has a 128-B line of its
  // own: its atomics kept evicting the line of k, parity and extent, which
  // every drain tile reads (large discharge: drain 0.072 -> 0.051 ms).
  alignas(128) unsigned long long append;
  unsigned long long append_pad[15];
};

// ---------------------------------------------------------------------------
// The FP32 form's hot word
// ---------------------------------------------------------------------------
// bits 0-11  cell (0xFFF: dead slot; grids have at most 2048 cells)
// bits 12-27 c: the particle's next collision candidacy knext as an offset
//            from the slot's epoch E, knext = E + c
// bits 28-30 weight class w: the particle's weight is W 2^(w-4) (4 unless
//            the discharge is rebalanced)
// bit  31    far: the knext array holds the candidacy (see hw_encode)
// A particle is a candidate at the pass of step k when c == k - E, which
// needs no read of the knext array and no change of the word from step to
// step: a particle that keeps its cell keeps its word, and the streaming
// pass does not store it.  Every sort re-expresses the offsets from the
// step it runs before (E := k), and the host forces one at least every
// kRebaseSteps steps, so k - E never reaches kCntMax.
constexpr uint32_t kHwDead = 0xFFFFFFFFu;
constexpr uint32_t kHwCell = 0xFFFu;
constexpr int kHwShift = 12;
constexpr uint32_t kCntMax = (1u << 16) - 1u;
constexpr int64_t kRebaseSteps = 16384;
static_assert(kRebaseSteps < (int64_t)kCntMax, "the epoch offset must stay below the far sentinel");
constexpr int kHwClassShift = 28;
constexpr uint32_t kHwClass = 7u << kHwClassShift;
constexpr uint32_t kHwFar = 1u << 31;
constexpr int kClassUnit = 4;   // the class of weight W
__host__ __device__ inline int hw_cell(uint32_t w) { return (int)(w & kHwCell); }
__host__ __device__ inline bool hw_live(uint32_t w) { return (w & kHwCell) != kHwCell; }
__host__ __device__ inline uint32_t hw_cnt(uint32_t w) { return (w >> kHwShift) & kCntMax; }
__host__ __device__ inline bool hw_far(uint32_t w) { return (w & kHwFar) != 0u; }
__host__ __device__ inline int hw_class(uint32_t w) { return (int)((w >> kHwClassShift) & 7u); }
// The hot word of a particle of weight class cls in `cell` whose next
// candidacy is step knext, for a slot with epoch E whose next pass is step k
// (E <= k < E + kCntMax):
//   k <= knext < E + kCntMax  c = knext - E;
//   knext < k (overdue)       far, c = k - E: a candidate at the next pass,
//                             as a candidacy in the past is;
//   knext >= E + kCntMax      far, c = kCntMax: never a candidate before the
//                             next re-expression, which reads the knext array.
__host__ __device__ inline uint32_t hw_encode(int cell, int64_t knext, int64_t k, int64_t E, int cls) {
  const uint32_t base = (uint32_t)cell | ((uint32_t)cls << kHwClassShift);
  const int64_t w = knext - E;
  if (knext >= k && w < (int64_t)kCntMax) return base | ((uint32_t)w << kHwShift);
  const uint32_t c = knext < k ? (uint32_t)(k - E) : kCntMax;
  return base | (c << kHwShift) | kHwFar;
}
// The particle's next candidacy (far_knext: its entry of the knext array).
__host__ __device__ inline int64_t hw_knext(uint32_t w, int32_t far_knext, int64_t E) {
  return hw_far(w) ? (int64_t)far_knext : E + (int64_t)hw_cnt(w);
}
// Whether the particle is a candidate at the pass of step k (kE = k - E).
__host__ __device__ inline bool hw_due(uint32_t w, uint32_t kE) { return hw_cnt(w) == kE; }
// The same word in another cell.
__host__ __device__ inline uint32_t hw_move(uint32_t w, int cell) {
  return (w & ~kHwCell) | (uint32_t)cell;
}

// ---------------------------------------------------------------------------
// Particle buffer views
// ---------------------------------------------------------------------------
// FP32 form: the fields every step streams (hw, off, vx) are separate
// arrays; the ones only collisions, emission, diagnostics and the sort touch
// (vy, vz, id) form one 16-B record per particle, so that handling a single
// particle costs one memory line for them instead of three.  knext is read
// and written only for far particles (see hw_encode).
struct Cold32 {
  float vy, vz;
  uint64_t id;
};
struct P32 {
  uint32_t *hw; float *off, *vx; int32_t *knext; Cold32 *cold;
};
struct P64 {
  double *x, *vx, *vy, *vz; int32_t *knext; uint64_t *id;
};
__host__ __device__ inline P32 view32(char *b, int64_t cap) {
  P32 p;
  p.hw = reinterpret_cast<uint32_t *>(b);
  p.off = reinterpret_cast<float *>(b + 4 * cap);
  p.vx = reinterpret_cast<float *>(b + 8 * cap);
  p.knext = reinterpret_cast<int32_t *>(b + 12 * cap);
  p.cold = reinterpret_cast<Cold32 *>(b + 16 * cap);   // cap is a multiple of 64
  return p;
}
__host__ __device__ inline P64 view64(char *b, int64_t cap) {
  P64 p;
  p.x = reinterpret_cast<double *>(b);
  p.vx = reinterpret_cast<double *>(b + 8 * cap);
  p.vy = reinterpret_cast<double *>(b + 16 * cap);
  p.vz = reinterpret_cast<double *>(b + 24 * cap);
  p.knext = reinterpret_cast<int32_t *>(b + 32 * cap);
  p.id = reinterpret_cast<uint64_t *>(b + 36 * cap);
  return p;
}
constexpr int64_t kBytes32 = 32, kBytes64 = 44;

// Global-address-space access.  The particle arrays are reached through
// pointers stored in the instance table, where the compiler no longer knows
// they are global memory and would emit FLAT instructions; FLAT operations
// also count against the LDS wait counter, so every LDS access after a store
// would wait for that store to reach memory.
//
// The vector forms below carry the non-temporal hint: each is used on data
// that a pass reads or writes once, in whole lines (the streaming pass
// touches every particle once per step), so those lines stream through L2
// instead of displacing lines that are reused (the LDS tables' sources, the
// deposits, the queues).  On the large discharge this took the streaming
// pass from 0.430 to 0.373 ms.  Single-element stores keep the plain form:
// their partial lines must merge in L2 (the sort's scatter with the hint took
// 2.9 ms instead of 1.25).
#define ECPIC_GLOBAL __attribute__((address_space(1)))
typedef int ecpic_iv4 __attribute__((ext_vector_type(4)));
typedef float ecpic_fv4 __attribute__((ext_vector_type(4)));
typedef double ecpic_dv2 __attribute__((ext_vector_type(2)));
template <class V, class T>
__device__ __forceinline__ V gload(const T *p) {
  return *(const ECPIC_GLOBAL V *)p;
}
template <class V, class T>
__device__ __forceinline__ void gstore(T *p, V v) {
  *(ECPIC_GLOBAL V *)p = v;
}
__device__ __forceinline__ int4 gload4(const int *p) {
  const ecpic_iv4 v = __builtin_nontemporal_load((const ECPIC_GLOBAL ecpic_iv4 *)p);
  return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float4 gload4(const float *p) {
  const ecpic_fv4 v = __builtin_nontemporal_load((const ECPIC_GLOBAL ecpic_fv4 *)p);
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ double2 gload2(const double *p) {
  const ecpic_dv2 v = __builtin_nontemporal_load((const ECPIC_GLOBAL ecpic_dv2 *)p);
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void gstore4(int *p, int a, int b, int c, int d) {
  ecpic_iv4 v = {a, b, c, d};
  __builtin_nontemporal_store(v, (ECPIC_GLOBAL ecpic_iv4 *)p);
}
// One 16-B queue record (plain: the drain's records are read once, in order).
__device__ __forceinline__ int4 gload_rec(const int4 *p) {
  const ecpic_iv4 v = *(const ECPIC_GLOBAL ecpic_iv4 *)p;
  return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gstore_rec(int4 *p, const int4 &r) {
  ecpic_iv4 v = {r.x, r.y, r.z, r.w};
  *(ECPIC_GLOBAL ecpic_iv4 *)p = v;
}
// One particle's cold record as one 16-B load / store.
__device__ __forceinline__ Cold32 gload_cold(const Cold32 *p) {
  const ecpic_iv4 v = *(const ECPIC_GLOBAL ecpic_iv4 *)p;
  return Cold32{__int_as_float(v.x), __int_as_float(v.y),
                (uint64_t)(uint32_t)v.z | ((uint64_t)(uint32_t)v.w << 32)};
}
__device__ __forceinline__ void gstore_cold(Cold32 *p, const Cold32 &c) {
  ecpic_iv4 v = {__float_as_int(c.vy), __float_as_int(c.vz), (int)(uint32_t)c.id,
                 (int)(uint32_t)(c.id >> 32)};
  *(ECPIC_GLOBAL ecpic_iv4 *)p = v;
}
__device__ __forceinline__ void gstore4(float *p, float a, float b, float c, float d) {
  ecpic_fv4 v = {a, b, c, d};
  __builtin_nontemporal_store(v, (ECPIC_GLOBAL ecpic_fv4 *)p);
}
__device__ __forceinline__ void gstore2(double *p, double a, double b) {
  ecpic_dv2 v = {a, b};
  __builtin_nontemporal_store(v, (ECPIC_GLOBAL ecpic_dv2 *)p);
}

// ---------------------------------------------------------------------------
// Values that are the same on every lane, made known as such to the compiler
// (they then live in scalar registers).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ int64_t uni(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xFFFFFFFFll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}
__device__ __forceinline__ double uni(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xFFFFFFFFll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and the uniform / normal variates.
// key = particle id, counter = (k, tag | species << 8, seed_lo, seed_hi).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint32_t k, uint32_t tag, uint64_t seed, uint64_t id) {
  uint32_t c0 = k, c1 = tag, c2 = (uint32_t)seed, c3 = (uint32_t)(seed >> 32);
  uint32_t k0 = (uint32_t)id, k1 = (uint32_t)(id >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ double u32d(uint32_t r) { return ((double)r + 0.5) * 0x1p-32; }
__device__ __forceinline__ double u52d(uint32_t a, uint32_t b) {
  const uint64_t m = ((uint64_t)a << 20) | (uint64_t)(b >> 12);
  return ((double)m + 0.5) * 0x1p-52;
}
__device__ __forceinline__ void box_muller(double ua, double ub, double &z0, double &z1) {
  const double r = sqrt(-2.0 * log(ua));
  const double a = kTWO_PI * ub;
  z0 = r * cos(a);
  z1 = r * sin(a);
}
// First candidate step after `base - 1`: base + floor(-ln u / (nu_max dt)).
__device__ __forceinline__ int32_t geometric(double base, double u, double nudt) {
  double g = floor(-log(u) / nudt);
  g = fmin(g, (double)kINT32_MAX);
  const double out = fmin(base + g, (double)kINT32_MAX);
  return (int32_t)out;
}
__device__ __forceinline__ int32_t next_candidate(uint64_t id, int64_t k, int s, uint64_t seed,
                                                  double nudt) {
  if (!(nudt > 0.0)) return kINT32_MAX;
  const uint4 r = philox((uint32_t)k, TAG_SKIP | (uint32_t)(s << 8), seed, id);
  return geometric((double)(k + 1), u52d(r.x, r.y), nudt);
}

// ---------------------------------------------------------------------------
// Closing a pass of one instance
// ---------------------------------------------------------------------------
// Whether the instance takes part in passes: active, not frozen by an error,
// and short of its k_stop.
__device__ __forceinline__ bool pass_open(CInst &I, const InstState &S) {
  return I.active && S.frozen == 0 && !(I.k_stop > 0 && S.k >= I.k_stop);
}

// Close a pass: clear the queues; in the passes that end a step (kEndsStep),
// new particles join the extents, the live count is updated and checked
// against the growth limit, and k advances.  Called by the 64 lanes of one
// wavefront for an open instance: lane (species << 5 | replica) takes one
// replica of the step's live and absorbed counts, the halves are summed with
// shuffles (exact integers), and lane 0 writes the state.  kFused: the live
// count comes from the pass's own tally instead of the previous count.
static_assert(kRep == 32, "one lane per (species, replica)");
template <bool kEndsStep, bool kFused>
__device__ inline void close_pass(CInst &I, InstState &S, int lane) {
  unsigned long long lv = 0, ab = 0;
  if (kEndsStep) {
    const int s = lane >> 5, r = lane & 31;
    if (s < I.nsp) {
      lv = S.step_live[s][r];
      ab = S.step_absorbed[s][r];
      S.step_live[s][r] = 0;
      S.step_absorbed[s][r] = 0;
    }
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) {
      lv += __shfl_xor(lv, o, 64);
      ab += __shfl_xor(ab, o, 64);
    }
  }
  const unsigned long long lv_s[2] = {lv, __shfl(lv, 32, 64)};
  const unsigned long long ab_s[2] = {ab, __shfl(ab, 32, 64)};
  if (lane != 0) return;
  for (int s = 0; s < I.nsp; ++s) {
    S.qcount[s] = 0;
    if (kEndsStep) {
      int64_t add = (int64_t)((S.append >> (32 * s)) & 0xFFFFFFFFull);
      if (S.extent[s] + add > I.cap[s]) add = I.cap[s] - S.extent[s];
      S.extent[s] += add;
      const int64_t live = kFused ? ((int64_t)lv_s[s] - (int64_t)ab_s[s] + add)
                                  : (S.n_live[s] - (int64_t)ab_s[s] + add);
      S.n_live[s] = live;
      if ((double)live > I.growth_limit * (double)I.n_init[s] && I.n_init[s] > 0)
        S.status |= ST_GROWTH;
    }
  }
  if (kEndsStep) {
    S.append = 0;
    S.k += 1;
    if (S.status != 0) S.frozen = 1;
  }
}

// ---------------------------------------------------------------------------
// Persistent grids over concatenated segments (instance x species)
// ---------------------------------------------------------------------------
// prefix[1..nseg] hold the segments' tile counts; this turns them into the
// exclusive prefix (prefix[0] = 0, prefix[nseg] = the total).  Up to 8
// segments thread 0 sums them; beyond, the first wavefront scans: each lane
// sums a run of consecutive counts (at most 16 for 512 discharges), the
// runs' sums are scanned with shuffles, and each lane adds its base back.  Every thread of the workgroup calls it after
// writing its counts (it synchronises on entry and on exit).
__device__ inline void tile_prefix(int *prefix, int nseg) {
  __syncthreads();
  if (nseg <= 8) {
    // A few discharges: a serial sum is shorter than the shuffle chain.
    if (threadIdx.x == 0) {
      prefix[0] = 0;
      for (int s = 2; s <= nseg; ++s) prefix[s] += prefix[s - 1];
    }
  } else if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const int per = (nseg + 63) / 64;
    const int b = 1 + lane * per, e = min(b + per, nseg + 1);
    int run = 0;
    for (int s = b; s < e; ++s) {
      run += prefix[s];
      prefix[s] = run;
    }
    int inc = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(inc, o, 64);
      if (lane >= o) inc += v;
    }
    const int base = inc - run;
    for (int s = b; s < e; ++s) prefix[s] += base;
    if (lane == 0) prefix[0] = 0;
  }
  __syncthreads();
}

// The segment that holds tile `tile` (< prefix[nseg]): the first s with
// prefix[s + 1] > tile, by bisection (empty segments are passed over).
__device__ __forceinline__ int segment_of(const int *prefix, int nseg, int64_t tile) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid + 1] <= tile)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

}  // namespace ecpic
