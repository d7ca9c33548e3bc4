// kernels_particles.hip -- the particle side of the EC-PIC step on gfx950.
//
// One persistent kernel template serves every particle pass.  The grid is a
// fixed number of workgroups (a multiple of the CU count); each workgroup
// takes an equal contiguous range of 4*BLOCK-particle tiles of the
// concatenated (instance, species) segments, so any number of instances of
// any size advance in one launch.  Per tile a thread owns 4 consecutive
// particles and reads them with 16-byte vector loads, so a wavefront streams
// 1 KB of each state array per instruction.
//
// Modes:
//   M_DEPOSIT   Eqs 2-3: fixed-point CIC weights of x^k into the LDS copy of
//               the node deposit, flushed to HBM with int64 atomics.
//   M_PUSH      Eqs 6-9: gather E^k, leapfrog, absorption at the electrodes,
//               secondary emission, central EEDF sample.
//   M_MCC       Section 2a collisions: null collisions of the particles due this step,
//               ionisation pairs appended, then k <- k+1.
//   M_FUSED     M_PUSH + M_MCC + the deposit of x^{k+1}, in one pass.
//   M_PULLBACK  v^{-1/2} = v^0 - (q/m) E^0 dt/2 (initial-state option).
//
// Gather tables (E, dt/h, neighbour ratios; for FP64 the nodes and widths)
// are staged in LDS when a workgroup enters a segment.  The deposit goes to
// an LDS int64 copy of the grid: each lane sums its own consecutive particles
// of one cell in registers (the usual case in a cell-sorted state) and adds
// the sum with one LDS atomic per node; a particle in another cell goes to
// LDS at once (the quadratic-spline deposit of second-order EC always does).
// At the end of a segment the nonzero LDS entries are added to HBM with one
// atomic each.
#include "device.h"
#include "kernels.h"

namespace ecpic {

constexpr double kHALF_ME_OVER_QE = (0.5 * kME) / kQE;
constexpr double kTWO_QE_OVER_ME = (2.0 * kQE) / kME;
constexpr double kTWO_ME_OVER_M = (2.0 * kME) / kMAR;
constexpr int kPPT = kParticlesPerThread;   // particles per thread per tile (a multiple of 4)
static_assert(kPPT % 4 == 0, "vector loads move 4 particles");
constexpr float kWalkLimit = 4194304.0f;    // |sigma| beyond 2^22 cells: out of any grid

// The grid parameters that locating and walking a particle need.  The
// streaming kernel reads them once per segment into registers: read through
// the instance table inside the particle loop they would be reloaded from
// memory for every particle, since the loop's stores could alias the table.
struct GridPar {
  int N, periodic, uniform;
  double dx;
};
__device__ __forceinline__ GridPar grid_par(CInst &I) {
  return GridPar{I.N, I.bc == 1 ? 1 : 0, I.uniform, I.dx};
}

// ---------------------------------------------------------------------------
// Locating positions (FP64 form) -- the deposit contract.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int locate64(const GridPar &G, const double *nodes, double x, double &xi) {
  const int N = G.N;
  int j;
  double f;
  if (G.uniform) {
    const double s = x / G.dx;
    const double jf = floor(s);
    j = (int)jf;
    if (j >= N) j = N - 1;
    f = s - (double)j;
  } else {
    int lo = 0, hi = N;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (nodes[mid] <= x) lo = mid;
      else hi = mid;
    }
    j = lo;
    f = (x - nodes[j]) / (nodes[j + 1] - nodes[j]);
  }
  xi = fmin(fmax(f, 0.0), 1.0);
  return j;
}

// FP32 state of an FP64 position: off = (float) xi, moved to the next cell when
// it rounds up to 1 (kept below 1 in the last cell of a bounded grid).
__device__ __forceinline__ void to_state32(CInst &I, double x, int &cell, float &off) {
  double xi;
  int j = locate64(grid_par(I), I.nodes, x, xi);
  float o = (float)xi;
  if (o >= 1.0f) {
    if (j + 1 < I.N) { j += 1; o = 0.0f; }
    else if (I.bc == 1) { j = 0; o = 0.0f; }
    else o = 0x1.fffffep-1f;
  }
  cell = j;
  off = o;
}

__device__ __forceinline__ void weights(double xi, int64_t &w0, int64_t &w1) {
  w1 = (int64_t)rint(xi * 4294967296.0);
  w0 = (int64_t)4294967296LL - w1;
}
// The same weights for an FP32 offset: off * 2^32 is exact in FP32 and below
// 2^32, so rounding it half-to-even in FP32 equals rint((double)off * 2^32).
__device__ __forceinline__ void weights32(float off, int64_t &w0, int64_t &w1) {
  const uint32_t r = (uint32_t)rintf(off * 4294967296.0f);
  w1 = (int64_t)r;
  w0 = (int64_t)4294967296LL - (int64_t)r;
}

// Second-order EC (uniform grids): quadratic-spline (S2) deposit to the
// nearest node n and its neighbours.  With d the signed distance to n in
// cells (n = j, d = xi for xi < 1/2; n = j + 1, d = xi - 1 otherwise),
// a = 1/2 - d and b = 1/2 + d formed in FP64, the fixed-point weights are
// wl = rint(a^2 2^31) to n - 1, wr = rint(b^2 2^31) to n + 1 and
// wc = 2^32 - wl - wr to n (the spline's (1/2-d)^2/2, 3/4-d^2, (1/2+d)^2/2).
__device__ __forceinline__ void weights_s2(int j, double xi, int &n, int64_t &wl, int64_t &wc,
                                           int64_t &wr) {
  const bool up = xi >= 0.5;
  n = up ? j + 1 : j;
  const double a = up ? 1.5 - xi : 0.5 - xi;
  const double b = up ? xi - 0.5 : 0.5 + xi;
  wl = (int64_t)rint((a * a) * 2147483648.0);
  wr = (int64_t)rint((b * b) * 2147483648.0);
  wc = (int64_t)4294967296LL - wl - wr;
}
// Node of an S2 weight at m in [-1, N+1]: beyond a Dirichlet end it goes to
// the electrode node, a periodic grid wraps it.
__device__ __forceinline__ int fold_s2(int m, int N, int periodic) {
  if (periodic) return m < 0 ? m + N : (m > N ? m - N : m);
  return min(max(m, 0), N);
}
// Linear gather of the cell-centred field between the two centres around
// (j, xi); the table holds N + 2 values, entry m being cell m - 1's field
// (entries 0 and N + 1 are the ghosts outside the ends).
__device__ __forceinline__ float gather_ec2_32(const float *E, int j, float off) {
  const bool up = off >= 0.5f;
  const int m = up ? j + 1 : j;
  const float t = up ? off - 0.5f : off + 0.5f;
  return ((1.0f - t) * E[m]) + (t * E[m + 1]);
}
__device__ __forceinline__ double gather_ec2_64(const double *E, int j, double xi) {
  const bool up = xi >= 0.5;
  const int m = up ? j + 1 : j;
  const double t = up ? xi - 0.5 : xi + 0.5;
  return (1.0 - t) * E[m] + t * E[m + 1];
}

// ---------------------------------------------------------------------------
// FP32 cell walk.  The contract is the cell-by-cell walk
//   while sigma < 0:  j -= 1 (wrap), sigma = 1 + sigma * (h_{j+1}/h_j)
//   while sigma >= 1: sigma = (sigma - 1) * (h_j/h_{j+1}), j += 1 (wrap)
// in FP32, with the ratios rounded to FP32.  Inside a run of cells whose FP32
// ratios are exactly 1 every step is sigma -= 1 (exact) or sigma += 1 (exact
// while sigma <= -1), so m steps collapse into one operation with the same
// result: sigma - m moving right, and fl(sigma + m) moving left (only the last
// step rounds; if it rounds up to 1 the contract's next step moves one cell
// right to offset 0).  The only ratios that are not 1 are met when leaving a
// run: h_hi/h_{hi+1} at its last cell and h_lo/h_{lo-1} before its first.
//
// Each cell's LDS entry is {dt/h_j, run (first | last << 16), ratio leaving
// the run forward, ratio leaving it backward}; a periodic grid uses runs of
// one cell (its walk wraps).  One walk step from cell j uses only j's entry:
// the collapsed move inside the run or, when sigma leaves the run, the move to
// its end and across into the next cell.  Almost every particle is done after
// the first step, which needs no data beyond the entry already read for it.
// ---------------------------------------------------------------------------
enum : int { W_IN = 0, W_LEFT = -1, W_RIGHT = 1, W_BAD = 2, W_MORE = 3, W_FIRST = 4 };

__device__ __forceinline__ int walk_step(const int4 T, int N, int periodic, int &j, float &sig) {
  const int lo = T.y & 0xFFFF, hi = T.y >> 16;
  if (sig >= 1.0f) {
    const float m = floorf(sig);
    const int avail = hi - j;
    if (m <= (float)avail) {
      j += (int)m;
      sig = sig - m;
      return W_IN;
    }
    float r = sig - (float)avail;       // exact: at the run's last cell
    r = (r - 1.0f) * __int_as_float(T.z);
    j = hi + 1;
    if (j >= N) {
      if (!periodic) return W_RIGHT;
      j -= N;
    }
    sig = r;
    return (r >= 1.0f) ? W_MORE : W_IN;
  }
  const float m = -floorf(sig);
  const int avail = j - lo;
  if (m <= (float)avail) {
    j -= (int)m;
    sig = sig + m;
    if (sig >= 1.0f) {   // rounded up to the right edge: next cell, offset 0
      sig = 0.0f;
      j += 1;
    }
    return W_IN;
  }
  float r = sig + (float)avail;         // exact: at the run's first cell
  j = lo - 1;
  if (j < 0) {
    if (!periodic) return W_LEFT;
    j += N;
  }
  const float tt = r * __int_as_float(T.w);
  r = 1.0f + tt;
  sig = r;
  return (r >= 0.0f && r < 1.0f) ? W_IN : W_MORE;
}

// A uniform grid is one run without wrap-around ratios: the whole walk is one
// floor (bounded), or one floor and a wrap (periodic).  A left walk that
// passes cell 0 of a bounded grid has left it, even when its last step
// rounds up to the right edge (the carry would bring it back to x = 0).
__device__ __forceinline__ int walk_uniform(int N, int periodic, int &j, float &sig) {
  const float m = floorf(sig);
  float r = sig - m;
  int jj = j + (int)m;
  if (!periodic && jj < 0) return W_LEFT;
  if (r >= 1.0f) {
    r = 0.0f;
    jj += 1;
  }
  if (periodic) {
    jj %= N;
    if (jj < 0) jj += N;
  } else if (jj >= N) {
    return W_RIGHT;
  }
  j = jj;
  sig = r;
  return W_IN;
}

// First walk step of a particle whose sigma left [0, 1): W_IN, W_LEFT/W_RIGHT,
// W_BAD (non-finite, or beyond any grid in a periodic box) or W_MORE.
__device__ __forceinline__ int walk_first(const GridPar &G, const int4 T, int &j, float &sig) {
  if (!(fabsf(sig) < kWalkLimit)) {
    if (sig != sig || G.periodic) return W_BAD;
    return sig < 0.0f ? W_LEFT : W_RIGHT;
  }
  if (G.uniform) return walk_uniform(G.N, G.periodic, j, sig);
  return walk_step(T, G.N, G.periodic, j, sig);
}

// ---------------------------------------------------------------------------
// Collisions (argon, analytic cross sections), in FP64 for both state forms.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double sig_el(double e) { return 1.0e-19 / (1.0 + e / 20.0); }
__device__ __forceinline__ double lnx_over_x(double e, double thr, double amp) {
  if (!(e > thr)) return 0.0;
  const double x = e / thr;
  return amp * log(x) / x;
}
__device__ __forceinline__ void iso_dir(double ua, double ub, double &dx, double &dy, double &dz) {
  const double ct = 1.0 - 2.0 * ua;
  const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
  const double a = kTWO_PI * ub;
  dx = ct;
  dy = st * cos(a);
  dz = st * sin(a);
}
__device__ __forceinline__ void gas_velocity(CInst &I, uint64_t id, int64_t k, int s,
                                             double &gx, double &gy, double &gz) {
  const uint4 g = philox((uint32_t)k, TAG_GAS | (uint32_t)(s << 8), I.seed, id);
  double z0, z1, z2, z3;
  box_muller(u32d(g.x), u32d(g.y), z0, z1);
  box_muller(u32d(g.z), u32d(g.w), z2, z3);
  gx = I.vti * z0;
  gy = I.vti * z1;
  gz = I.vti * z2;
}

// Electron null collision.  Returns the process (0 null, 1 elastic,
// 2 excitation, 3 ionisation); ej receives the ejected electron's velocity.
__device__ int collide_electron(CInst &I, uint64_t id, int64_t k, double &vx, double &vy,
                                double &vz, bool &bound, double ej[3]) {
  const uint4 r = philox((uint32_t)k, TAG_COLL, I.seed, id);
  const double u1 = u32d(r.x), u2 = u32d(r.y), u3 = u32d(r.z);
  const double v2 = (vx * vx + vy * vy) + vz * vz;
  const double speed = sqrt(v2);
  const double eps = kHALF_ME_OVER_QE * v2;
  const double nu_el = (I.n_g * sig_el(eps)) * speed;
  const double nu_ex = (I.n_g * lnx_over_x(eps, kEXC, 2.7e-20)) * speed;
  const double nu_iz = (I.n_g * lnx_over_x(eps, kION, 7.6e-20)) * speed;
  const double s_el_ex = nu_el + nu_ex;
  const double s_all = s_el_ex + nu_iz;
  const double R = u1 * I.nu_max[0];
  bound = s_all > I.nu_max[0];
  const int proc = (R < nu_el) ? 1 : ((R < s_el_ex) ? 2 : ((R < s_all) ? 3 : 0));
  if (proc == 0) return 0;
  double dx, dy, dz;
  iso_dir(u2, u3, dx, dy, dz);
  double s;
  if (proc == 1) {
    const double cos_chi = ((vx * dx + vy * dy) + vz * dz) / speed;
    const double f = 1.0 - kTWO_ME_OVER_M * (1.0 - cos_chi);
    s = speed * sqrt(f);
  } else if (proc == 2) {
    s = sqrt((eps - kEXC) * kTWO_QE_OVER_ME);
  } else {
    s = sqrt((0.5 * (eps - kION)) * kTWO_QE_OVER_ME);
  }
  vx = s * dx;
  vy = s * dy;
  vz = s * dz;
  if (proc == 3) {
    const uint4 q = philox((uint32_t)k, TAG_EJECT, I.seed, id);
    double ex, ey, ez;
    iso_dir(u32d(q.x), u32d(q.y), ex, ey, ez);
    ej[0] = s * ex;
    ej[1] = s * ey;
    ej[2] = s * ez;
  }
  return proc;
}

// Ion charge exchange with a gas atom drawn from the gas Maxwellian.
__device__ bool collide_ion(CInst &I, uint64_t id, int64_t k, double &vx, double &vy,
                            double &vz, bool &bound) {
  const uint4 r = philox((uint32_t)k, TAG_COLL | (1u << 8), I.seed, id);
  const double u1 = u32d(r.x);
  double gx, gy, gz;
  gas_velocity(I, id, k, 1, gx, gy, gz);
  const double ddx = vx - gx, ddy = vy - gy, ddz = vz - gz;
  const double g = sqrt((ddx * ddx + ddy * ddy) + ddz * ddz);
  const double nu = (I.n_g * kSIGMA_CX) * g;
  bound = nu > I.nu_max[1];
  const bool cx = (u1 * I.nu_max[1]) < nu;
  if (cx) {
    vx = gx;
    vy = gy;
    vz = gz;
  }
  return cx;
}

// ---------------------------------------------------------------------------
// Shared state of a workgroup
// ---------------------------------------------------------------------------
struct Smem {
  int seg_prefix[2 * kMaxInst + 1];
  unsigned long long ctr[kNctr];
};

// Sum over the 64 lanes of a wavefront (every lane gets the total).
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Per-thread accumulation of up to kPPT deposits: consecutive particles of a
// thread in one cell (the usual case after a cell sort) are summed in
// registers and added to LDS once; a different cell goes to LDS at once.
// LDS 64-bit atomics on scattered addresses cost less than a cross-lane merge.
struct DepAcc {
  bool has;
  int key;
  unsigned long long a0, a1;
  __device__ void init() { has = false; key = 0; a0 = 0; a1 = 0; }
  // Add the held run to the workgroup's LDS accumulator.
  __device__ void flush(int64_t *sA) {
    if (has) {
      atomicAdd(reinterpret_cast<unsigned long long *>(&sA[key]), a0);
      atomicAdd(reinterpret_cast<unsigned long long *>(&sA[key + 1]), a1);
    }
  }
  __device__ void add(int64_t *sA, int j, int64_t w0, int64_t w1) {
    if (!has) { has = true; key = j; a0 = (unsigned long long)w0; a1 = (unsigned long long)w1; }
    else if (j == key) { a0 += (unsigned long long)w0; a1 += (unsigned long long)w1; }
    else {
      atomicAdd(reinterpret_cast<unsigned long long *>(&sA[j]), (unsigned long long)w0);
      atomicAdd(reinterpret_cast<unsigned long long *>(&sA[j + 1]), (unsigned long long)w1);
    }
  }
};

// S2 deposit of one particle into the workgroup's LDS grid (the periodic
// fold of nodes 0 and N happens when the grid is flushed).
__device__ __forceinline__ void lds_deposit_s2(int64_t *sA, const GridPar &G, int j, double xi,
                                               int sh = 0) {
  int n;
  int64_t wl, wc, wr;
  weights_s2(j, xi, n, wl, wc, wr);
  wl <<= sh;
  wc <<= sh;
  wr <<= sh;
  atomicAdd(reinterpret_cast<unsigned long long *>(&sA[fold_s2(n - 1, G.N, G.periodic)]),
            (unsigned long long)wl);
  atomicAdd(reinterpret_cast<unsigned long long *>(&sA[n]), (unsigned long long)wc);
  atomicAdd(reinterpret_cast<unsigned long long *>(&sA[fold_s2(n + 1, G.N, G.periodic)]),
            (unsigned long long)wr);
}

// One weight straight into a deposit in HBM.  Periodic nodes 0 and N are one
// node whose total both entries hold (as a flushed LDS grid leaves them).
__device__ __forceinline__ void global_node_add(int64_t *A, const GridPar &G, int n, int64_t w) {
  if (G.periodic && (n == 0 || n == G.N)) {
    atomicAdd(reinterpret_cast<unsigned long long *>(&A[0]), (unsigned long long)w);
    atomicAdd(reinterpret_cast<unsigned long long *>(&A[G.N]), (unsigned long long)w);
  } else {
    atomicAdd(reinterpret_cast<unsigned long long *>(&A[n]), (unsigned long long)w);
  }
}
// A particle created in a pass (ionisation product, secondary electron) goes
// straight into the deposit of the next step with the instance's shape.
// sh: the power of two of the particle's weight in the deposit's unit.
__device__ __forceinline__ void global_deposit(CInst &I, int64_t *A, int j, double xi, int sh = 0) {
  const GridPar G = grid_par(I);
  if (I.gather == 2) {
    int n;
    int64_t wl, wc, wr;
    weights_s2(j, xi, n, wl, wc, wr);
    global_node_add(A, G, fold_s2(n - 1, G.N, G.periodic), wl << sh);
    global_node_add(A, G, n, wc << sh);
    global_node_add(A, G, fold_s2(n + 1, G.N, G.periodic), wr << sh);
  } else {
    int64_t w0, w1;
    weights(xi, w0, w1);
    global_node_add(A, G, j, w0 << sh);
    global_node_add(A, G, j + 1, w1 << sh);
  }
}

// Power of two of a particle's weight in the unit of the deposit: class - 4
// plus the instance's unit exponent (0 for every particle of a discharge that
// is not rebalanced).
__device__ __forceinline__ int weight_shift(int cls, int wunit) { return cls - kClassUnit + wunit; }

__device__ __forceinline__ void set_status(InstState &S, int bits) {
  atomicOr(&S.status, bits);
}

__device__ __forceinline__ bool eedf_due(CInst &I, int64_t k) {
  return I.eedf_every > 0 && k >= I.avg_start && ((k - I.avg_start) % I.eedf_every) == 0;
}

__device__ __forceinline__ void eedf_sample(CInst &I, double x, double vx, double vy,
                                            double vz, unsigned long long count = 1ull) {
  if (!(fabs(x - I.eedf_centre) < I.eedf_half)) return;
  const double eps = kHALF_ME_OVER_QE * ((vx * vx + vy * vy) + vz * vz);
  const double b = floor(eps / I.eedf_de);
  if (b < (double)I.eedf_bins) atomicAdd(&I.eedf[(int)b], count);
}

// Reserve a slot for a new particle of species s; -1 when the segment is full.
// All lanes of the wavefront that call this together (same instance and
// species) share one atomic: the first takes the whole group's slots.
__device__ __forceinline__ int64_t append_slot(CInst &I, InstState &S, int s) {
  const unsigned long long active = __ballot(true);
  const int lane = __lane_id();
  const int leader = __ffsll((long long)active) - 1;
  const int rank = __popcll(active & ((1ull << lane) - 1ull));
  unsigned long long old = 0;
  if (lane == leader)
    old = atomicAdd(&S.append, (unsigned long long)__popcll(active) << (32 * s));
  old = __shfl(old, leader, 64);
  const unsigned long long base = (old >> (32 * s)) & 0xFFFFFFFFull;
  const int64_t idx = S.extent[s] + (int64_t)(base + (unsigned long long)rank);
  if (idx >= I.cap[s]) {
    set_status(S, ST_CAPACITY);
    return -1;
  }
  return idx;
}
// One slot of each species (the electron and the ion of an ionisation) with
// one atomic; -1 where that species is full.
__device__ __forceinline__ void append_pair(CInst &I, InstState &S, int64_t &ie, int64_t &ii) {
  const unsigned long long active = __ballot(true);
  const int lane = __lane_id();
  const int leader = __ffsll((long long)active) - 1;
  const int rank = __popcll(active & ((1ull << lane) - 1ull));
  const unsigned long long n = (unsigned long long)__popcll(active);
  unsigned long long old = 0;
  if (lane == leader) old = atomicAdd(&S.append, n | (n << 32));
  old = __shfl(old, leader, 64);
  ie = S.extent[0] + (int64_t)((old & 0xFFFFFFFFull) + (unsigned long long)rank);
  ii = S.extent[1] + (int64_t)((old >> 32) + (unsigned long long)rank);
  if (ie >= I.cap[0]) {
    set_status(S, ST_CAPACITY);
    ie = -1;
  }
  if (ii >= I.cap[1]) {
    set_status(S, ST_CAPACITY);
    ii = -1;
  }
}

// ---------------------------------------------------------------------------
// Form traits
// ---------------------------------------------------------------------------
struct F32 {
  static constexpr int prec = 1;
  using V = float;
  using View = P32;
  static __device__ View view(CInst &I, int s, int buf) { return view32(I.pbuf[s][buf], I.cap[s]); }
};
struct F64 {
  static constexpr int prec = 0;
  using V = double;
  using View = P64;
  static __device__ View view(CInst &I, int s, int buf) { return view64(I.pbuf[s][buf], I.cap[s]); }
};

// Write a new particle (SEE electron or ionisation product).
// k1: the first step the particle takes part in; kn: its first candidacy;
// E: the slot's epoch; cls: its weight class (FP32 form).
template <class F>
__device__ void write_new(CInst &I, typename F::View P, int64_t idx, double x, int cell,
                         float off, double vx, double vy, double vz, uint64_t id, int32_t kn,
                         int64_t k1, int64_t E, int cls) {
  if constexpr (F::prec == 1) {
    const uint32_t w = hw_encode(cell, kn, k1, E, cls);
    P.hw[idx] = w;
    P.off[idx] = off;
    P.vx[idx] = (float)vx;
    gstore_cold(P.cold + idx, Cold32{(float)vy, (float)vz, id});
    if (hw_far(w)) P.knext[idx] = kn;
  } else {
    P.x[idx] = x;
    P.vx[idx] = vx;
    P.vy[idx] = vy;
    P.vz[idx] = vz;
    P.id[idx] = id;
    P.knext[idx] = kn;
  }
}

// Secondary emission by an ion absorbed at `wall` during step k.  The new
// electron goes straight into the electron deposit of step k+1 when `dep`.
template <class F>
__device__ void emit_secondary(CInst &I, InstState &S, Smem &sm, uint64_t ion_id, int wall,
                               int64_t k, int64_t E, int buf, bool dep, int64_t *A_next_e, int cls) {
  const uint4 r = philox((uint32_t)k, TAG_SEE | (1u << 8), I.seed, ion_id);
  if (!(u32d(r.x) < I.gamma_see)) return;
  const uint4 p = philox((uint32_t)k, TAG_SEE_POS | (1u << 8), I.seed, ion_id);
  const double vxm = I.vt_see * sqrt(-2.0 * log(u32d(r.y)));
  double zy, zz;
  box_muller(u32d(r.z), u32d(r.w), zy, zz);
  const double d = (vxm * I.dt) * u32d(p.x);
  const bool left = wall < 0;
  const double x = left ? d : I.L - d;
  const double vx = left ? vxm : -vxm;
  if (!(x >= 0.0 && x < I.L)) return;
  const uint64_t cid = (uint64_t)p.y | ((uint64_t)p.z << 32);
  const int32_t kn = next_candidate(cid, k, 0, I.seed, I.nudt[0]);
  int cell = 0;
  float off = 0.0f;
  double xi;
  int j;
  if constexpr (F::prec == 1) {
    to_state32(I, x, cell, off);
    j = cell;
    xi = (double)off;
  } else {
    j = locate64(grid_par(I), I.nodes, x, xi);
  }
  const int64_t idx = append_slot(I, S, 0);
  if (idx < 0) return;
  write_new<F>(I, F::view(I, 0, buf), idx, x, cell, off, vx, I.vt_see * zy, I.vt_see * zz, cid, kn, k + 1,
               E, cls);
  atomicAdd(&sm.ctr[C_SEE], 1ull);
  if (dep) global_deposit(I, A_next_e, j, xi, weight_shift(cls, I.wunit));
}

// ---------------------------------------------------------------------------
// The particle pass: a streaming kernel and a drain kernel.
//
// k_particles (persistent) reads the state with vector loads, pushes every
// live particle, deposits x^{k+1} into the LDS grid and writes the state back.
// Particles that leave the gap or are collision candidates this step (a few
// percent) are not handled in place: their indices go to a per-wavefront
// queue in LDS (slots from a ballot) and, kSpill at a time, to a per-segment
// queue in HBM (one atomic per chunk).  k_drain then processes those queues
// with full wavefronts: absorption tallies, secondary emission, the FP64
// collision arithmetic and ionisation products.  Keeping the rare, heavy code
// out of the streaming kernel keeps its register footprint small.
// ---------------------------------------------------------------------------
// Queue record (16 B): word 0 = particle index | kind << 30 (kind 0 =
// collision candidate, 1 / 2 = absorbed at the left / right electrode,
// 3 = non-finite state); then the particle's state as the pass leaves it,
// FP32 form: its hot word, vx and offset (as bits); FP64 form: 0 and vx (as
// two words).  The drain so reads none of the streamed arrays, only the
// particle's cold record (and, for far candidates, its knext).
constexpr int kSpill = 128;   // records moved to HBM per reservation
constexpr int kWaveQ = 192;   // per-wavefront LDS queue: kSpill - 1 carried + 64 new records fit
static_assert(kSpill - 1 + 64 <= kWaveQ, "wavefront queue too small");
constexpr int kQShift = 30;
constexpr int kQMask = (1 << kQShift) - 1;
__device__ __forceinline__ int qentry(int i, int kind) { return i | (kind << kQShift); }

// Tile prefix of the segments (inst, species) that advance in this pass.
// `count_of` selects the per-segment work (particle extent or queue length).
template <int BLOCK, class CountOf>
__device__ int64_t segment_prefix(const InstDev *insts, const InstState *states, int n_inst,
                                  int tile, int *prefix, CountOf count_of) {
  const int nseg = 2 * n_inst;
  const int t = threadIdx.x;
  for (int s = t; s < nseg; s += BLOCK) {
    CInst &I = cinst(insts)[s >> 1];
    const InstState &S = states[s >> 1];
    const int sp = s & 1;
    const bool ok = I.active && S.frozen == 0 && sp < I.nsp && !(I.k_stop > 0 && S.k >= I.k_stop);
    const int64_t n = ok ? count_of(S, sp) : 0;
    prefix[s + 1] = (int)((n + tile - 1) / tile);
  }
  tile_prefix(prefix, nseg);
  return prefix[nseg];
}

// Flush the per-workgroup counters of one segment to its instance state.
template <int BLOCK>
__device__ void flush_counters(Smem &sm, InstState *Sp, int sp) {
  __syncthreads();
  const int t = threadIdx.x;
  const int r = blockIdx.x & (kRep - 1);
  if (t < kNctr) {
    const unsigned long long v = sm.ctr[t];
    if (v) {
      atomicAdd(&Sp->ctr[t][r], v);
      if (t == C_PSTEPS) atomicAdd(&Sp->step_live[sp][r], v);
      else if (t >= C_ABS && t < C_ABS + 4) atomicAdd(&Sp->step_absorbed[(t - C_ABS) >> 1][r], v);
      sm.ctr[t] = 0;
    }
  }
  __syncthreads();
}

template <class F, int MODE>
__device__ void drain_one(CInst &I, InstState &S, Smem &sm, int sp, int buf, int64_t k, int64_t E,
                          typename F::View P, const int4 rec);

// INLINE (fused pass, discharges small enough that launches dominate): each
// wavefront drains its own queued particles itself, when its LDS queue
// fills and at the end of each segment, instead of moving them to the HBM
// queue for k_drain.  The results are the same (every product and counter
// is independent of who drains a particle); one launch per step is saved.
// The collision code makes this variant large (about 275 VGPRs); it is held
// to two wavefronts per SIMD (256 VGPRs, a few spills), which measured
// faster than one (resolved discharge, FP64: 38.3 against 47.9 us/step).
template <class F, int MODE, int BLOCK, bool INLINE = false>
__global__ void __launch_bounds__(BLOCK, INLINE ? 2 : 1)
k_particles(const InstDev *__restrict__ insts, InstState *__restrict__ states, int n_inst, int max_n) {
  constexpr int TILE = BLOCK * kPPT;
  __shared__ Smem sm;
  extern __shared__ __align__(16) unsigned char dsm[];
  const int t = threadIdx.x;
  const int lane = __lane_id();
  const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int np1 = max_n + 1;
  int64_t *sA = reinterpret_cast<int64_t *>(dsm);
  // FP32: the walk entry of every cell int4[max_n] (see walk_step), then the
  // gather table f32[np1 + 1] (N cells, N + 1 nodes, or N + 2 centres).
  const size_t a_bytes = ((size_t)np1 * 8 + 15) & ~(size_t)15;
  int4 *sT = reinterpret_cast<int4 *>(dsm + a_bytes);
  float *sE32 = reinterpret_cast<float *>(sT + max_n);
  // FP64: the gather table f64[np1 + 1], nodes f64[np1].
  double *sE64 = reinterpret_cast<double *>(sA + np1);
  double *sNodes = sE64 + np1 + 1;
  const size_t tables = (F::prec == 1) ? a_bytes + (size_t)max_n * 16 + (size_t)(np1 + 1) * 4
                                       : (size_t)np1 * 24 + 8;
  int4 *wq = reinterpret_cast<int4 *>(dsm + ((tables + 15) & ~(size_t)15)) + (t >> 6) * kWaveQ;
  int wq_n = 0;   // entries in this wavefront's queue (wavefront-uniform)

  if (t < kNctr) sm.ctr[t] = 0;
  if (MODE == M_DEPOSIT || MODE == M_FUSED)
    for (int j = t; j < np1; j += BLOCK) sA[j] = 0;
  const int64_t T = segment_prefix<BLOCK>(insts, states, n_inst, TILE, sm.seg_prefix,
                                          [](const InstState &S, int sp) { return S.extent[sp]; });
  const int64_t t0 = T * blockIdx.x / gridDim.x;
  const int64_t t1 = T * (blockIdx.x + 1) / gridDim.x;

  int seg = -1;
  CInst *Ip = nullptr;
  InstState *Sp = nullptr;
  int sp = 0, N = 0;
  int64_t k = 0, epoch = 0, ext = 0, seg_first = 0;
  uint32_t kE = 0;   // k - epoch: the hot-word offset of this pass's candidates
  typename F::View P;
  int64_t *A_out = nullptr;
  int4 *gq = nullptr;
  bool deposit_on = false;
  unsigned long long live_here = 0;
  // Per-segment constants, in scalar registers (see GridPar).
  GridPar G{0, 0, 0, 0.0};
  int gather = 0, wunit = 0;
  bool coll = false, due_eedf = false;
  float qmdt32 = 0.0f, hq32 = 0.0f;
  double qmdt = 0.0, hq = 0.0, dt = 0.0, L = 0.0;

  // Append this lane's entry (if any) to the wavefront queue; move whole
  // chunks of kSpill entries (or, at the end of a segment, all) to the
  // segment's HBM queue.  The reservation is an atomic on the segment's one
  // counter, which every wavefront of the device shares: chunks keep those
  // same-address atomics (which serialise) few.
  auto enqueue = [&](bool want, int4 rec) {
    const unsigned long long m = __ballot(want);
    if (want) wq[wq_n + __popcll(m & lt_mask)] = rec;
    wq_n += __popcll(m);
  };
  auto spill = [&](bool all) {
    const int n = all ? wq_n : (wq_n / kSpill) * kSpill;
    if (n == 0) return;
    if constexpr (INLINE) {
      // The wavefront's own stores of these particles (this pass) complete
      // before the drain rewrites them (the one field it reads back, an
      // FP64 position, it reads with an L2 load).
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      const int bufp = uni(Sp->parity);
      for (int e = lane; e < n; e += 64) drain_one<F, MODE>(*Ip, *Sp, sm, sp, bufp, k, epoch, P, wq[wq_n - n + e]);
      wq_n -= n;
      return;
    }
    unsigned long long b = 0;
    if (lane == 0) b = atomicAdd(&Sp->qcount[sp], (unsigned long long)n);
    b = __shfl(b, 0, 64);
    for (int e = lane; e < n; e += 64) gstore_rec(gq + b + e, wq[wq_n - n + e]);
    wq_n -= n;
  };
  auto flush = [&]() {
    spill(true);
    __syncthreads();
    if (deposit_on) {
      if (Ip->bc == 1 && t == 0) {
        const int64_t v = sA[0] + sA[N];
        sA[0] = v;
        sA[N] = v;
      }
      __syncthreads();
      for (int j = t; j <= N; j += BLOCK) {
        const int64_t v = sA[j];
        if (v != 0) {
          atomicAdd(reinterpret_cast<unsigned long long *>(&A_out[j]), (unsigned long long)v);
          sA[j] = 0;
        }
      }
    }
    const unsigned long long lw = wave_sum_u64(live_here);
    if (lane == 0 && lw) atomicAdd(&sm.ctr[C_PSTEPS], lw);
    live_here = 0;
    flush_counters<BLOCK>(sm, Sp, sp);
  };

  for (int64_t tile = t0; tile < t1; ++tile) {
    int s = seg < 0 ? segment_of(sm.seg_prefix, 2 * n_inst, tile) : seg;
    while (sm.seg_prefix[s + 1] <= tile) ++s;
    s = __builtin_amdgcn_readfirstlane(s);
    if (s != seg) {
      if (seg >= 0) flush();
      seg = s;
      Ip = &cinst(insts)[seg >> 1];
      Sp = &states[seg >> 1];
      sp = seg & 1;
      CInst &I = *Ip;
      N = I.N;
      // Per-segment values in scalar registers: read into vector registers,
      // every tile would wait at the loop's join for all outstanding memory
      // operations (the previous tile's stores included) before its loads.
      k = uni((int64_t)Sp->k);
      epoch = uni((int64_t)Sp->epoch);
      kE = (uint32_t)(k - epoch);
      ext = uni((int64_t)Sp->extent[sp]);
      seg_first = uni((int64_t)sm.seg_prefix[seg]);
      P = F::view(I, sp, Sp->parity);
      gq = I.queue[sp];
      const int par = (int)(k & 1);
      G = GridPar{uni(I.N), uni(I.bc == 1 ? 1 : 0), uni(I.uniform), uni(I.dx)};
      gather = uni(I.gather);
      wunit = uni(I.wunit);
      coll = (MODE == M_MCC || MODE == M_FUSED) && I.nudt[sp] > 0.0;
      due_eedf = (MODE == M_PUSH || MODE == M_FUSED) && sp == 0 && eedf_due(I, k);
      qmdt32 = uni(I.qmdt32[sp]);
      hq32 = uni(I.hq32[sp]);
      qmdt = uni(I.qmdt[sp]);
      hq = uni(I.hq[sp]);
      dt = uni(I.dt);
      L = uni(I.L);
      deposit_on = (MODE == M_DEPOSIT) || (MODE == M_FUSED);
      A_out = (MODE == M_DEPOSIT) ? I.A[par][sp] : I.A[par ^ 1][sp];
      if (MODE != M_MCC) {
        const int ne = (I.gather == 0) ? N : ((I.gather == 1) ? N + 1 : N + 2);
        if constexpr (F::prec == 1) {
          if (MODE != M_DEPOSIT) {
            for (int j = t; j < ne; j += BLOCK) sE32[j] = I.E32[j];
            if (MODE != M_PULLBACK) {
              if (I.uniform) {
                // one run spanning the grid: the first step's in-run test then
                // accepts every move that stays inside a bounded grid
                for (int j = t; j < N; j += BLOCK)
                  sT[j] = make_int4(__float_as_int(I.dtoh32u), (N - 1) << 16, 0, 0);
              } else {
                const bool per = I.bc == 1;
                for (int j = t; j < N; j += BLOCK) {
                  const int run = per ? (j | (j << 16)) : I.runs[j];
                  const int lo = run & 0xFFFF, hi = run >> 16;
                  sT[j] = make_int4(__float_as_int(I.dtoh32[j]), run, __float_as_int(I.rf32[hi]),
                                    __float_as_int(I.rb32[lo > 0 ? lo - 1 : N - 1]));
                }
              }
            }
          }
        } else {
          if (MODE != M_DEPOSIT)
            for (int j = t; j < ne; j += BLOCK) sE64[j] = I.E64[j];
          if (!I.uniform)
            for (int j = t; j <= N; j += BLOCK) sNodes[j] = I.nodes[j];
        }
      }
      __syncthreads();
    }
    CInst &I = *Ip;
    const int64_t base = (tile - seg_first) * TILE;
    const int64_t i0 = base + (int64_t)t * kPPT;
    const bool full = i0 + kPPT <= ext;
    DepAcc dep;
    dep.init();
    bool want[kPPT];
    int went[kPPT];

    if constexpr (F::prec == 1) {
      // ---------------- FP32-state form ----------------
      // hw: hot word (cell, candidacy offset from the epoch, class, far flag)
      uint32_t hw[kPPT];
      float o[kPPT], vx[kPPT];
      if (full) {
#pragma unroll
        for (int g = 0; g < kPPT; g += 4) {
          const int4 h4 = gload4(reinterpret_cast<const int *>(P.hw) + i0 + g);
          hw[g] = (uint32_t)h4.x; hw[g + 1] = (uint32_t)h4.y; hw[g + 2] = (uint32_t)h4.z; hw[g + 3] = (uint32_t)h4.w;
          const float4 o4 = gload4(P.off + i0 + g);
          o[g] = o4.x; o[g + 1] = o4.y; o[g + 2] = o4.z; o[g + 3] = o4.w;
          if (MODE != M_DEPOSIT) {
            const float4 v4 = gload4(P.vx + i0 + g);
            vx[g] = v4.x; vx[g + 1] = v4.y; vx[g + 2] = v4.z; vx[g + 3] = v4.w;
          }
        }
      } else {
#pragma unroll
        for (int q = 0; q < kPPT; ++q) {
          const int64_t i = i0 + q;
          const bool v = i < ext;
          hw[q] = v ? gload<uint32_t>(P.hw + i) : kHwDead;
          o[q] = v ? gload<float>(P.off + i) : 0.0f;
          vx[q] = v ? gload<float>(P.vx + i) : 0.0f;
        }
      }
      uint32_t hn[kPPT];
      float on[kPPT], vn[kPPT];
      if constexpr (MODE == M_PUSH || MODE == M_FUSED) {
        // Gather, push and first walk step of the thread's particles; then
        // the rare walks that go on (across more than one run boundary).
        int cn[kPPT], st[kPPT];
        bool more = false;
#pragma unroll
        for (int q = 0; q < kPPT; ++q) {
          const int j = hw_cell(hw[q]);
          cn[q] = j;
          on[q] = o[q];
          vn[q] = vx[q];
          st[q] = W_IN;
          if (!hw_live(hw[q])) continue;
          const float e = (gather == 0)   ? sE32[j]
                          : (gather == 1) ? ((1.0f - o[q]) * sE32[j]) + (o[q] * sE32[j + 1])
                                          : gather_ec2_32(sE32, j, o[q]);
          const float v1 = vx[q] + qmdt32 * e;
          const int4 T = sT[j];
          const float sig = o[q] + v1 * __int_as_float(T.x);
          // First walk step without branches: a move that stays inside the
          // run around j (j + floor(sigma) within [lo, hi], either direction)
          // ends at sigma - floor(sigma), moved one cell right when a left move
          // rounds up to 1 (see walk_step).  Anything else walks below.
          const float m = floorf(sig);
          const int jm = j + (int)m;
          const bool moved = sig < 0.0f || sig >= 1.0f;
          const bool inrun = fabsf(sig) < kWalkLimit && jm >= (T.y & 0xFFFF) && jm <= (T.y >> 16);
          const float r = sig - m;
          const bool up = r >= 1.0f;
          vn[q] = v1;
          cn[q] = moved ? (inrun ? (up ? jm + 1 : jm) : j) : j;
          on[q] = moved ? (inrun ? (up ? 0.0f : r) : sig) : sig;
          st[q] = (moved && !inrun) ? W_FIRST : W_IN;
          more |= moved && !inrun;
        }
        if (__ballot(more) != 0) {
#pragma unroll
          for (int q = 0; q < kPPT; ++q) {
            if (st[q] == W_FIRST) st[q] = walk_first(G, sT[cn[q]], cn[q], on[q]);
            int guard = 0;
            while (st[q] == W_MORE) {
              if (++guard > 4 * G.N + 64) {
                st[q] = W_BAD;
                break;
              }
              st[q] = walk_step(sT[cn[q]], G.N, G.periodic, cn[q], on[q]);
            }
          }
        }
#pragma unroll
        for (int q = 0; q < kPPT; ++q) {
          const bool live = hw_live(hw[q]);
          const int ii = (int)(i0 + q);
          const int wall = st[q];
          const float v1 = vn[q];
          const bool gone = live && (wall != W_IN || v1 != v1);   // absorbed or non-finite
          // a candidate this step (the drain re-checks far ones)
          const bool cand = MODE == M_FUSED && live && !gone && coll && hw_due(hw[q], kE);
          live_here += live ? 1u : 0u;
          want[q] = gone || cand;
          went[q] = qentry(ii, gone ? ((wall == W_BAD || v1 != v1) ? 3 : (wall < 0 ? 1 : 2)) : 0);
          // the word changes with the cell only (the drain rewrites a
          // candidate's word)
          hn[q] = !live ? hw[q] : (gone ? kHwDead : hw_move(hw[q], cn[q]));
          on[q] = gone ? o[q] : on[q];
          if (live && !gone) {
            const int jj = cn[q];
            const float sig = on[q];
            const int sh = weight_shift(hw_class(hw[q]), wunit);
            if (due_eedf) {
              const double x = I.uniform ? ((double)jj * I.dx + (double)sig * I.dx)
                                         : (I.nodes[jj] + (double)sig * I.h[jj]);
              if (fabs(x - I.eedf_centre) < I.eedf_half)
                eedf_sample(I, x, (double)v1, (double)P.cold[ii].vy, (double)P.cold[ii].vz, 1ull << sh);
            }
            if constexpr (MODE == M_FUSED) {
              if (gather == 2) {
                lds_deposit_s2(sA, G, jj, (double)sig, sh);
              } else {
                int64_t w0, w1;
                weights32(sig, w0, w1);
                dep.add(sA, jj, w0 << sh, w1 << sh);
              }
            }
          }
        }
      } else {
#pragma unroll
      for (int q = 0; q < kPPT; ++q) {
        want[q] = false;
        went[q] = 0;
        hn[q] = hw[q];
        on[q] = o[q];
        vn[q] = vx[q];
        if (!hw_live(hw[q])) continue;   // dead slot
        const int ii = (int)(i0 + q);
        const int j = hw_cell(hw[q]);
        if constexpr (MODE == M_DEPOSIT) {
          const int sh = weight_shift(hw_class(hw[q]), wunit);
          if (gather == 2) {
            lds_deposit_s2(sA, G, j, (double)o[q], sh);
          } else {
            int64_t w0, w1;
            weights32(o[q], w0, w1);
            dep.add(sA, j, w0 << sh, w1 << sh);
          }
        } else if constexpr (MODE == M_PULLBACK) {
          const float e = (gather == 0)   ? sE32[j]
                          : (gather == 1) ? ((1.0f - o[q]) * sE32[j]) + (o[q] * sE32[j + 1])
                                          : gather_ec2_32(sE32, j, o[q]);
          vn[q] = vx[q] - hq32 * e;
        } else if constexpr (MODE == M_MCC) {
          want[q] = coll && hw_due(hw[q], kE);
          went[q] = qentry(ii, 0);
        }
      }
      }
      if constexpr (MODE == M_DEPOSIT || MODE == M_FUSED) dep.flush(sA);
      if constexpr (MODE == M_PUSH || MODE == M_FUSED || MODE == M_PULLBACK || MODE == M_MCC) {
        if (full) {
#pragma unroll
          for (int g = 0; g < kPPT; g += 4) {
            // a hot word is stored only when one of the lane's four changed
            // (a cell change, an absorption): most particles keep theirs
            if constexpr (MODE != M_PULLBACK)
              if (((hn[g] ^ hw[g]) | (hn[g + 1] ^ hw[g + 1]) | (hn[g + 2] ^ hw[g + 2]) | (hn[g + 3] ^ hw[g + 3])) != 0u)
                gstore4(reinterpret_cast<int *>(P.hw) + i0 + g, (int)hn[g], (int)hn[g + 1], (int)hn[g + 2],
                        (int)hn[g + 3]);
            if constexpr (MODE == M_PUSH || MODE == M_FUSED)
              gstore4(P.off + i0 + g, on[g], on[g + 1], on[g + 2], on[g + 3]);
            if constexpr (MODE != M_MCC) gstore4(P.vx + i0 + g, vn[g], vn[g + 1], vn[g + 2], vn[g + 3]);
          }
        } else {
#pragma unroll
          for (int q = 0; q < kPPT; ++q) {
            const int64_t i = i0 + q;
            if (i < ext) {
              if constexpr (MODE != M_PULLBACK)
                if (hn[q] != hw[q]) gstore<uint32_t>(P.hw + i, hn[q]);
              if constexpr (MODE == M_PUSH || MODE == M_FUSED) gstore<float>(P.off + i, on[q]);
              if constexpr (MODE != M_MCC) gstore<float>(P.vx + i, vn[q]);
            }
          }
        }
      }
      // The queued particles, each with the state this pass leaves it in
      // (the drain then reads none of the streamed arrays).
      if constexpr (MODE == M_PUSH || MODE == M_MCC || MODE == M_FUSED) {
        if (__ballot(want[0] || want[1] || want[2] || want[3]) != 0) {
#pragma unroll
          for (int q = 0; q < kPPT; ++q) {
            // an absorbed particle's record keeps its last word (its weight class)
            const uint32_t hrec = ((unsigned)went[q] >> kQShift) != 0u ? hw[q] : hn[q];
            enqueue(want[q], make_int4(went[q], (int)hrec, __float_as_int(vn[q]), __float_as_int(on[q])));
            spill(false);   // at most 64 more: kSpill - 1 + 64 <= kWaveQ
          }
        }
      }
    } else {
      // ---------------- FP64 form ----------------
      double x[kPPT], vx[kPPT];
      int kn[kPPT];
      if (full) {
#pragma unroll
        for (int g = 0; g < kPPT; g += 4) {
          const double2 xa = gload2(P.x + i0 + g);
          const double2 xb = gload2(P.x + i0 + g + 2);
          x[g] = xa.x; x[g + 1] = xa.y; x[g + 2] = xb.x; x[g + 3] = xb.y;
          if (MODE != M_DEPOSIT) {
            const double2 va = gload2(P.vx + i0 + g);
            const double2 vb = gload2(P.vx + i0 + g + 2);
            vx[g] = va.x; vx[g + 1] = va.y; vx[g + 2] = vb.x; vx[g + 3] = vb.y;
          }
          if (MODE == M_MCC || MODE == M_FUSED) {
            const int4 k4 = gload4(P.knext + i0 + g);
            kn[g] = k4.x; kn[g + 1] = k4.y; kn[g + 2] = k4.z; kn[g + 3] = k4.w;
          }
        }
      } else {
#pragma unroll
        for (int q = 0; q < kPPT; ++q) {
          const int64_t i = i0 + q;
          const bool v = i < ext;
          x[q] = v ? gload<double>(P.x + i) : -1.0;
          vx[q] = v ? gload<double>(P.vx + i) : 0.0;
          kn[q] = v ? gload<int>(P.knext + i) : 0;
        }
      }
      double xn[kPPT], vn[kPPT];
#pragma unroll
      for (int q = 0; q < kPPT; ++q) {
        want[q] = false;
        went[q] = 0;
        xn[q] = x[q];
        vn[q] = vx[q];
        if (!(x[q] >= 0.0)) continue;   // dead slot
        const int ii = (int)(i0 + q);
        if constexpr (MODE == M_DEPOSIT) {
          double xi;
          const int j = locate64(G, sNodes, x[q], xi);
          if (gather == 2) {
            lds_deposit_s2(sA, G, j, xi);
          } else {
            int64_t w0, w1;
            weights(xi, w0, w1);
            dep.add(sA, j, w0, w1);
          }
        } else if constexpr (MODE == M_PULLBACK) {
          double xi;
          const int j = locate64(G, sNodes, x[q], xi);
          const double e = (gather == 0)   ? sE64[j]
                           : (gather == 1) ? (1.0 - xi) * sE64[j] + xi * sE64[j + 1]
                                           : gather_ec2_64(sE64, j, xi);
          vn[q] = vx[q] - hq * e;
        } else if constexpr (MODE == M_MCC) {
          want[q] = coll && kn[q] <= k;
          went[q] = qentry(ii, 0);
        } else {
          live_here += 1;
          double xi;
          const int j = locate64(G, sNodes, x[q], xi);
          const double e = (gather == 0)   ? sE64[j]
                           : (gather == 1) ? (1.0 - xi) * sE64[j] + xi * sE64[j + 1]
                                           : gather_ec2_64(sE64, j, xi);
          const double v1 = vx[q] + qmdt * e;
          double x1 = x[q] + v1 * dt;
          vn[q] = v1;
          int wall = 0;
          if (G.periodic) {
            if (!(fabs(x1) < 4.0 * L)) wall = 2;
            else {
              while (x1 < 0.0) x1 = x1 + L;
              while (x1 >= L) x1 = x1 - L;
            }
          } else if (!(x1 >= 0.0 && x1 < L)) {
            wall = (x1 < 0.0) ? -1 : ((x1 >= L) ? 1 : 2);
          }
          if (wall != 0) {
            xn[q] = -1.0;
            want[q] = true;
            went[q] = qentry(ii, (wall == 2) ? 3 : (wall < 0 ? 1 : 2));
          } else {
            xn[q] = x1;
            if (MODE == M_FUSED && coll && kn[q] <= k) {
              want[q] = true;
              went[q] = qentry(ii, 0);
            }
            if (due_eedf && fabs(x1 - I.eedf_centre) < I.eedf_half)
              eedf_sample(I, x1, v1, P.vy[ii], P.vz[ii]);
            if constexpr (MODE == M_FUSED) {
              double xi1;
              const int j1 = locate64(G, sNodes, x1, xi1);
              if (gather == 2) {
                lds_deposit_s2(sA, G, j1, xi1);
              } else {
                int64_t w0, w1;
                weights(xi1, w0, w1);
                dep.add(sA, j1, w0, w1);
              }
            }
          }
        }
      }
      if constexpr (MODE == M_DEPOSIT || MODE == M_FUSED) dep.flush(sA);
      if constexpr (MODE == M_PUSH || MODE == M_FUSED || MODE == M_PULLBACK) {
        if (full) {
#pragma unroll
          for (int g = 0; g < kPPT; g += 2) {
            if constexpr (MODE != M_PULLBACK) gstore2(P.x + i0 + g, xn[g], xn[g + 1]);
            gstore2(P.vx + i0 + g, vn[g], vn[g + 1]);
          }
        } else {
#pragma unroll
          for (int q = 0; q < kPPT; ++q) {
            const int64_t i = i0 + q;
            if (i < ext) {
              if constexpr (MODE != M_PULLBACK) gstore<double>(P.x + i, xn[q]);
              gstore<double>(P.vx + i, vn[q]);
            }
          }
        }
      }
      // The queued particles with their velocity after this pass.
      if constexpr (MODE == M_PUSH || MODE == M_MCC || MODE == M_FUSED) {
        if (__ballot(want[0] || want[1] || want[2] || want[3]) != 0) {
#pragma unroll
          for (int q = 0; q < kPPT; ++q) {
            const long long vb = __double_as_longlong(vn[q]);
            enqueue(want[q], make_int4(went[q], 0, (int)(vb & 0xFFFFFFFFll), (int)(vb >> 32)));
            spill(false);   // at most 64 more: kSpill - 1 + 64 <= kWaveQ
          }
        }
      }
    }
  }
  if (seg >= 0) flush();
}

// Energy and angle histograms of an absorbed particle (species sp, wall wi):
// energy bin floor(E * bins / emax), the last bin for E >= emax; angle to the
// wall normal theta = acos(|vx| / |v|), bin floor(theta_deg * abins / 90).
__device__ __forceinline__ void record_impact(CInst &I, int sp, int wi, double en, double vx, double v2,
                                              unsigned long long count) {
  const int nb = I.imp_bins, na = I.imp_abins;
  unsigned long long *row = I.impact + (size_t)(2 * sp + wi) * (size_t)(nb + 1 + na);
  const double fe = floor(en * I.imp_escale);
  const int be = (fe < (double)nb) ? (int)fe : nb;
  const double c = (v2 > 0.0) ? fmin(1.0, fabs(vx) / sqrt(v2)) : 1.0;
  const double th = acos(c) * (180.0 / 3.14159265358979323846);
  const int ba = min((int)floor(th * I.imp_ascale), na - 1);
  atomicAdd(&row[be], count);
  atomicAdd(&row[nb + 1 + ba], count);
}

// Velocity and id of a queued particle: vx from its queue record, the rest
// from its cold record.
__device__ __forceinline__ void load_particle(const P32 &P, int64_t i, const int4 &rec, double &vx,
                                              double &vy, double &vz, uint64_t &id) {
  const Cold32 c = gload_cold(P.cold + i);
  vx = (double)__int_as_float(rec.z);
  vy = (double)c.vy;
  vz = (double)c.vz;
  id = c.id;
}
__device__ __forceinline__ void load_particle(const P64 &P, int64_t i, const int4 &rec, double &vx,
                                              double &vy, double &vz, uint64_t &id) {
  vx = __longlong_as_double(((long long)rec.w << 32) | (long long)(uint32_t)rec.z);
  vy = P.vy[i];
  vz = P.vz[i];
  id = P.id[i];
}

// Handle one queued particle: absorption (tallies, secondary emission) or a
// null-collision candidate (collision, ionisation products, next candidate
// step).  Products go straight into the deposit of step k+1 in the fused pass.
template <class F, int MODE>
__device__ void drain_one(CInst &I, InstState &S, Smem &sm, int sp, int buf, int64_t k, int64_t E,
                          typename F::View P, const int4 rec) {
  const int entry = rec.x;
  const int64_t i = entry & kQMask;
  const int kind = (int)((unsigned)entry >> kQShift);
  if (kind == 3) {
    set_status(S, ST_NONFINITE);
    atomicAdd(&sm.ctr[C_NONFINITE], 1ull);
    return;
  }
  if constexpr (F::prec == 1) {
    // A far particle is queued only when its candidacy is overdue (see
    // hw_encode); one whose knext entry says otherwise is re-expressed and
    // is not a candidate.
    const uint32_t hw = (uint32_t)rec.y;
    if (kind == 0 && hw_far(hw)) {
      const int32_t kf = P.knext[i];
      if ((int64_t)kf > k) {
        P.hw[i] = hw_encode(hw_cell(hw), kf, k + 1, E, hw_class(hw));
        return;
      }
    }
  }
  double vxd, vy, vz;
  uint64_t id;
  load_particle(P, i, rec, vxd, vy, vz, id);
  // the particle's weight class (its record's word; FP64: class 4)
  const int cls = (F::prec == 1) ? hw_class((uint32_t)rec.y) : kClassUnit;
  const int sh = weight_shift(cls, I.wunit);
  if (kind != 0) {
    const int wi = kind - 1;
    atomicAdd(&sm.ctr[C_ABS + 2 * sp + wi], 1ull);
    const double v2 = (vxd * vxd + vy * vy) + vz * vz;
    const double en = (0.5 * I.mass[sp] / kQE) * v2;
    atomicAdd(&sm.ctr[C_EABS + 2 * sp + wi], (unsigned long long)rint(en * 65536.0) << sh);
    if (I.avg_every > 0 && k >= I.avg_start) record_impact(I, sp, wi, en, vxd, v2, 1ull << sh);
    if (sp == 1 && I.gamma_see > 0.0 && I.nsp > 1)
      emit_secondary<F>(I, S, sm, id, wi == 0 ? -1 : 1, k, E, buf, MODE == M_FUSED,
                        I.A[(k + 1) & 1][0], cls);
    return;
  }
  double ux = vxd, uy = vy, uz = vz;
  bool bound = false;
  bool scattered;   // a real collision: the velocity changed
  atomicAdd(&sm.ctr[C_CAND + sp], 1ull);
  if (sp == 0) {
    double ej[3];
    const int proc = collide_electron(I, id, k, ux, uy, uz, bound, ej);
    scattered = proc != 0;
    if (proc) atomicAdd(&sm.ctr[proc == 1 ? C_EL : (proc == 2 ? C_EX : C_IZ)], 1ull);
    if (proc == 3 && I.nsp > 1) {
      const uint4 ch = philox((uint32_t)k, TAG_CHILD, I.seed, id);
      const uint64_t eid = (uint64_t)ch.x | ((uint64_t)ch.y << 32);
      const uint64_t iid = (uint64_t)ch.z | ((uint64_t)ch.w << 32);
      double gx, gy, gz;
      gas_velocity(I, id, k, 0, gx, gy, gz);
      int64_t ie, ii;
      append_pair(I, S, ie, ii);
      int cc = 0;
      float oo = 0.0f;
      double xx = 0.0;
      if constexpr (F::prec == 1) {
        cc = hw_cell((uint32_t)rec.y);
        oo = __int_as_float(rec.w);
      } else {
        // an L2 load: in the inline drain this wavefront has just stored it
        xx = __hip_atomic_load(P.x + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      // the pair carries the primary's weight
      if (ie >= 0)
        write_new<F>(I, P, ie, xx, cc, oo, ej[0], ej[1], ej[2], eid,
                     next_candidate(eid, k, 0, I.seed, I.nudt[0]), k + 1, E, cls);
      if (ii >= 0)
        write_new<F>(I, F::view(I, 1, buf), ii, xx, cc, oo, gx, gy, gz, iid,
                     next_candidate(iid, k, 1, I.seed, I.nudt[1]), k + 1, E, cls);
      if constexpr (MODE == M_FUSED) {
        int j;
        double xi;
        if constexpr (F::prec == 1) {
          j = cc;
          xi = (double)oo;
        } else {
          j = locate64(grid_par(I), I.nodes, xx, xi);
        }
        const int par1 = (int)((k + 1) & 1);
        if (ie >= 0) global_deposit(I, I.A[par1][0], j, xi, sh);
        if (ii >= 0) global_deposit(I, I.A[par1][1], j, xi, sh);
      }
    }
  } else {
    scattered = collide_ion(I, id, k, ux, uy, uz, bound);
    if (scattered) atomicAdd(&sm.ctr[C_CX], 1ull);
  }
  if (bound) atomicAdd(&sm.ctr[C_BOUND], 1ull);
  // A null collision leaves the stored velocity as it is: its scattered
  // single-particle writes (each a partial line in HBM) are skipped.
  if (scattered) {
    if constexpr (F::prec == 1) {
      P.vx[i] = (float)ux;
      gstore_cold(P.cold + i, Cold32{(float)uy, (float)uz, id});
    } else {
      P.vx[i] = ux;
      P.vy[i] = uy;
      P.vz[i] = uz;
    }
  }
  const int32_t kn = next_candidate(id, k, sp, I.seed, I.nudt[sp]);
  if constexpr (F::prec == 1) {
    const uint32_t w = hw_encode(hw_cell((uint32_t)rec.y), kn, k + 1, E, cls);
    P.hw[i] = w;
    if (hw_far(w)) P.knext[i] = kn;
  } else {
    P.knext[i] = kn;
  }
}

// Drain the per-segment queues with full wavefronts (close_pass then closes
// the pass: in k_finalize, or in the next field launch between chained steps).
template <class F, int MODE>
__global__ void __launch_bounds__(kDrainTile)
k_drain(const InstDev *__restrict__ insts, InstState *__restrict__ states, int n_inst) {
  constexpr int BLOCK = kDrainTile;   // one queue entry per thread per tile
  __shared__ Smem sm;
  const int t = threadIdx.x;
  if (t < kNctr) sm.ctr[t] = 0;
  const int64_t T = segment_prefix<BLOCK>(insts, states, n_inst, BLOCK, sm.seg_prefix,
                                          [](const InstState &S, int sp) { return (int64_t)S.qcount[sp]; });
  const int64_t t0 = T * blockIdx.x / gridDim.x;
  const int64_t t1 = T * (blockIdx.x + 1) / gridDim.x;
  int seg = -1;
  InstState *Sp = nullptr;
  // per-segment values, in scalar registers
  int64_t qn = 0, k = 0, epoch = 0, first = 0;
  int buf = 0;
  for (int64_t tile = t0; tile < t1; ++tile) {
    int s = seg < 0 ? segment_of(sm.seg_prefix, 2 * n_inst, tile) : seg;
    while (sm.seg_prefix[s + 1] <= tile) ++s;
    s = __builtin_amdgcn_readfirstlane(s);
    if (s != seg) {
      if (seg >= 0) flush_counters<BLOCK>(sm, Sp, seg & 1);
      seg = s;
      Sp = &states[seg >> 1];
      qn = uni((int64_t)Sp->qcount[seg & 1]);
      k = uni((int64_t)Sp->k);
      epoch = uni((int64_t)Sp->epoch);
      buf = uni(Sp->parity);
      first = uni((int64_t)sm.seg_prefix[seg]);
    }
    CInst &I = cinst(insts)[seg >> 1];
    const int sp = seg & 1;
    const int64_t e = (tile - first) * BLOCK + t;
    if (e < qn)
      drain_one<F, MODE>(I, *Sp, sm, sp, buf, k, epoch, F::view(I, sp, buf), gload_rec(I.queue[sp] + e));
  }
  if (seg >= 0) flush_counters<BLOCK>(sm, Sp, seg & 1);
}

// Close a pass (see close_pass): one 64-lane workgroup per instance.
template <int MODE>
__global__ void __launch_bounds__(64)
k_finalize(const InstDev *__restrict__ insts, InstState *__restrict__ states, int n_inst) {
  const int i = blockIdx.x;
  if (i >= n_inst) return;
  CInst &I = cinst(insts)[i];
  InstState &S = states[i];
  if (!pass_open(I, S)) return;
  close_pass<MODE == M_MCC || MODE == M_FUSED, MODE == M_FUSED>(I, S, threadIdx.x);
}

// ---------------------------------------------------------------------------
// Initial load (Section 2b): one thread per particle.
// ---------------------------------------------------------------------------
template <class F>
__global__ void __launch_bounds__(256)
k_init(const InstDev *__restrict__ insts, InstState *__restrict__ states, int inst, int s,
       double t_ev) {
  CInst &I = cinst(insts)[inst];
  const int64_t n = I.n_init[s];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t id = (uint64_t)i;
  const uint32_t sb = (uint32_t)(s << 8);
  const uint4 r = philox(0u, TAG_INIT0 | sb, I.seed, id);
  const uint4 q = philox(0u, TAG_INIT1 | sb, I.seed, id);
  double x = u52d(r.x, r.y) * I.L;
  const double top = nextafter(I.L, 0.0);
  x = fmin(x, top);
  double z0, z1, z2, z3;
  box_muller(u32d(r.z), u32d(r.w), z0, z1);
  box_muller(u32d(q.x), u32d(q.y), z2, z3);
  const double vt = sqrt(t_ev * kQE / I.mass[s]);
  const double vx = vt * z0, vy = vt * z1, vz = vt * z2;
  const int32_t kn = (I.nudt[s] > 0.0) ? geometric(0.0, u52d(q.z, q.w), I.nudt[s]) : kINT32_MAX;
  const int buf = states[inst].parity;
  typename F::View P = F::view(I, s, buf);
  int cell = 0;
  float off = 0.0f;
  if constexpr (F::prec == 1) to_state32(I, x, cell, off);
  write_new<F>(I, P, i, x, cell, off, vx, vy, vz, id, kn, states[inst].k, states[inst].epoch, kClassUnit);
}

// ---------------------------------------------------------------------------
// Diagnostics of one instance: live counts, kinetic energy (2^-20 eV fixed
// point, order independent), max |vx| of the electrons.
// ---------------------------------------------------------------------------
template <class F>
__global__ void __launch_bounds__(256)
k_diag(const InstDev *__restrict__ insts, const InstState *__restrict__ states, int inst,
       unsigned long long *__restrict__ out) {
  // Wavefront sums, then block sums in LDS: one atomic per block and
  // quantity (same-address atomics from every wavefront would serialise).
  __shared__ unsigned long long red[4][3];
  __shared__ double redv[4];
  CInst &I = cinst(insts)[inst];
  const InstState &S = states[inst];
  const int wave = threadIdx.x >> 6;
  for (int s = 0; s < I.nsp; ++s) {
    typename F::View P = F::view(I, s, S.parity);
    const int64_t ext = S.extent[s];
    unsigned long long live = 0, ke = 0, wsum = 0;
    double vmax = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ext;
         i += (int64_t)gridDim.x * blockDim.x) {
      double vx, vy, vz;
      int sh = 0;
      if constexpr (F::prec == 1) {
        const uint32_t w = P.hw[i];
        if (!hw_live(w)) continue;
        sh = weight_shift(hw_class(w), I.wunit);
        vx = P.vx[i]; vy = P.cold[i].vy; vz = P.cold[i].vz;
      } else {
        if (!(P.x[i] >= 0.0)) continue;
        vx = P.vx[i]; vy = P.vy[i]; vz = P.vz[i];
      }
      live += 1;
      wsum += 1ull << sh;
      const double en = (0.5 * I.mass[s] / kQE) * ((vx * vx + vy * vy) + vz * vz);
      ke += (unsigned long long)rint(en * 1048576.0) << sh;
      vmax = fmax(vmax, fabs(vx));
    }
    live = wave_sum_u64(live);
    ke = wave_sum_u64(ke);
    wsum = wave_sum_u64(wsum);
    for (int o = 32; o > 0; o >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, o, 64));
    if (__lane_id() == 0) {
      red[wave][0] = live;
      red[wave][1] = ke;
      red[wave][2] = wsum;
      redv[wave] = vmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int nw = (int)(blockDim.x >> 6);
      for (int w = 1; w < nw; ++w) {
        live += red[w][0];
        ke += red[w][1];
        wsum += red[w][2];
        vmax = fmax(vmax, redv[w]);
      }
      if (live) {
        atomicAdd(&out[D_LIVE0 + s], live);
        atomicAdd(&out[D_KE0 + s], ke);
        if (s == 0) atomicAdd(&out[D_WE], wsum);
        if (s == 0) atomicMax(&out[D_VMAX], (unsigned long long)__double_as_longlong(vmax));
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Velocity moments and power of the averaged profiles (Section 3a), on the
// averaged steps, from x^k, v^{k-1/2} and E^k (before the push).  Per node,
// with linear (CIC) weights in FP64: sum w vx and sum w vx^2; per cell, the
// power given to the particles in it, sum vx E(x), E(x) being the gathered
// field (E_j for EC, linear for MC).  FP64 sums: their order, and so their
// last bits, may differ from run to run.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool avg_due(CInst &I, int64_t k) {
  return I.avg_every > 0 && k >= I.avg_start && ((k - I.avg_start) % I.avg_every) == 0;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <class F>
__global__ void __launch_bounds__(256)
k_moments(const InstDev *__restrict__ insts, const InstState *__restrict__ states, int n_inst,
          int max_n) {
  constexpr int BLOCK = 256, TILE = BLOCK * 4;
  __shared__ int prefix[2 * kMaxInst + 1];
  extern __shared__ __align__(16) unsigned char dsm[];
  const int np1 = max_n + 1;
  double *m1 = reinterpret_cast<double *>(dsm);
  double *m2 = m1 + np1;
  double *pw = m2 + np1;
  double *sE = pw + max_n;     // the gather table, up to np1 + 1 entries
  double *sNodes = sE + np1 + 1;   // FP64 form only
  const int t = threadIdx.x, lane = __lane_id();
  const int nseg = 2 * n_inst;
  for (int j = t; j < np1; j += BLOCK) { m1[j] = 0.0; m2[j] = 0.0; }
  for (int j = t; j < max_n; j += BLOCK) pw[j] = 0.0;
  for (int s = t; s < nseg; s += BLOCK) {
    CInst &I = cinst(insts)[s >> 1];
    const InstState &S = states[s >> 1];
    const bool ok = I.active && S.frozen == 0 && (s & 1) < I.nsp &&
                    !(I.k_stop > 0 && S.k >= I.k_stop) && I.moments && avg_due(I, S.k);
    prefix[s + 1] = ok ? (int)((S.extent[s & 1] + TILE - 1) / TILE) : 0;
  }
  tile_prefix(prefix, nseg);
  const int64_t T = prefix[nseg];
  const int64_t t0 = T * blockIdx.x / gridDim.x, t1 = T * (blockIdx.x + 1) / gridDim.x;
  int seg = -1, N = 0, gather = 0, wu = 0;
  CInst *Ip = nullptr;
  int64_t ext = 0;
  typename F::View P;
  GridPar G{0, 0, 0, 0.0};
  auto flush = [&]() {
    __syncthreads();
    CInst &I = *Ip;
    const int sp = seg & 1;
    for (int n = t; n <= N; n += BLOCK) {
      if (m1[n] != 0.0) atomicAdd(&I.accM1[sp][n], m1[n]);
      if (m2[n] != 0.0) atomicAdd(&I.accM2[sp][n], m2[n]);
      m1[n] = 0.0;
      m2[n] = 0.0;
      if (n < N) {
        if (pw[n] != 0.0) atomicAdd(&I.accP[sp][n], pw[n]);
        pw[n] = 0.0;
      }
    }
    __syncthreads();
  };
  for (int64_t tile = t0; tile < t1; ++tile) {
    int s = seg < 0 ? segment_of(prefix, nseg, tile) : seg;
    while (prefix[s + 1] <= tile) ++s;
    s = __builtin_amdgcn_readfirstlane(s);
    if (s != seg) {
      if (seg >= 0) flush();
      seg = s;
      Ip = &cinst(insts)[seg >> 1];
      CInst &I = *Ip;
      const InstState &S = states[seg >> 1];
      N = I.N;
      gather = I.gather;
      wu = I.wunit;
      G = grid_par(I);
      ext = uni((int64_t)S.extent[seg & 1]);
      P = F::view(I, seg & 1, S.parity);
      const int ne = (gather == 0) ? N : ((gather == 1) ? N + 1 : N + 2);
      for (int j = t; j < ne; j += BLOCK) sE[j] = I.E64[j];
      if (F::prec == 0 && !I.uniform)
        for (int j = t; j <= N; j += BLOCK) sNodes[j] = I.nodes[j];
      __syncthreads();
    }
    const int64_t base = (tile - prefix[seg]) * TILE;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = base + q * BLOCK + t;
      bool ok = i < ext;
      int j = 0;
      double xi = 0.0, vx = 0.0, fw = 1.0;   // fw: the particle's weight in deposit units
      if (ok) {
        if constexpr (F::prec == 1) {
          const uint32_t w = P.hw[i];
          j = hw_cell(w);
          ok = hw_live(w);
          if (ok) {
            xi = (double)P.off[i];
            vx = (double)P.vx[i];
            fw = ldexp(1.0, weight_shift(hw_class(w), wu));
          }
        } else {
          const double x = P.x[i];
          ok = x >= 0.0;
          if (ok) {
            j = locate64(G, sNodes, x, xi);
            vx = P.vx[i];
          }
        }
      }
      if (ok && gather == 2) {
        // quadratic-spline weights in FP64 (the deposit's shape), per lane
        const bool up = xi >= 0.5;
        const int n = up ? j + 1 : j;
        const double a = up ? 1.5 - xi : 0.5 - xi;
        const double b = up ? xi - 0.5 : 0.5 + xi;
        const double wl = fw * (0.5 * (a * a)), wr = fw * (0.5 * (b * b));
        const double wc = fw * ((1.0 - 0.5 * (a * a)) - 0.5 * (b * b));
        const int nl = fold_s2(n - 1, N, G.periodic), nr = fold_s2(n + 1, N, G.periodic);
        const double v2 = vx * vx;
        atomicAdd(&m1[nl], wl * vx);
        atomicAdd(&m1[n], wc * vx);
        atomicAdd(&m1[nr], wr * vx);
        atomicAdd(&m2[nl], wl * v2);
        atomicAdd(&m2[n], wc * v2);
        atomicAdd(&m2[nr], wr * v2);
        atomicAdd(&pw[j], fw * (vx * gather_ec2_64(sE, j, xi)));
        ok = false;
      }
      double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0, pp = 0.0;
      if (ok) {
        const double w0 = fw * (1.0 - xi), w1 = fw * xi;
        a0 = w0 * vx;
        a1 = w1 * vx;
        b0 = w0 * (vx * vx);
        b1 = w1 * (vx * vx);
        const double e = (gather == 0) ? sE[j] : (1.0 - xi) * sE[j] + xi * sE[j + 1];
        pp = fw * (vx * e);
      }
      // A cell-sorted state puts whole wavefronts in one cell: then the
      // wavefront sums its terms and one lane adds them (same-address LDS
      // atomics would serialise); otherwise every lane adds its own.
      const unsigned long long act = __ballot(ok);
      if (act == 0) continue;
      const int j0 = __shfl(j, __ffsll((long long)act) - 1, 64);
      if (__ballot(ok && j != j0) == 0) {
        a0 = wave_sum_f64(a0);
        a1 = wave_sum_f64(a1);
        b0 = wave_sum_f64(b0);
        b1 = wave_sum_f64(b1);
        pp = wave_sum_f64(pp);
        if (lane == 0) {
          atomicAdd(&m1[j0], a0);
          atomicAdd(&m1[j0 + 1], a1);
          atomicAdd(&m2[j0], b0);
          atomicAdd(&m2[j0 + 1], b1);
          atomicAdd(&pw[j0], pp);
        }
      } else if (ok) {
        atomicAdd(&m1[j], a0);
        atomicAdd(&m1[j + 1], a1);
        atomicAdd(&m2[j], b0);
        atomicAdd(&m2[j + 1], b1);
        atomicAdd(&pw[j], pp);
      }
    }
  }
  if (seg >= 0) flush();
}

// The FP32 hot words of instance inst, written with epoch E0, re-expressed
// for a next pass at step k1 with epoch k1 (pic_set_step, a restored
// checkpoint): the candidacies they stand for stay where they are.
__global__ void __launch_bounds__(256)
k_reencode(const InstDev *__restrict__ insts, const InstState *__restrict__ states, int inst,
           int64_t E0, int64_t k1) {
  CInst &I = cinst(insts)[inst];
  const InstState &S = states[inst];
  for (int s = 0; s < I.nsp; ++s) {
    const P32 P = view32(I.pbuf[s][S.parity], I.cap[s]);
    const int64_t ext = S.extent[s];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ext;
         i += (int64_t)gridDim.x * blockDim.x) {
      const uint32_t w = P.hw[i];
      if (!hw_live(w)) continue;
      const int64_t kn = hw_knext(w, hw_far(w) ? P.knext[i] : 0, E0);
      const uint32_t nw = hw_encode(hw_cell(w), kn, k1, k1, hw_class(w));
      P.hw[i] = nw;
      if (hw_far(nw)) P.knext[i] = (int32_t)kn;
    }
  }
}

void launch_reencode(const InstDev *insts, InstState *states, int inst, int64_t E0, int64_t k1,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_reencode, dim3(1024), dim3(256), 0, s, insts, states, inst, E0, k1);
}

__global__ void k_zero_deposit(const InstDev *__restrict__ insts, const InstState *__restrict__ states) {
  CInst &I = cinst(insts)[blockIdx.x];
  const InstState &S = states[blockIdx.x];
  if (!I.active) return;
  const int par = (int)(S.k & 1);
  for (int n = threadIdx.x; n <= I.N; n += blockDim.x) {
    I.A[par][0][n] = 0;
    if (I.nsp > 1) I.A[par][1][n] = 0;
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
size_t particle_lds_bytes(int prec, int max_n, int block) {
  const size_t np1 = (size_t)max_n + 1;
  const size_t tables =
      (prec == 1) ? ((np1 * 8 + 15) & ~(size_t)15) + (size_t)max_n * 16 + (np1 + 1) * 4
                  : np1 * 24 + 8;
  const size_t q = (size_t)(block / 64) * kWaveQ * sizeof(int4);
  return ((tables + 15) & ~(size_t)15) + q;
}

template <class F, int MODE, int BLOCK, bool INLINE = false>
static hipError_t launch_pk(const InstDev *insts, InstState *states, int n_inst, int grid,
                            int max_n, hipStream_t s) {
  const size_t lds = particle_lds_bytes(F::prec, max_n, BLOCK);
  hipLaunchKernelGGL((k_particles<F, MODE, BLOCK, INLINE>), dim3(grid), dim3(BLOCK), lds, s, insts, states,
                     n_inst, max_n);
  return hipGetLastError();
}

void launch_finalize(const InstDev *insts, InstState *states, int n_inst, hipStream_t s) {
  hipLaunchKernelGGL((k_finalize<M_FUSED>), dim3(n_inst), dim3(64), 0, s, insts, states, n_inst);
}

template <class F, int MODE>
static void launch_drain_mode(const InstDev *insts, InstState *states, int n_inst, int grid,
                              bool close, hipStream_t s) {
  hipLaunchKernelGGL((k_drain<F, MODE>), dim3(grid), dim3(kDrainTile), 0, s, insts, states, n_inst);
  if (close) hipLaunchKernelGGL((k_finalize<MODE>), dim3(n_inst), dim3(64), 0, s, insts, states, n_inst);
}
template <class F>
static hipError_t launch_drain_form(const InstDev *insts, InstState *states, int n_inst, int mode,
                                    int grid, bool close, hipStream_t s) {
  switch (mode) {
    case M_PUSH: launch_drain_mode<F, M_PUSH>(insts, states, n_inst, grid, close, s); break;
    case M_MCC: launch_drain_mode<F, M_MCC>(insts, states, n_inst, grid, close, s); break;
    case M_FUSED: launch_drain_mode<F, M_FUSED>(insts, states, n_inst, grid, close, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Drain workgroups that are resident on one CU at once, for the kernel as
// built (its registers bound it: three 256-thread workgroups per CU).  The
// persistent grid is sized to exactly that, since workgroups beyond it would
// run as a partly filled second round after the first.
template <class F>
static int drain_resident(int mode) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  if (mode == M_PUSH)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_drain<F, M_PUSH>, kDrainTile, 0);
  else if (mode == M_MCC)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_drain<F, M_MCC>, kDrainTile, 0);
  else if (mode == M_FUSED)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_drain<F, M_FUSED>, kDrainTile, 0);
  return e == hipSuccess && n > 0 ? n : 1;
}
int drain_blocks_per_cu(int prec, int mode) {
  return prec == 1 ? drain_resident<F32>(mode) : drain_resident<F64>(mode);
}

// The number of queued particles is only known on the device, so the drain
// grid is fixed and its workgroups split whatever the queues hold.
hipError_t launch_drain(const InstDev *insts, InstState *states, int n_inst, int prec, int mode,
                        int grid, bool close, hipStream_t s) {
  if (prec == 1) return launch_drain_form<F32>(insts, states, n_inst, mode, grid, close, s);
  return launch_drain_form<F64>(insts, states, n_inst, mode, grid, close, s);
}

template <class F>
static hipError_t launch_form(const InstDev *insts, InstState *states, int n_inst, int mode,
                              int block, int grid, int max_n, hipStream_t s) {
  if (mode == M_FUSED_INLINE) return launch_pk<F, M_FUSED, 256, true>(insts, states, n_inst, grid, max_n, s);
  if (mode == M_FUSED && block == 512)
    return launch_pk<F, M_FUSED, 512>(insts, states, n_inst, grid, max_n, s);
  if (mode == M_FUSED && block == 1024)
    return launch_pk<F, M_FUSED, 1024>(insts, states, n_inst, grid, max_n, s);
  switch (mode) {
    case M_DEPOSIT: return launch_pk<F, M_DEPOSIT, 256>(insts, states, n_inst, grid, max_n, s);
    case M_PUSH: return launch_pk<F, M_PUSH, 256>(insts, states, n_inst, grid, max_n, s);
    case M_MCC: return launch_pk<F, M_MCC, 256>(insts, states, n_inst, grid, max_n, s);
    case M_FUSED: return launch_pk<F, M_FUSED, 256>(insts, states, n_inst, grid, max_n, s);
    case M_PULLBACK: return launch_pk<F, M_PULLBACK, 256>(insts, states, n_inst, grid, max_n, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_particles(const InstDev *insts, InstState *states, int n_inst, int prec, int mode,
                            int block, int grid, int max_n, hipStream_t s) {
  if (prec == 1) return launch_form<F32>(insts, states, n_inst, mode, block, grid, max_n, s);
  return launch_form<F64>(insts, states, n_inst, mode, block, grid, max_n, s);
}

void launch_init(const InstDev *insts, InstState *states, int inst, int species, int prec,
                 double t_ev, int64_t n, hipStream_t s) {
  const int blocks = (int)((n + 255) / 256);
  if (blocks == 0) return;
  if (prec == 1)
    hipLaunchKernelGGL(k_init<F32>, dim3(blocks), dim3(256), 0, s, insts, states, inst, species, t_ev);
  else
    hipLaunchKernelGGL(k_init<F64>, dim3(blocks), dim3(256), 0, s, insts, states, inst, species, t_ev);
}

void launch_diag(const InstDev *insts, InstState *states, int inst, int prec, int64_t max_particles,
                 unsigned long long *out, hipStream_t s) {
  // About 32 particles per thread, at most 2048 blocks (8 per CU: enough
  // loads in flight for a large instance; 256 blocks took 0.99 ms for 64 M
  // particles), one atomic per block and quantity.
  const int64_t b = (max_particles + 8191) / 8192;
  const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(2048, b)));
  if (prec == 1)
    hipLaunchKernelGGL(k_diag<F32>, grid, dim3(256), 0, s, insts, states, inst, out);
  else
    hipLaunchKernelGGL(k_diag<F64>, grid, dim3(256), 0, s, insts, states, inst, out);
}

void launch_moments(const InstDev *insts, InstState *states, int n_inst, int prec, int grid, int max_n,
                    hipStream_t s) {
  const size_t np1 = (size_t)max_n + 1;
  const size_t lds = 8 * (np1 * 3 + 1 + (size_t)max_n + (prec == 0 ? np1 : 0));
  if (prec == 1)
    hipLaunchKernelGGL(k_moments<F32>, dim3(grid), dim3(256), lds, s, insts, states, n_inst, max_n);
  else
    hipLaunchKernelGGL(k_moments<F64>, dim3(grid), dim3(256), lds, s, insts, states, n_inst, max_n);
}

void launch_zero_deposit(const InstDev *insts, InstState *states, int n_inst, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_deposit, dim3(n_inst), dim3(256), 0, s, insts, states);
}

}  // namespace ecpic
