// api.cpp -- host side of the EC-PIC library: the C ABI of include/ecpic.h.
//
// The context owns host metadata only.  Device memory is the caller's arena:
// a static region (instance table, instance states, counters) followed by a
// pool from which every slot takes one block (grid arrays + particle buffers).
// The pool is managed on the host by a first-fit free list with coalescing,
// so slots can be filled and emptied while other slots run, without any
// device allocation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/ecpic.h"
#include "device.h"
#include "kernels.h"

using namespace ecpic;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// Pool allocator over [begin, end) of the arena (offsets), first fit.
// ---------------------------------------------------------------------------
struct Pool {
  size_t begin = 0, end = 0;
  std::map<size_t, size_t> free_;  // offset -> size
  void reset(size_t b, size_t e) {
    begin = b;
    end = e;
    free_.clear();
    if (e > b) free_[b] = e - b;
  }
  bool alloc(size_t bytes, size_t &off) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        off = it->first;
        const size_t rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest() const {
    size_t m = 0;
    for (auto &kv : free_) m = std::max(m, kv.second);
    return m;
  }
};

struct SlotHost {
  bool used = false;
  size_t off = 0, bytes = 0;
  pic_config cfg{};
  std::vector<double> nodes;
  RbScratch rb;                 // rebalancing scratch (rebalanced slots only)
};

// Grid block layout (offsets relative to the slot block).
struct GridLayout {
  size_t nodes, h, V, dtoh, rf, rb, runs, A[2][2], phi, E64, E32, accA[2], acc_phi, accM1[2], accM2[2],
      accP[2], eedf, impact, scount[2],
      scursor[2], queue[2], rb_flag[2], rb_words, rb_k64[2], rb_k32[2], rb_val[2], rb_temp, rb_temp_bytes,
      rb_items, particles, total;
};

int eff_bins(const pic_config &c) { return c.eedf_bins > 0 ? c.eedf_bins : 200; }
int eff_ibins(const pic_config &c) { return c.impact_bins > 0 ? c.impact_bins : 200; }
int eff_abins(const pic_config &c) { return c.impact_angle_bins > 0 ? c.impact_angle_bins : 90; }
// Impact counters per (species, wall): energy bins + overflow, then angle bins.
size_t impact_row(const pic_config &c) { return (size_t)eff_ibins(c) + 1 + (size_t)eff_abins(c); }
int64_t eff_cap(const pic_config &c) {
  int64_t cap = c.capacity > 0 ? c.capacity : 2 * c.n_per_species + 4096;
  return (cap + 63) / 64 * 64;
}
int bytes_per_particle(int prec) { return prec == PIC_FP32_STATE ? (int)kBytes32 : (int)kBytes64; }

// Scratch reserved for the rebalancing radix sorts of `items` entries (the
// size the sorts ask for is checked against it when the slot is set up).
size_t rb_temp_reserve(size_t items) { return ((size_t)64 << 20) + 8 * items; }

GridLayout layout(const pic_config &c) {
  GridLayout g{};
  const size_t N = (size_t)c.n_cells, n1 = N + 1;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += align_up(bytes); return r; };
  g.nodes = take(8 * n1);
  g.h = take(8 * N);
  g.V = take(8 * n1);
  g.dtoh = take(4 * N);
  g.rf = take(4 * N);
  g.rb = take(4 * N);
  g.runs = take(4 * N);
  for (int p = 0; p < 2; ++p)
    for (int s = 0; s < 2; ++s) g.A[p][s] = take(8 * n1);
  g.phi = take(8 * n1);
  g.E64 = take(8 * (n1 + 1));   // N cells, N + 1 nodes or N + 2 centres
  g.E32 = take(4 * (n1 + 1));
  g.accA[0] = take(8 * n1);
  g.accA[1] = take(8 * n1);
  g.acc_phi = take(8 * n1);
  for (int s = 0; s < 2; ++s) {
    g.accM1[s] = take(8 * n1);
    g.accM2[s] = take(8 * n1);
    g.accP[s] = take(8 * N);
  }
  g.eedf = take(8 * (size_t)eff_bins(c));
  g.impact = take(8 * 4 * impact_row(c));
  for (int s = 0; s < 2; ++s) g.scount[s] = take(8 * n1);
  for (int s = 0; s < 2; ++s) g.scursor[s] = take(8 * n1);
  // queue records of 16 B, at most one per particle and pass
  for (int s = 0; s < 2; ++s) g.queue[s] = take((s == 0 || c.n_species != 1) ? 16 * (size_t)eff_cap(c) : 0);
  // rebalancing: per-cell flags, the candidate list (both species) and the
  // radix sorts' scratch
  const bool rb = c.rebalance_ppc > 0;
  const size_t items = rb ? (size_t)(c.n_species == 1 ? 1 : 2) * (size_t)eff_cap(c) : 0;
  g.rb_items = items;
  for (int s = 0; s < 2; ++s) g.rb_flag[s] = take(rb ? N : 0);
  g.rb_words = take(rb ? 64 : 0);
  for (int b = 0; b < 2; ++b) g.rb_k64[b] = take(8 * items);
  for (int b = 0; b < 2; ++b) g.rb_k32[b] = take(4 * items);
  for (int b = 0; b < 2; ++b) g.rb_val[b] = take(4 * items);
  g.rb_temp_bytes = rb ? rb_temp_reserve(items) : 0;
  g.rb_temp = take(g.rb_temp_bytes);
  g.particles = o;
  const int nsp = c.n_species == 1 ? 1 : 2;
  o += (size_t)nsp * 2 * align_up((size_t)eff_cap(c) * bytes_per_particle(c.precision));
  g.total = o;
  return g;
}

size_t static_bytes(int n) {
  return align_up(sizeof(InstDev) * n) + align_up(sizeof(InstState) * n) + align_up(8 * D_NWORDS);
}

std::string validate(const pic_config &c) {
  if (c.n_cells == 0) return "";
  char buf[256];
  if (c.n_cells < 2 || c.n_cells > PIC_MAX_CELLS) {
    snprintf(buf, sizeof buf, "n_cells must be in [2, %d]", PIC_MAX_CELLS);
    return buf;
  }
  if (c.bc != PIC_BC_DIRICHLET_RF && c.bc != PIC_BC_PERIODIC) return "bc must be 0 or 1";
  if (c.gather != PIC_GATHER_EC && c.gather != PIC_GATHER_MC && c.gather != PIC_GATHER_EC2)
    return "gather must be 0, 1 or 2";
  if (c.gather == PIC_GATHER_EC2 && c.nodes) return "second-order EC needs a uniform grid";
  if (c.precision != PIC_FP64 && c.precision != PIC_FP32_STATE) return "precision must be 0 or 1";
  if (c.n_species != 1 && c.n_species != 2) return "n_species must be 1 or 2";
  if (c.nodes) {
    if (c.nodes[0] != 0.0) return "nodes[0] must be 0";
    for (int i = 0; i < c.n_cells; ++i)
      if (!std::isfinite(c.nodes[i + 1]) || !(c.nodes[i + 1] > c.nodes[i]))
        return "nodes must be finite and strictly increasing";
  } else if (!(c.gap_m > 0.0) || !std::isfinite(c.gap_m)) {
    return "gap_m must be positive";
  }
  if (!(c.dt_s > 0.0) || !std::isfinite(c.dt_s)) return "dt_s must be positive";
  if (c.n_per_species < 0) return "n_per_species must be >= 0";
  if (c.capacity != 0 && c.capacity < c.n_per_species) return "capacity below n_per_species";
  if (eff_cap(c) > ((int64_t)1 << 30)) return "capacity above 2^30";
  if (c.n_per_species > 0 && !(c.weight_m2 > 0.0) && !(c.n0_m3 > 0.0))
    return "need weight_m2 > 0 or n0_m3 > 0";
  if (!(c.te_ev >= 0.0) || !(c.ti_ev >= 0.0)) return "temperatures must be >= 0";
  if (c.collisions && (!(c.p_pa >= 0.0) || !(c.t_gas_k > 0.0))) return "need p_pa >= 0 and t_gas_k > 0";
  if (!(c.gamma_see >= 0.0 && c.gamma_see <= 1.0)) return "gamma_see must be in [0, 1]";
  if (c.eedf_bins < 0 || c.eedf_bins > PIC_MAX_EEDF_BINS) return "eedf_bins out of range";
  if (c.impact_bins < 0 || c.impact_bins > PIC_MAX_EEDF_BINS || c.impact_angle_bins < 0 ||
      c.impact_angle_bins > PIC_MAX_EEDF_BINS)
    return "impact bins out of range";
  if (!(c.impact_emax_ev >= 0.0) || !std::isfinite(c.impact_emax_ev)) return "impact_emax_ev must be >= 0";
  if (c.sort_interval < 0 || c.avg_every < 0 || c.eedf_every < 0) return "negative interval";
  if (c.nu_max_e < 0.0 || c.nu_max_i < 0.0) return "nu_max must be >= 0";
  if (!std::isfinite(c.v_rf) || !std::isfinite(c.f_rf) || !std::isfinite(c.phase))
    return "RF drive must be finite";
  if (c.rebalance_ppc < 0 || c.rebalance_every < 0) return "negative rebalancing parameter";
  if (c.rebalance_ppc > 0 && c.precision != PIC_FP32_STATE) return "rebalancing needs the FP32 state form";
  if (!(c.rebalance_dv_e >= 0.0) || !(c.rebalance_dv_i >= 0.0)) return "rebalance_dv must be >= 0";
  return "";
}

// Analytic argon cross sections (m^2), energy in eV.
double sig_el_h(double e) { return 1.0e-19 / (1.0 + e / 20.0); }
double lnx_h(double e, double thr, double amp) {
  if (!(e > thr)) return 0.0;
  const double x = e / thr;
  return amp * std::log(x) / x;
}
double nu_max_electron_h(double n_g) {
  // 1.02 n_g max_eps sum_p sigma_p(eps) v(eps) on a log scan of 200001 points
  // from 1e-3 to 1e5 eV: exponents -3 + i (8 / 200000), the last exactly 5.
  double best = 0.0;
  const int n = 200001;
  const double step = (5.0 - (-3.0)) / (double)(n - 1);
  for (int i = 0; i < n; ++i) {
    const double y = (i == n - 1) ? 5.0 : (double)i * step + (-3.0);
    const double e = std::pow(10.0, y);
    const double v = std::sqrt(((2.0 * kQE) / kME) * e);
    best = std::max(best, ((sig_el_h(e) + lnx_h(e, kEXC, 2.7e-20)) + lnx_h(e, kION, 7.6e-20)) * v);
  }
  return 1.02 * n_g * best;
}
double nu_max_ion_h(double n_g, double v0, double tg) {
  const double g = std::sqrt(4.0 * kQE * std::fabs(v0) / kMAR) + 6.0 * std::sqrt(kKB * tg / kMAR);
  return n_g * kSIGMA_CX * g;
}

}  // namespace

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct pic_ctx {
  hipStream_t stream = nullptr;
  hipStream_t capture_stream = nullptr;
  char *arena = nullptr;
  size_t arena_bytes = 0;
  int n_inst = 0;
  int prec = 0;
  int n_cu = 256;
  int device = 0;              // the device current at pic_init: the arena's
  int drain_per_cu[M_PULLBACK + 1] = {1, 1, 1, 1, 1};   // by pass mode
  Pool pool;
  std::vector<SlotHost> slots;
  std::vector<InstDev> host_inst;
  InstDev *d_inst = nullptr;
  InstState *d_state = nullptr;
  unsigned long long *d_diag = nullptr;
  int max_n = 2;
  int field_classes = 0;   // field_class bits of the used slots
  // more than four discharges that start with at least kBatchGridSlots
  // particles in all: the sort and drain grids are larger (see sort_grid)
  bool batch_grids = false;
  bool inline_drain = false;   // fused passes drain in the particle kernel (small contexts)
  // 1024 threads per block: measured fastest on the large workload.  Plain
  // launches: on every workload measured they beat graph replay (by about
  // 10 % on the small and resolved discharges, 1 % on the large one).
  pic_tuning tune{1024, 0, 0, 0, 0};
  int rebalance_every = 0;     // pic_step rebalances every this many steps (0 = never)
  int64_t host_step = 0;
  // steps since the last sort of every slot (each sort moves the FP32 hot
  // words' epoch to the current step; in the FP32 form pic_step and pic_mcc
  // force one before this reaches kRebaseSteps)
  int64_t since_rebase = 0;
  bool deposit_current = false;
  std::string err;
  // graphs: [0] one step, [1] one step + sort
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  int graph_max_n = -1;
  // timing
  bool timing = false;
  pic_kernel_time times{};
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_kind;   // 0 field, 1 particles, 2 sort, 3 drain (per pair)
  int ev_used = 0;
  int64_t timed_steps = 0;    // timed steps since timing was enabled
};

// Message of the last failure of a call that had no context to hold it
// (pic_init); returned by pic_last_error(NULL).
static thread_local std::string g_init_err;

static pic_status fail(pic_ctx *c, pic_status s, const std::string &m) {
  if (c) c->err = m;
  g_init_err = m;
  return s;
}
#define HIP_TRY(ctx, expr)                                                          \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) return fail(ctx, PIC_EDEVICE, std::string(#expr ": ") +   \
                                                          hipGetErrorString(e_));   \
  } while (0)

static void drop_graphs(pic_ctx *c) {
  for (auto &g : c->graph)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  c->graph_max_n = -1;
}

// Where the fused pass's queued particles are drained (pic_tuning.inline_drain):
// by default inline when at most kInlineDrainMaxDischarges discharges start
// with at most kInlineDrainMaxSlots particles in all.
static void choose_drain(pic_ctx *c) {
  int64_t total = 0;
  int used = 0;
  for (int i = 0; i < c->n_inst && i < (int)c->host_inst.size(); ++i)
    if (c->slots[i].used) {
      ++used;
      total += c->host_inst[i].n_init[0] + (c->host_inst[i].nsp > 1 ? c->host_inst[i].n_init[1] : 0);
    }
  const bool small = used <= kInlineDrainMaxDischarges && total <= kInlineDrainMaxSlots;
  c->inline_drain = c->tune.inline_drain == 1 || (c->tune.inline_drain == 0 && small);
  c->batch_grids = used > 4 && total >= kBatchGridSlots;
}

// Called whenever the set of slots changes: the grid bound and the grid
// sizes (which follow the slots' capacities) change with it, so the captured
// graphs are dropped.
static void recompute_max_n(pic_ctx *c) {
  int m = 2;
  c->field_classes = 0;
  for (auto &s : c->slots)
    if (s.used) {
      m = std::max(m, (int)s.cfg.n_cells);
      c->field_classes |= field_class((int)s.cfg.n_cells);
    }
  c->max_n = (m + 3) / 4 * 4;
  choose_drain(c);
  drop_graphs(c);
}

// Tiles of `tile` particles (or queue entries) that the slots' capacities
// can hold: workgroups of a persistent grid beyond that number would only
// start and exit, which costs microseconds on small discharges.
static int64_t capacity_tiles(const pic_ctx *c, int64_t tile) {
  int64_t t = 0;
  for (int i = 0; i < c->n_inst; ++i) {
    if (!c->slots[i].used) continue;
    const InstDev &I = c->host_inst[i];
    for (int s = 0; s < I.nsp; ++s) t += (I.cap[s] + tile - 1) / tile;
  }
  return std::max<int64_t>(t, 1);
}
static int capped(const pic_ctx *c, int64_t grid, int64_t tile) {
  return (int)std::max<int64_t>(1, std::min(grid, capacity_tiles(c, tile)));
}

// Workgroups of the persistent particle kernel (of `block` threads): per CU
// the tuned value, or as many as fit in the CU's 160 KB of LDS at once (so
// that every workgroup of the persistent grid is resident together), at most
// 8; never more than the tiles the capacities hold.
static int particle_grid(const pic_ctx *c, int block) {
  int per = c->tune.blocks_per_cu;
  if (per <= 0) {
    const size_t lds = particle_lds_bytes(c->prec, c->max_n, c->tune.block) + 8192;
    per = (int)std::min<size_t>(8, std::max<size_t>(1, (160 * 1024) / lds));
  }
  return capped(c, (int64_t)c->n_cu * per, (int64_t)block * kParticlesPerThread);
}
// The sort's chains (load, LDS rank, scattered stores) are latency bound:
// more workgroups than stay resident at once measured faster (per CU 4 / 8 /
// 16: sweep 3.31 / 3.16 / 3.00 ms per sort, large 1.077 / 1.056 / 1.044).
// Finer still (64, 128) the sorts kept shrinking (sweep 2.76, 2.68 ms), but
// a single large discharge's next streaming passes slowed by as much (each
// cell's particles come from more pieces, in a less regular order): a large
// batch (batch_grids) sorts with 128 per CU, other contexts with 16.  A
// batch of many small discharges pays each extra workgroup's set-up (a
// prefix over every segment): the served trace of small requests got slower
// with the larger grids (p50 0.70 -> 0.83 s).
static int sort_grid(const pic_ctx *c) {
  return capped(c, (int64_t)c->n_cu * (c->batch_grids ? 128 : 16), kSortTile);
}
// The sort's count keeps 16 per CU: each workgroup clears and flushes a
// histogram of the grid's cells, which the large batch grid multiplied
// (sweep count 136 us at 16 per CU, 234 us at 128).
static int count_grid(const pic_ctx *c) { return capped(c, (int64_t)c->n_cu * 16, kSortTile); }
// The persistent moments pass: four workgroups per CU.
static int moments_grid(const pic_ctx *c) { return capped(c, (int64_t)c->n_cu * 4, kSortTile); }
// The drain grid: four times the workgroups resident at once.  The queue's
// length is known only on the device, and with more workgroups than fit the
// ones that finish early take more tiles (times the resident count 1 / 2 /
// 4 / 8 / 16: sweep drain 0.279 / 0.278 / 0.261 / 0.255 / 0.283 ms, large
// 42.4 / 44.0 / 42.8 / 47.5 / 56.5 us: small queues pay the per-workgroup
// set-up).
// A large batch (batch_grids: long queues over many segments) takes eight
// times.
static int drain_grid(const pic_ctx *c, int mode) {
  return capped(c, (int64_t)c->n_cu * c->drain_per_cu[mode] * (c->batch_grids ? 8 : 4), kDrainTile);
}

// Fill InstDev for slot i from its config and block offset; write host arrays.
static pic_status setup_slot(pic_ctx *c, int i, const pic_config &cfg) {
  SlotHost &sl = c->slots[i];
  const GridLayout g = layout(cfg);
  size_t off = 0;
  if (!c->pool.alloc(g.total, off))
    return fail(c, PIC_ENOMEM, "slot pool cannot hold " + std::to_string(g.total) + " bytes");
  sl.used = true;
  sl.off = off;
  sl.bytes = g.total;
  sl.cfg = cfg;
  const int N = cfg.n_cells;
  char *base = c->arena + off;
  // Host copies of the grid arrays.
  std::vector<double> nodes(N + 1), h(N), V(N + 1);
  const bool uniform = cfg.nodes == nullptr;
  double L, dx = 0.0;
  if (uniform) {
    L = cfg.gap_m;
    dx = L / N;
    for (int n = 0; n <= N; ++n) nodes[n] = (double)n * dx;
    for (int j = 0; j < N; ++j) h[j] = dx;
  } else {
    for (int n = 0; n <= N; ++n) nodes[n] = cfg.nodes[n];
    L = nodes[N];
    for (int j = 0; j < N; ++j) h[j] = nodes[j + 1] - nodes[j];
  }
  sl.nodes = nodes;
  sl.cfg.nodes = nullptr;   // the caller's array is not kept
  for (int n = 1; n < N; ++n) V[n] = (h[n - 1] + h[n]) / 2.0;
  if (cfg.bc == PIC_BC_PERIODIC) {
    V[0] = (h[N - 1] + h[0]) / 2.0;
    V[N] = V[0];
  } else {
    V[0] = h[0] / 2.0;
    V[N] = h[N - 1] / 2.0;
  }
  const double dt = cfg.dt_s;
  std::vector<float> dtoh(N), rf(N), rb(N);
  for (int j = 0; j < N; ++j) {
    const double hn = h[(j + 1) % N];
    dtoh[j] = (float)(dt / h[j]);
    rf[j] = (float)(h[j] / hn);
    rb[j] = (float)(hn / h[j]);
  }
  // Runs of cells joined by unit ratios (both directions): the walk crosses
  // them in one step.  Cell j's run is [first, last], packed first | last << 16.
  std::vector<int> runs(N);
  for (int j = 0; j < N;) {
    int e = j;
    while (e + 1 < N && rf[e] == 1.0f && rb[e] == 1.0f) ++e;
    for (int i = j; i <= e; ++i) runs[i] = j | (e << 16);
    j = e + 1;
  }

  InstDev I;
  std::memset(&I, 0, sizeof I);
  I.active = 1;
  I.N = N;
  I.bc = cfg.bc;
  I.gather = cfg.gather;
  I.nsp = cfg.n_species == 1 ? 1 : 2;
  I.uniform = uniform ? 1 : 0;
  I.collisions = cfg.collisions;
  I.eedf_bins = eff_bins(cfg);
  I.avg_every = cfg.avg_every;
  I.eedf_every = cfg.eedf_every;
  I.avg_start = cfg.avg_start;
  I.k_stop = cfg.k_stop;
  const int64_t cap = eff_cap(cfg);
  I.cap[0] = cap;
  I.cap[1] = I.nsp > 1 ? cap : 0;
  I.n_init[0] = cfg.n_per_species;
  I.n_init[1] = I.nsp > 1 ? cfg.n_per_species : 0;
  I.L = L;
  I.dx = dx;
  I.dt = dt;
  I.hmin = *std::min_element(h.begin(), h.end());
  I.v_rf = cfg.v_rf;
  I.w_rf = kTWO_PI * cfg.f_rf;
  I.phase = cfg.phase;
  I.growth_limit = cfg.growth_limit > 0.0 ? cfg.growth_limit : 10.0;
  I.n_g = cfg.collisions ? cfg.p_pa / (kKB * cfg.t_gas_k) : 0.0;
  I.vti = cfg.t_gas_k > 0.0 ? std::sqrt(kKB * cfg.t_gas_k / kMAR) : 0.0;
  const double t_see = cfg.t_see_ev > 0.0 ? cfg.t_see_ev : 2.0;
  I.vt_see = std::sqrt(t_see * kQE / kME);
  I.gamma_see = cfg.gamma_see;
  double W = cfg.weight_m2;
  if (W == 0.0 && cfg.n_per_species > 0) W = cfg.n0_m3 * L / (double)cfg.n_per_species;
  // A rebalanced discharge keeps its deposit in units of W/16 (weights W 2^(w-4)).
  I.wunit = cfg.rebalance_ppc > 0 ? 4 : 0;
  I.W = std::ldexp(W, -I.wunit);
  I.rb_ppc = cfg.rebalance_ppc;
  {
    const double te[2] = {cfg.te_ev, cfg.ti_ev}, ms[2] = {kME, kMAR}, dvg[2] = {cfg.rebalance_dv_e, cfg.rebalance_dv_i};
    for (int s = 0; s < 2; ++s)
      I.rb_dv[s] = dvg[s] > 0.0 ? dvg[s] : 0.25 * std::sqrt(std::max(te[s], 1e-6) * kQE / ms[s]);
  }
  const double q[2] = {-kQE, kQE}, m[2] = {kME, kMAR};
  const double nu_e = cfg.nu_max_e > 0.0 ? cfg.nu_max_e : nu_max_electron_h(I.n_g);
  const double nu_i = cfg.nu_max_i > 0.0 ? cfg.nu_max_i : nu_max_ion_h(I.n_g, cfg.v_rf, cfg.t_gas_k);
  I.nu_max[0] = nu_e;
  I.nu_max[1] = nu_i;
  for (int s = 0; s < 2; ++s) {
    I.nudt[s] = cfg.collisions ? I.nu_max[s] * dt : 0.0;
    I.qmdt[s] = (q[s] / m[s]) * dt;
    I.qmdt32[s] = (float)I.qmdt[s];
    I.hq[s] = 0.5 * I.qmdt[s];
    I.hq32[s] = (float)I.hq[s];
    I.qW[s] = q[s] * I.W;     // per deposit unit
    I.mass[s] = m[s];
  }
  I.int_path = (cfg.bc == PIC_BC_DIRICHLET_RF) && (I.nsp == 1 || I.qW[0] == -I.qW[1]);
  I.cgauss = ((I.nsp == 1 ? I.qW[0] : I.qW[1]) * 0x1p-32) / kEPS0;
  I.eedf_de = (cfg.eedf_emax_ev > 0.0 ? cfg.eedf_emax_ev : 50.0) / I.eedf_bins;
  I.eedf_centre = 0.5 * L;
  I.eedf_half = 0.5 * (cfg.eedf_width_m > 0.0 ? cfg.eedf_width_m : 1e-3);
  I.dtoh32u = uniform ? (float)(dt / dx) : 0.0f;
  I.seed = cfg.seed;
  I.nodes = (double *)(base + g.nodes);
  I.h = (double *)(base + g.h);
  I.V = (double *)(base + g.V);
  I.dtoh32 = (float *)(base + g.dtoh);
  I.rf32 = (float *)(base + g.rf);
  I.rb32 = (float *)(base + g.rb);
  I.runs = (int *)(base + g.runs);
  for (int p = 0; p < 2; ++p)
    for (int s = 0; s < 2; ++s) I.A[p][s] = (int64_t *)(base + g.A[p][s]);
  I.phi = (double *)(base + g.phi);
  I.E64 = (double *)(base + g.E64);
  I.E32 = (float *)(base + g.E32);
  I.accA[0] = (double *)(base + g.accA[0]);
  I.accA[1] = (double *)(base + g.accA[1]);
  I.acc_phi = (double *)(base + g.acc_phi);
  for (int s = 0; s < 2; ++s) {
    I.accM1[s] = (double *)(base + g.accM1[s]);
    I.accM2[s] = (double *)(base + g.accM2[s]);
    I.accP[s] = (double *)(base + g.accP[s]);
  }
  I.eedf = (unsigned long long *)(base + g.eedf);
  I.impact = (unsigned long long *)(base + g.impact);
  I.imp_bins = eff_ibins(cfg);
  I.imp_abins = eff_abins(cfg);
  I.imp_escale = (double)I.imp_bins / (cfg.impact_emax_ev > 0.0 ? cfg.impact_emax_ev : 1000.0);
  I.imp_ascale = (double)I.imp_abins / 90.0;
  I.moments = cfg.moments ? 1 : 0;
  for (int s = 0; s < 2; ++s) {
    I.scount[s] = (unsigned long long *)(base + g.scount[s]);
    I.scursor[s] = (unsigned long long *)(base + g.scursor[s]);
    I.queue[s] = (int4 *)(base + g.queue[s]);
    I.rb_flag[s] = cfg.rebalance_ppc > 0 ? (unsigned char *)(base + g.rb_flag[s]) : nullptr;
  }
  sl.rb = RbScratch();
  if (cfg.rebalance_ppc > 0) {
    RbScratch &r = sl.rb;
    r.words = (unsigned long long *)(base + g.rb_words);
    for (int b = 0; b < 2; ++b) {
      r.k64[b] = (unsigned long long *)(base + g.rb_k64[b]);
      r.k32[b] = (uint32_t *)(base + g.rb_k32[b]);
      r.val[b] = (uint32_t *)(base + g.rb_val[b]);
    }
    r.temp = base + g.rb_temp;
    r.temp_bytes = g.rb_temp_bytes;
    r.items = (int64_t)g.rb_items;
    const size_t need = rb_sort_temp_bytes(r.items);
    if (need == 0 || need > r.temp_bytes) {
      c->pool.release(off, g.total);
      sl = SlotHost();
      return fail(c, PIC_ENOMEM, "rebalancing sort scratch: " + std::to_string(need) + " bytes asked, " +
                                     std::to_string(g.rb_temp_bytes) + " reserved");
    }
  }
  const size_t pb = align_up((size_t)cap * bytes_per_particle(cfg.precision));
  for (int s = 0; s < I.nsp; ++s)
    for (int b = 0; b < 2; ++b) I.pbuf[s][b] = base + g.particles + (size_t)(2 * s + b) * pb;
  c->host_inst[i] = I;

  hipStream_t st = c->stream;
  HIP_TRY(c, hipMemsetAsync(base, 0, g.queue[0], st));
  HIP_TRY(c, hipMemcpyAsync(I.nodes, nodes.data(), 8 * (N + 1), hipMemcpyHostToDevice, st));
  HIP_TRY(c, hipMemcpyAsync(I.h, h.data(), 8 * N, hipMemcpyHostToDevice, st));
  HIP_TRY(c, hipMemcpyAsync(I.V, V.data(), 8 * (N + 1), hipMemcpyHostToDevice, st));
  HIP_TRY(c, hipMemcpyAsync(I.dtoh32, dtoh.data(), 4 * N, hipMemcpyHostToDevice, st));
  HIP_TRY(c, hipMemcpyAsync(I.rf32, rf.data(), 4 * N, hipMemcpyHostToDevice, st));
  HIP_TRY(c, hipMemcpyAsync(I.rb32, rb.data(), 4 * N, hipMemcpyHostToDevice, st));
  HIP_TRY(c, hipMemcpyAsync(I.runs, runs.data(), 4 * N, hipMemcpyHostToDevice, st));
  HIP_TRY(c, hipMemcpyAsync(c->d_inst + i, &c->host_inst[i], sizeof(InstDev), hipMemcpyHostToDevice, st));
  InstState S;
  std::memset(&S, 0, sizeof S);
  S.extent[0] = cfg.n_per_species;
  S.extent[1] = I.nsp > 1 ? cfg.n_per_species : 0;
  S.n_live[0] = S.extent[0];
  S.n_live[1] = S.extent[1];
  HIP_TRY(c, hipMemcpyAsync(c->d_state + i, &S, sizeof S, hipMemcpyHostToDevice, st));
  // Initial load, deposit of x^0, optional pull-back (this slot only).
  const double T[2] = {cfg.te_ev, cfg.ti_ev};
  for (int s = 0; s < I.nsp; ++s)
    launch_init(c->d_inst, c->d_state, i, s, c->prec, T[s], cfg.n_per_species, st);
  HIP_TRY(c, hipGetLastError());
  // Wait for the host arrays to reach the device before they go out of scope.
  HIP_TRY(c, hipStreamSynchronize(st));
  return PIC_OK;
}

// Sort by cell and deposit the new load of one slot (only >= 0) or of all.
// The other slots must not be touched by the per-slot work; the kernels take
// every active instance, so deactivate the others while it runs.
static pic_status deposit_only(pic_ctx *c, int only) {
  hipStream_t st = c->stream;
  std::vector<int> saved(c->n_inst);
  for (int i = 0; i < c->n_inst; ++i) saved[i] = c->host_inst[i].active;
  if (only >= 0) {
    for (int i = 0; i < c->n_inst; ++i) {
      const int a = (i == only) ? saved[i] : 0;
      HIP_TRY(c, hipMemcpyAsync(&c->d_inst[i].active, &a, sizeof a, hipMemcpyHostToDevice, st));
    }
  }
  // The initial load is drawn in particle order: one sort leaves it in cell
  // order, as every later sort does, so the first steps stream sorted state
  // (on the large discharge the first sort of an unsorted load takes about
  // five times as long as the later ones).
  HIP_TRY(c, launch_sort(c->d_inst, c->d_state, c->n_inst, c->prec, sort_grid(c), count_grid(c), c->max_n, st));
  launch_zero_deposit(c->d_inst, c->d_state, c->n_inst, st);
  HIP_TRY(c, launch_particles(c->d_inst, c->d_state, c->n_inst, c->prec, M_DEPOSIT, 256,
                              particle_grid(c, 256), c->max_n, st));
  if (only >= 0 && c->slots[only].cfg.pullback) {
    launch_field(c->d_inst, c->d_state, c->n_inst, c->field_classes, 0, st);
    HIP_TRY(c, launch_particles(c->d_inst, c->d_state, c->n_inst, c->prec, M_PULLBACK, 256,
                                particle_grid(c, 256), c->max_n, st));
  }
  if (only >= 0) {
    for (int i = 0; i < c->n_inst; ++i)
      HIP_TRY(c, hipMemcpyAsync(&c->d_inst[i].active, &c->host_inst[i].active, sizeof(int32_t),
                                hipMemcpyHostToDevice, st));
  }
  HIP_TRY(c, hipStreamSynchronize(st));
  return PIC_OK;
}

static pic_status check_inst(pic_ctx *c, int inst) {
  if (!c) return PIC_EINVAL;
  if (inst < 0 || inst >= c->n_inst) return fail(c, PIC_EINVAL, "instance index out of range");
  if (!c->slots[inst].used) return fail(c, PIC_ESTATE, "slot is empty");
  return PIC_OK;
}

static pic_status status_of(int bits) {
  if (bits & ST_CAPACITY) return PIC_ECAPACITY;
  if (bits & ST_NONFINITE) return PIC_ENONFINITE;
  if (bits & ST_GROWTH) return PIC_EGROWTH;
  return PIC_OK;
}

static pic_status read_state(pic_ctx *c, int inst, InstState &S) {
  HIP_TRY(c, hipMemcpyAsync(&S, c->d_state + inst, sizeof S, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return PIC_OK;
}

// ---------------------------------------------------------------------------
// Timing helpers
// ---------------------------------------------------------------------------
static pic_status flush_events(pic_ctx *c) {
  if (c->ev_used == 0) return PIC_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int p = 0; p < c->ev_used; ++p) {
    float ms = 0.0f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[2 * p], c->ev[2 * p + 1]));
    switch (c->ev_kind[p]) {
      case 0: c->times.field_ms += ms; c->times.field_launches++; break;
      case 1: c->times.particle_ms += ms; c->times.particle_launches++; break;
      case 3: c->times.drain_ms += ms; c->times.drain_launches++; break;
      default: c->times.sort_ms += ms; c->times.sort_launches++; break;
    }
  }
  c->ev_used = 0;
  return PIC_OK;
}
static pic_status ev_begin(pic_ctx *c, int kind) {
  if ((size_t)(2 * c->ev_used + 2) > c->ev.size()) {
    pic_status s = flush_events(c);
    if (s != PIC_OK) return s;
  }
  c->ev_kind[c->ev_used] = kind;
  HIP_TRY(c, hipEventRecord(c->ev[2 * c->ev_used], c->stream));
  return PIC_OK;
}
static pic_status ev_end(pic_ctx *c) {
  HIP_TRY(c, hipEventRecord(c->ev[2 * c->ev_used + 1], c->stream));
  c->ev_used++;
  return PIC_OK;
}

// One step (and the sort when `sort`) as plain launches on stream st.
// Whether any slot accumulates averaged profiles (the moments kernel runs).
static bool any_averaging(const pic_ctx *c) {
  for (int i = 0; i < c->n_inst; ++i)
    if (c->slots[i].used && c->host_inst[i].avg_every > 0 && c->host_inst[i].moments) return true;
  return false;
}

// With `timed`, HIP events bracket the streaming kernel on every
// kPassTiming-th timed step, the sort on every sort, and the field and the
// drain (with its closing kernel, when launched) on every kFullTiming-th
// timed step.  Each event record costs the stream a few microseconds: with
// the streaming kernel bracketed on every step, a large-discharge step took
// about 1 % longer than untimed.
constexpr int64_t kPassTiming = 4;
constexpr int64_t kFullTiming = 16;

// One fused step.  close_prev: the previous step was left open and this
// step's field launch closes it first; leave_open: this step's closing kernel
// is not launched (the next step's field launch does its work).
static pic_status enqueue_step(pic_ctx *c, hipStream_t st, bool sort, bool timed,
                               bool close_prev = false, bool leave_open = false) {
  const int64_t n_timed = timed ? c->timed_steps++ : 0;
  const bool all = timed && n_timed % kFullTiming == 0;
  const bool pass = timed && n_timed % kPassTiming == 0;
  if (all) { pic_status r = ev_begin(c, 0); if (r) return r; }
  launch_field(c->d_inst, c->d_state, c->n_inst, c->field_classes, close_prev ? 7 : 3, st);
  HIP_TRY(c, hipGetLastError());
  if (any_averaging(c)) {
    launch_moments(c->d_inst, c->d_state, c->n_inst, c->prec, moments_grid(c), c->max_n, st);
    HIP_TRY(c, hipGetLastError());
  }
  if (all) { pic_status r = ev_end(c); if (r) return r; }
  if (pass) { pic_status r = ev_begin(c, 1); if (r) return r; }
  if (c->inline_drain) {
    HIP_TRY(c, launch_particles(c->d_inst, c->d_state, c->n_inst, c->prec, M_FUSED_INLINE, 256,
                                particle_grid(c, 256), c->max_n, st));
  } else {
    HIP_TRY(c, launch_particles(c->d_inst, c->d_state, c->n_inst, c->prec, M_FUSED, c->tune.block,
                                particle_grid(c, c->tune.block), c->max_n, st));
  }
  if (pass) { pic_status r = ev_end(c); if (r) return r; }
  if (all) { pic_status r = ev_begin(c, 3); if (r) return r; }
  if (c->inline_drain) {
    if (!leave_open) launch_finalize(c->d_inst, c->d_state, c->n_inst, st);
    HIP_TRY(c, hipGetLastError());
  } else {
    HIP_TRY(c, launch_drain(c->d_inst, c->d_state, c->n_inst, c->prec, M_FUSED, drain_grid(c, M_FUSED),
                            !leave_open, st));
  }
  if (all) { pic_status r = ev_end(c); if (r) return r; }
  if (sort) {
    if (timed) { pic_status r = ev_begin(c, 2); if (r) return r; }
    HIP_TRY(c, launch_sort(c->d_inst, c->d_state, c->n_inst, c->prec, sort_grid(c), count_grid(c), c->max_n, st));
    if (timed) { pic_status r = ev_end(c); if (r) return r; }
  }
  return PIC_OK;
}

static pic_status get_graph(pic_ctx *c, int which, hipGraphExec_t &out) {
  if (c->graph_max_n != c->max_n) drop_graphs(c);
  if (!c->graph[which]) {
    hipGraph_t g = nullptr;
    HIP_TRY(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
    pic_status r = enqueue_step(c, c->capture_stream, which == 1, false);
    hipError_t e = hipStreamEndCapture(c->capture_stream, &g);
    if (r != PIC_OK) return r;
    if (e != hipSuccess) return fail(c, PIC_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    HIP_TRY(c, hipGraphInstantiate(&c->graph[which], g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    c->graph_max_n = c->max_n;
  }
  out = c->graph[which];
  return PIC_OK;
}

// One instance's diagnostics from its reduction words (D_* layout: live
// counts, fixed-point kinetic energies, the electrons' max |vx|, deposit
// totals) and its state.
static void fill_diag(const pic_ctx *c, int inst, const InstState &S, const unsigned long long *w,
                      pic_diag *out) {
  const InstDev &I = c->host_inst[inst];
  std::memset(out, 0, sizeof *out);
  out->step = S.k;
  out->time_s = (double)S.k * I.dt;
  out->status = S.status;
  out->n_samples = S.n_samples;
  out->eedf_samples = S.eedf_samples;
  auto ctr = [&](int i) {
    unsigned long long v = 0;
    for (int r = 0; r < kRep; ++r) v += S.ctr[i][r];
    return v;
  };
  for (int s = 0; s < 2; ++s) {
    out->n_live[s] = s < I.nsp ? (int64_t)w[D_LIVE0 + s] : 0;
    out->extent[s] = S.extent[s];
    out->deposit_total[s] = s < I.nsp ? (int64_t)w[D_DEP0 + s] : 0;
    out->kinetic_j_m2[s] = I.W * kQE * ((double)w[D_KE0 + s] * 0x1p-20);
    for (int wl = 0; wl < 2; ++wl) {
      out->absorbed[s][wl] = (int64_t)ctr(C_ABS + 2 * s + wl);
      out->absorbed_energy_ev[s][wl] = (double)ctr(C_EABS + 2 * s + wl) / 65536.0;
    }
    out->candidates[s] = (int64_t)ctr(C_CAND + s);
  }
  out->field_j_m2 = S.field_energy;
  out->see_emitted = (int64_t)ctr(C_SEE);
  out->ionisations = (int64_t)ctr(C_IZ);
  out->excitations = (int64_t)ctr(C_EX);
  out->elastic = (int64_t)ctr(C_EL);
  out->charge_exchange = (int64_t)ctr(C_CX);
  out->bound_violations = (int64_t)ctr(C_BOUND);
  out->particle_steps = (int64_t)ctr(C_PSTEPS);
  out->ne_max_m3 = S.ne_max;
  out->wpe_dt_max = std::sqrt(S.ne_max * kQE * kQE / (kEPS0 * kME)) * I.dt;
  double vmax;
  std::memcpy(&vmax, &w[D_VMAX], 8);
  out->vmax_dt_over_dxmin = vmax * I.dt / I.hmin;
  // the electrons' mean energy, weighted (their summed weight in deposit units)
  const double w_e = (double)w[D_WE];
  const double mean_ev = w_e > 0 ? ((double)w[D_KE0] * 0x1p-20) / w_e : 0.0;
  const double te = 2.0 * mean_ev / 3.0;
  // lambda_De = sqrt(eps0 T_e / (n_e e)) with T_e in volts.
  out->lambda_de_over_dxmin = S.ne_max > 0 ? std::sqrt(kEPS0 * te / (S.ne_max * kQE)) / I.hmin : 0.0;
  out->nu_max[0] = I.nu_max[0];
  out->nu_max[1] = I.nu_max[1];
  for (int s = 0; s < 2; ++s) {
    out->merges[s] = (int64_t)S.ctr[C_MERGE][s];
    out->splits[s] = (int64_t)S.ctr[C_SPLIT][s];
  }
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int32_t pic_abi_version(void) { return PIC_ABI_VERSION; }

const char *pic_status_string(pic_status s) {
  switch (s) {
    case PIC_OK: return "ok";
    case PIC_EINVAL: return "invalid argument";
    case PIC_ENOMEM: return "arena or pool too small";
    case PIC_ECAPACITY: return "particle capacity exceeded";
    case PIC_ENONFINITE: return "non-finite particle state";
    case PIC_EGROWTH: return "runaway particle growth";
    case PIC_EDEVICE: return "HIP runtime error";
    case PIC_ESTATE: return "invalid state for this call";
  }
  return "unknown status";
}

size_t pic_slot_bytes(const pic_config *cfg) {
  if (!cfg || cfg->n_cells == 0) return 0;
  return align_up(layout(*cfg).total);
}

size_t pic_footprint(const pic_config *cfgs, int32_t n) {
  if (!cfgs || n <= 0 || n > PIC_MAX_INSTANCES) return 0;
  size_t b = static_bytes(n);
  for (int i = 0; i < n; ++i) b += pic_slot_bytes(&cfgs[i]);
  return b + kAlign;
}

pic_status pic_init(const pic_config *cfgs, int32_t n_inst, void *device_arena, size_t arena_bytes,
                    void *hip_stream, pic_ctx **out) {
  if (!out) return PIC_EINVAL;
  *out = nullptr;
  if (!cfgs || n_inst <= 0 || n_inst > PIC_MAX_INSTANCES || !device_arena)
    return fail(nullptr, PIC_EINVAL, "bad pic_init arguments");
  int prec = -1;
  for (int i = 0; i < n_inst; ++i) {
    const std::string why = validate(cfgs[i]);
    if (!why.empty()) return fail(nullptr, PIC_EINVAL, "config " + std::to_string(i) + ": " + why);
    if (cfgs[i].n_cells > 0) {
      if (prec >= 0 && cfgs[i].precision != prec)
        return fail(nullptr, PIC_EINVAL, "all instances of a context share one precision");
      prec = cfgs[i].precision;
    }
  }
  if (prec < 0) prec = cfgs[0].precision == PIC_FP32_STATE ? 1 : 0;
  const size_t need = pic_footprint(cfgs, n_inst);
  if (arena_bytes < need)
    return fail(nullptr, PIC_ENOMEM, "arena smaller than pic_footprint: " + std::to_string(need));

  pic_ctx *c = new pic_ctx();
  c->stream = (hipStream_t)hip_stream;
  c->arena = (char *)device_arena;
  c->arena_bytes = arena_bytes;
  c->n_inst = n_inst;
  c->prec = prec;
  c->slots.resize(n_inst);
  c->host_inst.resize(n_inst);
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    delete c;
    return PIC_EDEVICE;
  }
  c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  c->device = dev;
  if (noalloc_setup(dev) != hipSuccess) {
    delete c;
    return fail(nullptr, PIC_EDEVICE, "device address of the no-allocation scratch");
  }
  for (int m : {M_PUSH, M_MCC, M_FUSED}) c->drain_per_cu[m] = drain_blocks_per_cu(prec, m);
  if (hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return PIC_EDEVICE;
  }
  for (int i = 0; i < n_inst; ++i)
    if (cfgs[i].n_cells > 0 && cfgs[i].sort_interval > 0) {
      c->tune.sort_interval = cfgs[i].sort_interval;
      break;
    }
  for (int i = 0; i < n_inst; ++i)
    if (cfgs[i].n_cells > 0 && cfgs[i].rebalance_ppc > 0 && cfgs[i].rebalance_every > 0) {
      c->rebalance_every = cfgs[i].rebalance_every;
      break;
    }
  // Static region.
  size_t o = 0;
  c->d_inst = (InstDev *)(c->arena + o);
  o += align_up(sizeof(InstDev) * n_inst);
  c->d_state = (InstState *)(c->arena + o);
  o += align_up(sizeof(InstState) * n_inst);
  c->d_diag = (unsigned long long *)(c->arena + o);
  o += align_up(8 * D_NWORDS);
  c->pool.reset(align_up(o), arena_bytes);
  std::memset(c->host_inst.data(), 0, sizeof(InstDev) * n_inst);
  pic_status r = PIC_OK;
  if (hipMemsetAsync(c->arena, 0, o, c->stream) != hipSuccess) r = PIC_EDEVICE;
  for (int i = 0; i < n_inst && r == PIC_OK; ++i) {
    if (hipMemcpyAsync(c->d_inst + i, &c->host_inst[i], sizeof(InstDev), hipMemcpyHostToDevice,
                       c->stream) != hipSuccess)
      r = PIC_EDEVICE;
  }
  for (int i = 0; i < n_inst && r == PIC_OK; ++i)
    if (cfgs[i].n_cells > 0) r = setup_slot(c, i, cfgs[i]);
  if (r == PIC_OK) {
    recompute_max_n(c);
    r = deposit_only(c, -1);
  }
  if (r == PIC_OK) {
    // Pull-back: one field solve at k = 0 without accumulation, then the
    // half-step velocity correction of the instances that ask for it.
    bool any = false;
    for (int i = 0; i < n_inst; ++i) any |= (cfgs[i].n_cells > 0 && cfgs[i].pullback);
    if (any) {
      for (int i = 0; i < n_inst && r == PIC_OK; ++i)
        if (cfgs[i].n_cells > 0 && cfgs[i].pullback) r = deposit_only(c, i);
    }
  }
  if (r != PIC_OK) {
    g_init_err = c->err;
    pic_destroy(c);
    return r;
  }
  c->deposit_current = true;
  *out = c;
  return PIC_OK;
}

void pic_destroy(pic_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  for (auto e : c->ev) (void)hipEventDestroy(e);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  delete c;
}

const char *pic_last_error(const pic_ctx *c) { return c ? c->err.c_str() : g_init_err.c_str(); }

pic_status pic_deposit(pic_ctx *c) {
  if (!c) return PIC_EINVAL;
  launch_zero_deposit(c->d_inst, c->d_state, c->n_inst, c->stream);
  HIP_TRY(c, launch_particles(c->d_inst, c->d_state, c->n_inst, c->prec, M_DEPOSIT, 256,
                              particle_grid(c, 256), c->max_n, c->stream));
  c->deposit_current = true;
  return PIC_OK;
}

pic_status pic_poisson(pic_ctx *c) {
  if (!c) return PIC_EINVAL;
  if (!c->deposit_current) return fail(c, PIC_ESTATE, "deposit is stale: call pic_deposit first");
  launch_field(c->d_inst, c->d_state, c->n_inst, c->field_classes, 1, c->stream);
  HIP_TRY(c, hipGetLastError());
  if (any_averaging(c)) {
    launch_moments(c->d_inst, c->d_state, c->n_inst, c->prec, moments_grid(c), c->max_n, c->stream);
    HIP_TRY(c, hipGetLastError());
  }
  return PIC_OK;
}

pic_status pic_gather_push(pic_ctx *c) {
  if (!c) return PIC_EINVAL;
  HIP_TRY(c, launch_particles(c->d_inst, c->d_state, c->n_inst, c->prec, M_PUSH, 256,
                              particle_grid(c, 256), c->max_n, c->stream));
  HIP_TRY(c, launch_drain(c->d_inst, c->d_state, c->n_inst, c->prec, M_PUSH, drain_grid(c, M_PUSH), true, c->stream));
  c->deposit_current = false;
  return PIC_OK;
}

pic_status pic_mcc(pic_ctx *c) {
  if (!c) return PIC_EINVAL;
  HIP_TRY(c, launch_particles(c->d_inst, c->d_state, c->n_inst, c->prec, M_MCC, 256,
                              particle_grid(c, 256), c->max_n, c->stream));
  HIP_TRY(c, launch_drain(c->d_inst, c->d_state, c->n_inst, c->prec, M_MCC, drain_grid(c, M_MCC), true, c->stream));
  c->deposit_current = false;
  c->host_step++;
  if (++c->since_rebase >= kRebaseSteps && c->prec == PIC_FP32_STATE) return pic_sort(c);
  return PIC_OK;
}

pic_status pic_sort(pic_ctx *c) {
  if (!c) return PIC_EINVAL;
  HIP_TRY(c, launch_sort(c->d_inst, c->d_state, c->n_inst, c->prec, sort_grid(c), count_grid(c), c->max_n, c->stream));
  c->since_rebase = 0;
  return PIC_OK;
}

pic_status pic_rebalance(pic_ctx *c) {
  if (!c) return PIC_EINVAL;
  bool any = false;
  for (int i = 0; i < c->n_inst; ++i) any |= c->slots[i].used && c->host_inst[i].rb_ppc > 0;
  if (!any) return PIC_OK;
  // cell order (and the cell ranges the flags are read from)
  HIP_TRY(c, launch_sort(c->d_inst, c->d_state, c->n_inst, c->prec, sort_grid(c), count_grid(c), c->max_n, c->stream));
  for (int i = 0; i < c->n_inst; ++i) {
    if (!c->slots[i].used || c->host_inst[i].rb_ppc <= 0) continue;
    InstState S;
    pic_status r = read_state(c, i, S);
    if (r != PIC_OK) return r;
    if (S.frozen) continue;
    const hipError_t e = launch_rebalance(c->d_inst, c->d_state, i, c->host_inst[i].N, c->slots[i].rb, c->stream);
    if (e == hipErrorInvalidValue) return fail(c, PIC_ENOMEM, "rebalancing list beyond its scratch");
    if (e != hipSuccess) return fail(c, PIC_EDEVICE, std::string("rebalance: ") + hipGetErrorString(e));
  }
  // compact: the merged-away particles leave, the split children join the order
  HIP_TRY(c, launch_sort(c->d_inst, c->d_state, c->n_inst, c->prec, sort_grid(c), count_grid(c), c->max_n, c->stream));
  c->since_rebase = 0;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->deposit_current = false;
  for (int i = 0; i < c->n_inst; ++i) {
    if (!c->slots[i].used || c->host_inst[i].rb_ppc <= 0) continue;
    InstState S;
    pic_status r = read_state(c, i, S);
    if (r != PIC_OK) return r;
    if (S.status != 0) return status_of(S.status);
  }
  return PIC_OK;
}

pic_status pic_step(pic_ctx *c, int32_t n_steps) {
  if (!c || n_steps < 0) return PIC_EINVAL;
  bool any = false;
  for (auto &s : c->slots) any |= s.used;
  if (!any) return fail(c, PIC_ESTATE, "no active slot");
  if (!c->deposit_current) {
    pic_status r = pic_deposit(c);
    if (r != PIC_OK) return r;
  }
  const int S = c->tune.sort_interval;
  // With plain launches, a step followed by another in this call (and not
  // by a sort) is closed by the next step's field launch: one launch fewer
  // per step.  Every call returns with its last step closed.
  bool open = false;
  const int R = c->rebalance_every;
  for (int n = 0; n < n_steps; ++n) {
    // a sort at its interval, or (FP32 form) one that keeps the hot words'
    // epoch offsets in range (see kRebaseSteps)
    const bool sort = (S > 0 && ((c->host_step + 1) % S) == 0) ||
                      (c->prec == PIC_FP32_STATE && c->since_rebase + 1 >= kRebaseSteps);
    const bool rebal = R > 0 && ((c->host_step + 1) % R) == 0;
    if (c->timing || !c->tune.use_graph) {
      const bool leave_open = !sort && !rebal && n + 1 < n_steps;
      pic_status r = enqueue_step(c, c->stream, sort, c->timing, open, leave_open);
      if (r != PIC_OK) return r;
      open = leave_open;
    } else {
      hipGraphExec_t g = nullptr;
      pic_status r = get_graph(c, sort ? 1 : 0, g);
      if (r != PIC_OK) return r;
      HIP_TRY(c, hipGraphLaunch(g, c->stream));
    }
    c->host_step++;
    c->since_rebase = sort ? 0 : c->since_rebase + 1;
    if (rebal) {
      pic_status r = pic_rebalance(c);
      if (r != PIC_OK) return r;
      r = pic_deposit(c);
      if (r != PIC_OK) return r;
    }
  }
  return PIC_OK;
}

pic_status pic_diagnostics(pic_ctx *c, int32_t inst, pic_diag *out) {
  pic_status r = check_inst(c, inst);
  if (r != PIC_OK) return r;
  if (!out) return fail(c, PIC_EINVAL, "null output");
  HIP_TRY(c, hipMemsetAsync(c->d_diag, 0, 8 * D_NWORDS, c->stream));
  launch_diag(c->d_inst, c->d_state, inst, c->prec, std::max(c->host_inst[inst].cap[0], c->host_inst[inst].cap[1]),
              c->d_diag, c->stream);
  HIP_TRY(c, hipGetLastError());
  unsigned long long w[D_NWORDS];
  HIP_TRY(c, hipMemcpyAsync(w, c->d_diag, sizeof w, hipMemcpyDeviceToHost, c->stream));
  InstState S;
  r = read_state(c, inst, S);
  if (r != PIC_OK) return r;
  const InstDev &I = c->host_inst[inst];
  std::vector<int64_t> A(2 * (I.N + 1), 0);
  const int par = (int)(S.k & 1);
  for (int s = 0; s < I.nsp; ++s)
    HIP_TRY(c, hipMemcpy(A.data() + s * (I.N + 1), I.A[par][s], 8 * (I.N + 1), hipMemcpyDeviceToHost));
  const int upto = (I.bc == PIC_BC_PERIODIC) ? I.N : I.N + 1;
  for (int s = 0; s < I.nsp; ++s) {
    int64_t tot = 0;
    for (int n = 0; n < upto; ++n) tot += A[s * (I.N + 1) + n];
    w[D_DEP0 + s] = (unsigned long long)tot;
  }
  fill_diag(c, inst, S, w, out);
  return status_of(S.status);
}

pic_status pic_diagnostics_noalloc(pic_ctx *c, const int32_t *insts, int32_t n, pic_diag *out) {
  if (!c) return PIC_EINVAL;
  if (!insts || !out) return fail(c, PIC_EINVAL, "null instance list or output");
  if (n < 1 || n > kNoAllocMaxInst)
    return fail(c, PIC_EINVAL, "pic_diagnostics_noalloc takes 1 to " + std::to_string(kNoAllocMaxInst) +
                                   " instances per call, got " + std::to_string(n));
  for (int i = 0; i < n; ++i) {
    pic_status r = check_inst(c, insts[i]);
    if (r != PIC_OK) return r;
  }
  unsigned long long *scr = noalloc_scratch(c->device);
  if (!scr) return fail(c, PIC_EDEVICE, "no-allocation scratch was not set up on this device");
  hipStream_t st = c->stream;
  // The array keeps the previous call's records: clear this call's.
  launch_fill_zero(scr, n * kNoAllocRecord, st);
  for (int i = 0; i < n; ++i) {
    unsigned long long *rec = scr + (size_t)i * kNoAllocRecord;
    launch_diag(c->d_inst, c->d_state, insts[i], c->prec,
                std::max(c->host_inst[insts[i]].cap[0], c->host_inst[insts[i]].cap[1]), rec, st);
    launch_deposit_total(c->d_inst, c->d_state, insts[i], rec, st);
  }
  HIP_TRY(c, hipGetLastError());
  // Records come back in chunks through a buffer on the stack.
  constexpr int kChunk = 16;
  unsigned long long w[kChunk * kNoAllocRecord];
  pic_status worst = PIC_OK;
  for (int i0 = 0; i0 < n; i0 += kChunk) {
    const int m = std::min(kChunk, n - i0);
    HIP_TRY(c, hipMemcpyAsync(w, scr + (size_t)i0 * kNoAllocRecord, sizeof(unsigned long long) * m * kNoAllocRecord,
                              hipMemcpyDeviceToHost, st));
    for (int j = 0; j < m; ++j) {
      InstState S;
      pic_status r = read_state(c, insts[i0 + j], S);   // synchronises the stream
      if (r != PIC_OK) return r;
      fill_diag(c, insts[i0 + j], S, w + (size_t)j * kNoAllocRecord, out + i0 + j);
      if (worst == PIC_OK) worst = status_of(S.status);
    }
  }
  return worst;
}

pic_status pic_get_state(pic_ctx *c, int32_t inst, int32_t species, pic_state_view *v) {
  pic_status r = check_inst(c, inst);
  if (r != PIC_OK) return r;
  const InstDev &I = c->host_inst[inst];
  if (!v || species < 0 || species >= I.nsp) return fail(c, PIC_EINVAL, "bad species or view");
  InstState S;
  r = read_state(c, inst, S);
  if (r != PIC_OK) return r;
  const int64_t ext = S.extent[species];
  char *b = I.pbuf[species][S.parity];
  const int64_t cap = I.cap[species];
  std::vector<uint64_t> id(ext);
  std::vector<int32_t> kn(ext);
  int64_t live = 0;
  if (c->prec == PIC_FP32_STATE) {
    P32 P = view32(b, cap);
    std::vector<uint32_t> hw(ext);
    std::vector<int32_t> cell(ext);
    std::vector<float> off(ext), vx(ext), vy(ext), vz(ext);
    std::vector<Cold32> cold(ext);
    HIP_TRY(c, hipMemcpy(hw.data(), P.hw, 4 * ext, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(off.data(), P.off, 4 * ext, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(vx.data(), P.vx, 4 * ext, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(kn.data(), P.knext, 4 * ext, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(cold.data(), P.cold, sizeof(Cold32) * ext, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < ext; ++i) {
      vy[i] = cold[i].vy;
      vz[i] = cold[i].vz;
      id[i] = cold[i].id;
      // the hot word's cell and candidacy (absolute step)
      cell[i] = hw_live(hw[i]) ? hw_cell(hw[i]) : -1;
      if (hw_live(hw[i])) kn[i] = (int32_t)hw_knext(hw[i], kn[i], S.epoch);
    }
    for (int64_t i = 0; i < ext; ++i) live += cell[i] >= 0;
    if (live > v->n) { v->n = live; return fail(c, PIC_EINVAL, "view too small"); }
    int64_t o = 0;
    for (int64_t i = 0; i < ext; ++i) {
      if (cell[i] < 0) continue;
      if (v->wclass) v->wclass[o] = (uint8_t)hw_class(hw[i]);
      if (v->cell) v->cell[o] = cell[i];
      if (v->off) v->off[o] = off[i];
      if (v->vx) ((float *)v->vx)[o] = vx[i];
      if (v->vy) ((float *)v->vy)[o] = vy[i];
      if (v->vz) ((float *)v->vz)[o] = vz[i];
      if (v->id) v->id[o] = id[i];
      if (v->knext) v->knext[o] = kn[i];
      ++o;
    }
  } else {
    P64 P = view64(b, cap);
    std::vector<double> x(ext), vx(ext), vy(ext), vz(ext);
    HIP_TRY(c, hipMemcpy(x.data(), P.x, 8 * ext, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(vx.data(), P.vx, 8 * ext, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(vy.data(), P.vy, 8 * ext, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(vz.data(), P.vz, 8 * ext, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(kn.data(), P.knext, 4 * ext, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(id.data(), P.id, 8 * ext, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < ext; ++i) live += x[i] >= 0.0;
    if (live > v->n) { v->n = live; return fail(c, PIC_EINVAL, "view too small"); }
    int64_t o = 0;
    for (int64_t i = 0; i < ext; ++i) {
      if (!(x[i] >= 0.0)) continue;
      if (v->x) v->x[o] = x[i];
      if (v->vx) ((double *)v->vx)[o] = vx[i];
      if (v->vy) ((double *)v->vy)[o] = vy[i];
      if (v->vz) ((double *)v->vz)[o] = vz[i];
      if (v->id) v->id[o] = id[i];
      if (v->knext) v->knext[o] = kn[i];
      ++o;
    }
  }
  v->n = live;
  return status_of(S.status);
}

pic_status pic_set_state(pic_ctx *c, int32_t inst, int32_t species, const pic_state_view *v) {
  pic_status r = check_inst(c, inst);
  if (r != PIC_OK) return r;
  const InstDev &I = c->host_inst[inst];
  if (!v || species < 0 || species >= I.nsp || v->n < 0) return fail(c, PIC_EINVAL, "bad species or view");
  const int64_t n = v->n;
  if (n > I.cap[species]) return fail(c, PIC_ECAPACITY, "more particles than capacity");
  if (!v->vx || !v->vy || !v->vz || !v->id || !v->knext) return fail(c, PIC_EINVAL, "null array");
  if (c->prec == PIC_FP32_STATE) {
    if (!v->cell || !v->off) return fail(c, PIC_EINVAL, "null cell/off");
    for (int64_t i = 0; i < n; ++i) {
      const float o = v->off[i];
      const int w = v->wclass ? (int)v->wclass[i] : kClassUnit;
      if (w > 7 || (I.wunit == 0 && w != kClassUnit))
        return fail(c, PIC_EINVAL, "weight class of particle " + std::to_string(i) +
                                       " out of range (only 4 without rebalancing)");
      if (v->cell[i] < 0 || v->cell[i] >= I.N || !(o >= 0.0f && o < 1.0f) ||
          !std::isfinite(((float *)v->vx)[i]) || !std::isfinite(((float *)v->vy)[i]) ||
          !std::isfinite(((float *)v->vz)[i]) || v->knext[i] < 0)
        return fail(c, PIC_EINVAL, "particle " + std::to_string(i) + " out of range or non-finite");
    }
  } else {
    if (!v->x) return fail(c, PIC_EINVAL, "null x");
    for (int64_t i = 0; i < n; ++i) {
      if (!(v->x[i] >= 0.0 && v->x[i] < I.L) || !std::isfinite(((double *)v->vx)[i]) ||
          !std::isfinite(((double *)v->vy)[i]) || !std::isfinite(((double *)v->vz)[i]) ||
          v->knext[i] < 0)
        return fail(c, PIC_EINVAL, "particle " + std::to_string(i) + " out of range or non-finite");
    }
  }
  InstState S;
  r = read_state(c, inst, S);
  if (r != PIC_OK) return r;
  char *b = I.pbuf[species][S.parity];
  const int64_t cap = I.cap[species];
  if (n > 0) {
    if (c->prec == PIC_FP32_STATE) {
      P32 P = view32(b, cap);
      std::vector<uint32_t> hw(n);
      for (int64_t i = 0; i < n; ++i)
        hw[i] = hw_encode(v->cell[i], v->knext[i], S.k, S.epoch, v->wclass ? (int)v->wclass[i] : kClassUnit);
      HIP_TRY(c, hipMemcpy(P.hw, hw.data(), 4 * n, hipMemcpyHostToDevice));
      HIP_TRY(c, hipMemcpy(P.off, v->off, 4 * n, hipMemcpyHostToDevice));
      HIP_TRY(c, hipMemcpy(P.vx, v->vx, 4 * n, hipMemcpyHostToDevice));
      HIP_TRY(c, hipMemcpy(P.knext, v->knext, 4 * n, hipMemcpyHostToDevice));
      std::vector<Cold32> cold(n);
      for (int64_t i = 0; i < n; ++i)
        cold[i] = Cold32{((const float *)v->vy)[i], ((const float *)v->vz)[i], v->id[i]};
      HIP_TRY(c, hipMemcpy(P.cold, cold.data(), sizeof(Cold32) * n, hipMemcpyHostToDevice));
    } else {
      P64 P = view64(b, cap);
      HIP_TRY(c, hipMemcpy(P.x, v->x, 8 * n, hipMemcpyHostToDevice));
      HIP_TRY(c, hipMemcpy(P.vx, v->vx, 8 * n, hipMemcpyHostToDevice));
      HIP_TRY(c, hipMemcpy(P.vy, v->vy, 8 * n, hipMemcpyHostToDevice));
      HIP_TRY(c, hipMemcpy(P.vz, v->vz, 8 * n, hipMemcpyHostToDevice));
      HIP_TRY(c, hipMemcpy(P.knext, v->knext, 4 * n, hipMemcpyHostToDevice));
      HIP_TRY(c, hipMemcpy(P.id, v->id, 8 * n, hipMemcpyHostToDevice));
    }
  }
  S.extent[species] = n;
  S.n_live[species] = n;
  S.append &= ~(0xFFFFFFFFull << (32 * species));
  HIP_TRY(c, hipMemcpy(c->d_state + inst, &S, sizeof S, hipMemcpyHostToDevice));
  c->deposit_current = false;
  return PIC_OK;
}

pic_status pic_set_step(pic_ctx *c, int32_t inst, int64_t k) {
  pic_status r = check_inst(c, inst);
  if (r != PIC_OK) return r;
  if (k < 0 || k >= kINT32_MAX) return fail(c, PIC_EINVAL, "step out of range");
  InstState S;
  r = read_state(c, inst, S);
  if (r != PIC_OK) return r;
  if (c->prec == PIC_FP32_STATE) {
    // the FP32 hot words: re-expressed for a next pass at step k, with
    // epoch k
    launch_reencode(c->d_inst, c->d_state, inst, S.epoch, k, c->stream);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  S.k = k;
  S.epoch = k;
  HIP_TRY(c, hipMemcpy(c->d_state + inst, &S, sizeof S, hipMemcpyHostToDevice));
  c->deposit_current = false;
  return PIC_OK;
}

pic_status pic_get_fields(pic_ctx *c, int32_t inst, int64_t *A_e, int64_t *A_i, double *phi,
                          double *E, float *E32) {
  pic_status r = check_inst(c, inst);
  if (r != PIC_OK) return r;
  InstState S;
  r = read_state(c, inst, S);
  if (r != PIC_OK) return r;
  const InstDev &I = c->host_inst[inst];
  const int par = (int)(S.k & 1);
  const size_t n1 = (size_t)I.N + 1;
  const size_t ne = I.gather == PIC_GATHER_EC ? (size_t)I.N : (I.gather == PIC_GATHER_MC ? n1 : n1 + 1);
  if (A_e) HIP_TRY(c, hipMemcpy(A_e, I.A[par][0], 8 * n1, hipMemcpyDeviceToHost));
  if (A_i && I.nsp > 1) HIP_TRY(c, hipMemcpy(A_i, I.A[par][1], 8 * n1, hipMemcpyDeviceToHost));
  if (phi) HIP_TRY(c, hipMemcpy(phi, I.phi, 8 * n1, hipMemcpyDeviceToHost));
  if (E) HIP_TRY(c, hipMemcpy(E, I.E64, 8 * ne, hipMemcpyDeviceToHost));
  if (E32) HIP_TRY(c, hipMemcpy(E32, I.E32, 4 * ne, hipMemcpyDeviceToHost));
  return status_of(S.status);
}

pic_status pic_profiles(pic_ctx *c, int32_t inst, double *ne, double *ni, double *phi,
                        int64_t *eedf) {
  pic_status r = check_inst(c, inst);
  if (r != PIC_OK) return r;
  InstState S;
  r = read_state(c, inst, S);
  if (r != PIC_OK) return r;
  const InstDev &I = c->host_inst[inst];
  const SlotHost &sl = c->slots[inst];
  const size_t n1 = (size_t)I.N + 1;
  std::vector<double> acc(n1), V(n1);
  HIP_TRY(c, hipMemcpy(V.data(), I.V, 8 * n1, hipMemcpyDeviceToHost));
  const double nsm = (double)std::max(S.n_samples, 1);
  const double scale = I.W * 0x1p-32;
  double *dst[2] = {ne, ni};
  for (int s = 0; s < 2; ++s) {
    if (!dst[s]) continue;
    if (s >= I.nsp) {
      std::fill(dst[s], dst[s] + n1, 0.0);
      continue;
    }
    HIP_TRY(c, hipMemcpy(acc.data(), I.accA[s], 8 * n1, hipMemcpyDeviceToHost));
    for (size_t n = 0; n < n1; ++n) dst[s][n] = (acc[n] * scale) / (V[n] * nsm);
  }
  if (phi) {
    HIP_TRY(c, hipMemcpy(acc.data(), I.acc_phi, 8 * n1, hipMemcpyDeviceToHost));
    for (size_t n = 0; n < n1; ++n) phi[n] = acc[n] / nsm;
  }
  if (eedf) HIP_TRY(c, hipMemcpy(eedf, I.eedf, 8 * (size_t)I.eedf_bins, hipMemcpyDeviceToHost));
  (void)sl;
  return status_of(S.status);
}

pic_status pic_moments(pic_ctx *c, int32_t inst, int32_t species, double *ux, double *tx, double *power) {
  pic_status r = check_inst(c, inst);
  if (r != PIC_OK) return r;
  const InstDev &I = c->host_inst[inst];
  if (species < 0 || species >= I.nsp) return fail(c, PIC_EINVAL, "species out of range");
  if (!I.moments) return fail(c, PIC_ESTATE, "moments were not enabled for this instance");
  InstState S;
  r = read_state(c, inst, S);
  if (r != PIC_OK) return r;
  const size_t n1 = (size_t)I.N + 1, N = (size_t)I.N;
  std::vector<double> a(n1), m1(n1), m2(n1), p(N), h(N);
  HIP_TRY(c, hipMemcpy(a.data(), I.accA[species], 8 * n1, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(m1.data(), I.accM1[species], 8 * n1, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(m2.data(), I.accM2[species], 8 * n1, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(p.data(), I.accP[species], 8 * N, hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemcpy(h.data(), I.h, 8 * N, hipMemcpyDeviceToHost));
  if (I.bc == PIC_BC_PERIODIC) {   // node N is node 0 (the deposit is folded the same way)
    m1[0] += m1[N];
    m1[N] = m1[0];
    m2[0] += m2[N];
    m2[N] = m2[0];
  }
  const double mq = I.mass[species] / kQE;
  for (size_t n = 0; n < n1; ++n) {
    const double w = a[n] * 0x1p-32;   // sum of the particles' weights at node n
    const double u = w > 0.0 ? m1[n] / w : 0.0;
    if (ux) ux[n] = u;
    if (tx) tx[n] = w > 0.0 ? mq * (m2[n] / w - u * u) : 0.0;
  }
  const double ns = (double)std::max(S.n_samples, 1);
  if (power)
    for (size_t j = 0; j < N; ++j) power[j] = (I.qW[species] * p[j]) / (h[j] * ns);
  return status_of(S.status);
}

pic_status pic_impacts(pic_ctx *c, int32_t inst, int32_t species, int32_t wall, int64_t *energy,
                       int64_t *angle) {
  pic_status r = check_inst(c, inst);
  if (r != PIC_OK) return r;
  const InstDev &I = c->host_inst[inst];
  if (species < 0 || species > 1 || wall < 0 || wall > 1)
    return fail(c, PIC_EINVAL, "species and wall must be 0 or 1");
  InstState S;
  r = read_state(c, inst, S);
  if (r != PIC_OK) return r;
  const size_t row = (size_t)I.imp_bins + 1 + (size_t)I.imp_abins;
  const unsigned long long *src = I.impact + (size_t)(2 * species + wall) * row;
  if (energy) HIP_TRY(c, hipMemcpy(energy, src, 8 * ((size_t)I.imp_bins + 1), hipMemcpyDeviceToHost));
  if (angle)
    HIP_TRY(c, hipMemcpy(angle, src + I.imp_bins + 1, 8 * (size_t)I.imp_abins, hipMemcpyDeviceToHost));
  return status_of(S.status);
}

// ---------------------------------------------------------------------------
// Checkpoint and resume of one instance
// ---------------------------------------------------------------------------
namespace {
// What a checkpoint must agree on with the slot it is loaded into: the
// configuration that fixes the layout, the grid and the arithmetic.
struct CkptCfg {
  int32_t N, bc, gather, prec, nsp, collisions, avg_every, eedf_every, eedf_bins, imp_bins, imp_abins,
      moments, wunit, rb_ppc;
  int64_t cap[2], avg_start, k_stop;
  double L, W, dt, v_rf, w_rf, phase, n_g, t_gas, vt_see, gamma_see, nu_max[2], growth_limit,
      eedf_de, eedf_half, imp_escale, rb_dv[2];
  uint64_t seed;
};
struct CkptHeader {
  char magic[8];
  uint32_t version, prec;
  int64_t extent[2];
  uint64_t total;
  CkptCfg cfg;
};
constexpr uint32_t kCkptVersion = 2;
const char kCkptMagic[8] = {'E', 'C', 'P', 'I', 'C', 'C', 'K', '1'};

CkptCfg ckpt_cfg(const pic_ctx *c, int inst) {
  CkptCfg k;
  std::memset(&k, 0, sizeof k);
  const InstDev &I = c->host_inst[inst];
  const pic_config &g = c->slots[inst].cfg;
  k.N = I.N; k.bc = I.bc; k.gather = I.gather; k.prec = c->prec; k.nsp = I.nsp;
  k.collisions = I.collisions; k.avg_every = I.avg_every; k.eedf_every = I.eedf_every;
  k.eedf_bins = I.eedf_bins; k.imp_bins = I.imp_bins; k.imp_abins = I.imp_abins; k.moments = I.moments;
  k.cap[0] = I.cap[0]; k.cap[1] = I.cap[1]; k.avg_start = I.avg_start; k.k_stop = I.k_stop;
  k.L = I.L; k.W = I.W; k.dt = I.dt; k.v_rf = I.v_rf; k.w_rf = I.w_rf; k.phase = I.phase; k.n_g = I.n_g;
  k.t_gas = g.t_gas_k; k.vt_see = I.vt_see; k.gamma_see = I.gamma_see; k.nu_max[0] = I.nu_max[0];
  k.nu_max[1] = I.nu_max[1]; k.growth_limit = I.growth_limit; k.eedf_de = I.eedf_de;
  k.eedf_half = I.eedf_half; k.imp_escale = I.imp_escale; k.seed = I.seed;
  k.wunit = I.wunit; k.rb_ppc = I.rb_ppc; k.rb_dv[0] = I.rb_dv[0]; k.rb_dv[1] = I.rb_dv[1];
  return k;
}

// The device arrays of a checkpoint, in order: (pointer, bytes).
std::vector<std::pair<char *, size_t>> ckpt_arrays(const pic_ctx *c, int inst, const int64_t ext[2],
                                                   int parity) {
  const InstDev &I = c->host_inst[inst];
  const size_t n1 = (size_t)I.N + 1, N = (size_t)I.N;
  std::vector<std::pair<char *, size_t>> a;
  auto add = [&](void *p, size_t b) { a.emplace_back((char *)p, b); };
  add(I.accA[0], 8 * n1);
  add(I.accA[1], 8 * n1);
  add(I.acc_phi, 8 * n1);
  for (int s = 0; s < 2; ++s) {
    add(I.accM1[s], 8 * n1);
    add(I.accM2[s], 8 * n1);
    add(I.accP[s], 8 * N);
  }
  add(I.eedf, 8 * (size_t)I.eedf_bins);
  add(I.impact, 8 * 4 * ((size_t)I.imp_bins + 1 + (size_t)I.imp_abins));
  for (int s = 0; s < I.nsp; ++s) {
    const size_t e = (size_t)ext[s];
    char *b = I.pbuf[s][parity];
    if (c->prec == PIC_FP32_STATE) {
      const P32 P = view32(b, I.cap[s]);
      add(P.hw, 4 * e);
      add(P.off, 4 * e);
      add(P.vx, 4 * e);
      add(P.knext, 4 * e);
      add(P.cold, sizeof(Cold32) * e);
    } else {
      const P64 P = view64(b, I.cap[s]);
      add(P.x, 8 * e);
      add(P.vx, 8 * e);
      add(P.vy, 8 * e);
      add(P.vz, 8 * e);
      add(P.knext, 4 * e);
      add(P.id, 8 * e);
    }
  }
  return a;
}

size_t ckpt_total(const std::vector<std::pair<char *, size_t>> &a, size_t n_nodes) {
  size_t t = sizeof(CkptHeader) + sizeof(InstState) + 8 * n_nodes;
  for (auto &x : a) t += x.second;
  return t;
}
}  // namespace

pic_status pic_checkpoint_bytes(pic_ctx *c, int32_t inst, size_t *bytes) {
  pic_status r = check_inst(c, inst);
  if (r != PIC_OK) return r;
  if (!bytes) return fail(c, PIC_EINVAL, "null output");
  InstState S;
  r = read_state(c, inst, S);
  if (r != PIC_OK) return r;
  *bytes = ckpt_total(ckpt_arrays(c, inst, S.extent, S.parity), c->slots[inst].nodes.size());
  return PIC_OK;
}

pic_status pic_checkpoint_save(pic_ctx *c, int32_t inst, void *buf, size_t bytes) {
  pic_status r = check_inst(c, inst);
  if (r != PIC_OK) return r;
  if (!buf) return fail(c, PIC_EINVAL, "null buffer");
  InstState S;
  r = read_state(c, inst, S);
  if (r != PIC_OK) return r;
  const auto arrays = ckpt_arrays(c, inst, S.extent, S.parity);
  const std::vector<double> &nodes = c->slots[inst].nodes;
  const size_t total = ckpt_total(arrays, nodes.size());
  if (bytes < total) return fail(c, PIC_EINVAL, "checkpoint buffer smaller than pic_checkpoint_bytes");
  char *o = (char *)buf;
  CkptHeader h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, kCkptMagic, 8);
  h.version = kCkptVersion;
  h.prec = (uint32_t)c->prec;
  h.extent[0] = S.extent[0];
  h.extent[1] = S.extent[1];
  h.total = total;
  h.cfg = ckpt_cfg(c, inst);
  std::memcpy(o, &h, sizeof h);
  o += sizeof h;
  std::memcpy(o, &S, sizeof S);
  o += sizeof S;
  std::memcpy(o, nodes.data(), 8 * nodes.size());
  o += 8 * nodes.size();
  for (auto &a : arrays) {
    if (a.second) HIP_TRY(c, hipMemcpy(o, a.first, a.second, hipMemcpyDeviceToHost));
    o += a.second;
  }
  return status_of(S.status);
}

pic_status pic_checkpoint_load(pic_ctx *c, int32_t inst, const void *buf, size_t bytes) {
  pic_status r = check_inst(c, inst);
  if (r != PIC_OK) return r;
  if (!buf || bytes < sizeof(CkptHeader) + sizeof(InstState)) return fail(c, PIC_EINVAL, "checkpoint too short");
  const char *o = (const char *)buf;
  CkptHeader h;
  std::memcpy(&h, o, sizeof h);
  o += sizeof h;
  if (std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.version != kCkptVersion)
    return fail(c, PIC_EINVAL, "not a checkpoint of this library version");
  const CkptCfg mine = ckpt_cfg(c, inst);
  if (h.prec != (uint32_t)c->prec || std::memcmp(&h.cfg, &mine, sizeof mine) != 0)
    return fail(c, PIC_EINVAL, "checkpoint configuration differs from the slot's");
  const InstDev &I = c->host_inst[inst];
  for (int s = 0; s < 2; ++s)
    if (h.extent[s] < 0 || h.extent[s] > I.cap[s]) return fail(c, PIC_EINVAL, "checkpoint extent beyond capacity");
  const std::vector<double> &nodes = c->slots[inst].nodes;
  InstState S;
  std::memcpy(&S, o, sizeof S);
  o += sizeof S;
  if (std::memcmp(o, nodes.data(), 8 * nodes.size()) != 0)
    return fail(c, PIC_EINVAL, "checkpoint grid differs from the slot's");
  o += 8 * nodes.size();
  if (S.extent[0] != h.extent[0] || S.extent[1] != h.extent[1] || (S.parity != 0 && S.parity != 1))
    return fail(c, PIC_EINVAL, "corrupt checkpoint state");
  const auto arrays = ckpt_arrays(c, inst, S.extent, S.parity);
  const size_t total = ckpt_total(arrays, nodes.size());
  if (h.total != total || bytes < total) return fail(c, PIC_EINVAL, "checkpoint size mismatch");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (auto &a : arrays) {
    if (a.second) HIP_TRY(c, hipMemcpy(a.first, o, a.second, hipMemcpyHostToDevice));
    o += a.second;
  }
  // the FP32 hot words: re-expressed from the current step (the context's
  // sorts keep that epoch in range from here on)
  const int64_t E0 = S.epoch;
  S.epoch = S.k;
  HIP_TRY(c, hipMemcpy(c->d_state + inst, &S, sizeof S, hipMemcpyHostToDevice));
  if (c->prec == PIC_FP32_STATE) {
    launch_reencode(c->d_inst, c->d_state, inst, E0, S.k, c->stream);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  c->deposit_current = false;   // the next step rebuilds the deposit of x^k (exact)
  return PIC_OK;
}

pic_status pic_slot_reset(pic_ctx *c, int32_t inst, const pic_config *cfg) {
  if (!c || !cfg) return PIC_EINVAL;
  if (inst < 0 || inst >= c->n_inst) return fail(c, PIC_EINVAL, "instance index out of range");
  const std::string why = validate(*cfg);
  if (!why.empty()) return fail(c, PIC_EINVAL, why);
  if (cfg->n_cells > 0 && cfg->precision != c->prec)
    return fail(c, PIC_EINVAL, "precision differs from the context's");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (c->slots[inst].used) {
    pic_status r = pic_slot_release(c, inst);
    if (r != PIC_OK) return r;
  }
  if (cfg->n_cells == 0) return PIC_OK;
  if (c->pool.largest() < align_up(layout(*cfg).total))
    return fail(c, PIC_ENOMEM, "slot pool cannot hold this discharge");
  pic_status r = setup_slot(c, inst, *cfg);
  if (r != PIC_OK) return r;
  recompute_max_n(c);
  r = deposit_only(c, inst);
  if (r != PIC_OK) return r;
  if (c->tune.sort_interval == 0 && cfg->sort_interval > 0) c->tune.sort_interval = cfg->sort_interval;
  if (c->rebalance_every == 0 && cfg->rebalance_ppc > 0 && cfg->rebalance_every > 0)
    c->rebalance_every = cfg->rebalance_every;
  return PIC_OK;
}

pic_status pic_slot_release(pic_ctx *c, int32_t inst) {
  if (!c) return PIC_EINVAL;
  if (inst < 0 || inst >= c->n_inst) return fail(c, PIC_EINVAL, "instance index out of range");
  SlotHost &sl = c->slots[inst];
  if (!sl.used) return PIC_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  InstDev I;
  std::memset(&I, 0, sizeof I);
  c->host_inst[inst] = I;
  HIP_TRY(c, hipMemcpy(c->d_inst + inst, &I, sizeof I, hipMemcpyHostToDevice));
  InstState S;
  std::memset(&S, 0, sizeof S);
  HIP_TRY(c, hipMemcpy(c->d_state + inst, &S, sizeof S, hipMemcpyHostToDevice));
  c->pool.release(sl.off, sl.bytes);
  sl = SlotHost();
  recompute_max_n(c);
  return PIC_OK;
}

size_t pic_pool_free(const pic_ctx *c) { return c ? c->pool.largest() : 0; }

pic_status pic_set_tuning(pic_ctx *c, const pic_tuning *t) {
  if (!c || !t) return PIC_EINVAL;
  if (t->block != 256 && t->block != 512 && t->block != 1024)
    return fail(c, PIC_EINVAL, "block must be 256, 512 or 1024");
  if (t->blocks_per_cu < 0 || t->blocks_per_cu > 16)
    return fail(c, PIC_EINVAL, "blocks_per_cu in [0, 16] (0 = as many as fit)");
  if (t->sort_interval < 0) return fail(c, PIC_EINVAL, "sort_interval must be >= 0");
  if (t->inline_drain < 0 || t->inline_drain > 2) return fail(c, PIC_EINVAL, "inline_drain must be 0, 1 or 2");
  c->tune = *t;
  choose_drain(c);
  drop_graphs(c);
  return PIC_OK;
}

pic_status pic_get_tuning(const pic_ctx *c, pic_tuning *t) {
  if (!c || !t) return PIC_EINVAL;
  *t = c->tune;
  return PIC_OK;
}

pic_status pic_kernel_times(pic_ctx *c, int32_t enable, pic_kernel_time *out) {
  if (!c) return PIC_EINVAL;
  pic_status r = flush_events(c);
  if (r != PIC_OK) return r;
  if (out) *out = c->times;
  if (enable && !c->timing) {
    if (c->ev.empty()) {
      c->ev.resize(2 * 384);
      c->ev_kind.resize(384);
      for (auto &e : c->ev) HIP_TRY(c, hipEventCreate(&e));
    }
    c->times = pic_kernel_time{};
    c->timed_steps = 0;
  }
  c->timing = enable != 0;
  return PIC_OK;
}

int32_t pic_grid_refined(double L, double dx_min, double dx_max, double L_buff, double *nodes,
                         int32_t max_nodes) {
  if (!(L > 0.0) || !(dx_min > 0.0) || !(dx_max >= dx_min) || !(L_buff >= 0.0)) return -1;
  const int a = (int)std::lround(std::log2(L / dx_min));
  const int b = (int)std::lround(std::log2(L / dx_max));
  if (a < 0 || a > 24 || b < 0 || b > a) return -1;
  if (std::fabs(L / std::ldexp(1.0, a) - dx_min) > 1e-9 * dx_min) return -1;
  if (std::fabs(L / std::ldexp(1.0, b) - dx_max) > 1e-9 * dx_max) return -1;
  const int64_t U = (int64_t)1 << a;
  const int64_t smin = 1, smax = (int64_t)1 << (a - b);
  const double buff = L_buff / dx_min;
  // Dyadic refinement: split while larger than dx_max, or larger than dx_min
  // and overlapping a buffer; then split any cell more than twice a neighbour.
  std::vector<std::pair<int64_t, int64_t>> cells{{0, U}}, next;
  bool changed = true;
  while (changed) {
    changed = false;
    next.clear();
    for (auto &cl : cells) {
      const int64_t s = cl.second - cl.first;
      const bool in_buf = (double)cl.first < buff || (double)cl.second > (double)U - buff;
      if (s > smax || (in_buf && s > smin)) {
        const int64_t m = (cl.first + cl.second) / 2;
        next.push_back({cl.first, m});
        next.push_back({m, cl.second});
        changed = true;
      } else {
        next.push_back(cl);
      }
    }
    cells.swap(next);
  }
  changed = true;
  while (changed) {
    changed = false;
    next.clear();
    for (size_t i = 0; i < cells.size(); ++i) {
      const int64_t s = cells[i].second - cells[i].first;
      bool split = false;
      if (i > 0 && s > 2 * (cells[i - 1].second - cells[i - 1].first)) split = true;
      if (i + 1 < cells.size() && s > 2 * (cells[i + 1].second - cells[i + 1].first)) split = true;
      if (split) {
        const int64_t m = (cells[i].first + cells[i].second) / 2;
        next.push_back({cells[i].first, m});
        next.push_back({m, cells[i].second});
        changed = true;
      } else {
        next.push_back(cells[i]);
      }
    }
    cells.swap(next);
  }
  const int32_t N = (int32_t)cells.size();
  if (nodes && max_nodes >= N + 1) {
    const double unit = L / (double)U;
    for (int32_t i = 0; i < N; ++i) nodes[i] = (double)cells[i].first * unit;
    nodes[N] = (double)U * unit;
  }
  return N;
}

}  // extern "C"
