// kernels_sort.hip -- counting sort of the particles by cell, with compaction.
//
// Every sort_interval steps the particles of each (instance, species) segment
// are reordered by cell into the other particle buffer and absorbed particles
// are dropped.  In a sorted state a lane's consecutive particles share a cell
// (their deposit merges in registers before the LDS atomics) and each
// workgroup's share of the grid stays small.  Three passes:
//   count   per-workgroup LDS histogram of the live cells, added to HBM;
//   scan    one workgroup per instance: exclusive prefix of the counts gives
//           each cell's first destination slot;
//   scatter ranks within the tile from LDS atomics, one reservation per
//           (tile, cell) with an HBM atomic, then every field is copied to its
//           destination; a one-workgroup kernel then flips the buffers.
// Order within a cell is not defined; results depend on the particle set only.
#include "device.h"
#include "kernels.h"

namespace ecpic {

constexpr int kSB = 256;      // threads per workgroup
constexpr int kSPPT = 4;      // particles per thread per tile (a multiple of 4)
static_assert(kSPPT % 4 == 0, "records are loaded 4 at a time");
constexpr int kSTile = kSB * kSPPT;
static_assert(kSTile == kSortTile, "the host sizes the sort grid with kSortTile");

struct SortSmem {
  int seg_prefix[2 * kMaxInst + 1];
};

__device__ __forceinline__ int key_of(CInst &I, const P32 &P, int64_t i, const double *,
                                      const double *) {
  const uint32_t w = P.hw[i];
  return (hw_live(w) && hw_cell(w) < I.N) ? hw_cell(w) : -1;
}
__device__ __forceinline__ int key_of(CInst &I, const P64 &P, int64_t i, const double *nodes,
                                      const double *h) {
  const double x = P.x[i];
  if (!(x >= 0.0 && x < I.L)) return -1;
  if (I.uniform) {
    int j = (int)floor(x / I.dx);
    return j >= I.N ? I.N - 1 : j;
  }
  int lo = 0, hi = I.N;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (nodes[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Runs of equal keys in consecutive lanes of a wavefront (particles arrive
// nearly sorted by cell, so a wavefront holds few runs).  Returns whether this
// lane starts its run; len is the run's length and pos this lane's place in
// it.  Letting only the first lane of a run update a counter avoids the
// serialisation of many lanes updating one LDS address.
__device__ __forceinline__ bool key_run(int key, int &len, int &pos) {
  const int lane = __lane_id();
  const int prev = __shfl_up(key, 1, 64);
  const bool head = lane == 0 || key != prev;
  const unsigned long long heads = __ballot(head);
  const unsigned long long le = (2ull << lane) - 1ull;   // lanes 0..lane (all for lane 63)
  const int h = 63 - __clzll((long long)(heads & le));
  const unsigned long long above = heads & ~le;
  const int nxt = above ? __ffsll((long long)above) - 1 : 64;
  pos = lane - h;
  len = nxt - h;
  return head;
}

// Segment tile prefix over the instances that are not frozen.
__device__ void seg_prefix_setup(const InstDev *insts, const InstState *states, int n_inst,
                                 int *prefix, int tile = kSTile) {
  const int nseg = 2 * n_inst;
  for (int s = threadIdx.x; s < nseg; s += kSB) {
    CInst &I = cinst(insts)[s >> 1];
    const InstState &S = states[s >> 1];
    const bool ok = I.active && S.frozen == 0 && (s & 1) < I.nsp;
    const int64_t ext = ok ? S.extent[s & 1] : 0;
    prefix[s + 1] = (int)((ext + tile - 1) / tile);
  }
  tile_prefix(prefix, nseg);
}

template <class P>
__device__ __forceinline__ P make_view(CInst &I, int s, int buf);
template <>
__device__ __forceinline__ P32 make_view<P32>(CInst &I, int s, int buf) {
  return view32(I.pbuf[s][buf], I.cap[s]);
}
template <>
__device__ __forceinline__ P64 make_view<P64>(CInst &I, int s, int buf) {
  return view64(I.pbuf[s][buf], I.cap[s]);
}

constexpr int kCTile = kSB * 16;   // particles per tile of the count kernel

// Cell keys of particles i0..i0+3 (-1: dead or beyond the extent).
__device__ __forceinline__ void count_keys(CInst &I, const P32 &P, int64_t i0, int64_t ext,
                                           const double *, int *key) {
  if (i0 + 4 <= ext) {
    const int4 c = gload4(reinterpret_cast<const int *>(P.hw) + i0);
    const uint32_t cc[4] = {(uint32_t)c.x, (uint32_t)c.y, (uint32_t)c.z, (uint32_t)c.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) key[q] = (hw_live(cc[q]) && hw_cell(cc[q]) < I.N) ? hw_cell(cc[q]) : -1;
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) key[q] = (i0 + q < ext) ? key_of(I, P, i0 + q, nullptr, nullptr) : -1;
  }
}
__device__ __forceinline__ void count_keys(CInst &I, const P64 &P, int64_t i0, int64_t ext,
                                           const double *nodes, int *key) {
#pragma unroll
  for (int q = 0; q < 4; ++q) key[q] = (i0 + q < ext) ? key_of(I, P, i0 + q, nodes, nullptr) : -1;
}

template <class P>
__global__ void __launch_bounds__(kSB)
k_sort_count(const InstDev *__restrict__ insts, const InstState *__restrict__ states, int n_inst,
             int max_n) {
  __shared__ SortSmem sm;
  extern __shared__ __align__(16) unsigned char dsm[];
  unsigned int *hist = reinterpret_cast<unsigned int *>(dsm);
  double *sNodes = reinterpret_cast<double *>(dsm + 4 * ((max_n + 2) & ~1));
  for (int j = threadIdx.x; j < max_n; j += kSB) hist[j] = 0;
  seg_prefix_setup(insts, states, n_inst, sm.seg_prefix, kCTile);
  const int nseg = 2 * n_inst;
  const int64_t T = sm.seg_prefix[nseg];
  const int64_t t0 = T * blockIdx.x / gridDim.x, t1 = T * (blockIdx.x + 1) / gridDim.x;
  int seg = -1;
  CInst *Ip = nullptr;
  P view;
  int64_t ext = 0;
  auto flush = [&]() {
    __syncthreads();
    CInst &I = *Ip;
    for (int j = threadIdx.x; j < I.N; j += kSB) {
      const unsigned int v = hist[j];
      if (v) {
        atomicAdd(&I.scount[seg & 1][j], (unsigned long long)v);
        hist[j] = 0;
      }
    }
    __syncthreads();
  };
  for (int64_t tile = t0; tile < t1; ++tile) {
    int s = seg < 0 ? segment_of(sm.seg_prefix, nseg, tile) : seg;
    while (sm.seg_prefix[s + 1] <= tile) ++s;
    s = __builtin_amdgcn_readfirstlane(s);
    if (s != seg) {
      if (seg >= 0) flush();
      seg = s;
      Ip = &cinst(insts)[seg >> 1];
      const InstState &S = states[seg >> 1];
      ext = uni((int64_t)S.extent[seg & 1]);   // scalar: no wait on vector memory per tile
      view = make_view<P>(*Ip, seg & 1, S.parity);
      if (sizeof(P) == sizeof(P64) && !Ip->uniform)
        for (int j = threadIdx.x; j <= Ip->N; j += kSB) sNodes[j] = Ip->nodes[j];
      __syncthreads();
    }
    // The thread's particles: 4 groups of 4 consecutive ones, each group
    // read by one vector load that is contiguous across the wavefront.
    const int64_t base = (tile - sm.seg_prefix[seg]) * kCTile;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int64_t i0 = base + 4 * ((int64_t)g * kSB + threadIdx.x);
      int key[4];
      count_keys(*Ip, view, i0, ext, sNodes, key);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int len, pos;
        if (key_run(key[q], len, pos) && key[q] >= 0) atomicAdd(&hist[key[q]], (unsigned int)len);
      }
    }
  }
  if (seg >= 0) flush();
}

// One workgroup per instance: first destination slot of every cell.
__global__ void __launch_bounds__(kSB)
k_sort_scan(const InstDev *__restrict__ insts, InstState *__restrict__ states) {
  __shared__ unsigned long long tmp[kSB];
  CInst &I = cinst(insts)[blockIdx.x];
  InstState &S = states[blockIdx.x];
  if (!I.active || S.frozen != 0) return;
  const int N = I.N;
  const int t = threadIdx.x;
  for (int s = 0; s < I.nsp; ++s) {
    const int c = (N + kSB - 1) / kSB;
    const int lo = min(N, t * c), hi = min(N, lo + c);
    unsigned long long sum = 0;
    for (int j = lo; j < hi; ++j) sum += I.scount[s][j];
    tmp[t] = sum;
    __syncthreads();
    for (int off = 1; off < kSB; off <<= 1) {
      const unsigned long long v = (t >= off) ? tmp[t - off] : 0ull;
      __syncthreads();
      tmp[t] += v;
      __syncthreads();
    }
    unsigned long long run = (t > 0) ? tmp[t - 1] : 0ull;
    for (int j = lo; j < hi; ++j) {
      const unsigned long long cnt = I.scount[s][j];
      I.scursor[s][j] = run;
      run += cnt;
      I.scount[s][j] = 0;
    }
    if (t == kSB - 1) S.sort_live[s] = (int64_t)tmp[kSB - 1];
    __syncthreads();
  }
}

// One particle's fields in registers.
struct Rec32 {   // 4-byte fields only (the id as two words): kept in registers
  uint32_t hw; float off, vx, vy, vz; int knext; uint32_t id_lo, id_hi;
};
struct Rec64 {
  double x, vx, vy, vz; int knext; uint64_t id;
};
template <class P> struct RecOf;
template <> struct RecOf<P32> { using T = Rec32; };
template <> struct RecOf<P64> { using T = Rec64; };

// Load the 4 consecutive particles i0..i0+3 of a thread (vector loads when
// all four are inside the extent).
__device__ __forceinline__ void load_recs(const P32 &P, int64_t i0, int64_t ext, Rec32 *r, bool *ok) {
  if (i0 + 4 <= ext) {
    const int4 c = gload4(reinterpret_cast<const int *>(P.hw) + i0);
    const float4 o = gload4(P.off + i0), x = gload4(P.vx + i0);
    const uint32_t cc[4] = {(uint32_t)c.x, (uint32_t)c.y, (uint32_t)c.z, (uint32_t)c.w};
    // knext matters only for far particles (see hw_encode): the others'
    // entries are neither read nor moved
    int4 k = make_int4(0, 0, 0, 0);
    if (hw_far(cc[0]) || hw_far(cc[1]) || hw_far(cc[2]) || hw_far(cc[3])) k = gload4(P.knext + i0);
    const float oo[4] = {o.x, o.y, o.z, o.w}, xx[4] = {x.x, x.y, x.z, x.w};
    const int kk[4] = {k.x, k.y, k.z, k.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const ecpic_iv4 cd = *(const ECPIC_GLOBAL ecpic_iv4 *)(P.cold + i0 + q);
      r[q] = Rec32{cc[q], oo[q], xx[q], __int_as_float(cd.x), __int_as_float(cd.y), kk[q],
                   (uint32_t)cd.z, (uint32_t)cd.w};
      ok[q] = true;
    }
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = i0 + q;
      ok[q] = i < ext;
      r[q] = Rec32{kHwDead, 0.0f, 0.0f, 0.0f, 0.0f, 0, 0u, 0u};
      if (ok[q]) {
        const ecpic_iv4 cd = *(const ECPIC_GLOBAL ecpic_iv4 *)(P.cold + i);
        const uint32_t w = P.hw[i];
        r[q] = Rec32{w, P.off[i], P.vx[i], __int_as_float(cd.x), __int_as_float(cd.y),
                     hw_far(w) ? P.knext[i] : 0, (uint32_t)cd.z, (uint32_t)cd.w};
      }
    }
  }
}
__device__ __forceinline__ void load_recs(const P64 &P, int64_t i0, int64_t ext, Rec64 *r, bool *ok) {
  if (i0 + 4 <= ext) {
    const double2 xa = gload2(P.x + i0), xb = gload2(P.x + i0 + 2);
    const double2 ua = gload2(P.vx + i0), ub = gload2(P.vx + i0 + 2);
    const double2 va = gload2(P.vy + i0), vb = gload2(P.vy + i0 + 2);
    const double2 wa = gload2(P.vz + i0), wb = gload2(P.vz + i0 + 2);
    const int4 k = gload4(P.knext + i0);
    const ecpic_iv4 ia = *(const ECPIC_GLOBAL ecpic_iv4 *)(P.id + i0);
    const ecpic_iv4 ib = *(const ECPIC_GLOBAL ecpic_iv4 *)(P.id + i0 + 2);
    const double xx[4] = {xa.x, xa.y, xb.x, xb.y}, uu[4] = {ua.x, ua.y, ub.x, ub.y},
                 vv[4] = {va.x, va.y, vb.x, vb.y}, ww[4] = {wa.x, wa.y, wb.x, wb.y};
    const int kk[4] = {k.x, k.y, k.z, k.w};
    const uint64_t ii[4] = {(uint64_t)(uint32_t)ia.x | ((uint64_t)(uint32_t)ia.y << 32),
                            (uint64_t)(uint32_t)ia.z | ((uint64_t)(uint32_t)ia.w << 32),
                            (uint64_t)(uint32_t)ib.x | ((uint64_t)(uint32_t)ib.y << 32),
                            (uint64_t)(uint32_t)ib.z | ((uint64_t)(uint32_t)ib.w << 32)};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      r[q] = Rec64{xx[q], uu[q], vv[q], ww[q], kk[q], ii[q]};
      ok[q] = true;
    }
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = i0 + q;
      ok[q] = i < ext;
      if (ok[q]) r[q] = Rec64{P.x[i], P.vx[i], P.vy[i], P.vz[i], P.knext[i], P.id[i]};
    }
  }
}

__device__ __forceinline__ void store_rec(const P32 &P, int64_t d, const Rec32 &r) {
  gstore<uint32_t>(P.hw + d, r.hw);
  gstore<float>(P.off + d, r.off);
  gstore<float>(P.vx + d, r.vx);
  if (hw_far(r.hw)) gstore<int>(P.knext + d, r.knext);
  const ecpic_iv4 cd = {__float_as_int(r.vy), __float_as_int(r.vz), (int)r.id_lo, (int)r.id_hi};
  *(ECPIC_GLOBAL ecpic_iv4 *)(P.cold + d) = cd;
}
__device__ __forceinline__ void store_rec(const P64 &P, int64_t d, const Rec64 &r) {
  gstore<double>(P.x + d, r.x);
  gstore<double>(P.vx + d, r.vx);
  gstore<double>(P.vy + d, r.vy);
  gstore<double>(P.vz + d, r.vz);
  gstore<int>(P.knext + d, r.knext);
  gstore<uint64_t>(P.id + d, r.id);
}
// FP32 form: the hot word re-expressed from the slot's epoch E0 to the step k
// of the next pass, which becomes the epoch (see hw_encode).  A far word
// whose candidacy comes into range loses its knext entry; an overdue one
// gains it.
__device__ __forceinline__ void rebase_rec(Rec32 &r, int64_t E0, int64_t k) {
  const int64_t kn = hw_knext(r.hw, r.knext, E0);
  r.hw = hw_encode(hw_cell(r.hw), kn, k, k, hw_class(r.hw));
  r.knext = (int)kn;
}
__device__ __forceinline__ void rebase_rec(Rec64 &, int64_t, int64_t) {}
__device__ __forceinline__ int rec_key(CInst &I, const Rec32 &r, const double *) {
  return (hw_live(r.hw) && hw_cell(r.hw) < I.N) ? hw_cell(r.hw) : -1;
}
__device__ __forceinline__ int rec_key(CInst &I, const Rec64 &r, const double *nodes) {
  const double x = r.x;
  if (!(x >= 0.0 && x < I.L)) return -1;
  if (I.uniform) {
    const int j = (int)floor(x / I.dx);
    return j >= I.N ? I.N - 1 : j;
  }
  int lo = 0, hi = I.N;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (nodes[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

// The scatter.  A workgroup takes its contiguous range of tiles piece by
// piece (a piece: its tiles of one segment) in three phases:
//   1. an LDS histogram of the piece's cells (keys only);
//   2. one HBM atomic per nonzero cell reserves the piece's range of that
//      cell's destination slots;
//   3. every particle takes the next slot of its cell's range from an LDS
//      cursor and is copied there.
// Phase 3 has no barrier and no HBM atomic per tile, so its wavefronts stream
// independently.  Lanes with equal keys (particles arrive nearly sorted) take
// one cursor atomic per run and consecutive slots, so their stores coalesce.
// Order within a cell is not defined.
template <class P>
__global__ void __launch_bounds__(kSB)
k_sort_scatter(const InstDev *__restrict__ insts, InstState *__restrict__ states, int n_inst,
               int max_n) {
  __shared__ SortSmem sm;
  extern __shared__ __align__(16) unsigned char dsm[];
  // LDS: per-cell counts / cursors u32, per-cell destination bases u64 and,
  // FP64 only, the node positions to locate x.
  unsigned int *cnt = reinterpret_cast<unsigned int *>(dsm);
  unsigned long long *gbase = reinterpret_cast<unsigned long long *>(dsm + 4 * ((max_n + 2) & ~1));
  double *sNodes = reinterpret_cast<double *>(gbase + max_n);
  for (int j = threadIdx.x; j < max_n; j += kSB) cnt[j] = 0;
  seg_prefix_setup(insts, states, n_inst, sm.seg_prefix);
  const int nseg = 2 * n_inst;
  const int64_t T = sm.seg_prefix[nseg];
  const int64_t t0 = T * blockIdx.x / gridDim.x, t1 = T * (blockIdx.x + 1) / gridDim.x;
  int64_t tile = t0;
  while (tile < t1) {
    // the piece [tile, pe) of segment seg
    int seg = segment_of(sm.seg_prefix, nseg, tile);
    while (sm.seg_prefix[seg + 1] <= tile) ++seg;
    seg = uni(seg);
    const int64_t first = uni((int64_t)sm.seg_prefix[seg]);
    const int64_t pe = min(t1, uni((int64_t)sm.seg_prefix[seg + 1]));
    CInst &I = cinst(insts)[seg >> 1];
    const InstState &S = states[seg >> 1];
    const int64_t ext = uni((int64_t)S.extent[seg & 1]);
    const int par = uni(S.parity);
    const int64_t kS = uni((int64_t)S.k), E0 = uni((int64_t)S.epoch);
    const P src = make_view<P>(I, seg & 1, par);
    const P dst = make_view<P>(I, seg & 1, par ^ 1);
    const int N = I.N;
    if (sizeof(P) == sizeof(P64) && !I.uniform)
      for (int j = threadIdx.x; j <= N; j += kSB) sNodes[j] = I.nodes[j];
    __syncthreads();
    // 1. histogram of the piece's keys
    for (int64_t tt = tile; tt < pe; ++tt) {
      const int64_t i0 = (tt - first) * kSTile + (int64_t)threadIdx.x * kSPPT;
#pragma unroll
      for (int g = 0; g < kSPPT; g += 4) {
        int key[4];
        count_keys(I, src, i0 + g, ext, sNodes, key);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int len, pos;
          if (key_run(key[q], len, pos) && key[q] >= 0) atomicAdd(&cnt[key[q]], (unsigned int)len);
        }
      }
    }
    __syncthreads();
    // 2. reserve each cell's slots for the piece; the counts become cursors
    for (int j = threadIdx.x; j < N; j += kSB) {
      const unsigned int c = cnt[j];
      if (c) {
        gbase[j] = atomicAdd(&I.scursor[seg & 1][j], (unsigned long long)c);
        cnt[j] = 0;
      }
    }
    __syncthreads();
    // 3. copy every particle to the next slot of its cell
    for (int64_t tt = tile; tt < pe; ++tt) {
      const int64_t i0 = (tt - first) * kSTile + (int64_t)threadIdx.x * kSPPT;
      typename RecOf<P>::T r[kSPPT];
      bool ok[kSPPT];
#pragma unroll
      for (int g = 0; g < kSPPT; g += 4) load_recs(src, i0 + g, ext, r + g, ok + g);
#pragma unroll
      for (int q = 0; q < kSPPT; ++q) {
        const int key = ok[q] ? rec_key(I, r[q], sNodes) : -1;
        int len, pos;
        unsigned int b0 = 0;
        if (key_run(key, len, pos) && key >= 0) b0 = atomicAdd(&cnt[key], (unsigned int)len);
        b0 = __shfl(b0, __lane_id() - pos, 64);
        if (key >= 0) {
          rebase_rec(r[q], E0, kS);
          store_rec(dst, (int64_t)(gbase[key] + b0 + (unsigned int)pos), r[q]);
        }
      }
    }
    __syncthreads();
    // the cursors of the piece's cells back to zero for the next piece
    for (int j = threadIdx.x; j < N; j += kSB) cnt[j] = 0;
    __syncthreads();
    tile = pe;
  }
}

// Switch every sorted instance to the new buffer, whose hot words count from
// the current step.
__global__ void __launch_bounds__(256)
k_sort_finish(const InstDev *__restrict__ insts, InstState *__restrict__ states, int n_inst) {
  for (int i = threadIdx.x; i < n_inst; i += blockDim.x) {
    CInst &I = cinst(insts)[i];
    InstState &S = states[i];
    if (!I.active || S.frozen != 0) continue;
    for (int s = 0; s < I.nsp; ++s) {
      S.extent[s] = S.sort_live[s];
      S.n_live[s] = S.sort_live[s];
    }
    S.parity ^= 1;
    S.epoch = S.k;
  }
}

size_t sort_lds_bytes(int max_n, int prec) {
  return 4 * (size_t)((max_n + 2) & ~1) + 8 * (size_t)max_n + (prec == 0 ? 8 * (size_t)(max_n + 1) : 0);
}

hipError_t launch_sort(const InstDev *insts, InstState *states, int n_inst, int prec, int grid,
                       int count_grid, int max_n, hipStream_t s) {
  const size_t lds = sort_lds_bytes(max_n, prec);
  // The count needs only the histogram (and, FP64, the nodes to locate x).
  const size_t lds_count = 4 * (size_t)((max_n + 2) & ~1) + (prec == 0 ? 8 * (size_t)(max_n + 1) : 0);
  if (prec == 1)
    hipLaunchKernelGGL(k_sort_count<P32>, dim3(count_grid), dim3(kSB), lds_count, s, insts, states, n_inst, max_n);
  else
    hipLaunchKernelGGL(k_sort_count<P64>, dim3(count_grid), dim3(kSB), lds_count, s, insts, states, n_inst, max_n);
  hipLaunchKernelGGL(k_sort_scan, dim3(n_inst), dim3(kSB), 0, s, insts, states);
  if (prec == 1)
    hipLaunchKernelGGL(k_sort_scatter<P32>, dim3(grid), dim3(kSB), lds, s, insts, states, n_inst, max_n);
  else
    hipLaunchKernelGGL(k_sort_scatter<P64>, dim3(grid), dim3(kSB), lds, s, insts, states, n_inst, max_n);
  hipLaunchKernelGGL(k_sort_finish, dim3(1), dim3(256), 0, s, insts, states, n_inst);
  return hipGetLastError();
}

}  // namespace ecpic
