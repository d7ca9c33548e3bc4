// kernels_sort.hip -- counting sort of the particles by cell, with compaction.
//
// Every sort_interval steps the particles of each (instance, species) segment
// are reordered by cell into the other particle buffer and absorbed particles
// are dropped.  Sorted particles keep the deposit of a wavefront on one or two
// nodes (cheap to merge before the LDS atomics) and keep each workgroup's
// share of the grid small.  Three passes:
//   count   per-workgroup LDS histogram of the live cells, added to HBM;
//   scan    one workgroup per instance: exclusive prefix of the counts gives
//           each cell's first destination slot;
//   scatter ranks within a wavefront from ballots, one reservation per
//           (tile, cell) with an HBM atomic, then every field is copied to its
//           destination.  The last workgroup flips the buffers.
// Order within a cell is not defined; results depend on the particle set only.
#include "device.h"
#include "kernels.h"

namespace ecpic {

constexpr int kSB = 256;      // threads per workgroup
constexpr int kSPPT = 4;      // particles per thread per tile
constexpr int kSTile = kSB * kSPPT;

struct SortSmem {
  int seg_prefix[2 * kMaxInst + 1];
  int is_last;
};

__device__ __forceinline__ int key_of(const InstDev &I, const P32 &P, int64_t i, const double *,
                                      const double *) {
  const int c = P.cell[i];
  return (c >= 0 && c < I.N) ? c : -1;
}
__device__ __forceinline__ int key_of(const InstDev &I, const P64 &P, int64_t i, const double *nodes,
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

// Segment tile prefix over the instances that are not frozen.
__device__ void seg_prefix_setup(const InstDev *insts, const InstState *states, int n_inst,
                                 int *prefix) {
  const int nseg = 2 * n_inst;
  for (int s = threadIdx.x; s < nseg; s += blockDim.x) {
    const InstDev &I = insts[s >> 1];
    const InstState &S = states[s >> 1];
    const bool ok = I.active && S.frozen == 0 && (s & 1) < I.nsp;
    const int64_t ext = ok ? S.extent[s & 1] : 0;
    prefix[s + 1] = (int)((ext + kSTile - 1) / kSTile);
  }
  if (threadIdx.x == 0) prefix[0] = 0;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int s = 1; s <= nseg; ++s) prefix[s] += prefix[s - 1];
  __syncthreads();
}

template <class P>
__device__ __forceinline__ P make_view(const InstDev &I, int s, int buf);
template <>
__device__ __forceinline__ P32 make_view<P32>(const InstDev &I, int s, int buf) {
  return view32(I.pbuf[s][buf], I.cap[s]);
}
template <>
__device__ __forceinline__ P64 make_view<P64>(const InstDev &I, int s, int buf) {
  return view64(I.pbuf[s][buf], I.cap[s]);
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
  seg_prefix_setup(insts, states, n_inst, sm.seg_prefix);
  const int nseg = 2 * n_inst;
  const int64_t T = sm.seg_prefix[nseg];
  const int64_t t0 = T * blockIdx.x / gridDim.x, t1 = T * (blockIdx.x + 1) / gridDim.x;
  int seg = -1;
  const InstDev *Ip = nullptr;
  P view;
  int64_t ext = 0;
  auto flush = [&]() {
    __syncthreads();
    const InstDev &I = *Ip;
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
    int s = seg < 0 ? 0 : seg;
    while (sm.seg_prefix[s + 1] <= tile) ++s;
    s = __builtin_amdgcn_readfirstlane(s);
    if (s != seg) {
      if (seg >= 0) flush();
      seg = s;
      Ip = &insts[seg >> 1];
      const InstState &S = states[seg >> 1];
      ext = S.extent[seg & 1];
      view = make_view<P>(*Ip, seg & 1, S.parity);
      if (!Ip->uniform)
        for (int j = threadIdx.x; j <= Ip->N; j += kSB) sNodes[j] = Ip->nodes[j];
      __syncthreads();
    }
    const int64_t i0 = (tile - sm.seg_prefix[seg]) * kSTile + (int64_t)threadIdx.x * kSPPT;
    for (int q = 0; q < kSPPT; ++q) {
      const int64_t i = i0 + q;
      if (i >= ext) break;
      const int key = key_of(*Ip, view, i, sNodes, nullptr);
      if (key >= 0) atomicAdd(&hist[key], 1u);
    }
  }
  if (seg >= 0) flush();
}

// One workgroup per instance: first destination slot of every cell.
__global__ void __launch_bounds__(kSB)
k_sort_scan(const InstDev *__restrict__ insts, InstState *__restrict__ states) {
  __shared__ unsigned long long tmp[kSB];
  const InstDev &I = insts[blockIdx.x];
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

template <class P>
__device__ __forceinline__ void copy_particle(const P &src, int64_t i, const P &dst, int64_t d);
template <>
__device__ __forceinline__ void copy_particle<P32>(const P32 &src, int64_t i, const P32 &dst, int64_t d) {
  dst.cell[d] = src.cell[i];
  dst.off[d] = src.off[i];
  dst.vx[d] = src.vx[i];
  dst.vy[d] = src.vy[i];
  dst.vz[d] = src.vz[i];
  dst.knext[d] = src.knext[i];
  dst.id[d] = src.id[i];
}
template <>
__device__ __forceinline__ void copy_particle<P64>(const P64 &src, int64_t i, const P64 &dst, int64_t d) {
  dst.x[d] = src.x[i];
  dst.vx[d] = src.vx[i];
  dst.vy[d] = src.vy[i];
  dst.vz[d] = src.vz[i];
  dst.knext[d] = src.knext[i];
  dst.id[d] = src.id[i];
}

template <class P>
__global__ void __launch_bounds__(kSB)
k_sort_scatter(const InstDev *__restrict__ insts, InstState *__restrict__ states, int n_inst,
               int max_n, unsigned int *__restrict__ done) {
  __shared__ SortSmem sm;
  extern __shared__ __align__(16) unsigned char dsm[];
  unsigned int *cnt = reinterpret_cast<unsigned int *>(dsm);
  double *sNodes = reinterpret_cast<double *>(dsm + 4 * ((max_n + 2) & ~1));
  unsigned long long *gbase =
      reinterpret_cast<unsigned long long *>(sNodes + (max_n + 1));
  for (int j = threadIdx.x; j < max_n; j += kSB) cnt[j] = 0;
  seg_prefix_setup(insts, states, n_inst, sm.seg_prefix);
  const int nseg = 2 * n_inst;
  const int64_t T = sm.seg_prefix[nseg];
  const int64_t t0 = T * blockIdx.x / gridDim.x, t1 = T * (blockIdx.x + 1) / gridDim.x;
  const int lane = __lane_id();
  const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int seg = -1;
  const InstDev *Ip = nullptr;
  P src, dst;
  int64_t ext = 0;
  for (int64_t tile = t0; tile < t1; ++tile) {
    int s = seg < 0 ? 0 : seg;
    while (sm.seg_prefix[s + 1] <= tile) ++s;
    s = __builtin_amdgcn_readfirstlane(s);
    if (s != seg) {
      __syncthreads();
      seg = s;
      Ip = &insts[seg >> 1];
      const InstState &S = states[seg >> 1];
      ext = S.extent[seg & 1];
      src = make_view<P>(*Ip, seg & 1, S.parity);
      dst = make_view<P>(*Ip, seg & 1, S.parity ^ 1);
      if (!Ip->uniform)
        for (int j = threadIdx.x; j <= Ip->N; j += kSB) sNodes[j] = Ip->nodes[j];
      __syncthreads();
    }
    const InstDev &I = *Ip;
    const int64_t i0 = (tile - sm.seg_prefix[seg]) * kSTile + (int64_t)threadIdx.x * kSPPT;
    int key[kSPPT];
    unsigned int rank[kSPPT];
#pragma unroll
    for (int q = 0; q < kSPPT; ++q) {
      const int64_t i = i0 + q;
      key[q] = (i < ext) ? key_of(I, src, i, sNodes, nullptr) : -1;
      rank[q] = 0;
      // Ranks of equal keys within the wavefront, one LDS atomic per run.
      bool pending = key[q] >= 0;
      unsigned long long pm = __ballot(pending);
      while (pm) {
        const int leader = __ffsll((long long)pm) - 1;
        const int lkey = __shfl(key[q], leader, 64);
        const bool match = pending && key[q] == lkey;
        const unsigned long long mm = __ballot(match);
        unsigned int b = 0;
        if (lane == leader) b = atomicAdd(&cnt[lkey], (unsigned int)__popcll(mm));
        b = __shfl(b, leader, 64);
        if (match) {
          rank[q] = b + (unsigned int)__popcll(mm & lt_mask);
          pending = false;
        }
        pm &= ~mm;
      }
    }
    __syncthreads();
    // The first particle of each cell in the tile reserves the tile's range.
#pragma unroll
    for (int q = 0; q < kSPPT; ++q)
      if (key[q] >= 0 && rank[q] == 0)
        gbase[key[q]] = atomicAdd(&I.scursor[seg & 1][key[q]], (unsigned long long)cnt[key[q]]);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSPPT; ++q)
      if (key[q] >= 0) copy_particle<P>(src, i0 + q, dst, (int64_t)(gbase[key[q]] + rank[q]));
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSPPT; ++q)
      if (key[q] >= 0 && rank[q] == 0) cnt[key[q]] = 0;
  }
  // The last workgroup switches every sorted instance to the new buffer.
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) sm.is_last = (atomicAdd(done, 1u) == gridDim.x - 1);
  __syncthreads();
  if (sm.is_last) {
    __threadfence();
    for (int i = threadIdx.x; i < n_inst; i += kSB) {
      const InstDev &I = insts[i];
      InstState &S = states[i];
      if (!I.active || S.frozen != 0) continue;
      for (int s = 0; s < I.nsp; ++s) {
        S.extent[s] = S.sort_live[s];
        S.n_live[s] = S.sort_live[s];
      }
      S.parity ^= 1;
    }
    if (threadIdx.x == 0) *done = 0u;
  }
}

size_t sort_lds_bytes(int max_n) {
  return 4 * (size_t)((max_n + 2) & ~1) + 8 * (size_t)(max_n + 1) + 8 * (size_t)max_n;
}

hipError_t launch_sort(const InstDev *insts, InstState *states, int n_inst, int prec, int grid,
                       int max_n, unsigned int *done, hipStream_t s) {
  const size_t lds = sort_lds_bytes(max_n);
  if (prec == 1)
    hipLaunchKernelGGL(k_sort_count<P32>, dim3(grid), dim3(kSB), lds, s, insts, states, n_inst, max_n);
  else
    hipLaunchKernelGGL(k_sort_count<P64>, dim3(grid), dim3(kSB), lds, s, insts, states, n_inst, max_n);
  hipLaunchKernelGGL(k_sort_scan, dim3(n_inst), dim3(kSB), 0, s, insts, states);
  if (prec == 1)
    hipLaunchKernelGGL(k_sort_scatter<P32>, dim3(grid), dim3(kSB), lds, s, insts, states, n_inst, max_n, done);
  else
    hipLaunchKernelGGL(k_sort_scatter<P64>, dim3(grid), dim3(kSB), lds, s, insts, states, n_inst, max_n, done);
  return hipGetLastError();
}

}  // namespace ecpic
