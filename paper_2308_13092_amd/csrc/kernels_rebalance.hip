// kernels_rebalance.hip -- particle rebalancing toward a target number of
// particles per cell (the paper's Section 3d names it as the way to turn the
// fewer cells of a refined grid into fewer particles; it gives no algorithm).
//
// A pass over one rebalanced discharge, on its cell-sorted FP32 state at step
// k, per species (the particle's weight is W 2^(w-4) for its class w):
//   flags   cells with more than 2P particles merge, cells with fewer than P/2
//           (and at least one) split;
//   collect the merge candidates (class < 7 in merging cells) are listed with
//           their ids;
//   order   the list is sorted by id, then stably by (species, cell, class,
//           velocity bin floor(vx / dv)): within each group, id order;
//   merge   every full quadruple of a group (ids a < b < c < d) becomes two
//           particles of class w + 1 at the quadruple's mean offset, with
//           velocities v_mean +- delta e (delta^2 = <|v|^2> - |v_mean|^2, e the
//           unit vector of v_d - v_a, else v_c - v_b, else x); a and b keep
//           their ids and candidacies, c and d are marked dead;
//   split   every particle of class w > 0 in a splitting cell becomes two of
//           class w - 1 at its position and velocity: itself and a child with
//           the id of Philox words 0-1 (key = parent id, counter = (k, tag 8 |
//           species << 8, seed)) and a first candidacy drawn as at step k.
// Weight is kept exactly, momentum and energy to rounding.  The next cell sort
// drops the merged-away particles.  The two sorts come from hipCUB (stable
// LSD radix sorts), with scratch memory carved from the discharge's slot.
#include <hipcub/hipcub.hpp>

#include "device.h"
#include "kernels.h"

namespace ecpic {

constexpr uint32_t TAG_SPLIT = 8;
constexpr int kClassMax = 7;

// Velocity bin of a merge group, and the key that orders the groups.
__device__ __forceinline__ int vbin_of(float vx, double dv) {
  const double b = floor((double)vx / dv);
  return (int)fmin(fmax(b, -128.0), 127.0);
}
__device__ __forceinline__ uint32_t group_key(int sp, int cell, int cls, int vb) {
  return ((uint32_t)(sp * 2048 + cell) * 8u + (uint32_t)cls) * 256u + (uint32_t)(vb + 128);
}

// Per cell and species: 1 merge, 2 split, 0 nothing, from the cell ranges the
// cell sort leaves in scursor (each cell's end; its start is the previous
// cell's end).
__global__ void __launch_bounds__(256)
k_rb_flags(const InstDev *__restrict__ insts, int inst) {
  CInst &I = cinst(insts)[inst];
  const int N = I.N;
  const int64_t P = I.rb_ppc;
  for (int s = 0; s < I.nsp; ++s)
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) {
      const int64_t end = (int64_t)I.scursor[s][c];
      const int64_t start = c > 0 ? (int64_t)I.scursor[s][c - 1] : 0;
      const int64_t n = end - start;
      I.rb_flag[s][c] = n > 2 * P ? 1 : ((n > 0 && 2 * n < P) ? 2 : 0);
    }
}

// The merge candidates: (id, species << 31 | index), in any order.  Each
// block takes chunks of kRbChunk particles and reserves the list positions of
// a whole chunk with one atomic (one per wavefront would serialise on the
// counter when most particles are candidates).
constexpr int kRbPer = 16;
constexpr int kRbChunk = 256 * kRbPer;

__global__ void __launch_bounds__(256)
k_rb_collect(const InstDev *__restrict__ insts, const InstState *__restrict__ states, int inst,
             unsigned long long *__restrict__ keys, uint32_t *__restrict__ vals,
             unsigned long long *__restrict__ count) {
  __shared__ unsigned long long wsum[4];
  __shared__ unsigned long long base;
  CInst &I = cinst(insts)[inst];
  const InstState &S = states[inst];
  const int lane = __lane_id();
  const int wave = threadIdx.x >> 6;
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int s = 0; s < I.nsp; ++s) {
    const P32 P = view32(I.pbuf[s][S.parity], I.cap[s]);
    const int64_t ext = S.extent[s];
    for (int64_t c0 = (int64_t)blockIdx.x * kRbChunk; c0 < ext; c0 += (int64_t)gridDim.x * kRbChunk) {
      // this wavefront's slice of the chunk: kRbPer rows of 64 particles
      const int64_t w0 = c0 + (int64_t)wave * 64 * kRbPer;
      unsigned long long m[kRbPer];
      unsigned long long n_w = 0;
#pragma unroll
      for (int r = 0; r < kRbPer; ++r) {
        const int64_t i = w0 + (int64_t)r * 64 + lane;
        bool want = false;
        if (i < ext) {
          const uint32_t w = P.hw[i];
          want = hw_live(w) && hw_class(w) < kClassMax && I.rb_flag[s][hw_cell(w)] == 1;
        }
        m[r] = __ballot(want);
        n_w += (unsigned long long)__popcll(m[r]);
      }
      if (lane == 0) wsum[wave] = n_w;
      __syncthreads();
      if (threadIdx.x == 0) {
        const unsigned long long t = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        base = t ? atomicAdd(count, t) : 0ull;
      }
      __syncthreads();
      unsigned long long at = base;
      for (int v = 0; v < wave; ++v) at += wsum[v];
#pragma unroll
      for (int r = 0; r < kRbPer; ++r) {
        if ((m[r] >> lane) & 1ull) {
          const int64_t i = w0 + (int64_t)r * 64 + lane;
          const unsigned long long q = at + (unsigned long long)__popcll(m[r] & below);
          keys[q] = P.cold[i].id;
          vals[q] = ((uint32_t)s << 31) | (uint32_t)i;
        }
        at += (unsigned long long)__popcll(m[r]);
      }
      __syncthreads();   // wsum and base are rewritten by the next chunk
    }
  }
}

// The group key of each listed particle (in the list's current order).
__global__ void __launch_bounds__(256)
k_rb_keys(const InstDev *__restrict__ insts, const InstState *__restrict__ states, int inst,
          const uint32_t *__restrict__ vals, uint32_t *__restrict__ k32, int64_t n) {
  CInst &I = cinst(insts)[inst];
  const InstState &S = states[inst];
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(vals[j] >> 31);
    const int64_t i = vals[j] & 0x7FFFFFFFu;
    const P32 P = view32(I.pbuf[s][S.parity], I.cap[s]);
    const uint32_t w = P.hw[i];
    k32[j] = group_key(s, hw_cell(w), hw_class(w), vbin_of(P.vx[i], I.rb_dv[s]));
  }
}

// First index of the run of keys equal to keys[j] (keys sorted): a backward
// search in doubling steps, then bisection -- its loads stay near j.
__device__ __forceinline__ int64_t run_start(const uint32_t *keys, int64_t j) {
  const uint32_t key = keys[j];
  int64_t a = j;        // keys[a] == key
  int64_t b = -1;       // keys[b] != key, or b = -1
  for (int64_t step = 1;; step <<= 1) {
    const int64_t p = j - step;
    if (p < 0) break;
    if (keys[p] != key) {
      b = p;
      break;
    }
    a = p;
  }
  while (a - b > 1) {
    const int64_t mid = b + ((a - b) >> 1);
    if (keys[mid] == key) a = mid;
    else b = mid;
  }
  return a;
}

// One thread per list position: the first of every full quadruple of its
// group merges it.
__global__ void __launch_bounds__(256)
k_rb_merge(const InstDev *__restrict__ insts, InstState *__restrict__ states, int inst,
           const uint32_t *__restrict__ vals, const uint32_t *__restrict__ k32, int64_t n) {
  CInst &I = cinst(insts)[inst];
  InstState &S = states[inst];
  unsigned long long merges[2] = {0, 0};
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t key = k32[j];
    // a full quadruple starts here: j + 3 is in the same group, and j is at
    // a multiple of 4 from the group's start
    if (j + 3 >= n || k32[j + 3] != key) continue;
    if (((j - run_start(k32, j)) & 3) != 0) continue;
    const int s = (int)(vals[j] >> 31);
    const P32 P = view32(I.pbuf[s][S.parity], I.cap[s]);
    int64_t q[4];
    double vx[4], vy[4], vz[4], off[4];
    for (int t = 0; t < 4; ++t) {
      q[t] = vals[j + t] & 0x7FFFFFFFu;
      const Cold32 c = gload_cold(P.cold + q[t]);
      vx[t] = (double)P.vx[q[t]];
      vy[t] = (double)c.vy;
      vz[t] = (double)c.vz;
      off[t] = (double)P.off[q[t]];
    }
    // mean velocity and spread, in the order of the ids
    const double sx = ((vx[0] + vx[1]) + vx[2]) + vx[3];
    const double sy = ((vy[0] + vy[1]) + vy[2]) + vy[3];
    const double sz = ((vz[0] + vz[1]) + vz[2]) + vz[3];
    const double bx = sx * 0.25, by = sy * 0.25, bz = sz * 0.25;
    double e[4];
    for (int t = 0; t < 4; ++t) e[t] = (vx[t] * vx[t] + vy[t] * vy[t]) + vz[t] * vz[t];
    const double E2 = ((e[0] + e[1]) + e[2]) + e[3];
    const double d2 = E2 * 0.25 - ((bx * bx + by * by) + bz * bz);
    const double delta = sqrt(fmax(d2, 0.0));
    double dx = vx[3] - vx[0], dy = vy[3] - vy[0], dz = vz[3] - vz[0];
    double n2 = (dx * dx + dy * dy) + dz * dz;
    if (n2 == 0.0) {
      dx = vx[2] - vx[1];
      dy = vy[2] - vy[1];
      dz = vz[2] - vz[1];
      n2 = (dx * dx + dy * dy) + dz * dz;
    }
    if (n2 == 0.0) {
      dx = 1.0;
      dy = 0.0;
      dz = 0.0;
      n2 = 1.0;
    }
    const double nn = sqrt(n2);
    const double ux = dx / nn, uy = dy / nn, uz = dz / nn;
    float ob = (float)((((off[0] + off[1]) + off[2]) + off[3]) * 0.25);
    ob = fminf(ob, 0x1.fffffep-1f);
    const double va[3] = {bx + delta * ux, by + delta * uy, bz + delta * uz};
    const double vb[3] = {bx - delta * ux, by - delta * uy, bz - delta * uz};
    for (int t = 0; t < 2; ++t) {
      const double *v = t == 0 ? va : vb;
      const int64_t i = q[t];
      const uint32_t w = P.hw[i];
      P.hw[i] = (w & ~kHwClass) | ((uint32_t)(hw_class(w) + 1) << kHwClassShift);
      P.off[i] = ob;
      P.vx[i] = (float)v[0];
      const Cold32 c = gload_cold(P.cold + i);
      gstore_cold(P.cold + i, Cold32{(float)v[1], (float)v[2], c.id});
    }
    P.hw[q[2]] = kHwDead;
    P.hw[q[3]] = kHwDead;
    merges[s] += 1;
  }
  for (int s = 0; s < 2; ++s) {
    unsigned long long m = merges[s];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m += __shfl_xor(m, o, 64);
    if (__lane_id() == 0 && m) atomicAdd(&S.ctr[C_MERGE][s], m);
  }
}

// Splits, and the children appended after each species' extent (the count of
// appended children in added[s]).
__global__ void __launch_bounds__(256)
k_rb_split(const InstDev *__restrict__ insts, InstState *__restrict__ states, int inst,
           unsigned long long *__restrict__ added) {
  CInst &I = cinst(insts)[inst];
  InstState &S = states[inst];
  const int64_t k = S.k;
  for (int s = 0; s < I.nsp; ++s) {
    const P32 P = view32(I.pbuf[s][S.parity], I.cap[s]);
    const int64_t ext = S.extent[s];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ext;
         i += (int64_t)gridDim.x * blockDim.x) {
      const uint32_t w = P.hw[i];
      const bool want = hw_live(w) && hw_class(w) > 0 && I.rb_flag[s][hw_cell(w)] == 2;
      const unsigned long long m = __ballot(want);
      if (m == 0) continue;
      const int lane = __lane_id();
      const int leader = __ffsll((long long)m) - 1;
      unsigned long long b = 0;
      if (lane == leader) b = atomicAdd(&added[s], (unsigned long long)__popcll(m));
      b = __shfl(b, leader, 64);
      if (!want) continue;
      const int64_t at = ext + (int64_t)(b + (unsigned long long)__popcll(m & ((1ull << lane) - 1ull)));
      const int cls = hw_class(w) - 1;
      P.hw[i] = (w & ~kHwClass) | ((uint32_t)cls << kHwClassShift);
      if (at >= I.cap[s]) {
        atomicOr(&S.status, (int)ST_CAPACITY);
        continue;
      }
      const Cold32 c = gload_cold(P.cold + i);
      const uint4 r = philox((uint32_t)k, TAG_SPLIT | (uint32_t)(s << 8), I.seed, c.id);
      const uint64_t cid = (uint64_t)r.x | ((uint64_t)r.y << 32);
      const int32_t kn = next_candidate(cid, k - 1, s, I.seed, I.nudt[s]);
      const uint32_t cw = hw_encode(hw_cell(w), kn, k, S.epoch, cls);
      P.hw[at] = cw;
      P.off[at] = P.off[i];
      P.vx[at] = P.vx[i];
      if (hw_far(cw)) P.knext[at] = kn;
      gstore_cold(P.cold + at, Cold32{c.vy, c.vz, cid});
    }
  }
}

// The children join the extents (the next cell sort recounts the live ones).
__global__ void k_rb_finish(const InstDev *__restrict__ insts, InstState *__restrict__ states, int inst,
                            const unsigned long long *__restrict__ added) {
  CInst &I = cinst(insts)[inst];
  InstState &S = states[inst];
  if (threadIdx.x != 0) return;
  for (int s = 0; s < I.nsp; ++s) {
    int64_t a = (int64_t)added[s];
    if (S.extent[s] + a > I.cap[s]) a = I.cap[s] - S.extent[s];
    S.extent[s] += a;
    S.ctr[C_SPLIT][s] += (unsigned long long)added[s];
  }
}

__global__ void k_rb_zero(unsigned long long *p, int n) {
  if (threadIdx.x < n) p[threadIdx.x] = 0ull;
}

size_t rb_sort_temp_bytes(int64_t items) {
  // the larger of the two sorts' scratch, as the library queries it
  size_t t1 = 0, t2 = 0;
  hipcub::DoubleBuffer<unsigned long long> k64(nullptr, nullptr);
  hipcub::DoubleBuffer<uint32_t> k32(nullptr, nullptr), v(nullptr, nullptr);
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, t1, k64, v, (int)items, 0, 64) != hipSuccess) return 0;
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, t2, k32, v, (int)items, 0, 23) != hipSuccess) return 0;
  return t1 > t2 ? t1 : t2;
}

hipError_t launch_rebalance(const InstDev *insts, InstState *states, int inst, int N, const RbScratch &sc,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_rb_zero, dim3(1), dim3(64), 0, st, sc.words, 4);
  hipLaunchKernelGGL(k_rb_flags, dim3((N + 255) / 256), dim3(256), 0, st, insts, inst);
  hipLaunchKernelGGL(k_rb_collect, dim3(2048), dim3(256), 0, st, insts, states, inst, sc.k64[0], sc.val[0],
                     sc.words);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  unsigned long long n = 0;
  e = hipMemcpyAsync(&n, sc.words, sizeof n, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  if (n > 0) {
    if ((int64_t)n > sc.items) return hipErrorInvalidValue;
    hipcub::DoubleBuffer<unsigned long long> k64(sc.k64[0], sc.k64[1]);
    hipcub::DoubleBuffer<uint32_t> val(sc.val[0], sc.val[1]);
    size_t tb = sc.temp_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(sc.temp, tb, k64, val, (int)n, 0, 64, st);
    if (e != hipSuccess) return e;
    hipcub::DoubleBuffer<uint32_t> k32(sc.k32[0], sc.k32[1]);
    // the values in the id order, keyed by group
    uint32_t *vcur = val.Current();
    hipLaunchKernelGGL(k_rb_keys, dim3(2048), dim3(256), 0, st, insts, states, inst, vcur, k32.Current(),
                       (int64_t)n);
    hipcub::DoubleBuffer<uint32_t> val2(vcur, vcur == sc.val[0] ? sc.val[1] : sc.val[0]);
    tb = sc.temp_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(sc.temp, tb, k32, val2, (int)n, 0, 23, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rb_merge, dim3(2048), dim3(256), 0, st, insts, states, inst, val2.Current(),
                       k32.Current(), (int64_t)n);
  }
  hipLaunchKernelGGL(k_rb_split, dim3(2048), dim3(256), 0, st, insts, states, inst, sc.words + 2);
  hipLaunchKernelGGL(k_rb_finish, dim3(1), dim3(64), 0, st, insts, states, inst, sc.words + 2);
  return hipGetLastError();
}

}  // namespace ecpic
