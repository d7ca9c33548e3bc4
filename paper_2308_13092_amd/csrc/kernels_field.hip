// kernels_field.hip -- Poisson solve and field of every instance (Eqs 4-5).
//
// One workgroup per instance.  The paper solves the 3-point Poisson system by
// LU decomposition (Section 2), a sequential sweep of ~2N dependent steps.
// Here the same finite-volume system
//   (phi_{n+1}-phi_n)/h_n - (phi_n-phi_{n-1})/h_{n-1} = -Q_n/eps0,  n = 1..N-1
// is solved in its equivalent Gauss-law form, which is parallel:
//   E_j - E_{j-1} = Q_j/eps0   =>   E_j = E_0 + G_j,  G_j = (1/eps0) sum_{n=1..j} Q_n,
//   sum_j h_j E_j = phi_0 - phi_N fixes E_0,  phi_j = phi_0 - sum_{i<j} h_i E_i.
// When both species carry the same |q| W (or only electrons move), the charge
// prefix is an exact int64 prefix of the fixed-point deposit, so G_j takes a
// single rounding.  All prefix sums and reductions use a fixed blocking, so
// the result is bit-reproducible.
#include "device.h"
#include "kernels.h"

namespace ecpic {

// Threads per field workgroup: 256 for an instance of at most 512 cells
// (there the wider workgroup only adds barrier latency), 1024 above.  The
// choice follows each instance's own grid, never the batch it is in, since
// the FP64 prefix sums' blocking (and so their rounding) follows it.
constexpr int kFieldSmallCells = 512;

template <typename T>
__device__ __forceinline__ T wave_scan_inclusive(T v) {
  const int lane = __lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// In-place inclusive prefix sum of a[0..n) by the workgroup of FB threads:
// each thread sums a contiguous chunk, the chunk totals are scanned within
// each wavefront with shuffles, then across the wavefronts; the blocking is
// fixed, so the result is reproducible.  tmp holds FB / 64 values.  The
// 256-thread workgroup (grids of at most 512 cells) scans in its first
// wavefront alone, in 64 chunks: one barrier instead of three (small
// discharge 28.2 -> 27.7 us/step).  Callers synchronise before the call.
template <int FB, typename T>
__device__ void block_scan_inclusive(T *a, int n, T *tmp) {
  if constexpr (FB == 256) {
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x;
      const int c = (n + 63) / 64;
      const int lo = min(n, lane * c), hi = min(n, lo + c);
      T s = T(0);
      for (int i = lo; i < hi; ++i) {
        s += a[i];
        a[i] = s;
      }
      const T base = wave_scan_inclusive(s) - s;
      for (int i = lo; i < hi; ++i) a[i] += base;
    }
    __syncthreads();
    return;
  }
  constexpr int kFW = FB / 64;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int c = (n + FB - 1) / FB;
  const int lo = min(n, t * c), hi = min(n, lo + c);
  T s = T(0);
  for (int i = lo; i < hi; ++i) { s += a[i]; a[i] = s; }
  const T incl = wave_scan_inclusive(s);
  if (lane == 63) tmp[w] = incl;
  __syncthreads();
  if (w == 0) {
    T x = (lane < kFW) ? tmp[lane] : T(0);
    x = wave_scan_inclusive(x);
    if (lane < kFW) tmp[lane] = x;
  }
  __syncthreads();
  const T base = (incl - s) + ((w > 0) ? tmp[w - 1] : T(0));
  for (int i = lo; i < hi; ++i) a[i] += base;
  __syncthreads();
}

template <int FB, typename T>
__device__ T block_sum(T v, T *tmp) {
  constexpr int kFW = FB / 64;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  v = wave_sum(v);
  if (lane == 0) tmp[w] = v;
  __syncthreads();
  T r = T(0);
#pragma unroll
  for (int i = 0; i < kFW; ++i) r += tmp[i];
  __syncthreads();
  return r;
}

// block_sum of s and block_max of m together: the same per-value arithmetic
// with one exchange through LDS instead of two.
template <int FB>
__device__ void block_sum_max(double &s, double &m, double *tmps, double *tmpm) {
  constexpr int kFW = FB / 64;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  s = wave_sum(s);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if (lane == 0) {
    tmps[w] = s;
    tmpm[w] = m;
  }
  __syncthreads();
  double rs = 0.0, rm = 0.0;
#pragma unroll
  for (int i = 0; i < kFW; ++i) {
    rs += tmps[i];
    rm = fmax(rm, tmpm[i]);
  }
  __syncthreads();
  s = rs;
  m = rm;
}

template <int FB>
__device__ double block_max(double v, double *tmp) {
  constexpr int kFW = FB / 64;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if (lane == 0) tmp[w] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < kFW; ++i) r = fmax(r, tmp[i]);
  __syncthreads();
  return r;
}

// mode bit 0: accumulate the averaged profiles when due; bit 1: zero the
// deposit buffer of step k+1 (for the fused particle pass); bit 2: first close
// the previous fused step (what k_finalize does, when the host did not launch
// it on its own).
template <int kFB>
__global__ void __launch_bounds__(kFB)
k_field(const InstDev *__restrict__ insts, InstState *__restrict__ states, int mode) {
  constexpr int kFW = kFB / 64;
  __shared__ int64_t sA[2][kMaxCells + 1];
  __shared__ double sG[kMaxCells + 1];
  __shared__ double sE[kMaxCells + 1];
  __shared__ double sQ[kMaxCells + 1];
  __shared__ int64_t sD[kMaxCells + 1];
  __shared__ double sH[kMaxCells + 1];
  __shared__ int64_t tmpi[kFW];
  __shared__ double tmpd[kFW];
  __shared__ double tmpm[kFW];

  __shared__ int64_t s_k;
  __shared__ int s_open;

  CInst &I = cinst(insts)[blockIdx.x];
  InstState &S = states[blockIdx.x];
  if ((I.N <= kFieldSmallCells) != (kFB == 256)) return;   // the other launch's instance
  const int t = threadIdx.x;
  // The thread's nodes n = t + u kFB: both parities' deposits (the parity of
  // step k is known only after the close below), h and V, loaded first so
  // that their latency overlaps the close.  The deposits are final: the
  // close does not touch them.  An empty slot (not active) has no arrays:
  // nothing is loaded for it (it returns below).
  constexpr int kNPT = ((kFB == 256 ? kFieldSmallCells : kMaxCells) + kFB) / kFB;
  const int Nn = I.active ? I.N : -1;
  const int nsp0 = I.nsp;
  int64_t pa[2][2][kNPT];
  double ph[kNPT], pv[kNPT];
#pragma unroll
  for (int u = 0; u < kNPT; ++u) {
    const int n = t + u * kFB;
    pa[0][0][u] = pa[0][1][u] = pa[1][0][u] = pa[1][1][u] = 0;
    ph[u] = 0.0;
    pv[u] = 1.0;
    if (n <= Nn) {
      pa[0][0][u] = I.A[0][0][n];
      pa[1][0][u] = I.A[1][0][n];
      if (nsp0 > 1) {
        pa[0][1][u] = I.A[0][1][n];
        pa[1][1][u] = I.A[1][1][n];
      }
      if (n < Nn) ph[u] = I.h[n];
      pv[u] = I.V[n];
    }
  }
  int64_t k;
  if (mode & 4) {
    // The first wavefront closes the previous step; k and whether the
    // instance is still open reach the workgroup through LDS.
    if (t < 64) {
      if (pass_open(I, S)) close_pass<true, true>(I, S, t);
      if (t == 0) {
        s_k = S.k;
        s_open = pass_open(I, S) ? 1 : 0;
      }
    }
    __syncthreads();
    if (!s_open) return;
    k = s_k;
  } else {
    if (!pass_open(I, S)) return;
    k = S.k;
  }
  const int N = I.N;
  const int par = (int)(k & 1);
  const bool periodic = I.bc == 1;
  const int nsp = I.nsp;

  // The deposits, and from them (each thread for its own nodes, so without
  // a barrier in between) Q_n = sum_s (q_s W A_{s,n}) 2^-32 and the integer
  // Gauss-law differences.
  const bool int_path = !periodic && I.int_path;
#pragma unroll
  for (int u = 0; u < kNPT; ++u) {
    const int n = t + u * kFB;
    if (n > N) break;
    const int64_t a0 = par ? pa[1][0][u] : pa[0][0][u];
    const int64_t a1 = (nsp > 1) ? (par ? pa[1][1][u] : pa[0][1][u]) : 0;
    sA[0][n] = a0;
    sA[1][n] = a1;
    if (n < N) sH[n] = ph[u];
    double q = (I.qW[0] * (double)a0) * 0x1p-32;
    if (nsp > 1) q = q + (I.qW[1] * (double)a1) * 0x1p-32;
    sQ[n] = q;
    if (int_path && n < N) sD[n] = (n == 0) ? 0 : ((nsp > 1) ? (a1 - a0) : a0);
  }
  __syncthreads();
  const double t_k = (double)k * I.dt;
  const double phi0 = periodic ? 0.0 : I.v_rf * sin(I.w_rf * t_k + I.phase);
  const double phiN = 0.0;

  // G_j, j = 0..N-1 (G_0 = 0).
  if (int_path) {
    block_scan_inclusive<kFB, int64_t>(sD, N, tmpi);
    for (int n = t; n < N; n += kFB) sG[n] = I.cgauss * (double)sD[n];
  } else {
    double qbg = 0.0;
    if (periodic) {
      double part = 0.0;
      for (int n = t; n < N; n += kFB) part += sQ[n];
      qbg = block_sum<kFB, double>(part, tmpd) / I.L;
    }
    for (int n = t; n < N; n += kFB) {
      const double qn = periodic ? (sQ[n] - qbg * I.V[n]) : sQ[n];
      sG[n] = (n == 0) ? 0.0 : qn / kEPS0;
    }
    __syncthreads();
    block_scan_inclusive<kFB, double>(sG, N, tmpd);
  }

  // E_0 from sum_j h_j E_j = phi_0 - phi_N.  Each thread reads only the G_j
  // it wrote (the scan's chunks end with a barrier).
  double part = 0.0;
  for (int j = t; j < N; j += kFB) part += sH[j] * sG[j];
  const double hg = block_sum<kFB, double>(part, tmpd);
  const double e0 = (phi0 - phiN - hg) / I.L;
  // phi_j = phi_0 - sum_{i<j} h_i E_i  (sG, read before it is overwritten by
  // the same thread, becomes h_j E_j and then its prefix).
  for (int j = t; j < N; j += kFB) {
    const double e = e0 + sG[j];
    sE[j] = e;
    sG[j] = sH[j] * e;
  }
  __syncthreads();
  block_scan_inclusive<kFB, double>(sG, N, tmpd);
  for (int n = t; n <= N; n += kFB) {
    double p;
    if (n == 0) p = phi0;
    else if (n == N) p = phiN;
    else p = phi0 - sG[n - 1];
    I.phi[n] = p;
  }

  // Field handed to the particles.
  if (I.gather == 0) {
    for (int j = t; j < N; j += kFB) {
      I.E64[j] = sE[j];
      I.E32[j] = (float)sE[j];
    }
  } else if (I.gather == 2) {
    // Second-order EC: the cell fields at the N cell centres with a ghost
    // centre beyond each end, entry m = cell m - 1.  The S2 deposit puts the
    // weight beyond a Dirichlet end on the electrode node, which is the
    // energy of a ghost node at the electrode's potential: zero ghost field.
    // A periodic box wraps.
    for (int m = t; m <= N + 1; m += kFB) {
      double g;
      if (m >= 1 && m <= N) g = sE[m - 1];
      else if (periodic) g = (m == 0) ? sE[N - 1] : sE[0];
      else g = 0.0;
      I.E64[m] = g;
      I.E32[m] = (float)g;
    }
  } else {
    for (int n = t; n <= N; n += kFB) {
      double en;
      if (n > 0 && n < N) {
        en = (sH[n - 1] * sE[n - 1] + sH[n] * sE[n]) / (sH[n - 1] + sH[n]);
      } else if (periodic) {
        en = (sH[N - 1] * sE[N - 1] + sH[0] * sE[0]) / (sH[N - 1] + sH[0]);
      } else if (n == 0) {
        en = sE[0] - sQ[0] / kEPS0;
      } else {
        en = sE[N - 1] + sQ[N] / kEPS0;
      }
      I.E64[n] = en;
      I.E32[n] = (float)en;
    }
  }

  // Field energy and the density maximum (stability monitor 1b).
  double fe = 0.0;
  for (int j = t; j < N; j += kFB) fe += sH[j] * sE[j] * sE[j];
  double nm = 0.0;
#pragma unroll
  for (int u = 0; u < kNPT; ++u) {
    const int n = t + u * kFB;
    if (n <= N) nm = fmax(nm, ((double)sA[0][n] * I.W * 0x1p-32) / pv[u]);
  }
  block_sum_max<kFB>(fe, nm, tmpd, tmpm);
  if (t == 0) {
    S.field_energy = 0.5 * kEPS0 * fe;
    S.ne_max = nm;
  }

  // RF-averaged profiles (Section 3a).
  if ((mode & 1) && I.avg_every > 0 && k >= I.avg_start && ((k - I.avg_start) % I.avg_every) == 0) {
    for (int n = t; n <= N; n += kFB) {
      I.accA[0][n] += (double)sA[0][n];
      if (nsp > 1) I.accA[1][n] += (double)sA[1][n];
      I.acc_phi[n] += (n == 0) ? phi0 : ((n == N) ? phiN : phi0 - sG[n - 1]);
    }
    if (t == 0) S.n_samples += 1;
  }
  if ((mode & 1) && t == 0 && I.eedf_every > 0 && k >= I.avg_start &&
      ((k - I.avg_start) % I.eedf_every) == 0)
    S.eedf_samples += 1;
  // Clear the deposit of step k+1 for the fused particle pass.
  if (mode & 2) {
    for (int n = t; n <= N; n += kFB) {
      I.A[par ^ 1][0][n] = 0;
      if (nsp > 1) I.A[par ^ 1][1][n] = 0;
    }
  }
}

int field_class(int n_cells) { return n_cells <= kFieldSmallCells ? 1 : 2; }

void launch_field(const InstDev *insts, InstState *states, int n_inst, int classes, int mode,
                  hipStream_t s) {
  if (classes & 1)
    hipLaunchKernelGGL(k_field<256>, dim3(n_inst), dim3(256), 0, s, insts, states, mode);
  if (classes & 2)
    hipLaunchKernelGGL(k_field<1024>, dim3(n_inst), dim3(1024), 0, s, insts, states, mode);
}

}  // namespace ecpic
