// noalloc.hip -- the device scratch of pic_diagnostics_noalloc, the entry
// point for callers that cannot allocate memory.
//
// pic_diagnostics reduces an instance's particles into a few words of the
// caller's arena.  The no-allocation variant reduces several instances in one
// call into a fixed array of this library, `scratch`, one record of
// kNoAllocRecord words per instance of the call.  Every GPU the library runs
// on holds its own copy of the array until the process ends.  In host code
// the array's name is only a stand-in for it, so the host never passes it to a
// kernel or a copy: noalloc_setup() asks the runtime for the array's device
// address once per device (with that device current) and every use goes
// through that address.
#include <mutex>

#include "device.h"
#include "kernels.h"

namespace ecpic {

static __device__ __align__(256) unsigned long long scratch[kNoAllocMaxInst * kNoAllocRecord];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned long long *g_scratch[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;   // the caller makes it current
  void *p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch[device] = static_cast<unsigned long long *>(p);
  return hipSuccess;
}

unsigned long long *noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_scratch[device];
}

// Zero n words (a kernel rather than a memset, so that a captured stream
// records no memset node).
__global__ void __launch_bounds__(256) k_fill_zero(unsigned long long *p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0ull;
}

// Sum of instance inst's node deposit A_s of the current step into
// out[D_DEP0 + s] (periodic grids count the shared node 0 = N once).
__global__ void __launch_bounds__(256)
k_deposit_total(const InstDev *__restrict__ insts, const InstState *__restrict__ states, int inst,
                unsigned long long *__restrict__ out) {
  CInst &I = cinst(insts)[inst];
  const InstState &S = states[inst];
  const int par = (int)(S.k & 1);
  const int upto = (I.bc == 1) ? I.N : I.N + 1;
  for (int s = 0; s < I.nsp; ++s) {
    unsigned long long v = 0;
    for (int n = threadIdx.x; n < upto; n += blockDim.x) v += (unsigned long long)I.A[par][s][n];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (__lane_id() == 0) atomicAdd(&out[D_DEP0 + s], v);
  }
}

void launch_fill_zero(unsigned long long *p, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_zero, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
}

void launch_deposit_total(const InstDev *insts, const InstState *states, int inst,
                          unsigned long long *out, hipStream_t s) {
  hipLaunchKernelGGL(k_deposit_total, dim3(1), dim3(256), 0, s, insts, states, inst, out);
}

}  // namespace ecpic
