// Allocation-free variant of the batch EoS inversion, for callers that may
// not allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation).
//
// The inversion kernel needs one device word beyond its inputs and outputs:
// the count of inversions that did not converge.  ccake_eos_invert keeps it
// in memory the EoS handle allocated; this variant keeps it in a file-scope
// device array, `scratch`, whose device address is looked up once per
// device (hipGetSymbolAddress, with that device current) and then used for
// every kernel argument and copy.  Every call on a device shares that
// device's array, so calls that overlap on one device race on the counter.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ccake.h"
#include "common.h"
#include "kernels.h"
#include "runtime.h"

namespace ccake {

// 256 bytes per device, held until the process ends: word 0 is the failure
// counter of the current call, the rest is unused.
constexpr int SCRATCH_WORDS = 64;
static __device__ __align__(256) uint32_t scratch[SCRATCH_WORDS];

constexpr int MAX_DEVICES = 64;
static uint32_t* g_scratch_ptr[MAX_DEVICES];
static std::once_flag g_scratch_once[MAX_DEVICES];
static hipError_t g_scratch_err[MAX_DEVICES];

// device address of this device's scratch (nullptr on failure, with *err set)
static uint32_t* scratch_ptr(hipError_t* err) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *err = e;
    return nullptr;
  }
  if (dev < 0 || dev >= MAX_DEVICES) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::call_once(g_scratch_once[dev], [dev] {
    void* p = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? (uint32_t*)p : nullptr;
  });
  *err = g_scratch_err[dev];
  return g_scratch_ptr[dev];
}

// clears the first `words` words (a kernel, not a memset, so that a captured
// stream records an ordinary kernel node)
__global__ void k_clear_words(uint32_t* p, int words) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) p[i] = 0u;
}

}  // namespace ccake

using namespace ccake;

extern "C" ccake_status ccake_eos_invert_noalloc(ccake_eos* eos, int32_t mode, int32_t ncharge, int64_t n,
                                                 const double* in, double* out, int32_t* in_table, void* stream) {
  if (!eos || eos->magic != HANDLE_EOS) return CCAKE_E_ARG;
  if ((mode != 0 && mode != 1) || (ncharge != 0 && ncharge != 3) || n < 0 || (n > 0 && (!in || !out)))
    return fail(eos, CCAKE_E_ARG, "ccake_eos_invert_noalloc: bad arguments");
  hipError_t he = hipSuccess;
  uint32_t* bad = scratch_ptr(&he);
  if (!bad)
    return fail(eos, CCAKE_E_HIP, "ccake_eos_invert_noalloc: scratch address: %s", hipGetErrorString(he));
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(64), 0, s, bad, 1);
  he = hipGetLastError();
  if (he == hipSuccess) he = launch_eos_invert(eos->dev, mode, ncharge, n, in, out, in_table, bad, s);
  uint32_t nbad = 0;
  if (he == hipSuccess) he = hipMemcpyAsync(&nbad, bad, sizeof nbad, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess)
    return fail(eos, CCAKE_E_HIP, "ccake_eos_invert_noalloc: %s", hipGetErrorString(he));
  if (nbad) return fail(eos, CCAKE_E_EOS_NOCONV, "%u inversions did not converge", nbad);
  return CCAKE_OK;
}
