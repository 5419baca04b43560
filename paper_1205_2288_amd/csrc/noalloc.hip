// Fixed device array for the split-j partial sums of tsbts_force_noalloc, the variant of
// tsbts_force for callers that cannot allocate device memory.
//
// The array is a file-scope __device__ variable: every GPU the library runs on holds its
// own copy, at its own address, from the load of the code object until the process
// ends.  On the host its name is only a stand-in for the symbol, never a device address:
// the address is looked up once per device (hipGetSymbolAddress, with that device
// current) when the first context is created there, and every use on the host goes
// through that looked-up pointer.  All calls on one GPU share its copy.
#include <mutex>

#include "internal.hpp"

namespace tsbts {
namespace {

static_assert(TSBTS_NOALLOC_PARTIALS % 32 == 0, "whole 256-byte lines");

static __device__ __align__(256) double scratch[TSBTS_NOALLOC_PARTIALS];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;
  void *p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_ptr[device] = static_cast<double *>(p);
  return hipSuccess;
}

double *noalloc_partials(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_ptr[device];
}

}  // namespace tsbts
