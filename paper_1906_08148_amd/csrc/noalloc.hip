// Static device scratch for the entry point that allocates nothing
// (spamm_gershgorin_static): the per-leaf-row partial bounds of the
// Gershgorin kernels live in a file-scope device array instead of the
// caller's arena.  Each device holds its own copy of the array until the
// process ends; its address is looked up once per device, with that device
// current, when a context is created on it, and only that address is
// handed to kernels and copies.
#include <mutex>

#include "internal.h"

namespace spamm {

// Two doubles (min, max) per leaf row of the matrix.
static __device__ __align__(256) double scratch[2 * kGershStaticRows];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[device] = static_cast<double*>(p);
  return hipSuccess;
}

double* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_scratch[device];
}

}  // namespace spamm
