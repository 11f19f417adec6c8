// nflbm_diagnostics_noalloc: the diagnostics of nflbm_diagnostics with the
// reduction's partial records in a fixed device array of this library
// instead of a buffer it allocates, for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops, harnesses that forbid
// it).
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"
#include "nflbm.h"

using namespace nflbm;

namespace {

// Room for the partial records of the capped reduction grid plus the summed
// record, at the largest N: (2048 + 1) * 33 doubles, about 0.5 MiB.  Each
// device the library runs on holds its own copy until the process ends.
constexpr int kRecMax = 3 * kMaxComp + 9;
constexpr size_t kScratchDoubles = size_t(kDiagMaxBlocks + 1) * kRecMax;
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (the array's name
// is a host-side stand-in: only this address may be handed to kernels).
int scratch_on(int dev, double** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return -1;
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return 0;
}

}  // namespace

extern "C" int nflbm_diagnostics_noalloc(nflbm_sim* sim, int vcm_component, nflbm_diag* out) {
  if (!sim || !out) return sim_fail(sim, NFLBM_EINVAL, "NULL argument");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0)
    return sim_fail(sim, NFLBM_EDEVICE, "hipGetDevice failed");
  if (dev != sim_device(sim))
    return sim_fail(sim, NFLBM_EINVAL, "call with the simulation's device current");
  if (dev >= kMaxDevices) return sim_fail(sim, NFLBM_ENOTSUP, "device index above 63");
  // the records of the capped grid at this N must fit the array (always true
  // for N <= NFLBM_MAX_COMP; kept as the explicit size check)
  const size_t need = size_t(kDiagMaxBlocks + 1) * size_t(3 * kMaxComp + 9);
  if (need > kScratchDoubles) return sim_fail(sim, NFLBM_ENOTSUP, "diagnostic records exceed the fixed array");
  double* base = nullptr;
  if (scratch_on(dev, &base) != 0)
    return sim_fail(sim, NFLBM_EDEVICE, "hipGetSymbolAddress of the diagnostics array failed");
  const int rec = 3 * kMaxComp + 9;
  return diag_run(sim, vcm_component, base, kDiagMaxBlocks, base + size_t(kDiagMaxBlocks) * rec, out);
}
