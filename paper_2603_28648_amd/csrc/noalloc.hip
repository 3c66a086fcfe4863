// Fixed device scratch for the sigma entry point that allocates nothing
// (dmrg_sigma_noalloc): the stage-1 workspace of the FP64 sigma lives in one
// file-scope device array per GPU instead of a buffer the context allocates.
//
// In host code the array's name is only a host-side stand-in; its device
// address is looked up once per device with hipGetSymbolAddress (with that
// device current, at dmrg_create) and that address is what the descriptors
// and kernels use.  Every context on a device shares the one array, so
// dmrg_sigma_noalloc calls that overlap on one GPU race.
#include <map>
#include <mutex>

#include "noalloc.h"

static __device__ __align__(256) double scratch[dmrg::kNoAllocScratchDoubles];

namespace dmrg {

namespace {
std::mutex g_mu;
std::map<int, double*> g_ptr;  // device -> device address of scratch
}  // namespace

double* noalloc_scratch_init(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ptr.find(device);
  if (it != g_ptr.end()) return it->second;
  int cur = -1;
  DMRG_HIP(hipGetDevice(&cur));
  DMRG_REQUIRE(cur == device, kErrState, "noalloc scratch: the device must be current");
  void* p = nullptr;
  DMRG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  DMRG_REQUIRE(p != nullptr, kErrHip, "noalloc scratch: no device address");
  g_ptr[device] = static_cast<double*>(p);
  return static_cast<double*>(p);
}

double* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ptr.find(device);
  return it == g_ptr.end() ? nullptr : it->second;
}

}  // namespace dmrg
