// Static device workspace of the allocation-free local-energy entry point
// (nqs_eloc_noalloc): one fixed array per GPU, resolved to its device address
// once per device when a context is created there, and carved per call by the
// runtime's arena allocator.  Nothing here allocates after module load.
#include "internal.h"

#include <mutex>

namespace nqs {
namespace {

// The array itself.  In host code its name is only a stand-in for the device
// symbol: host code uses the address returned by hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

// With `device` current: look up this device's copy of the array (once).
hipError_t static_workspace_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_ptr[device] = p;
  return hipSuccess;
}

// Device address of the array on `device` (nullptr before the setup).
void* static_workspace(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

}  // namespace nqs
