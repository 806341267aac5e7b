// Fixed device scratch of the allocation-free matched filter (mf_full_noalloc).
//
// One file-scope device array per GPU, held by the loaded code object until
// the process ends.  Host code never passes the array's name to a kernel (on
// the host it is only a stand-in symbol): the device address of each GPU's
// copy is looked up once, with that GPU current, when the first context on it
// is created, and that address is what the kernels receive.
#include "internal.h"

#include <mutex>

namespace rbmf {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};
std::mutex g_busy[kMaxDevices];
}  // namespace

hipError_t noalloc_scratch_init(int device, void** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (g_addr[device] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_addr[device] = p;
  }
  *out = g_addr[device];
  return hipSuccess;
}

std::mutex& noalloc_scratch_lock(int device) { return g_busy[device < 0 || device >= kMaxDevices ? 0 : device]; }

}  // namespace rbmf
