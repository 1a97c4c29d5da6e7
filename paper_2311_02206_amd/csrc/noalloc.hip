// Static device scratch for the entry point that allocates nothing
// (hl_sort_keys_noalloc): callers that cannot call hipMalloc, such as code
// under HIP graph capture, tight serving loops and harnesses that forbid
// allocation, pass only their keys; the sort's second buffer and its count
// matrices live in this array.
//
// Each GPU the library runs on holds its own copy of the array for the rest
// of the process.  In host code `scratch` is only a host-side stand-in for
// the device symbol: its device address is looked up once per device (with
// that device current) and kept, and only that address is ever passed to
// kernels or copies.  Every call on one GPU shares that GPU's copy, so calls
// that overlap on one GPU race; the entry point synchronises its stream
// before returning, so calls made one after another from one thread do not.
#include <mutex>

#include "device.hpp"
#include "kernels.hpp"

namespace hl {

constexpr u64 kNoAllocScratchBytes = u64(64) << 20;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

u64 noalloc_scratch_bytes() { return kNoAllocScratchBytes; }

hipError_t noalloc_scratch(int device, void** ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace hl
