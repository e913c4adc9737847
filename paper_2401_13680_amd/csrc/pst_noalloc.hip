// Fixed device scratch of the allocation-free query profile
// (pst_mpdist_profile_noalloc): a file-scope device array, one per GPU the
// library runs on, held until the process ends.  Host code never uses the
// array's name as an address: static_scratch() looks the device address up
// once per device (with that device current) and hands out that pointer.
#include <mutex>

#include "pst_internal.h"

namespace pst {
namespace {

constexpr size_t kScratchBytes = (size_t)256 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices];
bool g_have[kMaxDevices];

}  // namespace

size_t static_scratch_bytes() { return kScratchBytes; }

hipError_t static_scratch(int device, void **ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_have[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[device] = p;
        g_have[device] = true;
    }
    *ptr = g_ptr[device];
    return hipSuccess;
}

}  // namespace pst
