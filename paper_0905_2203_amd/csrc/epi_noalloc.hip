// Device scratch of the allocation-free count (epi_count_noalloc): one
// file-scope device array, shared by every call on a device, holding the
// per-(segment, lane) records of the segment-parallel count.
//
// The array's name is a host-side stand-in in host code: kernels get the
// device address that hipGetSymbolAddress returns for the device, looked up
// once per device (with that device current) when a context is created.
#include <mutex>

#include "epi_internal.h"

namespace epi {

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
unsigned char *g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[device] = static_cast<unsigned char *>(p);
    return hipSuccess;
}

unsigned char *noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[device];
}

size_t noalloc_scratch_bytes() { return kScratchBytes; }

}  // namespace epi
