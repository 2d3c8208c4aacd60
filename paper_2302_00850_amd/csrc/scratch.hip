// Fixed device workspace of the non-allocating operator entry point
// (cola_dslash_apply_noalloc): the intermediate vectors of the composed
// operators live in one file-scope device array instead of memory the library
// allocates.  Each device that loads the library holds its own copy of the
// array until the process ends; its device address is taken once per device
// (hipGetSymbolAddress with that device current) and kept in a table.  Host
// code never passes the array's name to a kernel: on the host it names a
// stand-in, not device memory.
#include <mutex>

#include "handle.h"

namespace cola {

namespace {

__device__ __attribute__((aligned(256))) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void *g_addr[kMaxDevices];
std::mutex g_mu;

}  // namespace

int scratch_address(cola_handle_t *h, void **out) {
    *out = nullptr;
    const int dev = h->device;
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(h, COLA_EINVAL, "device index beyond the scratch address table");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        int cur = -1;
        COLA_HIP(h, hipGetDevice(&cur));
        if (cur != dev) COLA_HIP(h, hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) COLA_HIP(h, hipSetDevice(cur));
        COLA_HIP(h, e);
        if (!p) return set_error(h, COLA_EHIP, "hipGetSymbolAddress returned no address");
        g_addr[dev] = p;
    }
    *out = g_addr[dev];
    return COLA_OK;
}

}  // namespace cola
