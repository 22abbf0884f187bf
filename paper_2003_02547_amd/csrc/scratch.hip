// Device memory of the batch entry point that allocates nothing
// (oqp_batch_init_static): a file-scope array in the library's code object,
// one copy per GPU, held until the process ends.
//
// In host code the array's name only stands for the symbol; the device
// address of this GPU's copy comes from hipGetSymbolAddress, looked up once
// per device with that device current, and that address is what the batch
// hands to its kernels and copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)OQP_STATIC_DEV_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

}  // namespace

int static_dev_region(void** ptr, size_t* bytes)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(OQP_EDEVICE, "static device region: hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(OQP_EDEVICE, "static device region: device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(OQP_EDEVICE, "static device region: hipGetSymbolAddress: %s", hipGetErrorString(e));
        g_addr[dev] = p;
    }
    *ptr = g_addr[dev];
    *bytes = kScratchBytes;
    return OQP_OK;
}
