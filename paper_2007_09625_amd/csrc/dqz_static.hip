// dqz_static.hip -- compression that allocates nothing: the same kernels as
// dqz_compress_async, with their workspace in a fixed device array that the
// library's code object carries (one copy per GPU, resident until the
// process ends) instead of a context's allocation.
#include "../../include/dqz.h"
#include "dqz_internal.h"

#include <hip/hip_runtime.h>

#include <mutex>

namespace {

constexpr uint64_t kScratchBytes = 128ull << 20;
constexpr int kMaxDevices = 64;

// The workspace of every dqz_compress_async_static call on a GPU.  In host
// code this name is a stand-in for the symbol, not a device address: kernels
// and copies take the address hipGetSymbolAddress returns for the device.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

struct DeviceScratch {
    uint8_t *ptr = nullptr;   // this device's copy of `scratch`
    int ncu = 0;
    bool ready = false;
};
DeviceScratch g_dev[kMaxDevices];
std::mutex g_mu;

// The device address of `scratch` on `dev` (the current device), looked up
// once per device.
dqz_status device_scratch(int dev, DeviceScratch &out) {
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceScratch &d = g_dev[dev];
    if (!d.ready) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return DQZ_EHIP;
        }
        int ncu = 0;
        e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess || ncu <= 0) {
            (void)hipGetLastError();
            return DQZ_EHIP;
        }
        d.ptr = static_cast<uint8_t *>(p);
        d.ncu = ncu;
        d.ready = true;
    }
    out = d;
    return DQZ_OK;
}

}  // namespace

extern "C" dqz_status dqz_compress_async_static(const float *d_field, const dqz_shape *shape,
                                                const dqz_params *params, void *d_archive, uint64_t archive_cap,
                                                dqz_result *d_result, void *stream) {
    if (!d_result || (reinterpret_cast<uintptr_t>(d_result) & 7u)) return DQZ_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return DQZ_EHIP;
    }
    if (dev < 0 || dev >= kMaxDevices) return DQZ_EUNSUPPORTED;
    DeviceScratch ds;
    const dqz_status st = device_scratch(dev, ds);
    if (st != DQZ_OK) return st;
    uint64_t need = 0;
    return dqz::compress_on_workspace(ds.ptr, kScratchBytes, ds.ncu, d_field, shape, params, d_archive, archive_cap,
                                      reinterpret_cast<dqz::Readback *>(d_result),
                                      reinterpret_cast<hipStream_t>(stream), &need);
}
