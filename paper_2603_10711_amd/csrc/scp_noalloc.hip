// scp_problem_create_noalloc: the problem arena in a fixed device array of this library instead
// of caller memory, for callers that cannot allocate device memory.  The array is file-scope
// device memory of SCP_NOALLOC_MAX_BYTES per GPU, held until the process ends.  Host code never
// uses the array's name as an address: its device address on each GPU comes from
// hipGetSymbolAddress, called once per device with that device current.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/scp.h"
#include "scp_host.hpp"

namespace {

__device__ __align__(256) unsigned char scratch[SCP_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};     // device address of the array on each device (0: not yet looked up)
bool g_busy[kMaxDevices] = {};     // a live handle owns the array on that device

}  // namespace

namespace scp {

void noalloc_release(int dev) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (dev >= 0 && dev < kMaxDevices) g_busy[dev] = false;
}

}  // namespace scp

extern "C" scp_status scp_problem_create_noalloc(const scp_problem_desc* desc, void* hip_stream, scp_problem** out) {
    using namespace scp;
    if (!out) {
        set_create_error("out is NULL");
        return SCP_ERR_ARG;
    }
    *out = nullptr;
    const size_t need = scp_problem_device_bytes(desc);
    if (need == 0) return scp_problem_create(desc, nullptr, 0, hip_stream, out);   // reports the description error
    if (need > (size_t)SCP_NOALLOC_MAX_BYTES) {
        set_create_error("problem needs " + std::to_string(need) + " bytes of device memory, more than the " +
                         std::to_string((size_t)SCP_NOALLOC_MAX_BYTES) +
                         " bytes of the no-allocation arena; use scp_problem_create with a caller arena");
        return SCP_ERR_ARG;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_create_error(std::string("no usable current device: ") + hipGetErrorString(e));
        return SCP_ERR_HIP;
    }
    void* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (g_busy[dev]) {
            set_create_error("the no-allocation arena of this device is held by another live problem handle "
                             "(destroy it first)");
            return SCP_ERR_STATE;
        }
        if (!g_ptr[dev]) {
            e = hipGetSymbolAddress(&g_ptr[dev], HIP_SYMBOL(scratch));
            if (e != hipSuccess || !g_ptr[dev]) {
                g_ptr[dev] = nullptr;
                set_create_error(std::string("hipGetSymbolAddress of the no-allocation arena: ") + hipGetErrorString(e));
                return SCP_ERR_HIP;
            }
        }
        ptr = g_ptr[dev];
        g_busy[dev] = true;
    }
    // the arena starts from zero exactly as a caller arena does (scp_problem_create clears it)
    const scp_status st = scp_problem_create(desc, ptr, (size_t)SCP_NOALLOC_MAX_BYTES, hip_stream, out);
    if (st != SCP_OK) {
        noalloc_release(dev);
        return st;
    }
    problem_mark_noalloc(*out, dev);
    return SCP_OK;
}
