// fz_run_chain for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
// workspace that holds the intermediates between groups is a fixed array of
// FZ_STATIC_WORKSPACE_BYTES inside the library instead of a caller buffer.
//
// Each GPU the library runs on holds its own copy of the array from the first
// call on that device until the process ends.  Its device address is looked
// up once per device with hipGetSymbolAddress; host code never passes the
// array's own name to a kernel (on the host that name is only a stand-in, not
// a device address).  Every call on a GPU shares that GPU's array: two calls
// that overlap in time on one device (two streams, two threads) race on it.
// Nothing in the array needs to start at zero -- each group writes every
// element of its output before the next group reads it -- so it is never
// cleared.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "fz_internal.h"

namespace fz {

static __device__ __align__(256) unsigned char scratch[FZ_STATIC_WORKSPACE_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[MAX_DEVICES];

// Device address of `scratch` on the current device (looked up once).
static fz_status scratch_address(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(FZ_E_HIP, std::string("fz_run_chain_static: hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES)
        return fail(FZ_E_UNSUPPORTED, "fz_run_chain_static: device index " + std::to_string(dev) + " out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(FZ_E_HIP, std::string("fz_run_chain_static: hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FZ_OK;
}

}  // namespace fz

using namespace fz;

extern "C" {

fz_status fz_run_chain_static(const fz_plan* plan, const void* d_in, void* d_out, fz_point* d_points,
                              uint32_t* d_point_count, uint32_t point_capacity, void* stream)
{
    if (!plan || !d_in || !d_out) return fail(FZ_E_INVALID, "fz_run_chain_static: null plan or buffer");
    if (point_capacity > 0 && !d_points)
        return fail(FZ_E_INVALID, "fz_run_chain_static: capacity without a point buffer");
    const size_t need = workspace_bytes(*plan);
    if (need > FZ_STATIC_WORKSPACE_BYTES)
        return fail(FZ_E_WORKSPACE, "fz_run_chain_static: the plan needs " + std::to_string(need) +
                                        " bytes of workspace, more than the static " +
                                        std::to_string((size_t)FZ_STATIC_WORKSPACE_BYTES) + "; use fz_run_chain");
    void* ws = nullptr;
    if (need > 0) {
        const fz_status st = scratch_address(&ws);
        if (st != FZ_OK) return st;
    }
    return run_plan(*plan, d_in, d_out, d_points, d_point_count, point_capacity, ws, need > 0 ? FZ_STATIC_WORKSPACE_BYTES : 0,
                    stream);
}

}  // extern "C"
