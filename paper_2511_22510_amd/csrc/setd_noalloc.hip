// setd_noalloc.hip -- setd_run_noalloc: plan, initial condition, time steps and
// read-out of the final spectra in one call that allocates no device memory.
//
// The plan's workspace (item table, coefficient and twiddle tables, state,
// SETD2 carry, transform intermediates) lives in `scratch`, a fixed array of
// SETD_NOALLOC_MAX_WORKSPACE bytes in the library's device image.  Each device
// the library runs on holds its own copy from the first call on that device
// until the process ends.  In host code `scratch` only names the symbol: its
// device address is looked up once per device with hipGetSymbolAddress and
// that address is what the kernels receive.
#include <hip/hip_runtime.h>

#include <mutex>

#include "setd.h"
#include "setd_launch.hpp"
#include "setd_runtime.hpp"

static __device__ __align__(256) unsigned char scratch[SETD_NOALLOC_MAX_WORKSPACE];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on the first
// call per device, with that device current)
setd_status scratch_of_current_device(void** out)
{
    int dev = -1;
    SETD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return setd::fail(SETD_E_DEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return setd::fail(SETD_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                              hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return SETD_OK;
}

}  // namespace

extern "C" setd_status setd_run_noalloc(const setd_desc* desc, int64_t nsteps, double* dev_out, size_t cap,
                                        void* hip_stream)
{
    if (!desc || !dev_out) return setd::fail(SETD_E_INVAL, "null argument");
    if (nsteps < 0) return setd::fail(SETD_E_INVAL, "negative step count");
    setd::Plan p;
    setd_status st = p.init(*desc);
    if (st != SETD_OK) return st;
    if (p.lay.total > (size_t)SETD_NOALLOC_MAX_WORKSPACE)
        return setd::fail(SETD_E_NOMEM, "the plan needs %zu bytes of workspace; setd_run_noalloc holds at most %zu",
                          p.lay.total, (size_t)SETD_NOALLOC_MAX_WORKSPACE);
    const size_t need = 2 * p.nspec * (size_t)p.R;
    if (cap < need) return setd::fail(SETD_E_INVAL, "output holds %zu doubles, %zu needed", cap, need);
    void* ws = nullptr;
    if ((st = scratch_of_current_device(&ws)) != SETD_OK) return st;
    const hipStream_t s = (hipStream_t)hip_stream;
    p.no_alloc = true;
    // binding rewrites every table and clears every state buffer of the
    // layout, so nothing of an earlier call's contents is read
    if ((st = p.bind(ws, (size_t)SETD_NOALLOC_MAX_WORKSPACE, s)) != SETD_OK) return st;
    if ((st = p.step(nsteps)) != SETD_OK) return st;
    if ((st = p.ensure_phi()) != SETD_OK) return st;
    SETD_HIP(setd::launch_unpack(p.g, p.ws + p.lay.phi, p.Sb, p.R, (int64_t)p.nspec, dev_out, s));
    return SETD_OK;
}
