// setd_sde.hip -- scalar SETD schemes (Sec. 2) for batches of independent paths.
#include <hip/hip_runtime.h>

#include <cmath>

#include "setd.h"
#include "setd_device.hpp"
#include "setd_runtime.hpp"

namespace setd {

// Per-step factors of the schemes, with x = c h: e^x, (e^x - 1)/c, e^{x/2},
// sqrt((e^{2x} - 1)/(2c)) (their c -> 0 limits h, 1 and sqrt(h)).
struct SdeFactors {
    double E, fF, fmid, f4, sh;
};

// One thread per path; the path's state stays in registers for all steps.
__global__ void __launch_bounds__(256) k_sde(setd_sde_desc d, SdeFactors f, double* __restrict__ u_out,
                                             double* __restrict__ w_out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d.npaths) return;
    double u = d.u0, w = 0.0;
    for (int64_t n = 0; n < d.nsteps; n++) {
        double z1, z2;
        normal_pair(d.seed, (uint32_t)p, (uint32_t)n, 0u, 2u, z1, z2);
        const double dW = f.sh * z1;
        const double F = d.f1 * u + d.f3 * u * u * u;
        const double G = d.g0 + d.g1 * u;
        double kick;
        if (d.scheme == SETD_SDE_EM) kick = f.fmid * G * dW;
        else if (d.scheme == SETD_SDE_MILSTEIN) kick = f.fmid * G * (dW + 0.5 * d.g1 * (dW * dW - d.h));
        else kick = f.f4 * G * z1;
        u = f.E * u + f.fF * F + kick;
        w += dW;
    }
    u_out[p] = u;
    if (w_out) w_out[p] = w;
}

}  // namespace setd

extern "C" setd_status setd_sde_run(const setd_sde_desc* desc, double* dev_u, double* dev_w, void* hip_stream)
{
    using namespace setd;
    if (!desc) return fail(SETD_E_INVAL, "null descriptor");
    const setd_sde_desc& d = *desc;
    if (d.scheme < SETD_SDE_EM || d.scheme > SETD_SDE_SETD1) return fail(SETD_E_INVAL, "unknown scheme %d", d.scheme);
    if (!(d.h > 0.0) || !std::isfinite(d.h)) return fail(SETD_E_INVAL, "step h must be positive");
    if (d.nsteps < 0 || d.nsteps >= ((int64_t)1 << 32)) return fail(SETD_E_INVAL, "nsteps must be in [0, 2^32)");
    if (d.npaths < 0) return fail(SETD_E_INVAL, "negative path count");
    if (d.npaths == 0) return ok();
    if (!dev_u) return fail(SETD_E_INVAL, "null output");
    const double x = d.c * d.h;
    SdeFactors f;
    f.E = std::exp(x);
    f.fF = (d.c != 0.0) ? std::expm1(x) / d.c : d.h;
    f.fmid = std::exp(0.5 * x);
    f.f4 = (d.c != 0.0) ? std::sqrt(std::expm1(2.0 * x) / (2.0 * d.c)) : std::sqrt(d.h);
    f.sh = std::sqrt(d.h);
    const unsigned blocks = (unsigned)((d.npaths + 255) / 256);
    hipLaunchKernelGGL(k_sde, dim3(blocks), dim3(256), 0, (hipStream_t)hip_stream, d, f, dev_u, dev_w);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SETD_E_DEVICE, "k_sde launch failed: %s", hipGetErrorString(e));
    return ok();
}
