// FP64 tables, control blocks, copies and observable finalisation.
#include "setd_kernels.hpp"
#include "setd_launch.hpp"

namespace setd {

// ---------------------------------------------------------------- FP64 tables
// ETD coefficients per key (Sec. 4 step 3, Eq. SETD1/SETD2), with x = c h:
//   E = e^x, wa = h phi1 (SETD1) or h (phi1 + phi2) (SETD2), wb = -h phi2,
//   G = prod_i (N_i^2/L_i)^{1/2} sqrt(2 D(k) h phi1(2 Re x)).

__global__ void __launch_bounds__(256) k_coef(CoefArgs a)
{
    const int key = blockIdx.x * blockDim.x + threadIdx.x;
    if (key >= a.nkeys) return;
    double k2;
    if (a.mode == COEF_PER_MODE) {
        // a 2D lattice: one entry per |a0| (row) and stored column of the last
        // axis, in the padded row layout of the state
        const Geo& g = a.g;
        const int a0 = key / g.pitch, col = key % g.pitch;
        if (col >= g.kept[1]) {
            const int w = a.cplx_table ? 8 : 4;
            for (int i = 0; i < w; i++) {
                a.out64[w * (size_t)key + i] = 0.0;
                if (a.out32) reinterpret_cast<float*>(a.out32)[w * (size_t)key + i] = 0.0f;
            }
            return;
        }
        int a1 = col;
        if (g.cplx) {
            const int j1 = (col <= g.kp[1]) ? col : col + g.n[1] - g.kept[1];
            a1 = (j1 < g.n[1] / 2) ? j1 : j1 - g.n[1];
        }
        k2 = (a.dk[0] * a0) * (a.dk[0] * a0) + (a.dk[1] * a1) * (a.dk[1] * a1);
    } else if (a.mode == COEF_ISO) {
        k2 = a.dk[0] * a.dk[0] * (double)key;
    } else {
        const int a2 = key % a.keydim[2];
        const int rest = key / a.keydim[2];
        const int a1 = rest % a.keydim[1];
        const int a0 = rest / a.keydim[1];
        k2 = (a.dk[0] * a0) * (a.dk[0] * a0) + (a.dk[1] * a1) * (a.dk[1] * a1) + (a.dk[2] * a2) * (a.dk[2] * a2);
    }
    const cd c = {a.c0[0] + a.c2[0] * k2 + a.c4[0] * k2 * k2, a.c0[1] + a.c2[1] * k2 + a.c4[1] * k2 * k2};
    const cd x = {c.x * a.h, c.y * a.h};
    cd p1, p2;
    phi12(x, p1, p2);
    const double ex = exp(x.x);
    const cd E = {ex * cos(x.y), ex * sin(x.y)};
    cd wa, wb;
    if (a.order == 1) {
        wa = {a.h * p1.x, a.h * p1.y};
        wb = {0.0, 0.0};
    } else {
        wa = {a.h * (p1.x + p2.x), a.h * (p1.y + p2.y)};
        wb = {-a.h * p2.x, -a.h * p2.y};
    }
    const double Dk = a.D * (a.kpow == 2 ? k2 : 1.0);
    cd q1, q2;
    phi12({2.0 * x.x, 0.0}, q1, q2);
    const double var = 2.0 * Dk * a.h * q1.x;
    const double G = a.lat * sqrt(var > 0.0 ? var : 0.0);
    if (a.cplx_table) {
        double* o = a.out64 + 8 * (size_t)key;
        o[0] = E.x; o[1] = E.y; o[2] = wa.x; o[3] = wa.y; o[4] = wb.x; o[5] = wb.y; o[6] = G; o[7] = 0.0;
        if (a.out32) {
            float* f = reinterpret_cast<float*>(a.out32) + 8 * (size_t)key;
            for (int i = 0; i < 8; i++) f[i] = (float)o[i];
        }
    } else {
        double* o = a.out64 + 4 * (size_t)key;
        o[0] = E.x; o[1] = wa.x; o[2] = wb.x; o[3] = G;
        if (a.out32) {
            float* f = reinterpret_cast<float*>(a.out32) + 4 * (size_t)key;
            for (int i = 0; i < 4; i++) f[i] = (float)o[i];
        }
    }
}

// twiddles exp(-2 pi i k / n), k < n, in FP64 and rounded to FP32
__global__ void __launch_bounds__(256) k_twiddle(int n, double* out64, float* out32)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double s, c;
    sincospi(2.0 * (double)k / (double)n, &s, &c);
    out64[2 * k] = c;
    out64[2 * k + 1] = -s;
    out32[2 * k] = (float)c;
    out32[2 * k + 1] = (float)(-s);
}

// ---------------------------------------------------------------- control / copies
__global__ void k_ctrl_init(Ctrl* ctrl, int n, int64_t step)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ctrl[i].step = step;
    ctrl[i].done = 0u;
    ctrl[i].have_prev = 0;
    ctrl[i].nonfinite = 0;
}

__global__ void k_ctrl_set(Ctrl* ctrl, int n, int64_t step, int which)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (which == 0) ctrl[i].step = step;
    else ctrl[i].have_prev = 0;
}

__global__ void __launch_bounds__(256) k_fill64(double* p, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(256) k_copy16(uint4* dst, const uint4* src, int64_t n16)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Stored position of FFT index j on an axis of n points whose kept entries are
// 0..kp then the top (kept - kp - 1) indices (a full axis), or 0..kp only (the
// half-spectrum axis of a real field); -1 for an index dealiasing removed.
__device__ inline int stored_pos(int j, int n, int kept, int kp, bool half)
{
    if (j <= kp) return j;
    if (half) return -1;
    const int lo = n - (kept - kp - 1);
    return j >= lo ? j - (n - kept) : -1;
}

// Stored state of R realizations (rstride bytes apart, padded last axis) ->
// the unpruned FFT-order spectra of the ABI as interleaved doubles, realization
// r at out + 2 r nspec; removed modes are written as zero.
template <typename T>
__global__ void __launch_bounds__(256) k_unpack(Geo g, const char* phi, size_t rstride, int R, int64_t nspec,
                                                double* out)
{
    const int64_t total = (int64_t)R * nspec;
    const int last = g.ndim - 1;
    const int k1 = (g.ndim == 3) ? g.kept[1] : 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / nspec);
        int64_t e = i - (int64_t)r * nspec;
        const int jl = (int)(e % g.nh_last);
        e /= g.nh_last;
        int j1 = 0, j0 = 0;
        if (g.ndim == 3) {
            j1 = (int)(e % g.n[1]);
            j0 = (int)(e / g.n[1]);
        } else if (g.ndim == 2) {
            j0 = (int)e;
        }
        const int c = stored_pos(jl, g.n[last], g.kept[last], g.kp[last], !g.cplx);
        const int i1 = (g.ndim == 3) ? stored_pos(j1, g.n[1], g.kept[1], g.kp[1], false) : 0;
        const int i0 = (g.ndim >= 2) ? stored_pos(j0, g.n[0], g.kept[0], g.kp[0], false) : 0;
        double re = 0.0, im = 0.0;
        if (c >= 0 && i1 >= 0 && i0 >= 0) {
            const T* src = reinterpret_cast<const T*>(phi + (size_t)r * rstride) +
                           2 * (((size_t)i0 * k1 + i1) * g.pitch + c);
            re = (double)src[0];
            im = (double)src[1];
        }
        out[2 * i] = re;
        out[2 * i + 1] = im;
    }
}

// means per shell and the accumulated time series (kind = setd_obs_kind)
__global__ void k_obs_final(int kind, int nb, const double* acc, double* out, double* skacc, double wscale)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (kind == 1) {   // width
        if (b == 0) out[0] = sqrt(acc[0] * wscale);
        return;
    }
    if (b >= nb) return;
    const double cnt = acc[2 * nb + b];
    if (kind == 0) {
        out[b] = cnt > 0.0 ? acc[b] / cnt : 0.0;
        out[nb + b] = cnt;
    } else if (kind == 3) {
        out[b] = cnt > 0.0 ? acc[b] / cnt : 0.0;
        out[nb + b] = cnt > 0.0 ? acc[nb + b] / cnt : 0.0;
        out[2 * nb + b] = cnt;
    } else if (kind == 5) {
        skacc[b] += cnt > 0.0 ? acc[b] / cnt : 0.0;
        skacc[nb + b] = cnt;
        if (b == 0) {
            skacc[2 * nb] += 1.0;
            out[0] = skacc[2 * nb];
        }
    }
}

__global__ void k_obs_mean(int nb, const double* skacc, double* out)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const double m = skacc[2 * nb];
    out[b] = m > 0.0 ? skacc[b] / m : 0.0;
    out[nb + b] = skacc[nb + b];
}


void axis_shape(int precision, int n, int var, int* tile, int* lpt)
{
    const int tm = (precision == 32) ? (n <= 512 ? 16 : 8) : (n <= 512 ? 8 : 4);
    static const int tl[7] = {1, 1, 1, 2, 2, 1, 4};
    static const int lp[7] = {2, 1, 4, 1, 1, 1, 1};
    // register-kernel variants 4 + 2j / 5 + 2j share the tiles of 4 / 5, and
    // 12 + j take a quarter of tm
    const int v = (var >= 0 && var < 6) ? var : (var >= 6 && var < 12 ? 4 + (var - 4) % 2 : (var >= 12 && var < 16 ? 6 : 0));
    *tile = tm / tl[v] > 0 ? tm / tl[v] : 1;
    *lpt = lp[v];
}

hipError_t launch_coef(const CoefArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_coef, dim3((a.nkeys + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_twiddle(int n, double* out64, float* out32, hipStream_t s)
{
    hipLaunchKernelGGL(k_twiddle, dim3((n + 255) / 256), dim3(256), 0, s, n, out64, out32);
    return hipGetLastError();
}

hipError_t launch_ctrl_init(Ctrl* ctrl, int n, int64_t step, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctrl_init, dim3((n + 255) / 256), dim3(256), 0, s, ctrl, n, step);
    return hipGetLastError();
}

hipError_t launch_ctrl_set(Ctrl* ctrl, int n, int64_t step, int which, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctrl_set, dim3((n + 255) / 256), dim3(256), 0, s, ctrl, n, step, which);
    return hipGetLastError();
}

hipError_t launch_fill64(double* p, int64_t n, double v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    // every buffer of the workspace is a multiple of 16 bytes and 256-aligned
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 <= 0) return hipSuccess;
    int64_t blocks = (n16 + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s, reinterpret_cast<uint4*>(dst),
                       reinterpret_cast<const uint4*>(src), n16);
    return hipGetLastError();
}

hipError_t launch_unpack(const Geo& g, const void* phi, size_t rstride, int R, int64_t nspec, double* out,
                         hipStream_t s)
{
    const int64_t total = (int64_t)R * nspec;
    if (total <= 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (g.prec == 32)
        hipLaunchKernelGGL(k_unpack<float>, dim3((unsigned)blocks), dim3(256), 0, s, g,
                           reinterpret_cast<const char*>(phi), rstride, R, nspec, out);
    else
        hipLaunchKernelGGL(k_unpack<double>, dim3((unsigned)blocks), dim3(256), 0, s, g,
                           reinterpret_cast<const char*>(phi), rstride, R, nspec, out);
    return hipGetLastError();
}

hipError_t launch_obs_final(int kind, int nb, const double* acc, double* out, double* skacc, double wscale,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_obs_final, dim3((nb + 255) / 256), dim3(256), 0, s, kind, nb, acc, out, skacc, wscale);
    return hipGetLastError();
}

hipError_t launch_obs_mean(int nb, const double* skacc, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_obs_mean, dim3((nb + 255) / 256), dim3(256), 0, s, nb, skacc, out);
    return hipGetLastError();
}

}  // namespace setd
