// setd_launch_impl.hpp -- grid shapes and template dispatch of the SETD passes.
#pragma once

#include "setd_kernels.hpp"
#include "setd_launch.hpp"

namespace setd {

#define SETD_DISPATCH_N(N, CALL)                 \
    switch (N) {                                 \
    case 8: { constexpr int NN = 8; CALL; } break;       \
    case 16: { constexpr int NN = 16; CALL; } break;     \
    case 32: { constexpr int NN = 32; CALL; } break;     \
    case 64: { constexpr int NN = 64; CALL; } break;     \
    case 128: { constexpr int NN = 128; CALL; } break;   \
    case 256: { constexpr int NN = 256; CALL; } break;   \
    case 512: { constexpr int NN = 512; CALL; } break;   \
    case 1024: { constexpr int NN = 1024; CALL; } break; \
    default: return hipErrorInvalidValue;        \
    }

template <typename T>
hipError_t launch_row(const Geo& g, const Item* items, int nitems, int mode, int sub, hipStream_t s)
{
    const int last = g.ndim - 1;
    const int N = g.n[last];
    const int tpl = N / 8;
    const int lpw = tpl >= 256 ? 1 : 256 / tpl;
    RowArgs a;
    a.g = g;
    a.items = items;
    a.nrows = (g.ndim == 3) ? g.n[0] * g.n[1] : g.n[0];
    a.lpw = lpw;
    a.mode = mode;
    a.sub = sub;
    const int lines = g.cplx ? a.nrows : a.nrows / 2;
    dim3 grid((lines + lpw - 1) / lpw, nitems);
    dim3 block(lpw * tpl);
    const size_t lds = (size_t)lpw * N * 2 * sizeof(T);
    if (g.cplx) {
        SETD_DISPATCH_N(N, hipLaunchKernelGGL((k_row_cplx<T, NN>), grid, block, lds, s, a));
    } else {
        SETD_DISPATCH_N(N, hipLaunchKernelGGL((k_row_real<T, NN>), grid, block, lds, s, a));
    }
    return hipGetLastError();
}

template <typename T, int N>
static hipError_t launch_axis0_n(const Geo& g, const Item* items, int nitems, int mode, int sub, hipStream_t s)
{
    constexpr int TILE = tile_for<T>(N);
    AxisArgs a;
    a.g = g;
    a.items = items;
    a.ntiles = g.pitch / TILE;
    a.mode = mode;
    a.sub = sub;
    const int planes = (g.ndim == 3) ? g.kept[1] : 1;
    dim3 grid(a.ntiles * planes, nitems);
    dim3 block(TILE * (N / 8));
    const size_t lds = (size_t)TILE * N * 2 * sizeof(T);
    hipLaunchKernelGGL((k_axis0<T, N, TILE>), grid, block, lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_axis0(const Geo& g, const Item* items, int nitems, int mode, int sub, hipStream_t s)
{
    SETD_DISPATCH_N(g.n[0], return (launch_axis0_n<T, NN>(g, items, nitems, mode, sub, s)));
    return hipSuccess;
}

template <typename T, int N>
static hipError_t launch_axis1_n(const Geo& g, const Item* items, int nitems, int dir, int sub, hipStream_t s)
{
    constexpr int TILE = tile_for<T>(N);
    AxisArgs a;
    a.g = g;
    a.items = items;
    a.ntiles = g.pitch / TILE;
    a.mode = dir;
    a.sub = sub;
    dim3 grid(a.ntiles * g.n[0], nitems);
    dim3 block(TILE * (N / 8));
    const size_t lds = (size_t)TILE * N * 2 * sizeof(T);
    hipLaunchKernelGGL((k_axis1<T, N, TILE>), grid, block, lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_axis1(const Geo& g, const Item* items, int nitems, int dir, int sub, hipStream_t s)
{
    SETD_DISPATCH_N(g.n[1], return (launch_axis1_n<T, NN>(g, items, nitems, dir, sub, s)));
    return hipSuccess;
}

template <typename T>
hipError_t launch_linear(const Geo& g, const Item* items, int nitems, int sub, hipStream_t s)
{
    LinArgs a;
    a.g = g;
    a.items = items;
    a.total = g.kept[0] * (g.ndim == 3 ? g.kept[1] : 1) * g.pitch;
    a.sub = sub;
    dim3 grid((a.total + 255) / 256, nitems);
    hipLaunchKernelGGL((k_linear<T>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_observe(const Geo& g, const Item* items, int nitems, int kind, int nbins, double vol,
                          double* acc, hipStream_t s)
{
    ObsArgs a;
    a.g = g;
    a.items = items;
    a.nitems = nitems;
    a.kind = kind;
    a.nbins = nbins;
    a.total = g.kept[0] * (g.ndim == 3 ? g.kept[1] : 1) * g.pitch;
    a.vol = vol;
    a.acc = acc;
    int blocks = (a.total + 255) / 256;
    if (blocks > 128) blocks = 128;
    dim3 grid(blocks, nitems);
    const size_t lds = (size_t)3 * nbins * sizeof(double);
    hipLaunchKernelGGL((k_observe<T>), grid, dim3(256), lds, s, a);
    return hipGetLastError();
}

#define SETD_INSTANTIATE(T)                                                                                     \
    template hipError_t launch_row<T>(const Geo&, const Item*, int, int, int, hipStream_t);                     \
    template hipError_t launch_axis0<T>(const Geo&, const Item*, int, int, int, hipStream_t);                   \
    template hipError_t launch_axis1<T>(const Geo&, const Item*, int, int, int, hipStream_t);                   \
    template hipError_t launch_linear<T>(const Geo&, const Item*, int, int, hipStream_t);                       \
    template hipError_t launch_observe<T>(const Geo&, const Item*, int, int, int, double, double*, hipStream_t);

}  // namespace setd
