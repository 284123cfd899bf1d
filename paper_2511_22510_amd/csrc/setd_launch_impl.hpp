// setd_launch_impl.hpp -- grid shapes and template dispatch of the SETD passes.
//
// Every pass exists in a few variants that the plan's autotuner chooses from:
//   row pass : LDS padding (0 or one slot per 8) x line groups per block
//              (one wavefront or 256 threads)
//   axis pass: (column tile width, columns per thread) in
//              {(tm, 2), (tm, 1), (tm, 4), (tm/2, 1)}, tm = tile_max, with LDS
//              padding whenever the padded tile still fits 64 KiB; the axis-0
//              time step also has the register-update kernel k_axis0r with
//              tile tm/2 (variants 4, 6, 8, 10), tm (5, 7, 9, 11) or tm/4
//              (12 to 15), its items interleaved per column tile in groups of
//              1, 2, 4 or 8
#pragma once

#include <cmath>
#include <cstdlib>

#include "setd_kernels.hpp"
#include "setd_launch.hpp"

namespace setd {

#define SETD_DISPATCH_N(N, CALL)                         \
    switch (N) {                                         \
    case 8: { constexpr int NN = 8; CALL; } break;       \
    case 16: { constexpr int NN = 16; CALL; } break;     \
    case 32: { constexpr int NN = 32; CALL; } break;     \
    case 64: { constexpr int NN = 64; CALL; } break;     \
    case 128: { constexpr int NN = 128; CALL; } break;   \
    case 256: { constexpr int NN = 256; CALL; } break;   \
    case 512: { constexpr int NN = 512; CALL; } break;   \
    case 1024: { constexpr int NN = 1024; CALL; } break; \
    default: return hipErrorInvalidValue;                \
    }

template <typename T, int N, int PAD>
static hipError_t launch_row_np(const Geo& g, const Item* items, int nitems, int mode, int sub, int big_block,
                                int iter, bool kpz, hipStream_t s)
{
    constexpr int tpl = N / 8;
    // KPZ and phase-shift steps hold two lines per row (pair), KPZ with phase
    // shifts four; 256-thread blocks fall back to one wavefront's groups where
    // they would pass 64 KiB, and padded LDS to unpadded where even those would
    const bool ps = g.dealias == 2 && g.ndim >= 2 && mode == MODE_STEP;
    const bool kreal = kpz && !g.cplx;
    const int nlines = (ps && kreal) ? 4 : ((kreal || ps) ? 2 : 1);
    const int small = tpl >= 64 ? 1 : 64 / tpl;
    if constexpr (PAD > 0) {
        if ((size_t)small * lds_len<N, PAD>() * 2 * sizeof(T) * nlines > 65536)
            return launch_row_np<T, N, 0>(g, items, nitems, mode, sub, big_block, iter, kpz, s);
    }
    int lpw = big_block ? (tpl >= 256 ? 1 : 256 / tpl) : small;
    if ((size_t)lpw * lds_len<N, PAD>() * 2 * sizeof(T) * nlines > 65536) lpw = small;
    RowArgs a;
    a.g = g;
    a.items = items;
    a.nrows = (g.ndim == 3) ? g.n[0] * g.n[1] : g.n[0];
    a.lpw = lpw;
    a.iter = (g.cplx || mode != MODE_STEP) ? 1 : iter;
    a.mode = mode;
    a.sub = sub;
    const int lines = g.cplx ? a.nrows : (a.nrows + 1) / 2;
    const int groups = (lines + lpw - 1) / lpw;
    if (ps) {
        // phase shifts: the rows of pre and of its shifted copy (2D) or of the
        // four grids in big (3D), grid z; two (KPZ: four) lines per row group
        // in LDS, one group at a time
        a.iter = 1;
        dim3 gps(groups, nitems, g.ndim == 3 ? 4 : 2);
        const size_t lps = (size_t)lpw * lds_len<N, PAD>() * 2 * sizeof(T) * nlines;
        if (g.cplx) hipLaunchKernelGGL((k_row_cplx<T, N, PAD, false, true>), gps, dim3(lpw * tpl), lps, s, a);
        else if (kreal) hipLaunchKernelGGL((k_row_real<T, N, PAD, 4, false, false>), gps, dim3(lpw * tpl), lps, s, a);
        else hipLaunchKernelGGL((k_row_real<T, N, PAD, 3, false, false>), gps, dim3(lpw * tpl), lps, s, a);
        return hipGetLastError();
    }
    dim3 grid((groups + a.iter - 1) / a.iter, nitems);
    dim3 block(lpw * tpl);
    // KPZ steps hold two lines per row pair
    const size_t lds = (size_t)lpw * lds_len<N, PAD>() * 2 * sizeof(T) * nlines;
    if (g.cplx) {
        if (mode == MODE_IC) hipLaunchKernelGGL((k_row_cplx<T, N, PAD, true>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_row_cplx<T, N, PAD, false>), grid, block, lds, s, a);
    } else if (mode == MODE_IC) {
        if (g.dealias == 1) hipLaunchKernelGGL((k_row_real<T, N, PAD, 2, true, false>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_row_real<T, N, PAD, 2, false, false>), grid, block, lds, s, a);
    } else if (kpz) {
        if (a.iter > 1) {
            if (g.dealias == 1) hipLaunchKernelGGL((k_row_real<T, N, PAD, 1, true, true>), grid, block, lds, s, a);
            else hipLaunchKernelGGL((k_row_real<T, N, PAD, 1, false, true>), grid, block, lds, s, a);
        } else {
            if (g.dealias == 1) hipLaunchKernelGGL((k_row_real<T, N, PAD, 1, true, false>), grid, block, lds, s, a);
            else hipLaunchKernelGGL((k_row_real<T, N, PAD, 1, false, false>), grid, block, lds, s, a);
        }
    } else if (a.iter > 1) {
        if (g.dealias == 1) hipLaunchKernelGGL((k_row_real<T, N, PAD, 0, true, true>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_row_real<T, N, PAD, 0, false, true>), grid, block, lds, s, a);
    } else {
        if (g.dealias == 1) hipLaunchKernelGGL((k_row_real<T, N, PAD, 0, true, false>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_row_real<T, N, PAD, 0, false, false>), grid, block, lds, s, a);
    }
    return hipGetLastError();
}

// var: bit 0 = LDS padding, bit 1 = 256-thread blocks, bits 2-3 = log2 of the
// pair groups a workgroup takes in turn (real-field steps)
template <typename T>
hipError_t launch_row(const Geo& g, const Item* items, int nitems, int mode, int sub, int var, int kpz,
                      hipStream_t s)
{
    const int N = g.n[g.ndim - 1];
    const int big = (var >> 1) & 1;
    const int iter = 1 << ((var >> 2) & 3);
    const bool kp = kpz && mode == MODE_STEP;
    if (var & 1) {
        SETD_DISPATCH_N(N, return (launch_row_np<T, NN, 3>(g, items, nitems, mode, sub, big, iter, kp, s)));
    } else {
        SETD_DISPATCH_N(N, return (launch_row_np<T, NN, 0>(g, items, nitems, mode, sub, big, iter, kp, s)));
    }
    return hipSuccess;
}

template <typename T>
constexpr int tile_max(int n)
{
    return sizeof(T) == 4 ? (n <= 512 ? 16 : 8) : (n <= 512 ? 8 : 4);
}

template <typename T, int N, int TILE>
constexpr int tile_pad()
{
    return (size_t)TILE * lds_len<N, 3>() * 2 * sizeof(T) <= 65536 ? 3 : 0;
}

template <typename T, int N, int TILE, int LPT, bool AX0>
static hipError_t launch_axis_nt(const Geo& g, const Item* items, int nitems, int mode, int sub, bool kpz,
                                 hipStream_t s)
{
    constexpr int PAD = tile_pad<T, N, TILE>();
    AxisArgs a{};
    a.g = g;
    a.items = items;
    a.ntiles = g.pitch / TILE;
    a.per_item = a.ntiles * (AX0 ? ((g.ndim == 3) ? g.kept[1] : 1) : g.n[0]);
    // axis-1 mode -2: the forward transform into the noise intermediate npre
    a.alt = (!AX0 && mode == -2) ? 1 : 0;
    a.mode = a.alt ? -1 : mode;
    a.sub = sub;
    dim3 grid(a.per_item * nitems);
    dim3 block(TILE / LPT * (N / 8));
    const size_t lds = (size_t)TILE * lds_len<N, PAD>() * 2 * sizeof(T);
    if (AX0 && kpz) hipLaunchKernelGGL((k_axis0<T, N, TILE, PAD, true, LPT, false>), grid, block, lds, s, a);
    else if (AX0) hipLaunchKernelGGL((k_axis0<T, N, TILE, PAD, false, LPT, false>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((k_axis1<T, N, TILE, PAD, LPT>), grid, block, lds, s, a);
    return hipGetLastError();
}

// axis-0 pass of a plan with phase-shift dealiasing (k_axis0 with PS): the
// half-width tile, one column per thread, LDS for the lines and their shifted
// copies (padded only where both halves fit 64 KiB)
template <typename T, int N>
static hipError_t launch_axis0_ps(const Geo& g, const Item* items, int nitems, int mode, int sub, bool kpz,
                                  hipStream_t s)
{
    constexpr int TILE = tile_max<T>(N) / 2;
    constexpr int PAD = ((size_t)2 * TILE * lds_len<N, 3>() * 2 * sizeof(T) <= 65536) ? 3 : 0;
    constexpr size_t lds = (size_t)2 * TILE * lds_len<N, PAD>() * 2 * sizeof(T);
    static_assert(lds <= 65536, "phase-shift axis-0 tile exceeds 64 KiB of LDS");
    AxisArgs a{};
    a.g = g;
    a.items = items;
    a.ntiles = g.pitch / TILE;
    a.per_item = a.ntiles * ((g.ndim == 3) ? g.kept[1] : 1);
    a.mode = mode;
    a.sub = sub;
    if (kpz && g.ndim == 2)
        hipLaunchKernelGGL((k_axis0<T, N, TILE, PAD, true, 1, true>), dim3(a.per_item * nitems), dim3(TILE * (N / 8)),
                           lds, s, a);
    else
        hipLaunchKernelGGL((k_axis0<T, N, TILE, PAD, false, 1, true>), dim3(a.per_item * nitems), dim3(TILE * (N / 8)),
                           lds, s, a);
    return hipGetLastError();
}

// axis-1 passes of a 3D step with phase shifts (k_axis1 with PS): dir +1 takes
// pre and preb (grid z) to the four grids of big, -1 back; the half-width tile,
// one column per thread, two lines side by side in LDS
template <typename T, int N>
static hipError_t launch_axis1_ps(const Geo& g, const Item* items, int nitems, int dir, int sub, hipStream_t s)
{
    constexpr int TILE = tile_max<T>(N) / 2;
    constexpr int PAD = ((size_t)2 * TILE * lds_len<N, 3>() * 2 * sizeof(T) <= 65536) ? 3 : 0;
    constexpr size_t lds = (size_t)2 * TILE * lds_len<N, PAD>() * 2 * sizeof(T);
    static_assert(lds <= 65536, "phase-shift axis-1 tile exceeds 64 KiB of LDS");
    AxisArgs a{};
    a.g = g;
    a.items = items;
    a.ntiles = g.pitch / TILE;
    a.per_item = a.ntiles * g.n[0];
    a.mode = dir;
    a.sub = sub;
    hipLaunchKernelGGL((k_axis1<T, N, TILE, PAD, 1, true>), dim3(a.per_item * nitems, 1, 2), dim3(TILE * (N / 8)),
                       lds, s, a);
    return hipGetLastError();
}

// Hermitian planes of a real field's state array (which: 0 phi, 1 the F_{n-1}
// array / SETD2 carry); no-op for complex fields
template <typename T>
static hipError_t launch_hermitian_t(const Geo& g, const Item* items, int nitems, int which, int sub, hipStream_t s)
{
    if (g.cplx) return hipSuccess;
    HermArgs a;
    a.g = g;
    a.items = items;
    a.which = which;
    a.nplane = geo_rows(g);
    a.ncol = (2 * g.kp[g.ndim - 1] == g.n[g.ndim - 1]) ? 2 : 1;
    a.sub = sub;
    dim3 grid((a.nplane * a.ncol + 255) / 256, nitems);
    hipLaunchKernelGGL((k_hermitian<T>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// axis-0 pass with the update in registers (k_axis0r), one column per thread group
template <typename T, int N, int TILE>
static hipError_t launch_axis0r(const Geo& g, const Item* items, int nitems, int mode, int sub, bool kpz,
                                bool lean, int group, hipStream_t s)
{
    constexpr int PAD = tile_pad<T, N, TILE>();
    AxisArgs a{};
    a.g = g;
    a.items = items;
    a.ntiles = g.pitch / TILE;
    a.per_item = a.ntiles * ((g.ndim == 3) ? g.kept[1] : 1);
    a.mode = mode;
    a.sub = sub;
    dim3 grid(a.per_item * nitems);
    dim3 block(TILE * (N / 8));
    size_t lds = (size_t)TILE * lds_len<N, PAD>() * 2 * sizeof(T);
    // 3D lattices key their coefficients by |a|: the block stages the entries
    // of |a0| <= K0 for its columns in LDS when they fit in 64 KiB
    const size_t tab = (size_t)(g.kp[0] + 1) * TILE * (g.cplx ? 8 : 4) * sizeof(T);
    a.ctab = (g.ndim == 3 && tab <= 65536) ? 1 : 0;
    if (a.ctab && tab > lds) lds = tab;
    a.group = group < 1 ? 1 : (group > nitems ? nitems : group);
    if (lean) {
        if (g.cplx) hipLaunchKernelGGL((k_axis0r<T, N, TILE, PAD, 2, true>), grid, block, lds, s, a);
        else if (kpz) hipLaunchKernelGGL((k_axis0r<T, N, TILE, PAD, 1, true>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_axis0r<T, N, TILE, PAD, 0, true>), grid, block, lds, s, a);
    } else {
        if (g.cplx) hipLaunchKernelGGL((k_axis0r<T, N, TILE, PAD, 2, false>), grid, block, lds, s, a);
        else if (kpz) hipLaunchKernelGGL((k_axis0r<T, N, TILE, PAD, 1, false>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_axis0r<T, N, TILE, PAD, 0, false>), grid, block, lds, s, a);
    }
    return hipGetLastError();
}

template <typename T, int N, bool AX0>
static hipError_t launch_axis_n(const Geo& g, const Item* items, int nitems, int mode, int sub, int var,
                                bool kpz, bool lean, hipStream_t s)
{
    constexpr int TM = tile_max<T>(N);
    if constexpr (AX0) {
        // the register-update kernel does the time step under the 2/3 rule,
        // with buffer accesses into arrays of under 2 GiB per realization
        // (axis0_register_ok); other modes and plans take the tile-sweep
        // kernel.  A plan keeping the SETD2 carry steps with the register
        // kernel only.
        // variants 4 + 2j (tile TM/2), 5 + 2j (tile TM) and 12 + j (tile TM/4),
        // j = 0..3: items interleaved in groups of 2^j per column tile
        const bool reg = mode == MODE_STEP && axis0_register_ok(g, sizeof(T));
        if (reg && lean && var < 4) var = 4;
        if (reg && var >= 4) {
            const int group = 1 << (var >= 12 ? var - 12 : (var - 4) / 2);
            hipError_t e = (var >= 12) ? launch_axis0r<T, N, (TM >= 4 ? TM / 4 : 1)>(g, items, nitems, mode, sub, kpz, lean, group, s)
                           : ((var - 4) % 2 == 0)
                               ? launch_axis0r<T, N, (TM >= 2 ? TM / 2 : 1)>(g, items, nitems, mode, sub, kpz, lean, group, s)
                               : launch_axis0r<T, N, TM>(g, items, nitems, mode, sub, kpz, lean, group, s);
            // the register kernel keeps a 2D real field's column a_last = 0
            // Hermitian itself; 3D planes span several blocks
            if (e == hipSuccess && g.ndim == 3) e = launch_hermitian_t<T>(g, items, nitems, lean ? 1 : 0, sub, s);
            return e;
        }
        if (var >= 4) var = (var >= 12 || (var - 4) % 2 == 0) ? 3 : 0;
        if (g.dealias == 2) {
            hipError_t e = launch_axis0_ps<T, N>(g, items, nitems, mode, sub, kpz, s);
            if (e == hipSuccess && (mode == MODE_STEP || mode == MODE_IC || mode == MODE_RSN))
                e = launch_hermitian_t<T>(g, items, nitems, mode == MODE_RSN ? 2 : 0, sub, s);
            return e;
        }
    }
    hipError_t e;
    switch (var) {
    case 0: e = launch_axis_nt<T, N, TM, 2, AX0>(g, items, nitems, mode, sub, kpz, s); break;
    case 1: e = launch_axis_nt<T, N, TM, 1, AX0>(g, items, nitems, mode, sub, kpz, s); break;
    case 2: e = launch_axis_nt<T, N, TM, 4, AX0>(g, items, nitems, mode, sub, kpz, s); break;
    default: e = launch_axis_nt<T, N, TM / 2, 1, AX0>(g, items, nitems, mode, sub, kpz, s); break;
    }
    // the state a step or an initial condition wrote, or the transformed
    // real-space noise: Hermitian planes
    if (AX0 && e == hipSuccess && (mode == MODE_STEP || mode == MODE_IC || mode == MODE_RSN))
        e = launch_hermitian_t<T>(g, items, nitems, mode == MODE_RSN ? 2 : 0, sub, s);
    return e;
}

template <typename T>
hipError_t launch_axis0(const Geo& g, const Item* items, int nitems, int mode, int sub, int var, int kpz,
                        int lean, hipStream_t s)
{
    SETD_DISPATCH_N(g.n[0], return (launch_axis_n<T, NN, true>(g, items, nitems, mode, sub, var, kpz != 0,
                                                                lean != 0, s)));
    return hipSuccess;
}

template <typename T>
hipError_t launch_hermitian(const Geo& g, const Item* items, int nitems, int which, hipStream_t s)
{
    return launch_hermitian_t<T>(g, items, nitems, which, 0, s);
}

template <typename T>
hipError_t launch_axis1(const Geo& g, const Item* items, int nitems, int dir, int sub, int var, hipStream_t s)
{
    // dir +3 / -3: the phase-shift passes of a step (pre, preb <-> four grids)
    if (dir == 3 || dir == -3) {
        if (g.ndim != 3 || g.dealias != 2) return hipErrorInvalidValue;
        SETD_DISPATCH_N(g.n[1], return (launch_axis1_ps<T, NN>(g, items, nitems, dir / 3, sub, s)));
    }
    SETD_DISPATCH_N(g.n[1], return (launch_axis_n<T, NN, false>(g, items, nitems, dir, sub, var, false, false, s)));
    return hipSuccess;
}

// last-axis pass of the real-space noise (k_rsn_rows): thread groups of N/8
// threads, as many per block as fit 256 threads and 32 KiB of LDS
template <typename T, int N>
static hipError_t launch_rsn_rows_n(const Geo& g, const Item* items, int nitems, int sub, hipStream_t s)
{
    constexpr int TPL = N / 8, PAD = 3;
    constexpr int BY_THREADS = TPL >= 256 ? 1 : 256 / TPL;
    constexpr int BY_LDS = 32768 / (2 * lds_len<N, PAD>() * (int)sizeof(cx<T>));
    constexpr int CAP = BY_THREADS < BY_LDS ? BY_THREADS : BY_LDS;
    constexpr int LPB = CAP >= 1 ? (1 << ilog2(CAP)) : 1;
    RsnArgs a;
    a.g = g;
    a.items = items;
    a.nrows = (g.ndim == 3) ? g.n[0] * g.n[1] : g.n[0];
    a.ngroups = g.cplx ? a.nrows / 2 : a.nrows / 4;
    a.lpb = LPB;
    a.sub = sub;
    double sites = 1.0;
    for (int i = 0; i < g.ndim; i++) sites *= (double)g.n[i];
    a.scale = (g.cplx ? std::sqrt(0.5) : 1.0) / std::sqrt(sites);
    dim3 grid((a.ngroups + LPB - 1) / LPB, nitems);
    dim3 block(LPB * TPL);
    const size_t lds = (size_t)LPB * 2 * lds_len<N, PAD>() * sizeof(cx<T>);
    if (g.cplx) hipLaunchKernelGGL((k_rsn_rows<T, N, PAD, true>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((k_rsn_rows<T, N, PAD, false>), grid, block, lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rsn(const Geo& g, const Item* items, int nitems, int sub, int var1, int var0, hipStream_t s)
{
    if (g.ndim < 2 || !g.rsn) return hipErrorInvalidValue;
    hipError_t e = hipErrorInvalidValue;
    SETD_DISPATCH_N(g.n[g.ndim - 1], e = (launch_rsn_rows_n<T, NN>(g, items, nitems, sub, s)));
    if (e != hipSuccess) return e;
    if (g.ndim == 3) {
        SETD_DISPATCH_N(g.n[1], e = (launch_axis_n<T, NN, false>(g, items, nitems, -2, sub, var1, false, false, s)));
        if (e != hipSuccess) return e;
    }
    // the axis-0 transform writes eta_a into the noise array and keeps a real
    // field's Hermitian planes
    SETD_DISPATCH_N(g.n[0], e = (launch_axis_n<T, NN, true>(g, items, nitems, MODE_RSN, sub, var0, false, false, s)));
    return e;
}

template <typename T>
hipError_t launch_multi2d(const MultiClass (&cls)[4], int pass, int sub, hipStream_t s)
{
    static_assert(MULTI_SLOTS == 4, "one class slot per lattice size 64..512");
    int total = 0;
    if (pass == 0) {
        MultiRowArgs m{};
        for (int k = 0; k < MULTI_SLOTS; k++) {
            const int N = 64 << k, lpw = 256 / (N / 8);
            m.first[k] = total;
            RowArgs& a = m.a[k];
            a.g = cls[k].g;
            a.items = cls[k].items;
            a.nrows = N;
            a.lpw = lpw;
            a.iter = 1;
            a.mode = MODE_STEP;
            a.sub = sub;
            m.gx[k] = (N / 2 + lpw - 1) / lpw;
            if (cls[k].nitems > 0 && (cls[k].g.n[0] != N || cls[k].g.n[1] != N)) return hipErrorInvalidValue;
            total += cls[k].nitems * m.gx[k];
        }
        m.first[MULTI_SLOTS] = total;
        if (total == 0) return hipSuccess;
        // lpw lines of N + N/8 elements: 2048/N x 9N/8 = 2304 at every size
        hipLaunchKernelGGL((k_row_multi<T>), dim3(total), dim3(256), (size_t)2304 * sizeof(cx<T>), s, m);
    } else {
        MultiAxArgs m{};
        for (int k = 0; k < MULTI_SLOTS; k++) {
            const int tile = multi_tile(k), subs = multi_sub(k);
            m.first[k] = total;
            AxisArgs& a = m.a[k];
            a.g = cls[k].g;
            a.items = cls[k].items;
            m.bpi[k] = cls[k].nitems > 0 ? (cls[k].g.pitch / tile + subs - 1) / subs : 0;
            a.ntiles = m.bpi[k] * subs;
            a.per_item = m.bpi[k] * subs;
            a.mode = MODE_STEP;
            a.sub = sub;
            if (cls[k].nitems > 0 && cls[k].g.pitch % tile != 0) return hipErrorInvalidValue;
            total += cls[k].nitems * m.bpi[k];
        }
        m.first[MULTI_SLOTS] = total;
        if (total == 0) return hipSuccess;
        // 36 KiB at every size: tile x (N + N/8) elements x 2 reals
        hipLaunchKernelGGL((k_axis0_multi<T>), dim3(total), dim3(512), (size_t)8 * 576 * 2 * sizeof(T), s, m);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_linear(const Geo& g, const Item* items, int nitems, int sub, int mode, int64_t new_step,
                         hipStream_t s)
{
    LinArgs a;
    a.g = g;
    a.items = items;
    a.total = geo_rows(g) * g.pitch;
    a.sub = sub;
    a.mode = mode;
    a.new_step = new_step;
    dim3 grid((a.total + 255) / 256, nitems);
    hipLaunchKernelGGL((k_linear<T>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// 1D lattices: one launch takes nsteps steps (MODE_STEP) or draws the initial
// condition (MODE_IC)
template <typename T, int N, int DM, bool RS>
static hipError_t launch_line1d_n(const Geo& g, const Item* items, int nitems, int mode, int sub, int nsteps,
                                  int nl, hipStream_t s)
{
    // FP32 lines pad LDS by one slot per 8 (fewer bank conflicts in the
    // exchanges); FP64 lines would exceed 64 KiB of LDS with it
    constexpr int TPL = N / 8, LPB = 256 / TPL, PAD = sizeof(T) == 4 ? 3 : 0;
    constexpr int LL = lds_len<N, PAD>();
    Line1dArgs a;
    a.g = g;
    a.items = items;
    a.nitems = nitems;
    a.mode = mode;
    a.sub = sub;
    a.nsteps = nsteps;
    if (g.cplx) {
        a.nlines = nitems;
        const dim3 grid((unsigned)((a.nlines + LPB - 1) / LPB));
        const size_t lds = (size_t)LPB * ((RS || DM == 2) ? 2 : 1) * LL * sizeof(cx<T>);
        if (nl == NL_NONE) hipLaunchKernelGGL((k_line1d_cplx<T, N, PAD, DM, 1, RS>), grid, dim3(256), lds, s, a);
        else hipLaunchKernelGGL((k_line1d_cplx<T, N, PAD, DM, 0, RS>), grid, dim3(256), lds, s, a);
        return hipGetLastError();
    }
    a.nlines = (nitems + 1) / 2;
    const dim3 grid((unsigned)((a.nlines + LPB - 1) / LPB));
    const size_t lds = (size_t)LPB * 2 * LL * sizeof(cx<T>);
    if (nl == NL_KPZ) hipLaunchKernelGGL((k_line1d_real<T, N, PAD, DM, 1, RS>), grid, dim3(256), lds, s, a);
    else if (nl == NL_NONE) hipLaunchKernelGGL((k_line1d_real<T, N, PAD, DM, 2, RS>), grid, dim3(256), lds, s, a);
    else hipLaunchKernelGGL((k_line1d_real<T, N, PAD, DM, 0, RS>), grid, dim3(256), lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_line1d(const Geo& g, const Item* items, int nitems, int mode, int sub, int nsteps, int nl,
                         hipStream_t s)
{
    if (g.ndim != 1 || nitems <= 0) return hipErrorInvalidValue;
    // dealias 0 none, 1 the 2/3 rule, 2 phase shift
    if (g.dealias == 2 && g.rsn) {
        SETD_DISPATCH_N(g.n[0], return (launch_line1d_n<T, NN, 2, true>(g, items, nitems, mode, sub, nsteps, nl, s)));
    } else if (g.dealias == 1 && g.rsn) {
        SETD_DISPATCH_N(g.n[0], return (launch_line1d_n<T, NN, 1, true>(g, items, nitems, mode, sub, nsteps, nl, s)));
    } else if (g.dealias == 1) {
        SETD_DISPATCH_N(g.n[0], return (launch_line1d_n<T, NN, 1, false>(g, items, nitems, mode, sub, nsteps, nl, s)));
    } else if (g.dealias == 2) {
        SETD_DISPATCH_N(g.n[0], return (launch_line1d_n<T, NN, 2, false>(g, items, nitems, mode, sub, nsteps, nl, s)));
    } else if (g.rsn) {
        SETD_DISPATCH_N(g.n[0], return (launch_line1d_n<T, NN, 0, true>(g, items, nitems, mode, sub, nsteps, nl, s)));
    } else {
        SETD_DISPATCH_N(g.n[0], return (launch_line1d_n<T, NN, 0, false>(g, items, nitems, mode, sub, nsteps, nl, s)));
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_boxwidth(const BoxArgs& a, size_t ncls, hipStream_t s)
{
    int blocks = (a.total + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL((k_boxclass<T>), dim3(blocks), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t fb = (ncls + 255) / 256;
    if (fb > 1024) fb = 1024;
    hipLaunchKernelGGL(k_boxfinal, dim3((unsigned)fb), dim3(256), 0, s, a, ncls);
    return hipGetLastError();
}

template <typename T, int M>
static hipError_t launch_spectrum_m(const SpecArgs& a0, hipStream_t s)
{
    SpecArgs a = a0;
    constexpr int PAD = 3;
    constexpr int tpl = M / 8;
    const int lpb = tpl >= 256 ? 1 : 256 / tpl;
    dim3 grid((a.total + lpb - 1) / lpb, a.nitems);
    const size_t lds = (size_t)lpb * 2 * lds_len<M, PAD>() * 2 * sizeof(T);
    hipLaunchKernelGGL((k_spectrum<T, M, PAD>), grid, dim3(lpb * tpl), lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spectrum(const SpecArgs& a, int M, hipStream_t s)
{
    SETD_DISPATCH_N(M, return (launch_spectrum_m<T, NN>(a, s)));
    return hipSuccess;
}

template <typename T>
hipError_t launch_fdt_reduce(const Geo& g, const double* dacc, int total, int M, double* out, hipStream_t s)
{
    size_t blocks = ((size_t)total * M + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_fdt_reduce, dim3((unsigned)blocks), dim3(256), 0, s, g, dacc, total, M, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_observe(const Geo& g, const Item* items, int nitems, int kind, int nbins, double vol,
                          double* acc, int64_t kick, hipStream_t s)
{
    ObsArgs a;
    a.g = g;
    a.items = items;
    a.nitems = nitems;
    a.kind = kind;
    a.nbins = nbins;
    a.total = geo_rows(g) * g.pitch;
    a.vol = vol;
    a.acc = acc;
    a.kick = kick;
    int blocks = (a.total + 255) / 256;
    if (blocks > 128) blocks = 128;
    dim3 grid(blocks, nitems);
    const size_t lds = (size_t)3 * nbins * sizeof(double);
    hipLaunchKernelGGL((k_observe<T>), grid, dim3(256), lds, s, a);
    return hipGetLastError();
}

#define SETD_INSTANTIATE(T)                                                                                     \
    template hipError_t launch_row<T>(const Geo&, const Item*, int, int, int, int, int, hipStream_t);           \
    template hipError_t launch_axis0<T>(const Geo&, const Item*, int, int, int, int, int, int, hipStream_t);    \
    template hipError_t launch_axis1<T>(const Geo&, const Item*, int, int, int, int, hipStream_t);              \
    template hipError_t launch_linear<T>(const Geo&, const Item*, int, int, int, int64_t, hipStream_t);         \
    template hipError_t launch_observe<T>(const Geo&, const Item*, int, int, int, double, double*, int64_t, hipStream_t); \
    template hipError_t launch_spectrum<T>(const SpecArgs&, int, hipStream_t);                                    \
    template hipError_t launch_fdt_reduce<T>(const Geo&, const double*, int, int, double*, hipStream_t);         \
    template hipError_t launch_boxwidth<T>(const BoxArgs&, size_t, hipStream_t);                                  \
    template hipError_t launch_hermitian<T>(const Geo&, const Item*, int, int, hipStream_t);                      \
    template hipError_t launch_rsn<T>(const Geo&, const Item*, int, int, int, int, hipStream_t);

// the 1D line kernels, in translation units of their own (they compile in
// parallel with the others)
#define SETD_INSTANTIATE_LINES(T) \
    template hipError_t launch_line1d<T>(const Geo&, const Item*, int, int, int, int, int, hipStream_t);

}  // namespace setd
