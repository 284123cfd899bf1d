// setd_kernels.hpp -- kernels of one SETD time step on gfx950.
//
// A step of the pseudo-spectral algorithm (Sec. 4, algorithm box) is split
// into passes over lines of the lattice, each line transform held in
// registers and LDS (setd_device.hpp):
//
//   2D:  row pass (last axis)  : pre -> inverse FFT -> N[phi] -> forward FFT -> pre
//        axis-0 pass           : pre -> forward FFT -> F_a, ETD update with noise
//                                (Eq. SETD1 / SETD2) -> inverse FFT -> pre
//   3D:  axis-1 inverse, row pass, axis-1 forward, axis-0 pass.
//
// Between steps every realization keeps its stored spectral state phi (only
// the modes the 2/3 rule keeps), its previous nonlinear term (SETD2) and
// `pre`, the axis-0 inverse transform of phi restricted to the stored columns.
// All arrays are stored in the state precision; the last axis is padded to
// `pitch` so that every line segment starts on a 128-byte boundary.
#pragma once

#include <type_traits>

#include "setd_device.hpp"

namespace setd {

// ---------------------------------------------------------------- index maps
// signed wavenumber index of FFT position j on an axis of length n
__device__ __forceinline__ int sgn_idx(int j, int n) { return j < n / 2 ? j : j - n; }

// FFT position of stored index i on a full axis (low side 0..kp, then the top)
__device__ __forceinline__ int fft_pos(int i, int n, int kept, int kp) { return i <= kp ? i : i + n - kept; }

// stored index of FFT position j on a full axis, -1 if dealiased away
__device__ __forceinline__ int stored_idx(int j, int n, int kept, int kp)
{
    if (j <= kp) return j;
    const int i = j - n + kept;
    return i > kp ? i : -1;
}

__device__ __forceinline__ int ceil_isqrt(int m)
{
    if (m <= 0) return 0;
    int s = (int)sqrt((double)m);
    while (s * s > m) s--;
    while ((s + 1) * (s + 1) <= m) s++;
    return s * s == m ? s : s + 1;
}

// e^{i pi x}
template <typename T>
__device__ __forceinline__ cx<T> cispi(T x)
{
    T s, c;
    if constexpr (sizeof(T) == 4) sincospif(x, &s, &c);
    else sincospi(x, &s, &c);
    return {c, s};
}

// ---------------------------------------------------------------- coefficients
template <typename T>
struct Coef {
    cx<T> E, wa, wb;
    T G;
};

template <typename T>
__device__ __forceinline__ Coef<T> load_coef(const Item& it, int key)
{
    Coef<T> r;
    if (it.coef_cplx) {
        const T4<T>* p = reinterpret_cast<const T4<T>*>(it.coef) + 2 * (size_t)key;
        const T4<T> u = p[0], w = p[1];
        r.E = {u.a, u.b};
        r.wa = {u.c, u.d};
        r.wb = {w.a, w.b};
        r.G = w.c;
    } else {
        const T4<T> u = reinterpret_cast<const T4<T>*>(it.coef)[key];
        r.E = {u.a, T(0)};
        r.wa = {u.b, T(0)};
        r.wb = {u.c, T(0)};
        r.G = u.d;
    }
    return r;
}

// the same with the table's entry type known at compile time, through global
// loads at a 32-bit offset
template <typename T, bool CC>
__device__ __forceinline__ Coef<T> load_coef_t(const void* coef, int key)
{
    Coef<T> r;
    if constexpr (CC) {
        const uint32_t o = (uint32_t)key * (uint32_t)(8 * sizeof(T));
        const T4<T> u = gload4<T>(coef, o), w = gload4<T>(coef, o + 4 * sizeof(T));
        r.E = {u.a, u.b};
        r.wa = {u.c, u.d};
        r.wb = {w.a, w.b};
        r.G = w.c;
    } else {
        const T4<T> u = gload4<T>(coef, (uint32_t)key * (uint32_t)(4 * sizeof(T)));
        r.E = {u.a, T(0)};
        r.wa = {u.b, T(0)};
        r.wb = {u.c, T(0)};
        r.G = u.d;
    }
    return r;
}

// key of a mode in a shell-indexed table: |a|^2 (equal dk on every axis) or
// the separable (|a0|, |a1|, |a2|) index
// entry of a 2D lattice's per-mode table: row |a0| (c(k) and D(k) depend on
// k0 through k0^2 only, so a0 and -a0 share a row), column of the stored last axis
__device__ __forceinline__ int per_mode_key(const Geo& g, int a0, int col)
{
    return (a0 < 0 ? -a0 : a0) * g.pitch + col;
}

__device__ __forceinline__ int coef_key(const Item& it, int a0, int a1, int a2)
{
    if (it.coef_mode == COEF_ISO) return a0 * a0 + a1 * a1 + a2 * a2;
    return (abs(a0) * it.keydim[1] + abs(a1)) * it.keydim[2] + abs(a2);
}

// Fourier-space prefactor of the transformed nonlinearity (Sec. 5)
template <typename T>
__device__ __forceinline__ cx<T> nl_pref(const Item& it, T k2)
{
    const T p = (T)it.par0;
    switch (it.nl) {
    case NL_PHI3: return {-p, T(0)};
    case NL_PHI3_CONS: return {-p * k2, T(0)};
    case NL_KPZ: return {T(0.5) * p, T(0)};
    case NL_CGL: return {T(-1), -p};
    default: return {T(0), T(0)};
    }
}

// ---------------------------------------------------------------- noise (App. B)
// Unit noise eta_a of the stored modes for step n.  Complex modes draw
// (z1 + i z2)/sqrt2; on the a_d in {0, N_d/2} planes of a real field a
// self-conjugate mode takes z1 and a conjugate pair draws once, at the member
// with the smaller linear index, the other taking the conjugate.
// Draws are made for pairs of modes that differ only in the axis-0 position,
// j and j' = (j mod M) + (7 - j div M) M with M = N0/8 (bins q and 7 - q of
// one thread of the axis-0 pass): the pair's Philox counter is (P, n, r, 0),
// P the linear index of the member with j div M < 4 over the axis-0 extent
// N0/2, and that member takes words (x0, x1), the other (x2, x3).
struct NoiseSlot {
    uint32_t P;      // Philox counter word 0
    uint32_t half;   // 0: words (x0, x1), 1: words (x2, x3)
    int kind;        // 0: (z1 + i z2)/sqrt2, 1: z1, 2: (z1 - i z2)/sqrt2 drawn at the partner
};

__device__ __forceinline__ NoiseSlot noise_slot(const Geo& g, int j0, int j1, int jl)
{
    if (g.ndim == 1) {
        // one axis, position jl, M = N/8: a real line pairs a with a + 2M (the
        // Nyquist mode draws alone from block 2M, a = 0 and N/2 take z1); a
        // complex line pairs j with (j mod M) + (7 - j div M) M
        const int N = g.n[0], sh = __ffs(N) - 4, M = 1 << sh;
        NoiseSlot s;
        if (!g.cplx) {
            const int q = jl >> sh;
            s.kind = (jl == 0 || 2 * jl == N) ? 1 : 0;
            s.P = (2 * jl == N) ? (uint32_t)(2 * M) : (uint32_t)((jl & (M - 1)) + (q & 1) * M);
            s.half = (2 * jl == N) ? 0u : (uint32_t)(q >> 1);
        } else {
            const int q = jl >> sh;
            s.kind = 0;
            s.P = (uint32_t)((jl & (M - 1)) + ((q < 4 ? q : 7 - q) << sh));
            s.half = q >= 4 ? 1u : 0u;
        }
        return s;
    }
    const int last = g.ndim - 1;
    int d0 = j0, d1 = j1, kind = 0;
    if (!g.cplx && !(jl > 0 && 2 * jl < g.n[last])) {
        const int p0 = j0 ? g.n[0] - j0 : 0;
        const int p1 = (g.ndim == 3 && j1) ? g.n[1] - j1 : 0;
        if (p0 == j0 && p1 == j1) {
            kind = 1;
        } else if (p0 < j0 || (p0 == j0 && p1 < j1)) {
            kind = 2;
            d0 = p0;
            d1 = p1;
        }
    }
    // M = N0/8 is a power of two (lattice extents are)
    const int sh = g.n[0] >= 8 ? __ffs(g.n[0]) - 4 : 0;
    const int q = d0 >> sh;
    const uint32_t row = (uint32_t)(d0 - (q << sh) + ((q < 4 ? q : 7 - q) << sh));
    NoiseSlot s;
    s.P = ((g.ndim == 3) ? row * (uint32_t)g.n[1] + (uint32_t)d1 : row) * (uint32_t)g.nh_last + (uint32_t)jl;
    s.half = q >= 4 ? 1u : 0u;
    s.kind = kind;
    return s;
}

template <typename T>
__device__ __forceinline__ cx<T> eta_of(const uint32_t (&x)[4], const NoiseSlot& s)
{
    const T rs2 = T(0.70710678118654752440084436210484903928);
    T z1, z2;
    box_muller32(s.half ? x[2] : x[0], s.half ? x[3] : x[1], z1, z2);
    if (s.kind == 1) return {z1, T(0)};
    return {rs2 * z1, (s.kind == 2) ? -rs2 * z2 : rs2 * z2};
}

// one mode (one Philox block)
template <typename T>
__device__ __forceinline__ cx<T> noise_eta(const Geo& g, const Item& it, int j0, int j1, int jl, uint32_t n)
{
    const NoiseSlot s = noise_slot(g, j0, j1, jl);
    uint32_t x[4];
    philox_block(it.seed, s.P, n, it.r, 0u, x);
    return eta_of<T>(x, s);
}

// ---------------------------------------------------------------- step counter
// Called by thread 0 of every block of a realization's pass, after a block
// barrier (so every thread of the block has read the step counter): the last
// block to arrive advances the realization's step and marks its history valid.
// The counter is read only at the start of the next launch, and consecutive
// launches on a stream are ordered for all memory, so no fence is needed; a
// device-scope fence here would write back the whole L2 of the XCD from every
// block.
__device__ __forceinline__ void advance_step(Ctrl* c, unsigned blocks, int64_t nstep)
{
    const unsigned prior = atomicAdd(&c->done, 1u);
    if (prior == blocks - 1u) {
        atomicExch(&c->done, 0u);
        atomicExch(reinterpret_cast<unsigned long long*>(&c->step), (unsigned long long)(nstep + 1));
        atomicExch(&c->have_prev, 1);
    }
}

// ---------------------------------------------------------------- launch arguments
struct RowArgs {
    Geo g;
    const Item* items;
    int nrows;   // lines of the last axis per realization (n0 or n0*n1)
    int lpw;     // line groups per workgroup (row pairs for real fields)
    int iter;    // real fields: groups of lpw pairs a workgroup takes in turn
    int mode;    // MODE_STEP or MODE_IC
    int sub;     // sub-step of the scheduler tick
};

struct AxisArgs {
    Geo g;
    const Item* items;
    int ntiles;    // column tiles across the padded last axis
    int per_item;  // blocks per realization
    int mode;      // axis-0 pass: MODE_STEP / MODE_IC / MODE_SYNC; axis-1 pass: +1 inverse, -1 forward
    int sub;
    int ctab;      // register axis-0 kernel, keyed coefficients: stage them in LDS (the launch sized it)
    int alt;       // axis-1 pass: the noise intermediate npre in place of pre0
    int group;     // register axis-0 kernel: items interleaved per column tile (1: item after item)
};

struct LinArgs {
    Geo g;
    const Item* items;
    int total;   // stored elements per realization
    int sub;
    int mode;          // LIN_STEP / LIN_CARRY / LIN_RENOISE
    int64_t new_step;  // LIN_RENOISE: the step index the carry's noise is re-drawn for
};

template <typename T>
__device__ __forceinline__ const cx<T>* twid(const void* p) { return reinterpret_cast<const cx<T>*>(p); }

// Workgroups are dealt round-robin to the 8 XCDs.  Give every XCD a contiguous
// range of logical blocks, so that neighbouring column tiles (which can share
// 128-byte lines) meet in the same L2.
__device__ __forceinline__ unsigned xcd_logical(unsigned L, unsigned G)
{
    if (G % 8u != 0u) return L;
    return (L % 8u) * (G / 8u) + L / 8u;
}

// ---------------------------------------------------------------- row pass, real field
// Two real rows a, b travel as one complex line z = a + i b: the inverse uses
// Z_k = A_k + i B_k (k <= N/2) and conj(A_{N-k}) + i conj(B_{N-k}) above; the
// forward splits Z back into A_k = (Z_k + conj Z_{N-k})/2 and
// B_k = (Z_k - conj Z_{N-k})/(2i).  Block: lpw row pairs x N/8 threads; it
// takes iter consecutive groups of lpw pairs in turn.  With PF (prefetch) the
// loads of the next group are issued, into the registers the current group
// has just consumed, before the current group's transforms, so that the
// block's memory traffic overlaps its arithmetic (at the price of those
// registers).
// Rows are read and written with buffer accesses relative to the block's first
// row (the resource covers the block's rows that exist); a lane whose bin has
// no stored mode uses BUF_OOB, reads zero and writes nothing, so the loads are
// unconditional and all in flight together.
// KIND: 0 = phi^3 (Model A/B) step, 1 = KPZ step, 2 = initial condition,
// 3 = phi^3 step with phase shifts (dealias 2): the packed line and its copy
// moved by dx/2 along the row (e^{i pi a/N} per bin) go through the stages
// together and their transforms are averaged, the second moved back; 2D: rows
// of pre (sel 0) or of its axis-0-shifted copy preb (sel 1); 3D: rows of grid
// sel of the four grids in big; 4 = KPZ step with phase shifts (2D): the two
// rows' gradient lines and their copies moved along the row (four lines)
// through the inverse stages together, the squares of each pair packed, both
// packed lines forward and averaged, the second moved back; rows of pre and
// pre1 (sel 0) or of preb and pre1b (sel 1).
// DA: the 2/3 rule is on; then bins q = 0, 1 (k < N/4) always hold a stored
// mode, q = 6, 7 (k >= 3N/4) always its mirror, q = 3, 4 never any, and only
// q = 0..2 are written back, all decided at compile time.
// The body takes the block's grid position (bx, by) and thread: the kernel
// below passes its own, the shared launch of several lattice classes its
// position within the class.
template <typename T, int N, int PAD, int KIND, bool DA, bool PF>
__device__ __forceinline__ void row_real_body(const RowArgs& a, const int bx, const int by, const int tid,
                                              const int sel = 0)
{
    const Item it = a.items[by];
    if (a.sub >= it.steps) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    constexpr int TPL = N / 8;
    constexpr uint32_t ES = sizeof(cx<T>);
    const int l = tid / TPL, t = tid - l * TPL;
    // KPZ and phase-shift steps hold two lines per row pair in LDS, KPZ with
    // phase shifts four
    constexpr int LINES = KIND == 4 ? 4 : ((KIND == 1 || KIND == 3) ? 2 : 1);
    cx<T>* L = lds + l * LINES * lds_len<N, PAD>();
    const Geo& g = a.g;
    const int last = g.ndim - 1;
    LineTw<T, N> tw;
    line_tw_load(tw, t, twid<T>(last == 1 ? it.tw1 : it.tw2));
    // the transforms of a step share their twiddle powers
    LineTwP<T, N> twp;
    line_tw_expand(twp, tw);
    const int pitch = g.pitch;
    const int K = g.kp[last];
    // pair groups bx iter + i, i < niter (the same count in every lane)
    const int npair = (a.nrows + 1) / 2;
    const int ngrp = (npair + a.lpw - 1) / a.lpw;
    const int grp0 = bx * a.iter;
    // without prefetch the launch gives every workgroup one group
    const int niter = PF ? min(a.iter, ngrp - grp0) : 1;
    // rows of this block, clipped to the array
    const int row0 = 2 * grp0 * a.lpw;
    const int nrow = min(2 * a.lpw * niter, a.nrows - row0);
    const size_t boff = (size_t)row0 * pitch;
    cx<T>* const bufp =
        (g.ndim == 2 ? reinterpret_cast<cx<T>*>(((KIND == 3 || KIND == 4) && sel) ? it.preb : it.pre0)
                     : reinterpret_cast<cx<T>*>(it.big) + (KIND == 3 ? (size_t)sel * g.n[0] * g.n[1] * pitch : 0)) +
        boff;
    const rsrc_t rb = make_rsrc(bufp, (uint32_t)nrow * (uint32_t)pitch * ES);
    const uint32_t RS = (uint32_t)pitch * ES;   // bytes per row
    // the pair of lane group l in group i, whether it exists, and the byte
    // offset of its first row within the block (a wavefront can hold several
    // pairs); BUF_OOB plus a row offset stays out of range
    auto pair_of = [&](int i) { return (grp0 + i) * a.lpw + l; };
    auto pair_ok = [&](int i) { return 2 * pair_of(i) < a.nrows; };
    auto row_off = [&](int i) { return (uint32_t)(2 * (i * a.lpw + l)) * RS; };
    // stored column read for bin k (k itself, or N - k for the mirrored upper
    // half), BUF_OOB where the bin has no stored mode
    auto col_off = [&](int q, bool valid) -> uint32_t {
        const int k = t + q * TPL;
        if (!valid) return BUF_OOB;
        if (DA && q <= 1) return (uint32_t)k * ES;
        if (DA && q >= 6) return (uint32_t)(N - k) * ES;
        if (k <= K) return (uint32_t)k * ES;
        if (k >= N - K) return (uint32_t)(N - k) * ES;
        return BUF_OOB;
    };
    auto empty = [](int q) { return DA && (q == 3 || q == 4); };   // no stored mode in any lane
    // bin q of the lower half (k <= N/2 side) in the packing below
    auto lower = [&](int q) { return (DA && q <= 1) || (!(DA && q >= 6) && t + q * TPL <= K); };
    const T inv = (T)it.inv_vol;
    // Model A/B: rows a, b of a pair; KPZ: pre1 (d0 h) and pre (h) rows
    cx<T> A[2][8], X[2][8];
    auto load_rows = [&](int i) {
        const bool vi = pair_ok(i);
        const uint32_t oa = row_off(i);
#pragma unroll
        for (int s = 0; s < 2; s++) {
#pragma unroll
            for (int q = 0; q < 8; q++) {
                A[s][q] = czero<T>();
                X[s][q] = czero<T>();
                if (empty(q)) continue;
                const uint32_t c = col_off(q, vi) + oa + (s ? RS : 0u);
                if constexpr (KIND == 1 || KIND == 4) {
                    const rsrc_t rb2 =
                        make_rsrc(reinterpret_cast<cx<T>*>((KIND == 4 && sel) ? it.pre1b : it.pre1) + boff, (uint32_t)nrow * RS);
                    A[s][q] = bload<T>(rb2, c, 0);
                    X[s][q] = bload<T>(rb, c, 0);
                } else {
                    A[s][q] = bload<T>(rb, c, 0);
                }
            }
        }
    };
    if constexpr (KIND != 2 && PF) load_rows(0);

#pragma unroll 1
    for (int i = 0; i < niter; i++) {
        const int pair = pair_of(i);
        const bool valid = pair_ok(i);
        const uint32_t o0 = row_off(i), o1 = o0 + RS;
        cx<T> v[8];
        if constexpr (KIND != 2 && !PF) load_rows(i);
        if constexpr (KIND == 2) {
            // i.i.d. N(0, sigma^2) per site, Philox counter (site, 0, r, 1)
            const T sig = (T)it.ic_sigma;
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int n = t + q * TPL;
                v[q] = czero<T>();
                if (valid) {
                    T za, zb, zc, zd;
                    const uint32_t s0 = (uint32_t)(2 * pair) * (uint32_t)N + (uint32_t)n;
                    normal_pair(it.seed, s0, 0u, it.r, 1u, za, zb);
                    normal_pair(it.seed, s0 + (uint32_t)N, 0u, it.r, 1u, zc, zd);
                    v[q] = {sig * za, sig * zc};
                }
            }
        } else if constexpr (KIND == 1 || KIND == 4) {
            // |grad h|^2 with d0 h = IFFT[i k0 h] (from pre1) and d1 h = IFFT[i k1 h];
            // the two rows' lines go through the stages together (one set of
            // barriers, twice the independent work per exchange), interleaved in LDS
            // read from the item in global memory: indexing the private copy
            // with the run-time axis would keep all of it in scratch memory
            const T dkl = (T)a.items[by].dk[last];
            cx<T> w[2][8];
#pragma unroll
            for (int s = 0; s < 2; s++) {
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    const int k = t + q * TPL;
                    cx<T> z = czero<T>();
                    if (empty(q)) {
                    } else if (lower(q)) {
                        cx<T> Aq = A[s][q];
                        const T kk = (2 * k == N) ? T(0) : dkl * (T)k;
                        cx<T> B = {-kk * X[s][q].y, kk * X[s][q].x};
                        if (k == 0 || 2 * k == N) {
                            Aq.y = T(0);
                            B.y = T(0);
                        }
                        z = {Aq.x - B.y, Aq.y + B.x};
                    } else {
                        // mirrored bins (zeros where nothing is stored)
                        const T kk = dkl * (T)(N - k);
                        const cx<T> B = {-kk * X[s][q].y, kk * X[s][q].x};
                        z = {A[s][q].x + B.y, B.x - A[s][q].y};
                    }
                    w[s][q] = z;
                }
            }
            if (PF && i + 1 < niter) load_rows(i + 1);
            if constexpr (KIND == 4) {
                // the lines as they are and moved by dx/2 along the row: the
                // squares of each pair packed, both transformed forward and
                // averaged with the second moved back
                cx<T> w4[4][8], phs[8];
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    phs[q] = cispi<T>((T)sgn_idx(t + q * TPL, N) / (T)N);
#pragma unroll
                    for (int s = 0; s < 2; s++) {
                        w4[s][q] = w[s][q];
                        w4[2 + s][q] = cmul(phs[q], w[s][q]);
                    }
                }
                fft_lines<T, N, +1, PAD, 4>(w4, t, L, 4, 1, twp);
                cx<T> sq[2][8];
#pragma unroll
                for (int u = 0; u < 2; u++) {
#pragma unroll
                    for (int q = 0; q < 8; q++) {
                        const T x0 = w4[2 * u][q].x * inv, y0 = w4[2 * u][q].y * inv;
                        const T x1 = w4[2 * u + 1][q].x * inv, y1 = w4[2 * u + 1][q].y * inv;
                        sq[u][q] = {x0 * x0 + y0 * y0, x1 * x1 + y1 * y1};
                    }
                }
                fft_lines<T, N, -1, PAD, 2>(sq, t, L, 2, 1, twp);
#pragma unroll
                for (int q = 0; q < 8; q++) v[q] = T(0.5) * (sq[0][q] + cmulc(sq[1][q], phs[q]));
            } else {
                fft_lines<T, N, +1, PAD, 2>(w, t, L, 2, 1, twp);
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    const T x0 = w[0][q].x * inv, y0 = w[0][q].y * inv;
                    const T x1 = w[1][q].x * inv, y1 = w[1][q].y * inv;
                    v[q] = {x0 * x0 + y0 * y0, x1 * x1 + y1 * y1};
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int k = t + q * TPL;
                cx<T> z;
                if (empty(q)) {
                    z = czero<T>();
                } else if (lower(q)) {
                    cx<T> a0 = A[0][q], b0 = A[1][q];
                    if (k == 0 || 2 * k == N) {
                        a0.y = T(0);
                        b0.y = T(0);
                    }
                    z = {a0.x - b0.y, a0.y + b0.x};
                } else {
                    // mirrored bins (zeros where nothing is stored)
                    z = {A[0][q].x + A[1][q].y, A[1][q].x - A[0][q].y};
                }
                v[q] = z;
            }
            if (PF && i + 1 < niter) load_rows(i + 1);
            if constexpr (KIND == 3) {
                // phi^3 on the rows and on the rows moved by dx/2, through the
                // stages together; the mean of the transforms, the second
                // moved back, cancels the aliases along the row
                cx<T> w[2][8], phs[8];
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    phs[q] = cispi<T>((T)sgn_idx(t + q * TPL, N) / (T)N);
                    w[0][q] = v[q];
                    w[1][q] = cmul(phs[q], v[q]);
                }
                fft_lines<T, N, +1, PAD, 2>(w, t, L, 2, 1, twp);
#pragma unroll
                for (int u = 0; u < 2; u++) {
#pragma unroll
                    for (int q = 0; q < 8; q++) {
                        const T x = w[u][q].x * inv, y = w[u][q].y * inv;
                        w[u][q] = {x * x * x, y * y * y};
                    }
                }
                fft_lines<T, N, -1, PAD, 2>(w, t, L, 2, 1, twp);
#pragma unroll
                for (int q = 0; q < 8; q++) v[q] = T(0.5) * (w[0][q] + cmulc(w[1][q], phs[q]));
            } else {
                fft_line<T, N, +1, PAD>(v, t, L, 1, twp);
                // phi^3 in real space (Model A and B)
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    const T x = v[q].x * inv, y = v[q].y * inv;
                    v[q] = {x * x * x, y * y * y};
                }
            }
        }

        if constexpr (KIND != 3 && KIND != 4) fft_line<T, N, -1, PAD>(v, t, L, 1, twp);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; q++) {
            // under the 2/3 rule the split below reads bins k < 3N/8 and N - k > 5N/8 only
            if (DA && (q == 3 || q == 4)) continue;
            L[lds_slot<PAD>(t + q * TPL)] = v[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; q++) {
            // under the 2/3 rule only q <= 2 (k < 3N/8) can hold a stored mode
            if (DA && q > 2) continue;
            const int k = t + q * TPL;
            const cx<T> Zk = L[lds_slot<PAD>(k)], Zm = L[lds_slot<PAD>((N - k) & (N - 1))];
            const uint32_t c = (valid && ((DA && q <= 1) || k <= K)) ? (uint32_t)k * ES : BUF_OOB;
            bstore<T>(rb, c + o0, 0, {T(0.5) * (Zk.x + Zm.x), T(0.5) * (Zk.y - Zm.y)});
            bstore<T>(rb, c + o1, 0, {T(0.5) * (Zk.y + Zm.y), T(0.5) * (Zm.x - Zk.x)});
        }
    }
}

template <typename T, int N, int PAD, int KIND, bool DA, bool PF>
__global__ void __launch_bounds__(256) k_row_real(RowArgs a)
{
    row_real_body<T, N, PAD, KIND, DA, PF>(a, blockIdx.x, blockIdx.y, threadIdx.x, blockIdx.z);
}

// ---------------------------------------------------------------- row pass, complex field
// PS (dealias 2): the line and its copy moved by dx/2 (e^{i pi a/N} per bin)
// through the stages together, their transforms averaged with the second
// moved back; 2D: rows of pre (blockIdx.z 0) or of its axis-0-shifted copy
// preb (1); 3D: rows of grid blockIdx.z of the four grids in big.
template <typename T, int N, int PAD, bool IC, bool PS = false>
__global__ void __launch_bounds__(256) k_row_cplx(RowArgs a)
{
    const Item it = a.items[blockIdx.y];
    if (a.sub >= it.steps) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    constexpr int TPL = N / 8;
    const int tid = threadIdx.x;
    const int l = tid / TPL, t = tid - l * TPL;
    const int line = blockIdx.x * a.lpw + l;
    const bool valid = line < a.nrows;
    cx<T>* L = lds + l * (PS ? 2 : 1) * lds_len<N, PAD>();
    const Geo& g = a.g;
    const int last = g.ndim - 1;
    LineTw<T, N> tw;
    line_tw_load(tw, t, twid<T>(last == 1 ? it.tw1 : it.tw2));
    const int kept = g.kept[last], kp = g.kp[last];
    constexpr uint32_t ES = sizeof(cx<T>);
    // buffer resource over the block's lines that exist; per-lane offset of
    // this lane's line, BUF_OOB for bins without a stored mode
    const int line0 = blockIdx.x * a.lpw;
    const int nline = min(a.lpw, a.nrows - line0);
    // phase shifts: 2D rows of pre or preb, 3D rows of grid blockIdx.z of big
    cx<T>* const buf = g.ndim == 2 ? reinterpret_cast<cx<T>*>((PS && blockIdx.z) ? it.preb : it.pre0)
                                   : reinterpret_cast<cx<T>*>(it.big) +
                                         (PS ? (size_t)blockIdx.z * g.n[0] * g.n[1] * g.pitch : 0);
    const rsrc_t rb = make_rsrc(buf + (size_t)line0 * g.pitch,
                                (uint32_t)nline * (uint32_t)g.pitch * ES);
    const uint32_t lo = (uint32_t)l * (uint32_t)g.pitch * ES;
    auto col_off = [&](int q) -> uint32_t {
        const int i = stored_idx(t + q * TPL, N, kept, kp);
        return (valid && i >= 0) ? lo + (uint32_t)i * ES : BUF_OOB;
    };
    const T inv = (T)it.inv_vol;
    cx<T> v[8];
    if constexpr (IC) {
        const T sig = (T)it.ic_sigma;
#pragma unroll
        for (int q = 0; q < 8; q++) {
            v[q] = czero<T>();
            if (valid) {
                T z1, z2;
                const uint32_t s = (uint32_t)line * (uint32_t)N + (uint32_t)(t + q * TPL);
                normal_pair(it.seed, s, 0u, it.r, 1u, z1, z2);
                v[q] = {sig * z1, sig * z2};
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; q++) v[q] = bload<T>(rb, col_off(q), 0);
        if constexpr (PS) {
            cx<T> w[2][8], phs[8];
#pragma unroll
            for (int q = 0; q < 8; q++) {
                phs[q] = cispi<T>((T)sgn_idx(t + q * TPL, N) / (T)N);
                w[0][q] = v[q];
                w[1][q] = cmul(phs[q], v[q]);
            }
            fft_lines<T, N, +1, PAD, 2>(w, t, L, 2, 1, tw);
#pragma unroll
            for (int u = 0; u < 2; u++) {
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    const T x = w[u][q].x * inv, y = w[u][q].y * inv;
                    const T m = x * x + y * y;
                    w[u][q] = {m * x, m * y};
                }
            }
            fft_lines<T, N, -1, PAD, 2>(w, t, L, 2, 1, tw);
#pragma unroll
            for (int q = 0; q < 8; q++) v[q] = T(0.5) * (w[0][q] + cmulc(w[1][q], phs[q]));
        } else {
            fft_line<T, N, +1, PAD>(v, t, L, 1, tw);
            // |A|^2 A in real space (CGL)
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const T x = v[q].x * inv, y = v[q].y * inv;
                const T m = x * x + y * y;
                v[q] = {m * x, m * y};
            }
        }
    }
    if (!PS || IC) fft_line<T, N, -1, PAD>(v, t, L, 1, tw);
#pragma unroll
    for (int q = 0; q < 8; q++) bstore<T>(rb, col_off(q), 0, v[q]);
}

// ---------------------------------------------------------------- real-space noise, last axis
// Sec. 4 step 2's alternative on 2D/3D lattices: the noise is drawn per site
// and transformed, eta_a = DFT[eta_x]_a / sqrt(prod n).  This pass draws the
// site values of step n and transforms the lines of the last axis; the
// axis-1 (3D) and axis-0 passes finish the transform (MODE_RSN).
// With R lines of the last axis per realization (line r = i0 n1 + i1) a site
// is x = r N + c, and its Philox4x32-10 block is (x mod Q, n, realization, 3)
// with Box-Muller normals of the word pairs (x0, x1) and (x2, x3):
//   real field, Q = R N / 4: the sites x + m Q (lines rho + m R/4, m = 0..3,
//     column c) take z1, z2 of the first pair and z1, z2 of the second;
//   complex field, Q = R N / 2: line rho takes (z1 + i z2)/sqrt2 of the first
//     pair, line rho + R/2 that of the second.
// A thread group owns group rho and draws each block once: a real field's
// four lines travel as two complex lines (rho + i (rho + R/4), rho + R/2 +
// i (rho + 3R/4)), split into the four half spectra through LDS after the
// transform; a complex field's two lines are transformed as they are.  The
// stored columns go to npre (2D) or big (3D).  The scale 1/sqrt(prod n) (and
// 1/sqrt2 of a complex draw) multiplies the site values.
struct RsnArgs {
    Geo g;
    const Item* items;
    int nrows;     // lines of the last axis per realization (R)
    int ngroups;   // R/4 (real field) or R/2 (complex field)
    int lpb;       // thread groups per block
    int sub;
    double scale;
};

template <typename T, int N, int PAD, bool CPLX>
__global__ void __launch_bounds__(256) k_rsn_rows(RsnArgs a)
{
    const Item it = a.items[blockIdx.y];
    if (a.sub >= it.steps) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    constexpr int TPL = N / 8;
    constexpr int LL = lds_len<N, PAD>();
    const int tid = threadIdx.x;
    const int l = tid / TPL, t = tid - l * TPL;
    cx<T>* L = lds + l * 2 * LL;   // the group's two lines
    const Geo& g = a.g;
    const int last = g.ndim - 1;
    const int grp = blockIdx.x * a.lpb + l;
    const bool valid = grp < a.ngroups;
    const uint32_t n = (uint32_t)it.ctrl->step;
    const T sc = (T)a.scale;
    LineTw<T, N> tw;
    line_tw_load(tw, t, twid<T>(last == 1 ? it.tw1 : it.tw2));
    cx<T> v[2][8];
#pragma unroll
    for (int q = 0; q < 8; q++) {
        v[0][q] = czero<T>();
        v[1][q] = czero<T>();
        if (valid) {
            uint32_t x[4];
            philox_block(it.seed, (uint32_t)grp * (uint32_t)N + (uint32_t)(t + q * TPL), n, it.r, 3u, x);
            T z1, z2, z3, z4;
            box_muller32(x[0], x[1], z1, z2);
            box_muller32(x[2], x[3], z3, z4);
            v[0][q] = {sc * z1, sc * z2};
            v[1][q] = {sc * z3, sc * z4};
        }
    }
    fft_lines<T, N, -1, PAD, 2>(v, t, L, 1, LL, tw);
    cx<T>* const dst = reinterpret_cast<cx<T>*>(g.ndim == 2 ? it.npre : it.big);
    const size_t pitch = (size_t)g.pitch;
    const int K = g.kp[last];
    if constexpr (CPLX) {
        const int kept = g.kept[last];
        const size_t rows[2] = {(size_t)grp, (size_t)grp + (size_t)(a.nrows / 2)};
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int k = t + q * TPL;
            const int c = k <= K ? k : (k >= N - (kept - K - 1) ? k - (N - kept) : -1);
            if (valid && c >= 0) {
                dst[rows[0] * pitch + c] = v[0][q];
                dst[rows[1] * pitch + c] = v[1][q];
            }
        }
    } else {
        // Z = A + i B: A_k = (Z_k + conj Z_{N-k}) / 2, B_k = -i (Z_k - conj Z_{N-k}) / 2
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; q++) {
            L[lds_slot<PAD>(t + q * TPL)] = v[0][q];
            L[LL + lds_slot<PAD>(t + q * TPL)] = v[1][q];
        }
        __syncthreads();
        const size_t quarter = (size_t)(a.nrows / 4);
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int k = t + q * TPL;
            if (!(valid && k <= K)) continue;
            const int m = (N - k) & (N - 1);
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const cx<T> z = v[h][q], zm = L[h * LL + lds_slot<PAD>(m)];
                const cx<T> A = {T(0.5) * (z.x + zm.x), T(0.5) * (z.y - zm.y)};
                const cx<T> B = {T(0.5) * (z.y + zm.y), T(0.5) * (zm.x - z.x)};
                const size_t ra = (size_t)grp + (size_t)(2 * h) * quarter;
                dst[ra * pitch + k] = A;
                dst[(ra + quarter) * pitch + k] = B;
            }
        }
    }
}

// ---------------------------------------------------------------- axis-0 pass
// A block owns TILE adjacent columns of the stored last axis (3D: at one
// stored index of axis 1).  Each thread carries LPT columns: thread
// (c0, t) = (tid % CW, tid / CW), CW = TILE / LPT, holds elements t + q N0/8 of
// columns c0 + k CW, so the rows of a tile are contiguous segments in every
// global access.
//
// MODE_STEP: pre -> forward FFT -> F_a = pref * FFT[N] -> ETD update with the
//            noise of step n -> phi, F_{n-1} -> inverse FFT -> pre.
// MODE_IC:   pre (forward-transformed initial field) -> forward FFT -> phi.
// MODE_SYNC: phi -> inverse FFT -> pre.
// MODE_RECOVER: pre -> forward FFT / N0 -> phi, pre left as it is (the state
//            of a plan that keeps the SETD2 carry instead of phi; pre holds
//            the unscaled axis-0 inverse of phi, N0 a power of two).
// PS (phase-shift dealiasing, 2D and 3D): beside pre the pass keeps preb,
// the axis-0 inverse of e^{i pi a0/N0} phi.  A step transforms both forward
// (the passes before have already averaged each over the grids moved along
// the other axes), takes X = (X_pre + e^{-i pi a0/N0} X_preb) / 2 as the
// nonlinear term (the mean over the 2^d grids), and after the update
// transforms phi and e^{i pi a0/N0} phi back into pre and preb (KPZ: also
// i k0 of each into pre1 and pre1b); the second half of the LDS holds the
// shifted lines.
template <typename T, int N0, int TILE, int PAD, bool KPZ, int LPT, bool PS>
__global__ void __launch_bounds__(TILE / LPT * N0 / 8) k_axis0(AxisArgs a)
{
    const unsigned lg = xcd_logical(blockIdx.x, gridDim.x);
    const int item = (int)(lg / (unsigned)a.per_item);
    const int blk = (int)(lg % (unsigned)a.per_item);
    const Item it = a.items[item];
    if (a.sub >= it.steps) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    const Geo& g = a.g;
    constexpr int TPL = N0 / 8;
    constexpr int CW = TILE / LPT;
    constexpr int NTHR = CW * TPL;
    const int tid = threadIdx.x;
    const int c0 = tid % CW, t = tid / CW;
    const int tile = blk % a.ntiles, i1 = blk / a.ntiles;
    const int last = g.ndim - 1;
    const int keptl = g.kept[last];
    const size_t lstride = (g.ndim == 3) ? (size_t)g.kept[1] * g.pitch : (size_t)g.pitch;
    const size_t plane = (size_t)i1 * g.pitch + (size_t)tile * TILE;   // offset of the tile within a row
    int col[LPT];
    bool cv[LPT];
#pragma unroll
    for (int k = 0; k < LPT; k++) {
        col[k] = c0 + k * CW;   // column within the tile
        cv[k] = tile * TILE + col[k] < keptl;
    }
    // MODE_RSN transforms the real-space noise: npre in, eta_a out to noise
    const bool rsn_mode = a.mode == MODE_RSN;
    cx<T>* __restrict__ pre0 = reinterpret_cast<cx<T>*>(rsn_mode ? it.npre : it.pre0);
    cx<T>* __restrict__ phi = reinterpret_cast<cx<T>*>(rsn_mode ? it.noise : it.phi);
    cx<T>* __restrict__ prev = reinterpret_cast<cx<T>*>(it.prev);
    const cx<T>* __restrict__ rnoise = reinterpret_cast<const cx<T>*>(it.noise);
    cx<T>* __restrict__ preb = reinterpret_cast<cx<T>*>(it.preb);
    // the shifted lines' LDS: the second half
    cx<T>* const ldsb = lds + (PS ? TILE * lds_len<N0, PAD>() : 0);
    LineTw<T, N0> tw;
    line_tw_load(tw, t, twid<T>(it.tw0));
    cx<T>* L = lds + c0;   // line k at L + k * CW, element stride TILE
    cx<T>* LB = ldsb + c0;
    const int kept0 = g.kept[0], kp0 = g.kp[0];
    // e^{i pi a0/N0} of axis-0 position j (signed a0)
    auto shift0 = [&](int j) { return cispi<T>((T)sgn_idx(j, N0) / (T)N0); };

    int j1 = 0, a1 = 0;
    if (g.ndim == 3) {
        j1 = fft_pos(i1, g.n[1], g.kept[1], g.kp[1]);
        a1 = sgn_idx(j1, g.n[1]);
    }
    const T dk0 = (T)it.dk[0], dk1 = (T)it.dk[1], dk2 = (T)it.dk[2];

    cx<T> v[LPT][8];
    cx<T> vb[PS ? LPT : 1][8];
    int64_t nstep = 0;
    int hp = 0;
    if (a.mode == MODE_STEP) {
        nstep = it.ctrl->step;
        hp = it.ctrl->have_prev;
    }
    if (a.mode == MODE_SYNC) {
#pragma unroll
        for (int k = 0; k < LPT; k++) {
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int i0 = stored_idx(t + q * TPL, N0, kept0, kp0);
                v[k][q] = (cv[k] && i0 >= 0) ? phi[(size_t)i0 * lstride + plane + col[k]] : czero<T>();
                if constexpr (PS) vb[k][q] = cmul(shift0(t + q * TPL), v[k][q]);
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < LPT; k++) {
#pragma unroll
            for (int q = 0; q < 8; q++)
                v[k][q] = cv[k] ? pre0[(size_t)(t + q * TPL) * lstride + plane + col[k]] : czero<T>();
        }
        fft_lines<T, N0, -1, PAD, LPT>(v, t, L, TILE, CW, tw);
        if constexpr (PS) {
            // the shifted copy (a step only: the initial condition has none)
#pragma unroll
            for (int k = 0; k < LPT; k++) {
#pragma unroll
                for (int q = 0; q < 8; q++)
                    vb[k][q] = (cv[k] && a.mode == MODE_STEP) ? preb[(size_t)(t + q * TPL) * lstride + plane + col[k]]
                                                              : czero<T>();
            }
            fft_lines<T, N0, -1, PAD, LPT>(vb, t, LB, TILE, CW, tw);
#pragma unroll
            for (int k = 0; k < LPT; k++) {
#pragma unroll
                for (int q = 0; q < 8; q++) LB[k * CW + lds_slot<PAD>(t + q * TPL) * TILE] = vb[k][q];
            }
        }
#pragma unroll
        for (int k = 0; k < LPT; k++) {
#pragma unroll
            for (int q = 0; q < 8; q++) L[k * CW + lds_slot<PAD>(t + q * TPL) * TILE] = v[k][q];
        }
        __syncthreads();
        // Update the stored modes of the tile in a linear sweep, one mode per
        // thread at a time, with the state, history and coefficients of the
        // next mode fetched while the current one is computed.
        const bool use_prev = (a.mode == MODE_STEP) && it.order == 2 && hp;
        const int nst = kept0 * TILE;
        struct Fetch {
            cx<T> ph, pv;
            Coef<T> cf;
        };
        auto last_pos = [&](int colm, int& jlm, int& alm) {
            jlm = colm;
            alm = colm;
            if (g.cplx) {
                jlm = fft_pos(colm, g.n[last], keptl, g.kp[last]);
                alm = sgn_idx(jlm, g.n[last]);
            }
        };
        auto fetch = [&](int m) {
            Fetch f;
            f.ph = czero<T>();
            f.pv = czero<T>();
            f.cf = Coef<T>{czero<T>(), czero<T>(), czero<T>(), T(0)};
            if (m < nst && a.mode == MODE_STEP) {
                const int i0 = m / TILE, cc = m % TILE;
                const int colm = tile * TILE + cc;
                if (colm < keptl) {
                    const size_t si = (size_t)i0 * lstride + plane + cc;
                    f.ph = phi[si];
                    if (use_prev) f.pv = prev[si];
                    int key;
                    const int a0 = sgn_idx(fft_pos(i0, N0, kept0, kp0), N0);
                    if (it.coef_mode == COEF_PER_MODE) {
                        key = per_mode_key(g, a0, colm);
                    } else {
                        int jlm, alm;
                        last_pos(colm, jlm, alm);
                        key = (g.ndim == 3) ? coef_key(it, a0, a1, alm) : coef_key(it, a0, alm, 0);
                    }
                    f.cf = load_coef<T>(it, key);
                }
            }
            return f;
        };
        bool bad = false;
        Fetch cur = fetch(tid);
        for (int m = tid; m < nst; m += NTHR) {
            const Fetch nxt = fetch(m + NTHR);
            const int i0 = m / TILE, cc = m % TILE;
            const int colm = tile * TILE + cc;
            const int j0 = fft_pos(i0, N0, kept0, kp0);
            cx<T>* slot = lds + lds_slot<PAD>(j0) * TILE + cc;
            cx<T>* slotb = ldsb + lds_slot<PAD>(j0) * TILE + cc;
            // phase shifts: the mean over the four grids, and e^{i pi a0/N0}
            cx<T> sh = {T(1), T(0)};
            if constexpr (PS) {
                sh = shift0(j0);
                if (a.mode == MODE_STEP) *slot = T(0.5) * (*slot + cmulc(*slotb, sh));
            }
            if (colm < keptl) {
                const size_t si = (size_t)i0 * lstride + plane + cc;
                if (a.mode == MODE_IC || rsn_mode) {
                    phi[si] = *slot;
                } else if (a.mode == MODE_RECOVER) {
                    // pre holds the unscaled axis-0 inverse of phi: divide by N0
                    phi[si] = (T(1) / T(N0)) * *slot;
                } else {
                    int jlm, alm;
                    last_pos(colm, jlm, alm);
                    const int a0 = sgn_idx(j0, N0);
                    const T kl = (g.ndim == 3) ? dk2 * (T)alm : dk1 * (T)alm;
                    const T km = (g.ndim == 3) ? dk1 * (T)a1 : T(0);
                    const T k2 = (dk0 * (T)a0) * (dk0 * (T)a0) + km * km + kl * kl;
                    const cx<T> F = cmul(nl_pref<T>(it, k2), *slot);
                    // Fourier-space draws (App. B), or the transformed real-space noise
                    const cx<T> eta = g.rsn ? rnoise[si] : noise_eta<T>(g, it, j0, j1, jlm, (uint32_t)nstep);
                    cx<T> nw = cmul(cur.cf.E, cur.ph) + cmul(cur.cf.wa, F) + cur.cf.G * eta;
                    if (it.order == 2) {
                        nw = nw + cmul(cur.cf.wb, use_prev ? cur.pv : F);
                        prev[si] = F;
                    }
                    bad |= !(isfinite(nw.x) && isfinite(nw.y));
                    phi[si] = nw;
                    *slot = nw;
                }
                if constexpr (PS) *slotb = cmul(sh, *slot);
            } else {
                *slot = czero<T>();
                if constexpr (PS) *slotb = czero<T>();
            }
            cur = nxt;
        }
        // the rows the 2/3 rule removes
        for (int m = tid; m < (N0 - kept0) * TILE; m += NTHR) {
            const int row = kp0 + 1 + m / TILE;
            lds[lds_slot<PAD>(row) * TILE + (m % TILE)] = czero<T>();
            if constexpr (PS) ldsb[lds_slot<PAD>(row) * TILE + (m % TILE)] = czero<T>();
        }
        // one flag update per block
        if (__syncthreads_or(bad) && tid == 0) atomicOr(&it.ctrl->nonfinite, 1);
        // recovery reads pre and writes phi only; the noise transform writes eta_a only
        if (a.mode == MODE_RECOVER || rsn_mode) return;
#pragma unroll
        for (int k = 0; k < LPT; k++) {
#pragma unroll
            for (int q = 0; q < 8; q++) {
                v[k][q] = L[k * CW + lds_slot<PAD>(t + q * TPL) * TILE];
                if constexpr (PS) vb[k][q] = LB[k * CW + lds_slot<PAD>(t + q * TPL) * TILE];
            }
        }
    }
    // KPZ: i k0 phi for the second inverse (with phase shifts also of the
    // shifted copy)
    cx<T> v2[KPZ ? LPT : 1][8];
    cx<T> v2b[(KPZ && PS) ? LPT : 1][8];
    if constexpr (KPZ) {
#pragma unroll
        for (int k = 0; k < LPT; k++) {
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int j0 = t + q * TPL;
                const T kk = (2 * j0 == N0) ? T(0) : dk0 * (T)sgn_idx(j0, N0);
                v2[k][q] = {-kk * v[k][q].y, kk * v[k][q].x};
                if constexpr (PS) v2b[k][q] = {-kk * vb[k][q].y, kk * vb[k][q].x};
            }
        }
    }
    fft_lines<T, N0, +1, PAD, LPT>(v, t, L, TILE, CW, tw);
#pragma unroll
    for (int k = 0; k < LPT; k++) {
        if (cv[k]) {
#pragma unroll
            for (int q = 0; q < 8; q++) pre0[(size_t)(t + q * TPL) * lstride + plane + col[k]] = v[k][q];
        }
    }
    if constexpr (PS) {
        fft_lines<T, N0, +1, PAD, LPT>(vb, t, LB, TILE, CW, tw);
#pragma unroll
        for (int k = 0; k < LPT; k++) {
            if (cv[k]) {
#pragma unroll
                for (int q = 0; q < 8; q++) preb[(size_t)(t + q * TPL) * lstride + plane + col[k]] = vb[k][q];
            }
        }
    }
    if constexpr (KPZ) {
        cx<T>* __restrict__ pre1 = reinterpret_cast<cx<T>*>(it.pre1);
        fft_lines<T, N0, +1, PAD, LPT>(v2, t, L, TILE, CW, tw);
#pragma unroll
        for (int k = 0; k < LPT; k++) {
            if (cv[k]) {
#pragma unroll
                for (int q = 0; q < 8; q++) pre1[(size_t)(t + q * TPL) * lstride + plane + col[k]] = v2[k][q];
            }
        }
    }
    if constexpr (KPZ && PS) {
        cx<T>* __restrict__ pre1b = reinterpret_cast<cx<T>*>(it.pre1b);
        fft_lines<T, N0, +1, PAD, LPT>(v2b, t, LB, TILE, CW, tw);
#pragma unroll
        for (int k = 0; k < LPT; k++) {
            if (cv[k]) {
#pragma unroll
                for (int q = 0; q < 8; q++) pre1b[(size_t)(t + q * TPL) * lstride + plane + col[k]] = v2b[k][q];
            }
        }
    }
    if (a.mode == MODE_STEP) {
        // the last block of this realization advances its step counter
        __syncthreads();
        if (tid == 0) advance_step(it.ctrl, (unsigned)a.per_item, nstep);
    }
}

// ---------------------------------------------------------------- axis-0 pass, update in registers
// The time step of k_axis0 (MODE_STEP, 2/3 rule on), one column per thread
// group, with the ETD update done in the layout the column transform leaves in
// registers: thread t holds bins j = t + q N0/8 (q = 0..7).  The state and
// history of those bins do not depend on the transform, so they are requested
// before it starts, and the unit noise is drawn while they are in flight (a
// rolled loop with one Philox call site, its results rotated through a
// register array); the coefficient table (L2-resident, shared by all
// realizations) is read after the transform.  There is no LDS sweep.  (At
// four waves per SIMD the register budget allows only the noise to be
// prepared early; state and history are then read after the forward
// transform.)
//
// Under the 2/3 rule the bins of q = 0, 1, 6, 7 are always stored, those of
// q = 3, 4 (3N0/8 <= j < 5N0/8) never, those of q = 2, 5 in part; a stored
// bin's row is j (q <= 2) or j - N0 + kept0 (q >= 5).  Every array access is
// a buffer access at the per-lane offset of row t plus a uniform per-q offset;
// lanes without a stored mode (and padding columns past the stored last-axis
// modes) use BUF_OOB, so they read zeros and write nothing.  Padding columns
// are still transformed: every column is an independent line.
// KIND: 0 real field, 1 real field with the KPZ gradient, 2 complex field
// (complex coefficient entries).
//
// LEAN (SETD2 only): the realization stores, in place of phi and F_{n-1}, the
// carry Y_n = E phi_n + w_b F_{n-1} + G eta_n (Eq. SETD2 regrouped; the array
// of F_{n-1} holds it).  A step computes phi_{n+1} = Y_n + w_a F_n (w_a + w_b on
// a first step, where F_{-1} = F_0), transforms phi_{n+1} back into pre, and
// stores Y_{n+1} = E phi_{n+1} + w_b F_n + G eta_{n+1}, the noise of the next
// step drawn now: one stored array read and written instead of two.
//
// Occupancy target in waves per SIMD (a CU has 4 SIMDs): resident blocks per
// CU times waves per block over 4, with two blocks of 512 threads (one
// block's transforms overlapping another's memory traffic), three of 256, and
// one of 1024; double precision, with twice the registers, one block of 512
// or two of 256.
template <typename T, int NTHR>
constexpr int axis0r_waves()
{
    constexpr int w = NTHR / 64;   // waves per block
    constexpr int blocks = sizeof(T) == 8 ? (w >= 8 ? 1 : 2) : (w >= 16 ? 1 : (w >= 8 ? 2 : 3));
    return blocks * w / 4 > 1 ? blocks * w / 4 : 1;
}

// The body runs one column tile (blk) of one item with TILE * N0 / 8 threads
// (tid) and the LDS at byte lds_off; herm_sync says whether the block holding
// these threads also holds tile 0 of a 2D lattice (its Hermitian column needs
// a barrier of the whole block).  The kernel below runs one tile per block,
// the shared launch of several lattice classes one or more.
template <typename T, int N0, int TILE, int PAD, int KIND, bool LEAN>
__device__ __forceinline__ void axis0r_body(const AxisArgs& a, const int item, const int blk, const int tid,
                                            const unsigned lds_off, const bool herm_sync)
{
    constexpr bool KPZ = KIND == 1, CC = KIND == 2;
    const Item it = a.items[item];
    if (a.sub >= it.steps) return;
    extern __shared__ __align__(16) unsigned char smem_base[];
    unsigned char* const smem_raw = smem_base + lds_off;
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    const Geo& g = a.g;
    constexpr int TPL = N0 / 8;
    constexpr uint32_t ES = sizeof(cx<T>);
    constexpr uint32_t CS = (CC ? 8 : 4) * sizeof(T);   // bytes of a coefficient entry
    const int c0 = tid % TILE, t = tid / TILE;
    const int tile = blk % a.ntiles, i1 = blk / a.ntiles;
    const int last = g.ndim - 1;
    const int keptl = g.kept[last];
    const int kept0 = g.kept[0], kp0 = g.kp[0];
    // bytes of one row (axis-0 index) of the arrays of a realization
    const uint32_t lstride = ((g.ndim == 3) ? (uint32_t)g.kept[1] * g.pitch : (uint32_t)g.pitch) * ES;
    const int colm = tile * TILE + c0;
    const bool cv = colm < keptl;
    const uint32_t vrow = (uint32_t)t * lstride + ((uint32_t)i1 * g.pitch + colm) * ES;   // row t, this column
    const uint32_t vcol = cv ? vrow : BUF_OOB;
    const rsrc_t rpre = make_rsrc(it.pre0, (uint32_t)N0 * lstride);
    const rsrc_t rphi = make_rsrc(it.phi, (uint32_t)kept0 * lstride);
    const rsrc_t rprev = make_rsrc(it.prev, (uint32_t)kept0 * lstride);
    const rsrc_t rcoef = make_rsrc(it.coef, it.coef_bytes);
    // stored-row shift of bin q and whether this lane's bin of q is stored
    auto dq = [&](int q) { return q <= 2 ? 0 : kept0 - N0; };
    auto stored = [&](int q) {
        if (q == 3 || q == 4) return false;
        if (q == 2) return t + 2 * TPL <= kp0;
        if (q == 5) return t + 5 * TPL >= N0 - kp0;
        return true;
    };
    auto live = [](int q) { return q != 3 && q != 4; };
    auto voff = [&](int q) { return (q == 2 || q == 5) ? (stored(q) ? vcol : BUF_OOB) : vcol; };
    auto soff = [&](int q) { return (uint32_t)(q * TPL + dq(q)) * lstride; };

    int j1 = 0, a1 = 0;
    if (g.ndim == 3) {
        j1 = fft_pos(i1, g.n[1], g.kept[1], g.kp[1]);
        a1 = sgn_idx(j1, g.n[1]);
    }
    int jl = colm, al = colm;   // FFT position and signed index on the last axis
    if (CC) {
        jl = fft_pos(colm, g.n[last], keptl, g.kp[last]);
        al = sgn_idx(jl, g.n[last]);
    }

    const int64_t nstep = *(const SETD_GLOBAL int64_t*)&it.ctrl->step;
    const int hp = *(const SETD_GLOBAL int*)&it.ctrl->have_prev;

    cx<T> v[1][8];
    cx<T> ph[8], pv[8], eta[8];
#pragma unroll
    for (int q = 0; q < 8; q++) v[0][q] = bload<T>(rpre, vrow, (uint32_t)(q * TPL) * lstride);
    // at the highest occupancy target state and history are read after the
    // forward transform, with the coefficients, to stay within the register
    // budget
    constexpr bool EARLY = axis0r_waves<T, TILE * N0 / 8>() < 4;
    // state and history; with LEAN the carry Y_n in place of the state
    auto load_state = [&]() {
#pragma unroll
        for (int q = 0; q < 8; q++) {
            ph[q] = czero<T>();
            pv[q] = czero<T>();
            if (live(q)) {
                if constexpr (LEAN) {
                    ph[q] = bload<T>(rprev, voff(q), soff(q));
                } else {
                    ph[q] = bload<T>(rphi, voff(q), soff(q));
                    if (it.order == 2) pv[q] = bload<T>(rprev, voff(q), soff(q));
                }
            }
        }
    };
    if constexpr (EARLY) load_state();
    // unit noise of the six bins that can hold a stored mode (q = 0, 1, 2,
    // 5, 6, 7), while the loads are in flight: bins k and 7 - k share a Philox
    // block (a second one only where a Hermitian partner draws for one of
    // them, in the a_last = 0 plane of a real field)
    cx<T> elo[3], ehi[3];
#pragma unroll
    for (int k = 0; k < 3; k++) elo[k] = ehi[k] = czero<T>();
    // real-space noise (plans without the carry): eta_a of the step was
    // transformed into the noise array, which has the layout of phi
    const rsrc_t rnoise = make_rsrc(it.noise, g.rsn ? (uint32_t)kept0 * lstride : 0u);
    if (g.rsn) {
#pragma unroll
        for (int k = 0; k < 3; k++) {
            elo[k] = bload<T>(rnoise, voff(k), soff(k));
            ehi[2 - k] = bload<T>(rnoise, voff(7 - k), soff(7 - k));
        }
    }
    const uint32_t nn = (uint32_t)(LEAN ? nstep + 1 : nstep);
    // off the a_last in {0, N_last/2} planes of a real field the pair's block
    // is the one of row t + k N0/8 (bin k half 0, bin 7 - k half 1); on them a
    // Hermitian partner may draw instead (noise_slot)
    const bool herm = !g.cplx && !(jl > 0 && 2 * jl < g.n[last]);
    const uint32_t S = (g.ndim == 3) ? (uint32_t)g.n[1] * (uint32_t)g.nh_last : (uint32_t)g.nh_last;
    const uint32_t rest = (g.ndim == 3) ? (uint32_t)j1 * (uint32_t)g.nh_last + (uint32_t)jl : (uint32_t)jl;
#pragma unroll 1
    for (int k = 0; k < (g.rsn ? 0 : 3); k++) {
        const int ja = t + k * TPL, jb = t + (7 - k) * TPL;
        NoiseSlot sa, sb;
        if (herm) {
            sa = noise_slot(g, ja, j1, jl);
            sb = noise_slot(g, jb, j1, jl);
        } else {
            sa = {(uint32_t)ja * S + rest, 0u, 0};
            sb = {sa.P, 1u, 0};
        }
        uint32_t x[4];
        philox_block(it.seed, sa.P, nn, it.r, 0u, x);
        cx<T> ea = eta_of<T>(x, sa);
        if (sb.P != sa.P) philox_block(it.seed, sb.P, nn, it.r, 0u, x);
        cx<T> eb = eta_of<T>(x, sb);
        // bins 0, 1, 6, 7 always hold a stored mode, 2 and 5 as stored() says
        if (!(cv && (k < 2 || stored(2)))) ea = czero<T>();
        if (!(cv && (k < 2 || stored(5)))) eb = czero<T>();
        elo[0] = elo[1];
        elo[1] = elo[2];
        elo[2] = ea;
        ehi[2] = ehi[1];
        ehi[1] = ehi[0];
        ehi[0] = eb;
    }
#pragma unroll
    for (int q = 0; q < 8; q++) eta[q] = q < 3 ? elo[q] : (q > 4 ? ehi[q - 5] : czero<T>());
    LineTw<T, N0> tw;
    line_tw_load(tw, t, twid<T>(it.tw0));
    cx<T>* L = lds + c0;   // element e of the column at L + e * TILE

    fft_lines<T, N0, -1, PAD, 1>(v, t, L, TILE, 0, tw);
    const bool per_mode = it.coef_mode == COEF_PER_MODE;
    // per-mode table rows |a0|: bins q <= 2 (a0 = t + q N0/8) read row
    // t + q N0/8, bins q >= 5 (a0 = t + q N0/8 - N0) row
    // (N0/8 - 1 - t) + N0 - (q + 1) N0/8 + 1: a lane part and a uniform part each
    const uint32_t vcoef = ((uint32_t)t * g.pitch + colm) * CS;
    const uint32_t vcoefn = ((uint32_t)(TPL - 1 - t) * g.pitch + colm) * CS;
    // Keyed coefficients (3D): the block needs the entries of |a0| = 0..K0 for
    // its TILE columns only, and a0 and -a0 share one.  Each is gathered once
    // into LDS, which the transform leaves free until the inverse starts.
    constexpr int NW = CC ? 2 : 1;   // T4 words per entry
    T4<T>* const ctab = reinterpret_cast<T4<T>*>(smem_raw);
    const bool staged = !KPZ && !per_mode && a.ctab;   // KPZ lattices are 2D
    if (staged) {
        __syncthreads();   // every lane has read its last transform values
        const int nent = (kp0 + 1) * TILE;
        for (int e = tid; e < nent; e += TILE * N0 / 8) {
            const int m = e / TILE, c = e - m * TILE;
            const int col = tile * TILE + c;
            int alc = col;
            if (CC) alc = sgn_idx(fft_pos(col, g.n[last], keptl, g.kp[last]), g.n[last]);
            const int key = (g.ndim == 3) ? coef_key(it, m, a1, alc) : coef_key(it, m, alc, 0);
            const uint32_t vo = col < keptl ? (uint32_t)key * CS : BUF_OOB;
#pragma unroll
            for (int w = 0; w < NW; w++) ctab[e * NW + w] = bload4<T>(rcoef, vo, (uint32_t)w * 4u * sizeof(T));
        }
        __syncthreads();
    }
    auto load_coef_q = [&](int q) {
        // lanes without a stored mode read nothing
        const bool st = cv && stored(q);
        if (staged) {
            const int a0 = sgn_idx(t + q * TPL, N0);
            const int m = st ? (a0 < 0 ? -a0 : a0) : 0;
            const T4<T>* ce = ctab + (m * TILE + c0) * NW;
            Coef<T> c;
            const T4<T> u = ce[0];
            if constexpr (CC) {
                const T4<T> w = ce[1];
                c.E = {u.a, u.b};
                c.wa = {u.c, u.d};
                c.wb = {w.a, w.b};
                c.G = w.c;
            } else {
                c.E = {u.a, T(0)};
                c.wa = {u.b, T(0)};
                c.wb = {u.c, T(0)};
                c.G = u.d;
            }
            return c;
        }
        uint32_t vo, so;
        if (per_mode) {
            // entry (|a0|, column) of the table
            vo = st ? (q >= 5 ? vcoefn : vcoef) : BUF_OOB;
            so = (uint32_t)(q >= 5 ? N0 - (q + 1) * TPL + 1 : q * TPL) * g.pitch * CS;
        } else {
            const int a0 = sgn_idx(t + q * TPL, N0);
            const int key = (g.ndim == 3) ? coef_key(it, a0, a1, al) : coef_key(it, a0, al, 0);
            vo = st ? (uint32_t)key * CS : BUF_OOB;
            so = 0;
        }
        Coef<T> c;
        if constexpr (CC) {
            const T4<T> u = bload4<T>(rcoef, vo, so), w = bload4<T>(rcoef, vo, so + 4 * sizeof(T));
            c.E = {u.a, u.b};
            c.wa = {u.c, u.d};
            c.wb = {w.a, w.b};
            c.G = w.c;
        } else {
            const T4<T> u = bload4<T>(rcoef, vo, so);
            c.E = {u.a, T(0)};
            c.wa = {u.b, T(0)};
            c.wb = {u.c, T(0)};
            c.G = u.d;
        }
        return c;
    };
    const bool use_prev = it.order == 2 && hp;
    const T dk0 = (T)it.dk[0], dk1 = (T)it.dk[1], dk2 = (T)it.dk[2];
    const T kl = (g.ndim == 3) ? dk2 * (T)al : dk1 * (T)al;
    const T km = (g.ndim == 3) ? dk1 * (T)a1 : T(0);
    // Fourier prefactor of the nonlinearity, affine in k^2: P0 + P2 k^2 (real
    // for real fields)
    const cx<T> P0 = nl_pref<T>(it, T(0)), P2 = nl_pref<T>(it, T(1)) - P0;
    // non-finite detection without branches: x - x is 0 for finite x and NaN
    // for NaN or infinity
    T nfacc = T(0);
    v[0][3] = czero<T>();
    v[0][4] = czero<T>();
    cx<T> ysv[3];   // LEAN: the new carry of bins q = 0..2 (Hermitian column below)
    // the six bins in two groups of three (q = 0..2, then 5..7): each group
    // reads its coefficients (and, when not read early, state and history)
    // and is updated and stored before the next group's reads
#pragma unroll
    for (int grp = 0; grp < 2; grp++) {
        const int qb = grp == 0 ? 0 : 5;
        cx<T> gph[3], gpv[3];
        Coef<T> cf[3];
#pragma unroll
        for (int u = 0; u < 3; u++) {
            const int q = qb + u;
            if constexpr (EARLY) {
                gph[u] = ph[q];
                gpv[u] = pv[q];
            } else if constexpr (LEAN) {
                gph[u] = bload<T>(rprev, voff(q), soff(q));
                gpv[u] = czero<T>();
            } else {
                gph[u] = bload<T>(rphi, voff(q), soff(q));
                gpv[u] = it.order == 2 ? bload<T>(rprev, voff(q), soff(q)) : czero<T>();
            }
            cf[u] = load_coef_q(q);
        }
#pragma unroll
        for (int u = 0; u < 3; u++) {
            const int q = qb + u;
            // lanes without a stored mode compute on zeros and store nothing
            const bool st = cv && stored(q);
            const T k0 = dk0 * (T)sgn_idx(t + q * TPL, N0);
            const T k2 = k0 * k0 + km * km + kl * kl;
            cx<T> F;
            if constexpr (CC) F = cmul(P0 + k2 * P2, v[0][q]);
            else F = (P0.x + k2 * P2.x) * v[0][q];
            cx<T> nw;
            if constexpr (LEAN) {
                // phi_{n+1} = Y_n + w F_n, Y_{n+1} = E phi_{n+1} + w_b F_n + G eta_{n+1}
                cx<T> y;
                if constexpr (CC) {
                    const cx<T> w = hp ? cf[u].wa : cf[u].wa + cf[u].wb;
                    nw = gph[u] + cmul(w, F);
                    y = cmul(cf[u].E, nw) + cmul(cf[u].wb, F) + cf[u].G * eta[q];
                } else {
                    const T w = hp ? cf[u].wa.x : cf[u].wa.x + cf[u].wb.x;
                    nw = gph[u] + w * F;
                    y = cf[u].E.x * nw + cf[u].wb.x * F + cf[u].G * eta[q];
                }
                bstore<T>(rprev, voff(q), soff(q), y);
                if (grp == 0) ysv[u] = y;
            } else {
                if constexpr (CC) {
                    nw = cmul(cf[u].E, gph[u]) + cmul(cf[u].wa, F) + cf[u].G * eta[q];
                    if (it.order == 2) nw = nw + cmul(cf[u].wb, use_prev ? gpv[u] : F);
                } else {
                    nw = cf[u].E.x * gph[u] + cf[u].wa.x * F + cf[u].G * eta[q];
                    if (it.order == 2) nw = nw + cf[u].wb.x * (use_prev ? gpv[u] : F);
                }
                if (it.order == 2) bstore<T>(rprev, voff(q), soff(q), F);
                bstore<T>(rphi, voff(q), soff(q), nw);
            }
            v[0][q] = st ? nw : czero<T>();
            nfacc += (v[0][q].x - v[0][q].x) + (v[0][q].y - v[0][q].y);
        }
    }
    // one flag update per block
    const bool bad = !(nfacc == nfacc);
    if (__syncthreads_or(bad) && tid == 0) atomicOr(&it.ctrl->nonfinite, 1);

    // Hermitian column a_last = 0 of a 2D real field (the rule of
    // k_hermitian): rows j and N0 - j are both in this block, the lower one
    // (q <= 2) independent; row 0 is self-conjugate.  LDS is free between the
    // barrier above and the one that opens the inverse transform.
    if constexpr (!CC) {
        if (g.ndim == 2 && herm_sync) {
            if (tile == 0 && c0 == 0) {
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    if (!stored(q)) continue;
                    const int sl = lds_slot<PAD>(t + q * TPL) * TILE;
                    lds[sl] = v[0][q];
                    if constexpr (LEAN) lds[sl + 1] = ysv[q];
                }
            }
            __syncthreads();
            if (tile == 0 && c0 == 0) {
#pragma unroll
                for (int q = 5; q < 8; q++) {
                    if (!stored(q)) continue;
                    const int sl = lds_slot<PAD>(N0 - (t + q * TPL)) * TILE;
                    const cx<T> pv = lds[sl];
                    v[0][q] = {pv.x, -pv.y};
                    if constexpr (LEAN) {
                        const cx<T> py = lds[sl + 1];
                        bstore<T>(rprev, voff(q), soff(q), {py.x, -py.y});
                    } else {
                        bstore<T>(rphi, voff(q), soff(q), v[0][q]);
                    }
                }
                if (t == 0) {
                    v[0][0].y = T(0);
                    if constexpr (LEAN) bstore<T>(rprev, voff(0), soff(0), {ysv[0].x, T(0)});
                    else bstore<T>(rphi, voff(0), soff(0), v[0][0]);
                }
            }
        }
    }

    cx<T> v2[1][8];
    if constexpr (KPZ) {
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int j0 = t + q * TPL;
            const T kk = (2 * j0 == N0) ? T(0) : dk0 * (T)sgn_idx(j0, N0);
            v2[0][q] = {-kk * v[0][q].y, kk * v[0][q].x};
        }
    }
    fft_lines<T, N0, +1, PAD, 1>(v, t, L, TILE, 0, tw);
#pragma unroll
    for (int q = 0; q < 8; q++) bstore<T>(rpre, vcol, (uint32_t)(q * TPL) * lstride, v[0][q]);
    if constexpr (KPZ) {
        const rsrc_t rpre1 = make_rsrc(it.pre1, (uint32_t)N0 * lstride);
        fft_lines<T, N0, +1, PAD, 1>(v2, t, L, TILE, 0, tw);
#pragma unroll
        for (int q = 0; q < 8; q++) bstore<T>(rpre1, vcol, (uint32_t)(q * TPL) * lstride, v2[0][q]);
    }
    // the last block of this realization advances its step counter
    __syncthreads();
    if (tid == 0) advance_step(it.ctrl, (unsigned)a.per_item, nstep);
}

template <typename T, int N0, int TILE, int PAD, int KIND, bool LEAN>
__global__ void __launch_bounds__(TILE * N0 / 8)
__attribute__((amdgpu_waves_per_eu(axis0r_waves<T, TILE * N0 / 8>())))
k_axis0r(AxisArgs a)
{
    // Logical blocks in groups of `group` items: within a group, consecutive
    // blocks take one block position (column tile) of each of the group's
    // items in turn, so the coefficient rows of a tile, which every item
    // reads, are used group times while in L2; an XCD's contiguous range of
    // logical blocks covers whole groups.  group 1: one item after the other.
    const unsigned lg = xcd_logical(blockIdx.x, gridDim.x);
    const unsigned P = (unsigned)a.per_item, G = (unsigned)a.group;
    const unsigned nit = gridDim.x / P;
    const unsigned grp = lg / (G * P), w = lg % (G * P);
    const unsigned gsz = min(G, nit - grp * G);   // items in this group (the last may hold fewer)
    const int item = (int)(grp * G + w % gsz);
    const int blk = (int)(w / gsz);
    axis0r_body<T, N0, TILE, PAD, KIND, LEAN>(a, item, blk, threadIdx.x, 0u, blk % a.ntiles == 0);
}

// ---------------------------------------------------------------- launches shared by lattice classes
// The 2D real-field classes of a serving tick that differ only in the lattice
// size (square N = 64, 128, 256 or 512; complex64; 2/3 rule; SETD2 carry;
// the phi^3 nonlinearities) advance in one launch per pass.  The arguments
// hold one slot per size; a block finds its slot from the slots' first blocks
// and runs that size's body, so every slot's body is compiled once and its
// arguments are read at fixed offsets.  Row pass: 256-thread blocks at every
// size (the same LDS, 18 KiB).  Axis-0 pass: 512-thread blocks; tile 8 for
// N = 512 and 16 otherwise, and for N <= 128 a block holds SUB = 2 or 4
// sub-blocks of one item (sub-block k runs tile SUB b + k of the item's
// b-th block; those past its last tile read and store nothing), so that all
// threads of a block meet the same barriers; every size uses 36 KiB of LDS.
constexpr int MULTI_SLOTS = 4;   // N = 64 << slot

__host__ __device__ constexpr int multi_tile(int slot) { return slot == 3 ? 8 : 16; }
__host__ __device__ constexpr int multi_sub(int slot) { return 512 / (multi_tile(slot) * ((64 << slot) / 8)); }

struct MultiRowArgs {
    RowArgs a[MULTI_SLOTS];
    int first[MULTI_SLOTS + 1];   // first block of each slot; first[MULTI_SLOTS] = the grid
    int gx[MULTI_SLOTS];          // blocks per item
};

struct MultiAxArgs {
    AxisArgs a[MULTI_SLOTS];      // a[s].per_item counts sub-blocks; a[s].ntiles covers them
    int first[MULTI_SLOTS + 1];
    int bpi[MULTI_SLOTS];         // blocks per item
};

// the slot of block b: the last one whose first block is <= b (empty slots
// share their successor's first block)
__device__ __forceinline__ int multi_slot(const int (&first)[MULTI_SLOTS + 1], int b)
{
    int s = 0;
#pragma unroll
    for (int i = 1; i < MULTI_SLOTS; i++)
        if (b >= first[i]) s = i;
    return s;
}

template <typename T, int SLOT>
__device__ __forceinline__ void row_multi_slot(const MultiRowArgs& m, int b)
{
    constexpr int N = 64 << SLOT;
    const int local = b - m.first[SLOT];
    row_real_body<T, N, 3, 0, true, false>(m.a[SLOT], local % m.gx[SLOT], local / m.gx[SLOT], threadIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(256) k_row_multi(MultiRowArgs m)
{
    const int b = blockIdx.x;
    switch (multi_slot(m.first, b)) {
    case 0: row_multi_slot<T, 0>(m, b); break;
    case 1: row_multi_slot<T, 1>(m, b); break;
    case 2: row_multi_slot<T, 2>(m, b); break;
    default: row_multi_slot<T, 3>(m, b); break;
    }
}

template <typename T, int SLOT>
__device__ __forceinline__ void axis0_multi_slot(const MultiAxArgs& m, int lg)
{
    constexpr int N0 = 64 << SLOT, TILE = multi_tile(SLOT), SUB = multi_sub(SLOT);
    constexpr int SUBT = TILE * N0 / 8;   // threads of a sub-block
    constexpr int PAD = 3;
    constexpr unsigned SUBLDS = (unsigned)(TILE * lds_len<N0, PAD>() * 2 * sizeof(T));
    const int local = lg - m.first[SLOT];
    const int item = local / m.bpi[SLOT], blk = local % m.bpi[SLOT];
    const int k = (int)threadIdx.x / SUBT;
    axis0r_body<T, N0, TILE, PAD, 0, true>(m.a[SLOT], item, blk * SUB + k, (int)threadIdx.x - k * SUBT,
                                           (unsigned)k * SUBLDS, blk == 0);
}

// (the four bodies in one function need more registers than any of them
// alone: at the three waves per SIMD targeted here they fit without spills)
template <typename T>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(3)))
k_axis0_multi(MultiAxArgs m)
{
    const int lg = (int)xcd_logical(blockIdx.x, gridDim.x);
    switch (multi_slot(m.first, lg)) {
    case 0: axis0_multi_slot<T, 0>(m, lg); break;
    case 1: axis0_multi_slot<T, 1>(m, lg); break;
    case 2: axis0_multi_slot<T, 2>(m, lg); break;
    default: axis0_multi_slot<T, 3>(m, lg); break;
    }
}

// ---------------------------------------------------------------- axis-1 pass (3D)
// mode +1: stored axis-1 entries of pre -> inverse FFT -> big
// mode -1: big -> forward FFT -> stored axis-1 entries of pre
// PS (phase-shift dealiasing, 3D): big holds four grids, 2 s0 + s1, s0 = 1 for
// the grid moved by dx/2 along axis 0 (the source preb instead of pre), s1 = 1
// for the grid moved along axis 1 (e^{i pi a1/N1} per mode).  blockIdx.z picks
// s0; mode +1 writes both grids of that source, mode -1 transforms both
// forward and keeps their mean, the second moved back, in pre or preb.  One
// column per thread; the two lines sit side by side in LDS (stride 2 TILE).
template <typename T, int N1, int TILE, int PAD, int LPT, bool PS = false>
__global__ void __launch_bounds__(TILE / LPT * N1 / 8) k_axis1(AxisArgs a)
{
    const unsigned lg = xcd_logical(blockIdx.x, gridDim.x);
    const int item = (int)(lg / (unsigned)a.per_item);
    const int blk = (int)(lg % (unsigned)a.per_item);
    const Item it = a.items[item];
    if (a.sub >= it.steps) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    const Geo& g = a.g;
    constexpr int TPL = N1 / 8;
    constexpr int CW = TILE / LPT;
    const int tid = threadIdx.x;
    const int c0 = tid % CW, t = tid / CW;
    const int tile = blk % a.ntiles, n0 = blk / a.ntiles;
    const int pitch = g.pitch, kept1 = g.kept[1], kp1 = g.kp[1];
    int col[LPT];
    bool cv[LPT];
#pragma unroll
    for (int k = 0; k < LPT; k++) {
        col[k] = tile * TILE + c0 + k * CW;
        cv[k] = col[k] < g.kept[2];
    }
    LineTw<T, N1> tw;
    line_tw_load(tw, t, twid<T>(it.tw1));
    if constexpr (PS) {
        static_assert(LPT == 1, "one column per thread");
        const int s0 = (int)blockIdx.z;
        const size_t gsz = (size_t)g.n[0] * N1 * pitch;   // elements of one grid of big
        cx<T>* __restrict__ src = reinterpret_cast<cx<T>*>(s0 ? it.preb : it.pre0) + (size_t)n0 * kept1 * pitch;
        cx<T>* __restrict__ b0 = reinterpret_cast<cx<T>*>(it.big) + (size_t)(2 * s0) * gsz + (size_t)n0 * N1 * pitch;
        cx<T>* __restrict__ b1 = b0 + gsz;
        cx<T> w[2][8], sh[8];
#pragma unroll
        for (int q = 0; q < 8; q++) sh[q] = cispi<T>((T)sgn_idx(t + q * TPL, N1) / (T)N1);
        if (a.mode > 0) {
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int i = stored_idx(t + q * TPL, N1, kept1, kp1);
                w[0][q] = (cv[0] && i >= 0) ? src[(size_t)i * pitch + col[0]] : czero<T>();
                w[1][q] = cmul(sh[q], w[0][q]);
            }
            fft_lines<T, N1, +1, PAD, 2>(w, t, lds + c0, 2 * TILE, TILE, tw);
            if (cv[0]) {
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    b0[(size_t)(t + q * TPL) * pitch + col[0]] = w[0][q];
                    b1[(size_t)(t + q * TPL) * pitch + col[0]] = w[1][q];
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < 8; q++) {
                w[0][q] = cv[0] ? b0[(size_t)(t + q * TPL) * pitch + col[0]] : czero<T>();
                w[1][q] = cv[0] ? b1[(size_t)(t + q * TPL) * pitch + col[0]] : czero<T>();
            }
            fft_lines<T, N1, -1, PAD, 2>(w, t, lds + c0, 2 * TILE, TILE, tw);
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int i = stored_idx(t + q * TPL, N1, kept1, kp1);
                if (cv[0] && i >= 0) src[(size_t)i * pitch + col[0]] = T(0.5) * (w[0][q] + cmulc(w[1][q], sh[q]));
            }
        }
        return;
    }
    cx<T>* __restrict__ small = reinterpret_cast<cx<T>*>(a.alt ? it.npre : it.pre0) + (size_t)n0 * kept1 * pitch;
    cx<T>* __restrict__ big = reinterpret_cast<cx<T>*>(it.big) + (size_t)n0 * N1 * pitch;
    cx<T>* L = lds + c0;
    cx<T> v[LPT][8];
    if (a.mode > 0) {
#pragma unroll
        for (int k = 0; k < LPT; k++) {
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int i = stored_idx(t + q * TPL, N1, kept1, kp1);
                v[k][q] = (cv[k] && i >= 0) ? small[(size_t)i * pitch + col[k]] : czero<T>();
            }
        }
        fft_lines<T, N1, +1, PAD, LPT>(v, t, L, TILE, CW, tw);
#pragma unroll
        for (int k = 0; k < LPT; k++) {
            if (cv[k]) {
#pragma unroll
                for (int q = 0; q < 8; q++) big[(size_t)(t + q * TPL) * pitch + col[k]] = v[k][q];
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < LPT; k++) {
#pragma unroll
            for (int q = 0; q < 8; q++) v[k][q] = cv[k] ? big[(size_t)(t + q * TPL) * pitch + col[k]] : czero<T>();
        }
        fft_lines<T, N1, -1, PAD, LPT>(v, t, L, TILE, CW, tw);
#pragma unroll
        for (int k = 0; k < LPT; k++) {
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int i = stored_idx(t + q * TPL, N1, kept1, kp1);
                if (cv[k] && i >= 0) small[(size_t)i * pitch + col[k]] = v[k][q];
            }
        }
    }
}

// ---------------------------------------------------------------- linear update (F = 0)
template <typename T>
__global__ void __launch_bounds__(256) k_linear(LinArgs a)
{
    const Item it = a.items[blockIdx.y];
    if (a.sub >= it.steps) return;
    const Geo& g = a.g;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nstep = it.ctrl->step;
    const int last = g.ndim - 1;
    bool bad = false;
    if (idx < a.total) {
        const int col = idx % g.pitch;
        const int rest = idx / g.pitch;
        const int i1 = (g.ndim == 3) ? rest % g.kept[1] : 0;
        const int i0 = (g.ndim == 3) ? rest / g.kept[1] : rest;
        if (col < g.kept[last]) {
            const int j0 = fft_pos(i0, g.n[0], g.kept[0], g.kp[0]);
            const int a0 = sgn_idx(j0, g.n[0]);
            int j1 = 0, a1 = 0;
            if (g.ndim == 3) {
                j1 = fft_pos(i1, g.n[1], g.kept[1], g.kp[1]);
                a1 = sgn_idx(j1, g.n[1]);
            }
            int jl = col, al = col;
            if (g.cplx) {
                jl = fft_pos(col, g.n[last], g.kept[last], g.kp[last]);
                al = sgn_idx(jl, g.n[last]);
            }
            const int key = (it.coef_mode == COEF_PER_MODE) ? per_mode_key(g, a0, col)
                            : (g.ndim == 3) ? coef_key(it, a0, a1, al) : coef_key(it, a0, al, 0);
            const Coef<T> cf = load_coef<T>(it, key);
            // Fourier-space draws, or the transformed real-space noise (separate
            // storage only: plans with it keep no carry)
            const cx<T> eta = g.rsn ? reinterpret_cast<const cx<T>*>(it.noise)[idx]
                                    : noise_eta<T>(g, it, j0, j1, jl, (uint32_t)nstep);
            cx<T>* phi = reinterpret_cast<cx<T>*>(it.phi);
            cx<T>* carry = reinterpret_cast<cx<T>*>(it.prev);
            cx<T> nw;
            if (a.mode == LIN_RENOISE) {
                // the carry drew G eta_n; it gets G eta_new instead
                const cx<T> eta2 = noise_eta<T>(g, it, j0, j1, jl, (uint32_t)a.new_step);
                nw = carry[idx] + cf.G * (eta2 - eta);
                carry[idx] = nw;
            } else {
                nw = cmul(cf.E, phi[idx]) + cf.G * eta;
                if (a.mode == LIN_CARRY) carry[idx] = nw;
                else phi[idx] = nw;
            }
            bad = !(isfinite(nw.x) && isfinite(nw.y));
        }
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(&it.ctrl->nonfinite, 1);
    if (a.mode == LIN_STEP && threadIdx.x == 0) advance_step(it.ctrl, gridDim.x, nstep);
}

// ---------------------------------------------------------------- Hermitian planes
// A real field's spectrum is Hermitian, phi_{-a} = conj(phi_a) (App. A).  On
// the planes a_last in {0, N_last/2} of the stored half spectrum both members
// of a conjugate pair are stored; transform round-off breaks the pairing, and
// the anti-Hermitian part, invisible to the real-space nonlinearity, would
// grow like e^{c h} per step where Re c > 0.  As for the noise (App. B), the
// member with the smaller linear index is independent and its partner takes
// its conjugate; self-conjugate modes are made real.  One thread per stored
// mode of the planes; partners only read independent members, which no
// thread writes.
struct HermArgs {
    Geo g;
    const Item* items;
    int which;    // 0: phi, 1: the F_{n-1} array (the SETD2 carry of lean plans), 2: the noise array
    int nplane;   // stored modes per plane and realization
    int ncol;     // planes: 1 (a_last = 0), or 2 when a_last = N_last/2 is stored
    int sub;
};

template <typename T>
__global__ void __launch_bounds__(256) k_hermitian(HermArgs a)
{
    const Item it = a.items[blockIdx.y];
    if (a.sub >= it.steps) return;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.nplane * a.ncol) return;
    const Geo& g = a.g;
    const int last = g.ndim - 1;
    const int c = idx / a.nplane, rest = idx % a.nplane;
    const int jl = c == 0 ? 0 : g.n[last] / 2;
    const int col = c == 0 ? 0 : g.kept[last] - 1;
    const int i1 = (g.ndim == 3) ? rest % g.kept[1] : 0;
    const int i0 = (g.ndim == 3) ? rest / g.kept[1] : rest;
    const int j0 = fft_pos(i0, g.n[0], g.kept[0], g.kp[0]);
    const int j1 = (g.ndim == 3) ? fft_pos(i1, g.n[1], g.kept[1], g.kp[1]) : 0;
    const int p0 = j0 ? g.n[0] - j0 : 0;
    const int p1 = (g.ndim == 3 && j1) ? g.n[1] - j1 : 0;
    const uint32_t nh = (uint32_t)g.nh_last;
    const uint32_t e = (g.ndim == 3) ? ((uint32_t)j0 * (uint32_t)g.n[1] + (uint32_t)j1) * nh + (uint32_t)jl
                                     : (uint32_t)j0 * nh + (uint32_t)jl;
    const uint32_t ep = (g.ndim == 3) ? ((uint32_t)p0 * (uint32_t)g.n[1] + (uint32_t)p1) * nh + (uint32_t)jl
                                      : (uint32_t)p0 * nh + (uint32_t)jl;
    cx<T>* arr = reinterpret_cast<cx<T>*>(a.which == 2 ? it.noise : (a.which ? it.prev : it.phi));
    const size_t lstride = (g.ndim == 3) ? (size_t)g.kept[1] * g.pitch : (size_t)g.pitch;
    const size_t own = (size_t)i0 * lstride + (size_t)i1 * g.pitch + col;
    if (ep == e) {
        arr[own].y = T(0);
    } else if (ep < e) {
        const int ip0 = stored_idx(p0, g.n[0], g.kept[0], g.kp[0]);
        const int ip1 = (g.ndim == 3) ? stored_idx(p1, g.n[1], g.kept[1], g.kp[1]) : 0;
        const cx<T> v = arr[(size_t)ip0 * lstride + (size_t)ip1 * g.pitch + col];
        arr[own] = {v.x, -v.y};
    }
}

// ---------------------------------------------------------------- FP64 observables
struct ObsArgs {
    Geo g;
    const Item* items;
    int nitems;
    int kind;       // RED_SK / RED_WIDTH / RED_TWOTIME / RED_RESPONSE
    int nbins;
    int total;      // stored elements per realization
    double vol;     // prod L_i / N_i^2
    double* acc;    // [3 * nbins] sums (re, im, weight)
    int64_t kick;   // RED_RESPONSE: the step whose noise is the kick
};

// Per stored mode: weight w = 2 for interior modes of a real field (a and -a),
// shell ceil|a|.  Sums go to LDS bins in FP64, then once per block to HBM.
template <typename T>
__global__ void __launch_bounds__(256) k_observe(ObsArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* sb = reinterpret_cast<double*>(smem_raw);
    const int nb = a.nbins;
    for (int i = threadIdx.x; i < 3 * nb; i += blockDim.x) sb[i] = 0.0;
    __syncthreads();
    const Geo& g = a.g;
    const Item& it = a.items[blockIdx.y];
    const int last = g.ndim - 1;
    const cx<T>* phi = reinterpret_cast<const cx<T>*>(it.phi);
    const cx<T>* snap = reinterpret_cast<const cx<T>*>(it.snap);
    const double invR = 1.0 / (double)a.nitems;
    double wacc = 0.0;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < a.total; idx += gridDim.x * blockDim.x) {
        const int col = idx % g.pitch;
        if (col >= g.kept[last]) continue;
        const int rest = idx / g.pitch;
        const int i1 = (g.ndim == 3) ? rest % g.kept[1] : 0;
        const int i0 = (g.ndim == 3) ? rest / g.kept[1] : rest;
        const int a0 = sgn_idx(fft_pos(i0, g.n[0], g.kept[0], g.kp[0]), g.n[0]);
        const int a1 = (g.ndim == 3) ? sgn_idx(fft_pos(i1, g.n[1], g.kept[1], g.kp[1]), g.n[1]) : 0;
        int al = col;
        if (g.cplx) al = sgn_idx(fft_pos(col, g.n[last], g.kept[last], g.kp[last]), g.n[last]);
        const double w = (!g.cplx && col > 0 && 2 * col < g.n[last]) ? 2.0 : 1.0;
        const cx<T> p = phi[idx];
        const double px = (double)p.x, py = (double)p.y;
        if (a.kind == RED_WIDTH) {
            if (a0 != 0 || a1 != 0 || al != 0) wacc += w * (px * px + py * py);
            continue;
        }
        const int b = ceil_isqrt(a0 * a0 + a1 * a1 + al * al);
        if (a.kind == RED_RESPONSE) {
            // linear response by the noise correlation (App. C): phi_a(n)
            // conj eta_a(n') / G_a with the step's own unit noise, regenerated
            // in the state precision, and G_a of the coefficient table
            const int ew = it.coef_cplx ? 8 : 4;   // table words per entry
            const int entry = (it.coef_mode == COEF_PER_MODE) ? per_mode_key(g, a0, col)
                              : ((g.ndim == 3) ? coef_key(it, a0, a1, al) : coef_key(it, a0, al, 0));
            const double G = (double)reinterpret_cast<const T*>(it.coef)[(size_t)entry * ew + (it.coef_cplx ? 6 : 3)];
            if (!(G > 0.0)) continue;
            const int j0 = fft_pos(i0, g.n[0], g.kept[0], g.kp[0]);
            const int j1 = (g.ndim == 3) ? fft_pos(i1, g.n[1], g.kept[1], g.kp[1]) : 0;
            const int jl = g.cplx ? fft_pos(col, g.n[last], g.kept[last], g.kp[last]) : col;
            const cx<T> e = noise_eta<T>(g, it, j0, j1, jl, (uint32_t)a.kick);
            const double ex = (double)e.x, ey = (double)e.y;
            const double re = (px * ex + py * ey) / G * invR;
            const double im = (py * ex - px * ey) / G * invR;
            if (w == 2.0) {
                atomicAdd(&sb[b], 2.0 * re);
            } else {
                atomicAdd(&sb[b], re);
                atomicAdd(&sb[nb + b], im);
            }
            if (blockIdx.y == 0) atomicAdd(&sb[2 * nb + b], w);
            continue;
        }
        if (a.kind == RED_SK) {
            atomicAdd(&sb[b], w * a.vol * (px * px + py * py) * invR);
        } else {
            const cx<T> s = snap[idx];
            const double sx = (double)s.x, sy = (double)s.y;
            const double re = (px * sx + py * sy) * a.vol * invR;
            const double im = (py * sx - px * sy) * a.vol * invR;
            if (w == 2.0) {
                atomicAdd(&sb[b], 2.0 * re);
            } else {
                atomicAdd(&sb[b], re);
                atomicAdd(&sb[nb + b], im);
            }
        }
        if (blockIdx.y == 0) atomicAdd(&sb[2 * nb + b], w);
    }
    if (a.kind == RED_WIDTH) atomicAdd(&sb[0], wacc);
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * nb; i += blockDim.x)
        if (sb[i] != 0.0) atomicAdd(&a.acc[i], sb[i]);
}

// ---------------------------------------------------------------- 1D lattices
// A line of N sites is a whole lattice: one group of N/8 threads holds a
// line's transform (thread t: bins t + q N/8), and the state stays in
// registers for all steps of a launch, so HBM sees the state once per launch.
// Real fields pair two realizations in one complex line (z = h1 + i h2, as
// the row pass of the other lattices does); complex fields take a line each.
struct Line1dArgs {
    Geo g;
    const Item* items;
    int nitems;
    int nlines;   // realization pairs (real fields) or realizations (complex)
    int mode;     // MODE_STEP or MODE_IC
    int sub;      // sub-step of the scheduler tick
    int nsteps;   // MODE_STEP: steps of this launch
};

// Twiddles of a line kernel: every power in registers (FP32) or the stage
// bases only (FP64, whose registers are twice as wide).
template <typename T, int N, int KIND>
constexpr bool line1d_twp() { return sizeof(T) == 4; }

template <typename T, int N, int KIND>
using Line1dTw = typename std::conditional<line1d_twp<T, N, KIND>(), LineTwP<T, N>, LineTw<T, N>>::type;

template <typename T, int N, int KIND>
__device__ __forceinline__ void line1d_tw(Line1dTw<T, N, KIND>& tw, int t, const cx<T>* tab)
{
    LineTw<T, N> base;
    line_tw_load(base, t, tab);
    if constexpr (line1d_twp<T, N, KIND>()) line_tw_expand(tw, base);
    else tw = base;
}

// Real field, realizations 2l and 2l + 1 of line l.  Rounding in the packed
// transforms couples the two channels, so a realization's bits depend on its
// partner: the server keeps every job's realizations on lines of their own.  Thread t keeps the stored
// modes a = t + q N/8 (q < 4, and a = N/2 in slot 4 of thread 0) of both
// realizations.  A step: pack z = A + i B from the two half spectra (the bins
// above N/2 are conj(A_{N-k}) + i conj(B_{N-k}), read back through LDS),
// inverse transform, the nonlinearity of each real part, forward transform,
// split W into the two spectra through LDS, and the update of Eq. SETD1/SETD2
// per realization with its own noise, table and step.  KIND 0: phi^3 (Model A,
// and Model B with its k^2 in the prefactor), 1: KPZ ((lambda/2) h'^2 from the
// line of h + i h' per realization pair), 2: no nonlinearity.
template <typename T, int N, int PAD, int DM, int KIND, bool RS>
__global__ void __launch_bounds__(256) k_line1d_real(Line1dArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr bool DA = DM == 1, PS = DM == 2;   // 2/3 truncation, phase shift
    constexpr int TPL = N / 8, M = N / 8;
    constexpr int LPB = 256 / TPL;
    constexpr int LL = lds_len<N, PAD>();
    constexpr int QS = DA ? 3 : (PS ? 4 : 5);    // register slots of stored modes
    const Geo& g = a.g;
    const int tid = threadIdx.x;
    const int l = tid / TPL, t = tid - l * TPL;
    const int line = blockIdx.x * LPB + l;
    cx<T>* L = reinterpret_cast<cx<T>*>(smem_raw) + (size_t)l * 2 * LL;
    const int ra = 2 * line, rb = 2 * line + 1;
    const bool va = line < a.nlines && ra < a.nitems, vb = line < a.nlines && rb < a.nitems;
    const Item& ia = a.items[va ? ra : 0];
    const Item& ib = a.items[vb ? rb : (va ? ra : 0)];
    const bool acta = va && a.sub < ia.steps, actb = vb && a.sub < ib.steps;
    const int K = DA ? (N - 1) / 3 : (PS ? N / 2 - 1 : N / 2);
    Line1dTw<T, N, KIND> tw;
    line1d_tw<T, N, KIND>(tw, t, twid<T>(ia.tw0));
    const T inv = (T)ia.inv_vol;
    // mode of slot q, and whether it is stored
    auto mode_of = [&](int q) { return t + q * M; };
    auto stored = [&](int q) { return q < 4 ? (t + q * M <= K) : (DM == 0 && t == 0); };
    // phase shift: e^{i pi a/N} of bin t + qM (signed a), the grid moved by dx/2
    cx<T> phs[PS ? 8 : 1];
    if constexpr (PS) {
#pragma unroll
        for (int q = 0; q < 8; q++) phs[q] = cispi<T>((T)sgn_idx(t + q * M, N) / (T)N);
    }

    cx<T> pa[QS], pb[QS];
    if (a.mode == MODE_IC) {
        // per site: h = sigma z1 of the Philox block (site, 0, r, 1)
        cx<T> v[8];
#pragma unroll
        for (int q = 0; q < 8; q++) {
            T z1a = T(0), z2a, z1b = T(0), z2b;
            const uint32_t site = (uint32_t)(t + q * M);
            if (va) normal_pair(ia.seed, site, 0u, ia.r, 1u, z1a, z2a);
            if (vb) normal_pair(ib.seed, site, 0u, ib.r, 1u, z1b, z2b);
            v[q] = {(T)ia.ic_sigma * z1a, (T)ib.ic_sigma * z1b};
        }
        fft_line<T, N, -1, PAD>(v, t, L, 1, tw);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; q++) L[lds_slot<PAD>(t + q * M)] = v[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < QS; q++) {
            const int k = mode_of(q) & (N - 1);
            const cx<T> Zk = L[lds_slot<PAD>(k)], Zm = L[lds_slot<PAD>((N - k) & (N - 1))];
            pa[q] = {T(0.5) * (Zk.x + Zm.x), T(0.5) * (Zk.y - Zm.y)};
            pb[q] = {T(0.5) * (Zk.y + Zm.y), T(0.5) * (Zm.x - Zk.x)};
            if (!stored(q)) pa[q] = pb[q] = czero<T>();
        }
        cx<T>* phia = reinterpret_cast<cx<T>*>(ia.phi);
        cx<T>* phib = reinterpret_cast<cx<T>*>(ib.phi);
#pragma unroll
        for (int q = 0; q < QS; q++) {
            if (!stored(q)) continue;
            const int m = mode_of(q);
            if (m == 0 || 2 * m == N) {
                pa[q].y = T(0);
                pb[q].y = T(0);
            }
            if (va) phia[m] = pa[q];
            if (vb) phib[m] = pb[q];
        }
        return;
    }

    // state, F_{n-1}, coefficients and steps of both realizations
    cx<T> fa[QS], fb[QS];
    Coef<T> ca[QS], cb[QS];
    const cx<T>* phia0 = reinterpret_cast<const cx<T>*>(ia.phi);
    const cx<T>* phib0 = reinterpret_cast<const cx<T>*>(ib.phi);
    const cx<T>* preva = reinterpret_cast<const cx<T>*>(ia.prev);
    const cx<T>* prevb = reinterpret_cast<const cx<T>*>(ib.prev);
    const int64_t stepa = va ? ia.ctrl->step : 0, stepb = vb ? ib.ctrl->step : 0;
    const int hpa = va ? ia.ctrl->have_prev : 0, hpb = vb ? ib.ctrl->have_prev : 0;
    const bool o2 = ia.order == 2;
#pragma unroll
    for (int q = 0; q < QS; q++) {
        pa[q] = pb[q] = fa[q] = fb[q] = czero<T>();
        ca[q] = cb[q] = Coef<T>{czero<T>(), czero<T>(), czero<T>(), T(0)};
        if (!stored(q)) continue;
        const int m = mode_of(q);
        // a realization that does not step in this launch is no partner: its
        // channel stays zero, as for the missing partner of an odd count
        if (acta) {
            pa[q] = phia0[m];
            if (o2 && hpa) fa[q] = preva[m];
            ca[q] = load_coef_t<T, false>(ia.coef, m);   // real fields: real tables, keyed by |a|
        }
        if (actb) {
            pb[q] = phib0[m];
            if (o2 && hpb) fb[q] = prevb[m];
            cb[q] = load_coef_t<T, false>(ib.coef, m);
        }
        if (m == 0 || 2 * m == N) {
            pa[q].y = T(0);
            pb[q].y = T(0);
        }
    }
    const T dka = (T)ia.dk[0], dkb = (T)ib.dk[0];
    const cx<T> pra = nl_pref<T>(ia, T(0)), prb = nl_pref<T>(ib, T(0));
    // real-space noise of step s: site x = t + qM of both realizations from
    // Philox blocks (x mod N/4, n, r, 3): block t + hM gives sites q = h,
    // h + 2 (half 0) and h + 4, h + 6 (half 1)
    auto site_noise = [&](cx<T> (&e)[8], int s) {
#pragma unroll
        for (int q = 0; q < 8; q++) e[q] = czero<T>();
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const uint32_t P = (uint32_t)(t + h * M);
            uint32_t x[4];
            T z1, z2, z3, z4;
            if (acta) {
                philox_block(ia.seed, P, (uint32_t)(stepa + s), ia.r, 3u, x);
                box_muller32(x[0], x[1], z1, z2);
                box_muller32(x[2], x[3], z3, z4);
                e[h].x = z1;
                e[h + 2].x = z2;
                e[h + 4].x = z3;
                e[h + 6].x = z4;
            }
            if (actb) {
                philox_block(ib.seed, P, (uint32_t)(stepb + s), ib.r, 3u, x);
                box_muller32(x[0], x[1], z1, z2);
                box_muller32(x[2], x[3], z3, z4);
                e[h].y = z1;
                e[h + 2].y = z2;
                e[h + 4].y = z3;
                e[h + 6].y = z4;
            }
        }
    };
    (void)site_noise;
    const T rsq = (T)(1.0 / sqrt((double)N));

#pragma unroll 1
    for (int s = 0; s < a.nsteps; s++) {
        if constexpr (KIND != 2) {
            // pack the two half spectra (KPZ: of h and h' per realization)
            __syncthreads();
#pragma unroll
            for (int q = 0; q < QS; q++) {
                if (q == 4 && t != 0) continue;
                const int m = mode_of(q);
                cx<T> A = pa[q], B = pb[q];
                if constexpr (KIND == 1) {
                    // h' = i k h, the Nyquist derivative dropped
                    const T kk = (2 * m == N) ? T(0) : (T)m;
                    A = {-kk * dka * pa[q].y, kk * dka * pa[q].x};
                    B = {-kk * dkb * pb[q].y, kk * dkb * pb[q].x};
                }
                L[lds_slot<PAD>(m)] = A;
                L[LL + lds_slot<PAD>(m)] = B;
            }
            __syncthreads();
            cx<T> z[8];
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int k = t + q * M;
                // bins whose mode (k or N - k) is not stored are zero
                if ((DA && (q == 3 || q == 4)) || (k <= N / 2 ? k : N - k) > K) {
                    z[q] = czero<T>();
                } else if (k <= N / 2) {
                    const cx<T> A = L[lds_slot<PAD>(k)], B = L[LL + lds_slot<PAD>(k)];
                    z[q] = {A.x - B.y, A.y + B.x};
                } else {
                    const cx<T> A = L[lds_slot<PAD>(N - k)], B = L[LL + lds_slot<PAD>(N - k)];
                    z[q] = {A.x + B.y, B.x - A.y};
                }
            }
            if constexpr (PS) {
                // the nonlinearity on the grid and on the grid shifted by
                // dx/2, through the stages together; the mean of the two
                // transforms (the second shifted back) cancels single aliases
                cx<T> w[2][8];
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    w[0][q] = z[q];
                    w[1][q] = cmul(phs[q], z[q]);
                }
                fft_lines<T, N, +1, PAD, 2>(w, t, L, 2, 1, tw);
#pragma unroll
                for (int u = 0; u < 2; u++) {
#pragma unroll
                    for (int q = 0; q < 8; q++) {
                        const T x = w[u][q].x * inv, y = w[u][q].y * inv;
                        w[u][q] = (KIND == 1) ? cx<T>{x * x, y * y} : cx<T>{x * x * x, y * y * y};
                    }
                }
                fft_lines<T, N, -1, PAD, 2>(w, t, L, 2, 1, tw);
#pragma unroll
                for (int q = 0; q < 8; q++) z[q] = T(0.5) * (w[0][q] + cmulc(w[1][q], phs[q]));
            } else {
                fft_line<T, N, +1, PAD>(z, t, L, 1, tw);
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    const T x = z[q].x * inv, y = z[q].y * inv;
                    z[q] = (KIND == 1) ? cx<T>{x * x, y * y} : cx<T>{x * x * x, y * y * y};
                }
            }
            if constexpr (PS) {
                // (the mean is already transformed; site noise, if drawn,
                // goes through the forward stages alone into the second half)
                cx<T> e[RS ? 8 : 1];
                if constexpr (RS) {
                    site_noise(e, s);
                    fft_line<T, N, -1, PAD>(e, t, L, 1, tw);
                }
                __syncthreads();
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    L[lds_slot<PAD>(t + q * M)] = z[q];
                    if constexpr (RS) L[LL + lds_slot<PAD>(t + q * M)] = e[q];
                }
                __syncthreads();
            } else if constexpr (RS) {
                // the nonlinearity and the site noise of both realizations
                // through the forward stages together (interleaved in LDS)
                cx<T> w2[2][8];
                site_noise(w2[1], s);
#pragma unroll
                for (int q = 0; q < 8; q++) w2[0][q] = z[q];
                fft_lines<T, N, -1, PAD, 2>(w2, t, L, 2, 1, tw);
                __syncthreads();
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    L[lds_slot<PAD>(t + q * M)] = w2[0][q];
                    L[LL + lds_slot<PAD>(t + q * M)] = w2[1][q];
                }
                __syncthreads();
            } else {
                fft_line<T, N, -1, PAD>(z, t, L, 1, tw);
                __syncthreads();
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    if (DA && (q == 3 || q == 4)) continue;
                    L[lds_slot<PAD>(t + q * M)] = z[q];
                }
                __syncthreads();
            }
        } else if constexpr (RS) {
            cx<T> e[8];
            site_noise(e, s);
            fft_line<T, N, -1, PAD>(e, t, L, 1, tw);
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 8; q++) L[LL + lds_slot<PAD>(t + q * M)] = e[q];
            __syncthreads();
        }
        // split W into the two spectra with the model prefactor
        cx<T> F1[QS], F2[QS];
#pragma unroll
        for (int q = 0; q < QS; q++) {
            F1[q] = F2[q] = czero<T>();
            if constexpr (KIND != 2) {
                const int k = mode_of(q) & (N - 1);
                const cx<T> Zk = L[lds_slot<PAD>(k)], Zm = L[lds_slot<PAD>((N - k) & (N - 1))];
                const cx<T> wa = {T(0.5) * (Zk.x + Zm.x), T(0.5) * (Zk.y - Zm.y)};
                const cx<T> wb = {T(0.5) * (Zk.y + Zm.y), T(0.5) * (Zm.x - Zk.x)};
                const T k2a = (dka * (T)k) * (dka * (T)k), k2b = (dkb * (T)k) * (dkb * (T)k);
                // Model B: -u k^2; the others a constant
                const T sa = (ia.nl == NL_PHI3_CONS) ? -(T)ia.par0 * k2a : pra.x;
                const T sb = (ib.nl == NL_PHI3_CONS) ? -(T)ib.par0 * k2b : prb.x;
                F1[q] = sa * wa;
                F2[q] = sb * wb;
            }
        }
        cx<T> ea[QS], eb[QS];
        if constexpr (RS) {
            // the transformed site noise of both realizations, split
#pragma unroll
            for (int q = 0; q < QS; q++) {
                const int k = mode_of(q) & (N - 1);
                const cx<T> Ek = L[LL + lds_slot<PAD>(k)], Em = L[LL + lds_slot<PAD>((N - k) & (N - 1))];
                ea[q] = {rsq * T(0.5) * (Ek.x + Em.x), rsq * T(0.5) * (Ek.y - Em.y)};
                eb[q] = {rsq * T(0.5) * (Ek.y + Em.y), rsq * T(0.5) * (Em.x - Ek.x)};
            }
        } else {
            // Fourier draws: block t serves modes t and t + 2M, block t + M
            // serves t + M and t + 3M, block 2M the Nyquist mode (thread 0)
#pragma unroll
            for (int h = 0; h < 2; h++) {
                uint32_t xa[4], xb[4];
                const uint32_t P = (uint32_t)(t + h * M);
                if (acta) philox_block(ia.seed, P, (uint32_t)(stepa + s), ia.r, 0u, xa);
                if (actb) philox_block(ib.seed, P, (uint32_t)(stepb + s), ib.r, 0u, xb);
#pragma unroll
                for (int u = 0; u < 2; u++) {
                    const int q = h + 2 * u;
                    if (q >= QS) continue;
                    NoiseSlot ns;
                    ns.P = P;
                    ns.half = (uint32_t)u;
                    ns.kind = (q == 0 && t == 0) ? 1 : 0;
                    ea[q] = acta ? eta_of<T>(xa, ns) : czero<T>();
                    eb[q] = actb ? eta_of<T>(xb, ns) : czero<T>();
                }
            }
            if constexpr (DM == 0) {
                ea[4] = eb[4] = czero<T>();
                if (t == 0) {
                    uint32_t xa[4], xb[4];
                    NoiseSlot ns;
                    ns.P = (uint32_t)(2 * M);
                    ns.half = 0u;
                    ns.kind = 1;
                    if (acta) {
                        philox_block(ia.seed, ns.P, (uint32_t)(stepa + s), ia.r, 0u, xa);
                        ea[4] = eta_of<T>(xa, ns);
                    }
                    if (actb) {
                        philox_block(ib.seed, ns.P, (uint32_t)(stepb + s), ib.r, 0u, xb);
                        eb[4] = eta_of<T>(xb, ns);
                    }
                }
            }
        }
        // Eq. SETD1 / SETD2 (the first step of a fresh state takes F_{n-1} = F_n)
        const bool upa = o2 && (s > 0 || hpa), upb = o2 && (s > 0 || hpb);
#pragma unroll
        for (int q = 0; q < QS; q++) {
            if (!stored(q)) continue;
            const int m = mode_of(q);
            cx<T> na = cmul(ca[q].E, pa[q]) + cmul(ca[q].wa, F1[q]) + ca[q].G * ea[q];
            cx<T> nb = cmul(cb[q].E, pb[q]) + cmul(cb[q].wa, F2[q]) + cb[q].G * eb[q];
            if (o2) {
                na = na + cmul(ca[q].wb, upa ? fa[q] : F1[q]);
                nb = nb + cmul(cb[q].wb, upb ? fb[q] : F2[q]);
                fa[q] = F1[q];
                fb[q] = F2[q];
            }
            if (m == 0 || 2 * m == N) {
                na.y = T(0);
                nb.y = T(0);
            }
            if (acta) pa[q] = na;
            if (actb) pb[q] = nb;
        }
    }
    cx<T>* phia = reinterpret_cast<cx<T>*>(ia.phi);
    cx<T>* phib = reinterpret_cast<cx<T>*>(ib.phi);
    cx<T>* pva = reinterpret_cast<cx<T>*>(ia.prev);
    cx<T>* pvb = reinterpret_cast<cx<T>*>(ib.prev);
    bool bada = false, badb = false;
#pragma unroll
    for (int q = 0; q < QS; q++) {
        if (!stored(q)) continue;
        const int m = mode_of(q);
        if (acta) {
            phia[m] = pa[q];
            if (o2 && a.nsteps > 0) pva[m] = fa[q];
            bada |= !(isfinite(pa[q].x) && isfinite(pa[q].y));
        }
        if (actb) {
            phib[m] = pb[q];
            if (o2 && a.nsteps > 0) pvb[m] = fb[q];
            badb |= !(isfinite(pb[q].x) && isfinite(pb[q].y));
        }
    }
    if (bada) atomicOr(&ia.ctrl->nonfinite, 1);
    if (badb) atomicOr(&ib.ctrl->nonfinite, 1);
    // every thread has read the step counters before thread 0 of the line
    // advances them
    __syncthreads();
    if (t == 0) {
        if (acta) {
            ia.ctrl->step = stepa + a.nsteps;
            if (a.nsteps > 0) ia.ctrl->have_prev = 1;
        }
        if (actb) {
            ib.ctrl->step = stepb + a.nsteps;
            if (a.nsteps > 0) ib.ctrl->have_prev = 1;
        }
    }
}

// Complex field, one realization per line: thread t keeps bins j = t + q N/8
// of phi (FFT order).  KIND 0: CGL, F = -(1 + i beta) FFT[|phi|^2 phi];
// 1: no nonlinearity.  The noise block t + qM (q < 4) serves bins q and 7 - q.
template <typename T, int N, int PAD, int DM, int KIND, bool RS>
__global__ void __launch_bounds__(256) k_line1d_cplx(Line1dArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr bool DA = DM == 1, PS = DM == 2;   // 2/3 truncation, phase shift
    constexpr int TPL = N / 8, M = N / 8;
    constexpr int LPB = 256 / TPL;
    constexpr int LL = lds_len<N, PAD>();
    const Geo& g = a.g;
    const int tid = threadIdx.x;
    const int l = tid / TPL, t = tid - l * TPL;
    const int line = blockIdx.x * LPB + l;
    // one line of LDS per line, two where a second line shares the stages
    // (the launcher sizes the allocation the same way)
    constexpr int LSTR = (RS || PS) ? 2 * LL : LL;
    cx<T>* L = reinterpret_cast<cx<T>*>(smem_raw) + (size_t)l * LSTR;
    const bool valid = line < a.nlines;
    const Item& it = a.items[valid ? line : 0];
    const bool act = valid && a.sub < it.steps;
    Line1dTw<T, N, 2> tw;
    line1d_tw<T, N, 2>(tw, t, twid<T>(it.tw0));
    const T inv = (T)it.inv_vol;
    const int kept = g.kept[0], kp = g.kp[0];
    int si[8];
#pragma unroll
    for (int q = 0; q < 8; q++) si[q] = (DA && (q == 3 || q == 4)) ? -1 : stored_idx(t + q * M, N, kept, kp);
    cx<T>* phi = reinterpret_cast<cx<T>*>(it.phi);
    cx<T> p[8];
    if (a.mode == MODE_IC) {
        // per site: phi = sigma (z1 + i z2) of the Philox block (site, 0, r, 1)
#pragma unroll
        for (int q = 0; q < 8; q++) {
            T z1 = T(0), z2 = T(0);
            if (valid) normal_pair(it.seed, (uint32_t)(t + q * M), 0u, it.r, 1u, z1, z2);
            p[q] = {(T)it.ic_sigma * z1, (T)it.ic_sigma * z2};
        }
        fft_line<T, N, -1, PAD>(p, t, L, 1, tw);
        if (valid) {
#pragma unroll
            for (int q = 0; q < 8; q++)
                if (si[q] >= 0) phi[si[q]] = p[q];
        }
        return;
    }
    cx<T> fp[8];
    Coef<T> cf[8];
    const int64_t step0 = valid ? it.ctrl->step : 0;
    const int hp = valid ? it.ctrl->have_prev : 0;
    const bool o2 = it.order == 2;
    const cx<T>* prev0 = reinterpret_cast<const cx<T>*>(it.prev);
#pragma unroll
    for (int q = 0; q < 8; q++) {
        p[q] = fp[q] = czero<T>();
        cf[q] = Coef<T>{czero<T>(), czero<T>(), czero<T>(), T(0)};
        if (si[q] < 0 || !valid) continue;
        p[q] = phi[si[q]];
        if (o2 && hp) fp[q] = prev0[si[q]];
        cf[q] = load_coef_t<T, true>(it.coef, coef_key(it, sgn_idx(t + q * M, N), 0, 0));   // complex tables
    }
    const cx<T> pref = nl_pref<T>(it, T(0));
    const T rsq = (T)(1.0 / sqrt((double)N));
    bool bad = false;
#pragma unroll 1
    for (int s = 0; s < a.nsteps; s++) {
        cx<T> F[8], eta[8];
        // real-space noise: site x = t + qM takes (z1 + i z2)/sqrt2 of half
        // q div 4 of the Philox block (t + (q mod 4) M, n, r, 3)
        cx<T> e[8];
        if constexpr (RS) {
            const T rs2 = T(0.70710678118654752440084436210484903928);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                e[q] = e[q + 4] = czero<T>();
                if (!act) continue;
                uint32_t x[4];
                T z1, z2, z3, z4;
                philox_block(it.seed, (uint32_t)(t + q * M), (uint32_t)(step0 + s), it.r, 3u, x);
                box_muller32(x[0], x[1], z1, z2);
                box_muller32(x[2], x[3], z3, z4);
                e[q] = {rs2 * z1, rs2 * z2};
                e[q + 4] = {rs2 * z3, rs2 * z4};
            }
        }
        if constexpr (KIND == 0) {
            cx<T> z[2][8];
#pragma unroll
            for (int q = 0; q < 8; q++) z[0][q] = p[q];
            if constexpr (PS) {
                // the grid and the grid shifted by dx/2 together
                cx<T> phs[8];
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    phs[q] = cispi<T>((T)sgn_idx(t + q * M, N) / (T)N);
                    z[1][q] = cmul(phs[q], p[q]);
                }
                fft_lines<T, N, +1, PAD, 2>(z, t, L, 2, 1, tw);
#pragma unroll
                for (int u = 0; u < 2; u++) {
#pragma unroll
                    for (int q = 0; q < 8; q++) {
                        const T x = z[u][q].x * inv, y = z[u][q].y * inv;
                        const T m2 = x * x + y * y;
                        z[u][q] = {m2 * x, m2 * y};
                    }
                }
                fft_lines<T, N, -1, PAD, 2>(z, t, L, 2, 1, tw);
#pragma unroll
                for (int q = 0; q < 8; q++) z[0][q] = T(0.5) * (z[0][q] + cmulc(z[1][q], phs[q]));
            } else {
                fft_line<T, N, +1, PAD>(z[0], t, L, 1, tw);
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    const T x = z[0][q].x * inv, y = z[0][q].y * inv;
                    const T m2 = x * x + y * y;
                    z[0][q] = {m2 * x, m2 * y};
                }
            }
            if constexpr (RS && PS) {
                // the mean is already transformed: the site noise alone
                fft_line<T, N, -1, PAD>(e, t, L, 1, tw);
            } else if constexpr (RS) {
                // the nonlinearity and the site noise through the forward
                // stages together
#pragma unroll
                for (int q = 0; q < 8; q++) z[1][q] = e[q];
                fft_lines<T, N, -1, PAD, 2>(z, t, L, 2, 1, tw);
#pragma unroll
                for (int q = 0; q < 8; q++) e[q] = z[1][q];
            } else if constexpr (!PS) {
                fft_line<T, N, -1, PAD>(z[0], t, L, 1, tw);
            }
#pragma unroll
            for (int q = 0; q < 8; q++) F[q] = (si[q] >= 0) ? cmul(pref, z[0][q]) : czero<T>();
        } else {
#pragma unroll
            for (int q = 0; q < 8; q++) F[q] = czero<T>();
            if constexpr (RS) fft_line<T, N, -1, PAD>(e, t, L, 1, tw);
        }
        if constexpr (RS) {
#pragma unroll
            for (int q = 0; q < 8; q++) eta[q] = rsq * e[q];
        }
        if constexpr (!RS) {
#pragma unroll
            for (int q = 0; q < 4; q++) {
                eta[q] = eta[7 - q] = czero<T>();
                if (DA && q == 3) continue;
                if (!act || (si[q] < 0 && si[7 - q] < 0)) continue;
                uint32_t x[4];
                philox_block(it.seed, (uint32_t)(t + q * M), (uint32_t)(step0 + s), it.r, 0u, x);
                NoiseSlot ns;
                ns.P = (uint32_t)(t + q * M);
                ns.kind = 0;
                ns.half = 0u;
                eta[q] = eta_of<T>(x, ns);
                ns.half = 1u;
                eta[7 - q] = eta_of<T>(x, ns);
            }
        }
        const bool up = o2 && (s > 0 || hp);
#pragma unroll
        for (int q = 0; q < 8; q++) {
            if (si[q] < 0) continue;
            cx<T> nw = cmul(cf[q].E, p[q]) + cmul(cf[q].wa, F[q]) + cf[q].G * eta[q];
            if (o2) {
                nw = nw + cmul(cf[q].wb, up ? fp[q] : F[q]);
                fp[q] = F[q];
            }
            if (act) p[q] = nw;
        }
    }
    cx<T>* pv = reinterpret_cast<cx<T>*>(it.prev);
    if (act) {
#pragma unroll
        for (int q = 0; q < 8; q++) {
            if (si[q] < 0) continue;
            phi[si[q]] = p[q];
            if (o2 && a.nsteps > 0) pv[si[q]] = fp[q];
            bad |= !(isfinite(p[q].x) && isfinite(p[q].y));
        }
    }
    if (bad) atomicOr(&it.ctrl->nonfinite, 1);
    __syncthreads();
    if (t == 0 && act) {
        it.ctrl->step = step0 + a.nsteps;
        if (a.nsteps > 0) it.ctrl->have_prev = 1;
    }
}

// ---------------------------------------------------------------- box-averaged width (Sec. 5 KPZ)
// With h(x) = N^-d sum_a h_a e^{2 pi i a.x/N}, the mean over boxes of l^d
// sites of |box mean|^2 is N^-2d sum_c |A_c|^2 with A_c = sum_{a = c mod N/l}
// h_a D_l(a), D_l(a) = prod_i (1/l) sum_{u < l} e^{2 pi i a_i u/N}, and the
// mean of |h|^2 is N^-2d sum_a |h_a|^2 (Parseval): the box variance needs no
// transform.  D_l vanishes on the multiples of N/l other than 0, so the mode
// a = 0 is alone in its class and cancels; it is left out of both sums.  Per
// stored mode of one realization the kernel adds to the class sums of every
// level l = 2^j (an interior mode of a real field adds its mirror -a to the
// class of -a with the conjugate value).  The coarse levels, whose few
// classes every mode reaches, are summed in LDS first.
__device__ __forceinline__ double2 box_dirichlet(int a, int l, int N)
{
    const int am = ((a % N) + N) % N;
    if (am == 0) return make_double2(1.0, 0.0);
    if ((am * l) % N == 0) return make_double2(0.0, 0.0);
    const double num = sinpi((double)am * l / N), den = sinpi((double)am / N);
    double s, c;
    sincospi((double)am * (l - 1) / N, &s, &c);
    const double m = num / (l * den);
    return make_double2(m * c, m * s);
}

constexpr int BOX_LDS = 1024;   // complex class sums held in LDS per block

template <typename T>
__global__ void __launch_bounds__(256) k_boxclass(BoxArgs a)
{
    __shared__ double lcls[2 * BOX_LDS];
    __shared__ double red[256];
    for (int i = threadIdx.x; i < 2 * a.nlds; i += blockDim.x) lcls[i] = 0.0;
    __syncthreads();
    const Geo& g = a.g;
    const Item& it = a.items[a.r];
    const int last = g.ndim - 1;
    const cx<T>* phi = reinterpret_cast<const cx<T>*>(it.phi);
    double s2 = 0.0;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < a.total; idx += gridDim.x * blockDim.x) {
        const int col = idx % g.pitch;
        if (col >= g.kept[last]) continue;
        const int rest = idx / g.pitch;
        const int i1 = (g.ndim == 3) ? rest % g.kept[1] : 0;
        const int i0 = (g.ndim == 3) ? rest / g.kept[1] : rest;
        int ai[3] = {sgn_idx(fft_pos(i0, g.n[0], g.kept[0], g.kp[0]), g.n[0]), 0, 0};
        if (g.ndim == 3) ai[1] = sgn_idx(fft_pos(i1, g.n[1], g.kept[1], g.kp[1]), g.n[1]);
        ai[last] = g.cplx ? sgn_idx(fft_pos(col, g.n[last], g.kept[last], g.kp[last]), g.n[last]) : col;
        if (ai[0] == 0 && ai[1] == 0 && ai[last] == 0) continue;
        const bool mirror = !g.cplx && col > 0 && 2 * col < g.n[last];
        const cx<T> p = phi[idx];
        const double hx = (double)p.x, hy = (double)p.y;
        s2 += (mirror ? 2.0 : 1.0) * (hx * hx + hy * hy);
        size_t off = 0;
        for (int j = 1; j <= a.J; j++) {
            const int l = 1 << j, P = a.N >> j;
            size_t cls_size = 1;
            for (int d = 0; d < g.ndim; d++) cls_size *= (size_t)P;
            double2 D = make_double2(1.0, 0.0);
            bool zero = false;
            for (int d = 0; d < g.ndim; d++) {
                const double2 e = box_dirichlet(ai[d], l, a.N);
                if (e.x == 0.0 && e.y == 0.0) zero = true;
                D = make_double2(D.x * e.x - D.y * e.y, D.x * e.y + D.y * e.x);
            }
            if (!zero) {
                const double vx = hx * D.x - hy * D.y, vy = hx * D.y + hy * D.x;
                size_t c = 0, cm = 0;
                for (int d = 0; d < g.ndim; d++) {
                    c = c * P + (size_t)(((ai[d] % P) + P) % P);
                    cm = cm * P + (size_t)(((-ai[d] % P) + P) % P);
                }
                c += off;
                cm += off;
                if (c >= a.lds_base) {
                    atomicAdd(&lcls[2 * (c - a.lds_base)], vx);
                    atomicAdd(&lcls[2 * (c - a.lds_base) + 1], vy);
                } else {
                    atomicAdd(&a.cls[2 * c], vx);
                    atomicAdd(&a.cls[2 * c + 1], vy);
                }
                if (mirror) {
                    if (cm >= a.lds_base) {
                        atomicAdd(&lcls[2 * (cm - a.lds_base)], vx);
                        atomicAdd(&lcls[2 * (cm - a.lds_base) + 1], -vy);
                    } else {
                        atomicAdd(&a.cls[2 * cm], vx);
                        atomicAdd(&a.cls[2 * cm + 1], -vy);
                    }
                }
            }
            off += cls_size;
        }
    }
    red[threadIdx.x] = s2;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(&a.sums[0], red[0]);
    for (int i = threadIdx.x; i < 2 * a.nlds; i += blockDim.x)
        if (lcls[i] != 0.0) atomicAdd(&a.cls[2 * a.lds_base + i], lcls[i]);
}

// sum_c |A_c|^2 per level, one atomic per block and level
static __global__ void __launch_bounds__(256) k_boxfinal(BoxArgs a, size_t ncls)
{
    __shared__ double red[16];
    for (int j = threadIdx.x; j < 16; j += blockDim.x) red[j] = 0.0;
    __syncthreads();
    const int nd = a.g.ndim;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncls; c += (size_t)gridDim.x * blockDim.x) {
        size_t off = 0;
        int j = 1;
        for (; j < a.J; j++) {
            size_t sz = 1;
            for (int d = 0; d < nd; d++) sz *= (size_t)(a.N >> j);
            if (c < off + sz) break;
            off += sz;
        }
        const double x = a.cls[2 * c], y = a.cls[2 * c + 1];
        const double v = x * x + y * y;
        if (v != 0.0) atomicAdd(&red[j], v);
    }
    __syncthreads();
    for (int j = 1 + (int)threadIdx.x; j <= a.J; j += blockDim.x)
        if (red[j] != 0.0) atomicAdd(&a.sums[j], red[j]);
}

// ---------------------------------------------------------------- time-frequency observables (App. C)

// One line per (stored mode, realization): the window phi_a(m) and the kicks
// xi_a(m) = G_a eta_a(n0 + m) of the steps taken from the samples go through
// the unscaled transform with e^{+2 pi i b m / M} together; an interior mode
// of a real field adds its mirror -a (the conjugate transforms at -w_b, read
// back through LDS); FP64 sums per shell and frequency.
template <typename T, int M, int PAD>
__global__ void __launch_bounds__(256) k_spectrum(SpecArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    constexpr int TPL = M / 8;
    constexpr int LL = lds_len<M, PAD>();
    const int tid = threadIdx.x;
    const int lpb = (int)blockDim.x / TPL;
    const int l = tid / TPL, t = tid - l * TPL;
    const int idx = blockIdx.x * lpb + l;     // stored element of the realization
    const Item& it = a.items[blockIdx.y];
    const Geo& g = a.g;
    const int last = g.ndim - 1;
    cx<T>* L = lds + l * 2 * LL;
    // the mode of this line, its shell, weight, G and D(k); lanes of lines
    // without a mode compute on zeros (they share the block's barriers)
    bool use = idx < a.total;
    int col = 0, i0 = 0, i1 = 0;
    if (use) {
        col = idx % g.pitch;
        const int rest = idx / g.pitch;
        i1 = (g.ndim == 3) ? rest % g.kept[1] : 0;
        i0 = (g.ndim == 3) ? rest / g.kept[1] : rest;
        use = col < g.kept[last];
    }
    const int j0 = fft_pos(i0, g.n[0], g.kept[0], g.kp[0]);
    const int j1 = (g.ndim == 3) ? fft_pos(i1, g.n[1], g.kept[1], g.kp[1]) : 0;
    const int jl = g.cplx ? fft_pos(col, g.n[last], g.kept[last], g.kp[last]) : col;
    const int a0 = sgn_idx(j0, g.n[0]);
    const int a1 = (g.ndim == 3) ? sgn_idx(j1, g.n[1]) : 0;
    const int al = g.cplx ? sgn_idx(jl, g.n[last]) : col;
    double G = 0.0, Da = 0.0;
    if (use) {
        const int ew = it.coef_cplx ? 8 : 4;
        const int entry = (it.coef_mode == COEF_PER_MODE) ? per_mode_key(g, a0, col)
                          : ((g.ndim == 3) ? coef_key(it, a0, a1, al) : coef_key(it, a0, al, 0));
        G = (double)reinterpret_cast<const T*>(it.coef)[(size_t)entry * ew + (it.coef_cplx ? 6 : 3)];
        const double k0 = it.dk[0] * a0;
        const double k1 = (g.ndim == 3) ? it.dk[1] * a1 : 0.0;
        const double kl = it.dk[last] * al;
        Da = a.D * (a.kpow == 2 ? k0 * k0 + k1 * k1 + kl * kl : 1.0);
        use = G > 0.0 && Da > 0.0;
    }
    const double w = (!g.cplx && col > 0 && 2 * col < g.n[last]) ? 2.0 : 1.0;
    const int shell = ceil_isqrt(a0 * a0 + a1 * a1 + al * al);

    cx<T> v[2][8];
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const int m = t + q * TPL;
        v[0][q] = czero<T>();
        v[1][q] = czero<T>();
        if (use) {
            v[0][q] = *reinterpret_cast<const cx<T>*>(a.series + (size_t)m * a.slot + (size_t)blockIdx.y * a.rstride +
                                                      (size_t)idx * sizeof(cx<T>));
            const cx<T> e = noise_eta<T>(g, it, j0, j1, jl, (uint32_t)(a.step0 + m));
            v[1][q] = {(T)G * e.x, (T)G * e.y};
        }
    }
    LineTw<T, M> tw;
    line_tw_load(tw, t, reinterpret_cast<const cx<T>*>(a.tw));
    fft_lines<T, M, +1, PAD, 2>(v, t, L, 1, LL, tw);
    // the transforms at -w_b for the mirror of an interior real mode
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; q++) {
        L[lds_slot<PAD>(t + q * TPL)] = v[0][q];
        L[LL + lds_slot<PAD>(t + q * TPL)] = v[1][q];
    }
    __syncthreads();
    if (!use) return;   // no barrier follows
    const int nb = a.nbins;
    const double invR = 1.0 / (double)a.nitems;
    const double cC = a.vol * a.h / M * invR, cX = a.vol / (2.0 * Da * M) * invR;
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const int b = t + q * TPL;
        const double px = v[0][q].x, py = v[0][q].y, xx = v[1][q].x, xy = v[1][q].y;
        double c2 = px * px + py * py;
        double xr = px * xx + py * xy, xi = py * xx - px * xy;   // phi conj(xi)
        if (a.dacc) {
            // FDT check (Sec. 5): 2 Im chi - (w_b / D_a) C of this mode (its own
            // frequencies; the mirror of an interior mode is counted at the end),
            // w_b h = 2 pi b / M with b signed
            const int bs = (2 * b < M) ? b : b - M;
            const double wh = 6.283185307179586476925 * (double)bs / (double)M;
            atomicAdd(&a.dacc[(size_t)idx * M + b], a.vol / (Da * M) * invR * (xi - wh * c2));
        }
        if (w == 2.0) {
            const int bm = (M - b) & (M - 1);
            const cx<T> pm = L[lds_slot<PAD>(bm)], km = L[LL + lds_slot<PAD>(bm)];
            const double qx = pm.x, qy = pm.y, yx = km.x, yy = km.y;
            c2 += qx * qx + qy * qy;
            xr += qx * yx + qy * yy;         // conj(phi(-b) conj xi(-b))
            xi -= qy * yx - qx * yy;
        }
        atomicAdd(&a.acc[(size_t)shell * M + b], cC * c2);
        atomicAdd(&a.acc[((size_t)nb + shell) * M + b], cX * xr);
        atomicAdd(&a.acc[((size_t)2 * nb + shell) * M + b], cX * xi);
    }
    if (blockIdx.y == 0 && t == 0) atomicAdd(&a.acc[(size_t)3 * nb * M + shell], w);
}

// Sums of the FDT deviations: out[0] += w |Delta|, out[1] += Delta of the modes
// stored with their partner (w = 1); an interior mode of a real field stands
// for -a as well, whose deviations are -Delta_{a,-b}.
static __global__ void __launch_bounds__(256) k_fdt_reduce(Geo g, const double* dacc, int total, int M, double* out)
{
    __shared__ double ra[256], rs[256];
    double sa = 0.0, ss = 0.0;
    const int last = g.ndim - 1;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)total * M;
         i += (size_t)gridDim.x * blockDim.x) {
        const int col = (int)((i / (size_t)M) % (size_t)g.pitch);
        if (col >= g.kept[last]) continue;
        const double v = dacc[i];
        const bool twice = !g.cplx && col > 0 && 2 * col < g.n[last];
        sa += (twice ? 2.0 : 1.0) * fabs(v);
        if (!twice) ss += v;
    }
    ra[threadIdx.x] = sa;
    rs[threadIdx.x] = ss;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            ra[threadIdx.x] += ra[threadIdx.x + st];
            rs[threadIdx.x] += rs[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(&out[0], ra[0]);
        atomicAdd(&out[1], rs[0]);
    }
}

}  // namespace setd
