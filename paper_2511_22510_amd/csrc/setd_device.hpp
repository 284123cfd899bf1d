// setd_device.hpp -- device building blocks of the gfx950 SETD path.
//
//  * cx<T>: complex numbers in float or double.
//  * fft_line<T, N, SIGN, PAD>: one length-N line transform held by N/8
//    threads, 8 values per thread.  Stockham autosort stages (radix 2/4 first,
//    then radix 8) with the values exchanged through LDS between stages.
//    Thread t holds elements t + q N/8 (q = 0..7) on entry and output bins
//    t + q N/8 on exit, so the first stage reads and the last stage writes in
//    the layout in which lines are loaded from and stored to global memory.
//    Each thread keeps one base twiddle per radix-8 stage in registers
//    (LineTw) or, for kernels that run several transforms, all seven powers
//    of it (LineTwP).
//  * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller normals
//    for the Fourier-space noise of App. B (two modes per Philox block) and
//    the initial condition (one block per site).
//  * phi1(x) = (e^x - 1)/x and phi2(x) = (e^x - 1 - x)/x^2 in FP64 for the ETD
//    coefficients of Eq. SETD1/SETD2, by Taylor series for |x| < 1 and closed
//    forms otherwise.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "setd_types.hpp"

namespace setd {

template <typename T>
struct cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.x, s * a.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) { return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> czero() { return {T(0), T(0)}; }

// ---------------------------------------------------------------- global memory
// Loads and stores through the global address space at a 32-bit byte offset
// from a wave-uniform base, so that the compiler emits global (not flat)
// instructions with the base in scalar registers; callers guarantee that the
// offset fits 32 bits.
template <typename T>
struct vec2;
template <>
struct vec2<float> {
    typedef float __attribute__((ext_vector_type(2))) type;
};
template <>
struct vec2<double> {
    typedef double __attribute__((ext_vector_type(2))) type;
};
#define SETD_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ cx<T> gload(const void* base, uint32_t off)
{
    typedef typename vec2<T>::type V;
    const V u = *(const SETD_GLOBAL V*)((const SETD_GLOBAL char*)base + off);
    return {u.x, u.y};
}

template <typename T>
__device__ __forceinline__ void gstore(void* base, uint32_t off, cx<T> v)
{
    typedef typename vec2<T>::type V;
    V u;
    u.x = v.x;
    u.y = v.y;
    *(SETD_GLOBAL V*)((SETD_GLOBAL char*)base + off) = u;
}

template <typename T>
struct alignas(4 * sizeof(T)) T4 {
    T a, b, c, d;
};

template <typename T>
__device__ __forceinline__ T4<T> gload4(const void* base, uint32_t off)
{
    typedef T __attribute__((ext_vector_type(4))) V;
    const V u = *(const SETD_GLOBAL V*)((const SETD_GLOBAL char*)base + off);
    return {u.x, u.y, u.z, u.w};
}

// ---------------------------------------------------------------- buffer access
// Raw buffer loads and stores: a 128-bit resource in scalar registers holds the
// base and byte size of an array (third word 0x00020000, the gfx9-family
// format for untyped dword access), and each access adds a 32-bit per-lane
// offset and a wave-uniform offset.  A lane whose per-lane offset is at or past
// the size reads zero and writes nothing, which is how masked lanes are
// expressed (BUF_OOB; every array addressed this way is under 2 GiB).
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr uint32_t BUF_OOB = 0x80000000u;

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ cx<T> bload(rsrc_t r, uint32_t voff, uint32_t soff)
{
    if constexpr (sizeof(T) == 4) {
        const u32x2 u = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
        return {__uint_as_float(u.x), __uint_as_float(u.y)};
    } else {
        const u32x4 u = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
        return {__hiloint2double((int)u.y, (int)u.x), __hiloint2double((int)u.w, (int)u.z)};
    }
}

template <typename T>
__device__ __forceinline__ void bstore(rsrc_t r, uint32_t voff, uint32_t soff, cx<T> v)
{
    if constexpr (sizeof(T) == 4) {
        u32x2 u;
        u.x = __float_as_uint(v.x);
        u.y = __float_as_uint(v.y);
        __builtin_amdgcn_raw_buffer_store_b64(u, r, (int)voff, (int)soff, 0);
    } else {
        const unsigned long long a = (unsigned long long)__double_as_longlong(v.x);
        const unsigned long long b = (unsigned long long)__double_as_longlong(v.y);
        u32x4 u;
        u.x = (unsigned)a;
        u.y = (unsigned)(a >> 32);
        u.z = (unsigned)b;
        u.w = (unsigned)(b >> 32);
        __builtin_amdgcn_raw_buffer_store_b128(u, r, (int)voff, (int)soff, 0);
    }
}

template <typename T>
__device__ __forceinline__ T4<T> bload4(rsrc_t r, uint32_t voff, uint32_t soff)
{
    if constexpr (sizeof(T) == 4) {
        const u32x4 u = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
        return {__uint_as_float(u.x), __uint_as_float(u.y), __uint_as_float(u.z), __uint_as_float(u.w)};
    } else {
        const u32x4 u = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
        const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff + 16, 0);
        return {__hiloint2double((int)u.y, (int)u.x), __hiloint2double((int)u.w, (int)u.z),
                __hiloint2double((int)w.y, (int)w.x), __hiloint2double((int)w.w, (int)w.z)};
    }
}

// ---------------------------------------------------------------- butterflies
// a * (SIGN i)
template <int SIGN, typename T>
__device__ __forceinline__ cx<T> mul_si(cx<T> a)
{
    if constexpr (SIGN > 0) return {-a.y, a.x};
    else return {a.y, -a.x};
}

template <int SIGN, typename T>
__device__ __forceinline__ void dft2(cx<T>* u)
{
    cx<T> d = u[0] - u[1];
    u[0] = u[0] + u[1];
    u[1] = d;
}

// X_k = sum_r u_r exp(SIGN 2 pi i r k / 4), in place on u[0..3] (stride S)
template <int SIGN, int S, typename T>
__device__ __forceinline__ void dft4s(cx<T>* u)
{
    cx<T> s02 = u[0] + u[2 * S], d02 = u[0] - u[2 * S];
    cx<T> s13 = u[S] + u[3 * S], d13 = mul_si<SIGN>(u[S] - u[3 * S]);
    u[0] = s02 + s13;
    u[2 * S] = s02 - s13;
    u[S] = d02 + d13;
    u[3 * S] = d02 - d13;
}

template <int SIGN, typename T>
__device__ __forceinline__ void dft4(cx<T>* u) { dft4s<SIGN, 1>(u); }

template <int SIGN, typename T>
__device__ __forceinline__ void dft8(cx<T>* u)
{
    // even / odd halves, then combine with W8^k, W8 = exp(SIGN 2 pi i / 8)
    dft4s<SIGN, 2>(u);       // u0 u2 u4 u6 -> E0 E1 E2 E3
    dft4s<SIGN, 2>(u + 1);   // u1 u3 u5 u7 -> O0 O1 O2 O3
    const T r = T(0.70710678118654752440084436210484903928);
    cx<T> o1 = u[3], o2 = u[5], o3 = u[7];
    // o1 * W8 = r (x - SIGN y, SIGN x + y); o3 * W8^3 = r (-x - SIGN y, SIGN x - y);
    // the factor r is applied inside the final fused multiply-adds
    const cx<T> d1 = {o1.x - T(SIGN) * o1.y, T(SIGN) * o1.x + o1.y};
    const cx<T> w2 = mul_si<SIGN>(o2);
    const cx<T> d3 = {-o3.x - T(SIGN) * o3.y, T(SIGN) * o3.x - o3.y};
    const cx<T> e0 = u[0], e1 = u[2], e2 = u[4], e3 = u[6], o0 = u[1];
    u[0] = e0 + o0;
    u[4] = e0 - o0;
    u[1] = {fma(r, d1.x, e1.x), fma(r, d1.y, e1.y)};
    u[5] = {fma(-r, d1.x, e1.x), fma(-r, d1.y, e1.y)};
    u[2] = e2 + w2;
    u[6] = e2 - w2;
    u[3] = {fma(r, d3.x, e3.x), fma(r, d3.y, e3.y)};
    u[7] = {fma(-r, d3.x, e3.x), fma(-r, d3.y, e3.y)};
}

template <int R, int SIGN, typename T>
__device__ __forceinline__ void dft(cx<T>* u)
{
    if constexpr (R == 2) dft2<SIGN>(u);
    else if constexpr (R == 4) dft4<SIGN>(u);
    else dft8<SIGN>(u);
}

// ---------------------------------------------------------------- line FFT
constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// Stage plan of a length-N line: a radix R0 in {2, 4, 8} first, then radix 8.
template <int N>
struct FftPlan {
    static constexpr int LG = ilog2(N);
    static constexpr int R0 = (LG % 3 == 0) ? 8 : (1 << (LG % 3));
    static constexpr int NST = (LG % 3 == 0) ? LG / 3 : LG / 3 + 1;
};

// LDS slot of element e with one pad slot after every 2^PAD elements
// (PAD = 0: no padding).  Spreads the strided Stockham writes over the banks.
template <int PAD>
__device__ __forceinline__ int lds_slot(int e)
{
    if constexpr (PAD > 0) return e + (e >> PAD);
    else return e;
}

template <int N, int PAD>
constexpr int lds_len() { return PAD > 0 ? N + (N >> PAD) : N; }

// Per-thread twiddles: for the radix-8 stage after NS combined points, thread
// t multiplies its inputs r = 1..7 by w^r with w = exp(-2 pi i (t mod NS) / (8 NS)).
// Only the base w of each stage is kept; its powers are formed by products.
template <typename T, int N>
struct LineTw {
    cx<T> w[FftPlan<N>::NST > 1 ? FftPlan<N>::NST - 1 : 1];
};

// tw[k] = exp(-2 pi i k / N) for k < N (FP64-evaluated table in state precision)
template <typename T, int N>
__device__ __forceinline__ void line_tw_load(LineTw<T, N>& L, int t, const cx<T>* __restrict__ tw)
{
    constexpr int NST = FftPlan<N>::NST;
    int ns = FftPlan<N>::R0;
#pragma unroll
    for (int s = 0; s + 1 < NST; s++) {
        L.w[s] = gload<T>(tw, (uint32_t)((t & (ns - 1)) * (N / (ns * 8))) * (uint32_t)sizeof(cx<T>));
        ns *= 8;
    }
}

// First stage (no twiddles).  Thread t owns butterflies j = t + b N/8,
// b < 8/R0, whose inputs are elements j + r N/R0, i.e. v[b + (8/R0) r].
template <typename T, int N, int R, int SIGN>
__device__ __forceinline__ void fft_stage0(cx<T>* v)
{
    constexpr int NB = 8 / R;
#pragma unroll
    for (int b = 0; b < NB; b++) {
        cx<T> u[R];
#pragma unroll
        for (int r = 0; r < R; r++) u[r] = v[b + NB * r];
        dft<R, SIGN>(u);
#pragma unroll
        for (int r = 0; r < R; r++) v[b + NB * r] = u[r];
    }
}

// Powers w, w^2, ..., w^7 of a stage's base twiddle.
template <typename T>
__device__ __forceinline__ void tw_powers(cx<T> w, cx<T> (&p)[7])
{
    p[0] = w;
    p[1] = cmul(w, w);
    p[2] = cmul(p[1], w);
    p[3] = cmul(p[1], p[1]);
    p[4] = cmul(p[3], w);
    p[5] = cmul(p[2], p[2]);
    p[6] = cmul(p[3], p[2]);
}

// Radix-8 stage: input r is multiplied by w^r (forward) or conj(w)^r
// (inverse) before the butterfly, p holding w^1..w^7.
template <typename T, int SIGN>
__device__ __forceinline__ void fft_stage8(cx<T>* v, const cx<T> (&p)[7])
{
#pragma unroll
    for (int r = 1; r < 8; r++) v[r] = (SIGN < 0) ? cmul(v[r], p[r - 1]) : cmulc(v[r], p[r - 1]);
    dft8<SIGN>(v);
}

// Twiddles of a line transform with every power formed once per thread (for
// kernels that run several transforms with the same t and have the registers).
template <typename T, int N>
struct LineTwP {
    cx<T> p[FftPlan<N>::NST > 1 ? FftPlan<N>::NST - 1 : 1][7];
};

template <typename T, int N>
__device__ __forceinline__ void line_tw_expand(LineTwP<T, N>& P, const LineTw<T, N>& L)
{
#pragma unroll
    for (int s = 0; s + 1 < FftPlan<N>::NST; s++) tw_powers(L.w[s], P.p[s]);
}

// twiddle multiplication and butterfly of radix-8 stage s (s >= 0 after the first)
template <typename T, int N, int SIGN>
__device__ __forceinline__ void tw_stage(cx<T>* v, const LineTw<T, N>& L, int s)
{
    cx<T> p[7];
    tw_powers(L.w[s], p);
    fft_stage8<T, SIGN>(v, p);
}

template <typename T, int N, int SIGN>
__device__ __forceinline__ void tw_stage(cx<T>* v, const LineTwP<T, N>& P, int s)
{
    fft_stage8<T, SIGN>(v, P.p[s]);
}

// Slot distance of element e0 + d from element e0 for a power-of-two d when no
// multiple of 2^PAD lies in (e0, e0 + d] other than those d itself implies
// (see fft_exchange): d plus one pad slot per 2^PAD.
template <int PAD>
constexpr int slot_step(int d) { return PAD > 0 ? d + (d >> PAD) : d; }

// Write the outputs of a stage (radix R, NS points combined before it) to
// their Stockham positions (j / NS) NS R + j mod NS + r NS, then read the next
// stage's inputs back in the natural layout t + q N/8.  Element e of line k
// lives at lds[k * lstep + lds_slot<PAD>(e) * stride]; the NL lines of a thread
// share the two block barriers of the exchange.
// Every address is one per-thread base plus a compile-time offset: with
// A = (j / NS) NS R and power-of-two NS, R, 2^PAD, the positions A + j mod NS
// + r NS cross a multiple of 2^PAD exactly where r NS does when NS R >= 2^PAD
// (offset slot_step(r NS)) and never otherwise (offset r NS); the reads
// t + q N/8 with t < N/8 likewise sit at slot(t) + slot_step(q N/8).
template <typename T, int N, int R, int NS, int PAD, int NL>
__device__ __forceinline__ void fft_exchange(cx<T> (&v)[NL][8], int t, cx<T>* lds, int stride, int lstep)
{
    constexpr int NB = 8 / R;
    constexpr bool LIN = PAD == 0 || NS * R >= (1 << PAD);
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int j = t + b * (N / 8);
        const int base = (j / NS) * NS * R + (j & (NS - 1));
        cx<T>* p = lds + lds_slot<PAD>(base) * stride;
#pragma unroll
        for (int k = 0; k < NL; k++) {
#pragma unroll
            for (int r = 0; r < R; r++) p[k * lstep + (LIN ? slot_step<PAD>(r * NS) : r * NS) * stride] = v[k][b + NB * r];
        }
    }
    __syncthreads();
    const cx<T>* p = lds + lds_slot<PAD>(t) * stride;
#pragma unroll
    for (int k = 0; k < NL; k++) {
#pragma unroll
        for (int q = 0; q < 8; q++) v[k][q] = p[k * lstep + slot_step<PAD>(q * (N / 8)) * stride];
    }
}

// NL independent line transforms X_k = sum_m x_m exp(SIGN 2 pi i k m / N),
// unscaled, held by the same threads (same t, same twiddles).  Every thread of
// the block must call it (it contains block barriers).
template <typename T, int N, int SIGN, int PAD, int NL, typename TW>
__device__ __forceinline__ void fft_lines(cx<T> (&v)[NL][8], int t, cx<T>* lds, int stride, int lstep, const TW& tw)
{
    static_assert(N >= 8 && (N & (N - 1)) == 0, "power-of-two line length >= 8");
    constexpr int R0 = FftPlan<N>::R0;
    constexpr int NST = FftPlan<N>::NST;
#pragma unroll
    for (int k = 0; k < NL; k++) fft_stage0<T, N, R0, SIGN>(v[k]);
    if constexpr (NST > 1) {
        fft_exchange<T, N, R0, 1, PAD, NL>(v, t, lds, stride, lstep);
#pragma unroll
        for (int k = 0; k < NL; k++) tw_stage<T, N, SIGN>(v[k], tw, 0);
    }
    if constexpr (NST > 2) {
        fft_exchange<T, N, 8, R0, PAD, NL>(v, t, lds, stride, lstep);
#pragma unroll
        for (int k = 0; k < NL; k++) tw_stage<T, N, SIGN>(v[k], tw, 1);
    }
    if constexpr (NST > 3) {
        fft_exchange<T, N, 8, R0 * 8, PAD, NL>(v, t, lds, stride, lstep);
#pragma unroll
        for (int k = 0; k < NL; k++) tw_stage<T, N, SIGN>(v[k], tw, 2);
    }
}

// One line held by the calling thread group.
template <typename T, int N, int SIGN, int PAD, typename TW>
__device__ __forceinline__ void fft_line(cx<T> (&v)[8], int t, cx<T>* lds, int stride, const TW& tw)
{
    fft_lines<T, N, SIGN, PAD, 1>(reinterpret_cast<cx<T>(&)[1][8]>(v), t, lds, stride, 0, tw);
}

// ---------------------------------------------------------------- Philox
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                              uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; i++) {
        if (i > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
}

// Box-Muller normals from one Philox block with counter (e, n, r, tag): the
// word pairs give two 53-bit integers m = x_a 2^21 + (x_b >> 11) and the
// uniforms u = (m + 1/2) 2^-53 in (0, 1).
__device__ __forceinline__ void normal_pair(uint64_t seed, uint32_t e, uint32_t n, uint32_t r, uint32_t tag,
                                            double& z1, double& z2)
{
    uint32_t c0 = e, c1 = n, c2 = r, c3 = tag;
    philox4x32_10(c0, c1, c2, c3, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
    const uint64_t m1 = ((uint64_t)c0 << 21) | (uint64_t)(c1 >> 11);
    const uint64_t m2 = ((uint64_t)c2 << 21) | (uint64_t)(c3 >> 11);
    const double u1 = ((double)m1 + 0.5) * 0x1p-53;
    const double u2 = ((double)m2 + 0.5) * 0x1p-53;
    const double rad = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    z1 = rad * c;
    z2 = rad * s;
}

// Single precision: the same uniforms rounded to float, formed without FP64
// arithmetic, and the transcendental functions of the hardware (base-2
// logarithm, square root, sine and cosine of 2 pi x).  For u1 >= 1/2 the
// logarithm is taken of the exactly formed 1 - u1, by its series
// -om (1 + om/2 + om^2/3 + ...) when om = 1 - u1 < 1/64.
__device__ __forceinline__ void normal_pair(uint64_t seed, uint32_t e, uint32_t n, uint32_t r, uint32_t tag,
                                            float& z1, float& z2)
{
    uint32_t c0 = e, c1 = n, c2 = r, c3 = tag;
    philox4x32_10(c0, c1, c2, c3, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
    const float ln2 = 0.69314718055994530942f;
    float lg;
    if (c0 >= 0x80000000u) {
        const float om = fmaf((float)(0xffffffffu - c0), 0x1p-32f, ((float)(0x1fffffu - (c1 >> 11)) + 0.5f) * 0x1p-53f);
        if (om < 0.015625f) {
            const float p = fmaf(om, fmaf(om, fmaf(om, fmaf(om, 1.0f / 6.0f, 0.2f), 0.25f), 1.0f / 3.0f), 0.5f);
            lg = -om * fmaf(om, p, 1.0f);
        } else {
            lg = __builtin_amdgcn_logf(1.0f - om) * ln2;
        }
    } else {
        lg = __builtin_amdgcn_logf(fmaf((float)c0, 0x1p-32f, ((float)(c1 >> 11) + 0.5f) * 0x1p-53f)) * ln2;
    }
    const float rad = __builtin_amdgcn_sqrtf(-2.0f * lg);
    const float u2 = fmaf((float)c2, 0x1p-32f, ((float)(c3 >> 11) + 0.5f) * 0x1p-53f);
    z1 = rad * __builtin_amdgcn_cosf(u2);
    z2 = rad * __builtin_amdgcn_sinf(u2);
}

// ---------------------------------------------------------------- noise normals
// The Fourier-space noise takes two modes' normals from one Philox block: the
// words are used in pairs (x0, x1) and (x2, x3), each word a uniform
// u = (x + 1/2) 2^-32 in (0, 1), and Box-Muller gives
// z1 = sqrt(-2 ln u1) cos(2 pi u2), z2 = sqrt(-2 ln u1) sin(2 pi u2).
__device__ __forceinline__ void philox_block(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                             uint32_t (&x)[4])
{
    philox4x32_10(c0, c1, c2, c3, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
    x[0] = c0;
    x[1] = c1;
    x[2] = c2;
    x[3] = c3;
}

__device__ __forceinline__ void box_muller32(uint32_t a, uint32_t b, double& z1, double& z2)
{
    const double u1 = ((double)a + 0.5) * 0x1p-32;
    const double u2 = ((double)b + 0.5) * 0x1p-32;
    const double rad = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    z1 = rad * c;
    z2 = rad * s;
}

// Single precision, without branches: u1 < 1/2 is formed directly; for
// u1 >= 1/2 the exactly formed om = 1 - u1 (from the complement of the word)
// gives ln u1 by the series -om (1 + om/2 + om^2/3 + ...) when om < 1/64 and
// by the hardware logarithm of 1 - om otherwise.
__device__ __forceinline__ void box_muller32(uint32_t a, uint32_t b, float& z1, float& z2)
{
    const float ln2 = 0.69314718055994530942f;
    const bool hi = a >= 0x80000000u;
    const float u1 = fmaf((float)a, 0x1p-32f, 0x1p-33f);
    const float om = fmaf((float)(0xffffffffu - a), 0x1p-32f, 0x1p-33f);
    const float p = fmaf(om, fmaf(om, fmaf(om, fmaf(om, 1.0f / 6.0f, 0.2f), 0.25f), 1.0f / 3.0f), 0.5f);
    const float lser = -om * fmaf(om, p, 1.0f);
    const float llog = __builtin_amdgcn_logf(hi ? 1.0f - om : u1) * ln2;
    const float lg = (hi && om < 0.015625f) ? lser : llog;
    const float rad = __builtin_amdgcn_sqrtf(-2.0f * lg);
    const float u2 = fmaf((float)b, 0x1p-32f, 0x1p-33f);
    z1 = rad * __builtin_amdgcn_cosf(u2);
    z2 = rad * __builtin_amdgcn_sinf(u2);
}

// ---------------------------------------------------------------- phi functions (FP64)
struct cd {
    double x, y;
};
__device__ __forceinline__ cd cd_mul(cd a, cd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cd cd_div(cd a, cd b)
{
    // Smith's algorithm
    if (fabs(b.x) >= fabs(b.y)) {
        const double r = b.y / b.x, den = b.x + b.y * r;
        return {(a.x + a.y * r) / den, (a.y - a.x * r) / den};
    }
    const double r = b.x / b.y, den = b.x * r + b.y;
    return {(a.x * r + a.y) / den, (a.y * r - a.x) / den};
}

__device__ __forceinline__ void phi12(cd x, cd& p1, cd& p2)
{
    const double ax = hypot(x.x, x.y);
    if (ax < 1.0) {
        // Taylor series phi1 = sum_k x^k/(k+1)!, phi2 = sum_k x^k/(k+2)!, 24 terms
        cd s1 = {0.0, 0.0}, s2 = {0.0, 0.0}, xk = {1.0, 0.0};
        double f1 = 1.0, f2 = 0.5;   // 1/(k+1)! and 1/(k+2)! at k = 0
        for (int k = 0; k < 24; k++) {
            s1.x += f1 * xk.x;
            s1.y += f1 * xk.y;
            s2.x += f2 * xk.x;
            s2.y += f2 * xk.y;
            xk = cd_mul(xk, x);
            f1 /= (double)(k + 2);
            f2 /= (double)(k + 3);
        }
        p1 = s1;
        p2 = s2;
    } else {
        const double s = sin(0.5 * x.y);
        const cd em = {expm1(x.x) * cos(x.y) - 2.0 * s * s, exp(x.x) * sin(x.y)};
        p1 = cd_div(em, x);
        p2 = cd_div({em.x - x.x, em.y - x.y}, cd_mul(x, x));
    }
}

}  // namespace setd
