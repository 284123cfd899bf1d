// setd_device.hpp -- device building blocks of the gfx950 SETD path.
//
//  * cx<T>: complex numbers in float or double.
//  * fft_line<T, N, SIGN>: one length-N line transform held by N/8 threads,
//    8 values per thread.  Stockham autosort stages (radix 2/4 first, then
//    radix 8) with the values exchanged through LDS between stages.  Thread t
//    holds elements t + q N/8 (q = 0..7) on entry and output bins t + q N/8 on
//    exit, so the first stage reads and the last stage writes in the layout in
//    which lines are loaded from and stored to global memory.
//  * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller normals
//    for the Fourier-space noise of App. B.
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
    // o1 * W8 = r (x - SIGN y, SIGN x + y); o3 * W8^3 = r (-x - SIGN y, SIGN x - y)
    cx<T> w1 = {r * (o1.x - T(SIGN) * o1.y), r * (T(SIGN) * o1.x + o1.y)};
    cx<T> w2 = mul_si<SIGN>(o2);
    cx<T> w3 = {r * (-o3.x - T(SIGN) * o3.y), r * (T(SIGN) * o3.x - o3.y)};
    cx<T> e0 = u[0], e1 = u[2], e2 = u[4], e3 = u[6], o0 = u[1];
    u[0] = e0 + o0;
    u[4] = e0 - o0;
    u[1] = e1 + w1;
    u[5] = e1 - w1;
    u[2] = e2 + w2;
    u[6] = e2 - w2;
    u[3] = e3 + w3;
    u[7] = e3 - w3;
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

// One Stockham stage of radix R after NS points have been combined.  Thread t
// owns butterflies j = t + b N/8, b < 8/R, whose inputs are elements
// j + r N/R, i.e. v[b + (8/R) r].  Twiddles come from tw[k] = exp(-2 pi i k/N).
template <typename T, int N, int R, int NS, int SIGN>
__device__ __forceinline__ void fft_stage(cx<T>* v, int t, const cx<T>* __restrict__ tw)
{
    constexpr int NB = 8 / R;
#pragma unroll
    for (int b = 0; b < NB; b++) {
        cx<T> u[R];
#pragma unroll
        for (int r = 0; r < R; r++) u[r] = v[b + NB * r];
        if constexpr (NS > 1) {
            const int j = t + b * (N / 8);
            const int jm = j & (NS - 1);
            constexpr int TS = N / (NS * R);
#pragma unroll
            for (int r = 1; r < R; r++) {
                const cx<T> w = tw[jm * r * TS];
                u[r] = (SIGN < 0) ? cmul(u[r], w) : cmulc(u[r], w);
            }
        }
        dft<R, SIGN>(u);
#pragma unroll
        for (int r = 0; r < R; r++) v[b + NB * r] = u[r];
    }
}

// Write the outputs of a stage to their Stockham positions
// (j / NS) NS R + j mod NS + r NS, then read the next stage's inputs back in
// the natural layout t + q N/8.  lds[e * stride] holds element e of the line.
template <typename T, int N, int R, int NS>
__device__ __forceinline__ void fft_exchange(cx<T>* v, int t, cx<T>* lds, int stride)
{
    constexpr int NB = 8 / R;
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int j = t + b * (N / 8);
        const int base = (j / NS) * NS * R + (j & (NS - 1));
#pragma unroll
        for (int r = 0; r < R; r++) lds[(base + r * NS) * stride] = v[b + NB * r];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; q++) v[q] = lds[(t + q * (N / 8)) * stride];
}

// Full line transform X_k = sum_m x_m exp(SIGN 2 pi i k m / N), unscaled.
// Every thread of the block must call it (it contains block barriers).
template <typename T, int N, int SIGN>
__device__ __forceinline__ void fft_line(cx<T>* v, int t, cx<T>* lds, int stride, const cx<T>* __restrict__ tw)
{
    static_assert(N >= 8 && (N & (N - 1)) == 0, "power-of-two line length >= 8");
    constexpr int LG = ilog2(N);
    constexpr int R0 = (LG % 3 == 0) ? 8 : (1 << (LG % 3));
    constexpr int NST = (LG % 3 == 0) ? LG / 3 : LG / 3 + 1;
    fft_stage<T, N, R0, 1, SIGN>(v, t, tw);
    if constexpr (NST > 1) {
        fft_exchange<T, N, R0, 1>(v, t, lds, stride);
        fft_stage<T, N, 8, R0, SIGN>(v, t, tw);
    }
    if constexpr (NST > 2) {
        fft_exchange<T, N, 8, R0>(v, t, lds, stride);
        fft_stage<T, N, 8, R0 * 8, SIGN>(v, t, tw);
    }
    if constexpr (NST > 3) {
        fft_exchange<T, N, 8, R0 * 8>(v, t, lds, stride);
        fft_stage<T, N, 8, R0 * 64, SIGN>(v, t, tw);
    }
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
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
}

// Two 53-bit integers from one Philox block with counter (e, n, r, tag).
__device__ __forceinline__ void philox_m53(uint64_t seed, uint32_t e, uint32_t n, uint32_t r, uint32_t tag,
                                           uint64_t& m1, uint64_t& m2)
{
    uint32_t c0 = e, c1 = n, c2 = r, c3 = tag;
    philox4x32_10(c0, c1, c2, c3, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
    m1 = ((uint64_t)c0 << 21) | (uint64_t)(c1 >> 11);
    m2 = ((uint64_t)c2 << 21) | (uint64_t)(c3 >> 11);
}

// Box-Muller on u = (m + 1/2) 2^-53 in (0, 1).
__device__ __forceinline__ void box_muller(uint64_t m1, uint64_t m2, double& z1, double& z2)
{
    const double u1 = ((double)m1 + 0.5) * 0x1p-53;
    const double u2 = ((double)m2 + 0.5) * 0x1p-53;
    const double rad = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    z1 = rad * c;
    z2 = rad * s;
}

__device__ __forceinline__ void box_muller(uint64_t m1, uint64_t m2, float& z1, float& z2)
{
    // ln u1: for u1 > 1/2 take log1p of the exactly formed -(1 - u1)
    float lg;
    if (m1 >= (1ull << 52)) {
        const double om = ((double)((1ull << 53) - m1) - 0.5) * 0x1p-53;
        lg = log1pf(-(float)om);
    } else {
        lg = logf((float)(((double)m1 + 0.5) * 0x1p-53));
    }
    const float rad = sqrtf(-2.0f * lg);
    const float u2 = (float)(((double)m2 + 0.5) * 0x1p-53);
    float s, c;
    sincospif(2.0f * u2, &s, &c);
    z1 = rad * c;
    z2 = rad * s;
}

template <typename T>
__device__ __forceinline__ void normal_pair(uint64_t seed, uint32_t e, uint32_t n, uint32_t r, uint32_t tag,
                                            T& z1, T& z2)
{
    uint64_t m1, m2;
    philox_m53(seed, e, n, r, tag, m1, m2);
    box_muller(m1, m2, z1, z2);
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
