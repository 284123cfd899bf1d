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

// ---------------------------------------------------------------- coefficients
template <typename T>
struct Coef {
    cx<T> E, wa, wb;
    T G;
};

template <typename T>
struct alignas(4 * sizeof(T)) T4 {
    T a, b, c, d;
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

__device__ __forceinline__ int coef_key(const Item& it, int a0, int a1, int a2)
{
    if (it.iso) return a0 * a0 + a1 * a1 + a2 * a2;
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
// Unit noise eta_a of the stored mode at FFT positions (j0, j1, jl) for step n.
template <typename T>
__device__ __forceinline__ cx<T> noise_eta(const Geo& g, const Item& it, int j0, int j1, int jl, uint32_t n)
{
    const T rs2 = T(0.70710678118654752440084436210484903928);
    const int last = g.ndim - 1;
    const uint32_t e = (g.ndim == 3) ? ((uint32_t)j0 * (uint32_t)g.n[1] + (uint32_t)j1) * (uint32_t)g.nh_last + (uint32_t)jl
                                     : (uint32_t)j0 * (uint32_t)g.nh_last + (uint32_t)jl;
    T z1, z2;
    if (g.cplx || (jl > 0 && 2 * jl < g.n[last])) {
        normal_pair<T>(it.seed, e, n, it.r, 0u, z1, z2);
        return {rs2 * z1, rs2 * z2};
    }
    // a_d in {0, N_d/2}: the conjugate partner -a lies on the same plane
    const int p0 = j0 ? g.n[0] - j0 : 0;
    const int p1 = (g.ndim == 3 && j1) ? g.n[1] - j1 : 0;
    const uint32_t ep = (g.ndim == 3) ? ((uint32_t)p0 * (uint32_t)g.n[1] + (uint32_t)p1) * (uint32_t)g.nh_last + (uint32_t)jl
                                      : (uint32_t)p0 * (uint32_t)g.nh_last + (uint32_t)jl;
    if (ep == e) {
        normal_pair<T>(it.seed, e, n, it.r, 0u, z1, z2);
        return {z1, T(0)};
    }
    if (e < ep) {
        normal_pair<T>(it.seed, e, n, it.r, 0u, z1, z2);
        return {rs2 * z1, rs2 * z2};
    }
    normal_pair<T>(it.seed, ep, n, it.r, 0u, z1, z2);
    return {rs2 * z1, -rs2 * z2};
}

// ---------------------------------------------------------------- launch arguments
struct RowArgs {
    Geo g;
    const Item* items;
    int nrows;   // lines of the last axis per realization (n0 or n0*n1)
    int lpw;     // line groups per workgroup (row pairs for real fields)
    int mode;    // MODE_STEP or MODE_IC
    int sub;     // sub-step of the scheduler tick
};

struct AxisArgs {
    Geo g;
    const Item* items;
    int ntiles;  // column tiles across the padded last axis
    int mode;    // axis-0 pass: MODE_STEP / MODE_IC / MODE_SYNC; axis-1 pass: +1 inverse, -1 forward
    int sub;
};

struct LinArgs {
    Geo g;
    const Item* items;
    int total;   // stored elements per realization
    int sub;
};

template <typename T>
__device__ __forceinline__ const cx<T>* twid(const void* p) { return reinterpret_cast<const cx<T>*>(p); }

// ---------------------------------------------------------------- row pass, real field
// Two real rows a, b travel as one complex line z = a + i b: the inverse uses
// Z_k = A_k + i B_k (k <= N/2) and conj(A_{N-k}) + i conj(B_{N-k}) above; the
// forward splits Z back into A_k = (Z_k + conj Z_{N-k})/2 and
// B_k = (Z_k - conj Z_{N-k})/(2i).  Block: lpw row pairs x N/8 threads.
template <typename T, int N>
__global__ void __launch_bounds__(256) k_row_real(RowArgs a)
{
    const Item& it = a.items[blockIdx.y];
    if (a.sub >= it.steps) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    constexpr int TPL = N / 8;
    const int tid = threadIdx.x;
    const int l = tid / TPL, t = tid - l * TPL;
    const int pair = blockIdx.x * a.lpw + l;
    const bool valid = 2 * pair < a.nrows;
    cx<T>* L = lds + l * N;
    const Geo& g = a.g;
    const int last = g.ndim - 1;
    const cx<T>* tw = twid<T>(last == 1 ? it.tw1 : it.tw2);
    const int pitch = g.pitch;
    const int K = g.kp[last];
    cx<T>* buf = reinterpret_cast<cx<T>*>(g.ndim == 2 ? it.pre0 : it.big);
    const size_t r0 = (size_t)(2 * pair) * pitch, r1 = r0 + pitch;
    const T inv = (T)it.inv_vol;
    cx<T> v[8];

    if (a.mode == MODE_IC) {
        // i.i.d. N(0, sigma^2) per site, Philox counter (site, 0, r, 1)
        const T sig = (T)it.ic_sigma;
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int n = t + q * TPL;
            v[q] = czero<T>();
            if (valid) {
                T za, zb, zc, zd;
                const uint32_t s0 = (uint32_t)(2 * pair) * (uint32_t)N + (uint32_t)n;
                normal_pair<T>(it.seed, s0, 0u, it.r, 1u, za, zb);
                normal_pair<T>(it.seed, s0 + (uint32_t)N, 0u, it.r, 1u, zc, zd);
                v[q] = {sig * za, sig * zc};
            }
        }
    } else if (it.nl == NL_KPZ) {
        // |grad h|^2 with d0 h = IFFT[i k0 h] (from pre1) and d1 h = IFFT[i k1 h]
        const cx<T>* buf2 = reinterpret_cast<const cx<T>*>(it.pre1);
        const T dkl = (T)it.dk[last];
        T gsq[2][8];
#pragma unroll
        for (int s = 0; s < 2; s++) {
            const size_t rr = s ? r1 : r0;
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int k = t + q * TPL;
                cx<T> z = czero<T>();
                if (valid) {
                    if (k <= K) {
                        cx<T> A = buf2[rr + k];
                        const cx<T> X = buf[rr + k];
                        const T kk = (2 * k == N) ? T(0) : dkl * (T)k;
                        cx<T> B = {-kk * X.y, kk * X.x};
                        if (k == 0 || 2 * k == N) {
                            A.y = T(0);
                            B.y = T(0);
                        }
                        z = {A.x - B.y, A.y + B.x};
                    } else if (k >= N - K) {
                        const int m = N - k;
                        const cx<T> A = buf2[rr + m];
                        const cx<T> X = buf[rr + m];
                        const T kk = dkl * (T)m;
                        const cx<T> B = {-kk * X.y, kk * X.x};
                        z = {A.x + B.y, B.x - A.y};
                    }
                }
                v[q] = z;
            }
            fft_line<T, N, +1>(v, t, L, 1, tw);
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const T x = v[q].x * inv, y = v[q].y * inv;
                gsq[s][q] = x * x + y * y;
            }
        }
#pragma unroll
        for (int q = 0; q < 8; q++) v[q] = {gsq[0][q], gsq[1][q]};
    } else {
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int k = t + q * TPL;
            cx<T> z = czero<T>();
            if (valid) {
                if (k <= K) {
                    cx<T> A = buf[r0 + k], B = buf[r1 + k];
                    if (k == 0 || 2 * k == N) {
                        A.y = T(0);
                        B.y = T(0);
                    }
                    z = {A.x - B.y, A.y + B.x};
                } else if (k >= N - K) {
                    const cx<T> A = buf[r0 + (N - k)], B = buf[r1 + (N - k)];
                    z = {A.x + B.y, B.x - A.y};
                }
            }
            v[q] = z;
        }
        fft_line<T, N, +1>(v, t, L, 1, tw);
        // phi^3 in real space (Model A and B)
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const T x = v[q].x * inv, y = v[q].y * inv;
            v[q] = {x * x * x, y * y * y};
        }
    }

    fft_line<T, N, -1>(v, t, L, 1, tw);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; q++) L[t + q * TPL] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const int k = t + q * TPL;
        if (valid && k <= K) {
            const cx<T> Zk = L[k], Zm = L[(N - k) & (N - 1)];
            buf[r0 + k] = {T(0.5) * (Zk.x + Zm.x), T(0.5) * (Zk.y - Zm.y)};
            buf[r1 + k] = {T(0.5) * (Zk.y + Zm.y), T(0.5) * (Zm.x - Zk.x)};
        }
    }
}

// ---------------------------------------------------------------- row pass, complex field
template <typename T, int N>
__global__ void __launch_bounds__(256) k_row_cplx(RowArgs a)
{
    const Item& it = a.items[blockIdx.y];
    if (a.sub >= it.steps) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    constexpr int TPL = N / 8;
    const int tid = threadIdx.x;
    const int l = tid / TPL, t = tid - l * TPL;
    const int line = blockIdx.x * a.lpw + l;
    const bool valid = line < a.nrows;
    cx<T>* L = lds + l * N;
    const Geo& g = a.g;
    const int last = g.ndim - 1;
    const cx<T>* tw = twid<T>(last == 1 ? it.tw1 : it.tw2);
    const int kept = g.kept[last], kp = g.kp[last];
    cx<T>* buf = reinterpret_cast<cx<T>*>(g.ndim == 2 ? it.pre0 : it.big) + (size_t)line * g.pitch;
    const T inv = (T)it.inv_vol;
    cx<T> v[8];
    if (a.mode == MODE_IC) {
        const T sig = (T)it.ic_sigma;
#pragma unroll
        for (int q = 0; q < 8; q++) {
            v[q] = czero<T>();
            if (valid) {
                T z1, z2;
                const uint32_t s = (uint32_t)line * (uint32_t)N + (uint32_t)(t + q * TPL);
                normal_pair<T>(it.seed, s, 0u, it.r, 1u, z1, z2);
                v[q] = {sig * z1, sig * z2};
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int i = stored_idx(t + q * TPL, N, kept, kp);
            v[q] = (valid && i >= 0) ? buf[i] : czero<T>();
        }
        fft_line<T, N, +1>(v, t, L, 1, tw);
        // |A|^2 A in real space (CGL)
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const T x = v[q].x * inv, y = v[q].y * inv;
            const T m = x * x + y * y;
            v[q] = {m * x, m * y};
        }
    }
    fft_line<T, N, -1>(v, t, L, 1, tw);
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const int i = stored_idx(t + q * TPL, N, kept, kp);
        if (valid && i >= 0) buf[i] = v[q];
    }
}

// ---------------------------------------------------------------- axis-0 pass
// A block owns TILE adjacent columns of the stored last axis (3D: at one
// stored index of axis 1).  Thread (c, t) = (tid % TILE, tid / TILE) holds
// elements t + q N0/8 of column c, so each row of the tile is one contiguous
// 128-byte segment in every global access.
//
// MODE_STEP: pre -> forward FFT -> F_a = pref * FFT[N] -> ETD update with the
//            noise of step n -> phi, F_{n-1} -> inverse FFT -> pre.
// MODE_IC:   pre (forward-transformed initial field) -> forward FFT -> phi.
// MODE_SYNC: phi -> inverse FFT -> pre.
template <typename T, int N0, int TILE>
__global__ void __launch_bounds__(1024) k_axis0(AxisArgs a)
{
    const Item& it = a.items[blockIdx.y];
    if (a.sub >= it.steps) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    const Geo& g = a.g;
    constexpr int TPL = N0 / 8;
    const int tid = threadIdx.x;
    const int c = tid % TILE, t = tid / TILE;
    const int tile = blockIdx.x % a.ntiles, i1 = blockIdx.x / a.ntiles;
    const int col = tile * TILE + c;
    const int last = g.ndim - 1;
    const bool cv = col < g.kept[last];
    const size_t lstride = (g.ndim == 3) ? (size_t)g.kept[1] * g.pitch : (size_t)g.pitch;
    const size_t poff = (size_t)i1 * g.pitch + col;
    cx<T>* pre0 = reinterpret_cast<cx<T>*>(it.pre0);
    cx<T>* phi = reinterpret_cast<cx<T>*>(it.phi);
    cx<T>* prev = reinterpret_cast<cx<T>*>(it.prev);
    const cx<T>* tw = twid<T>(it.tw0);
    cx<T>* L = lds + c;
    const int kept0 = g.kept[0], kp0 = g.kp[0];

    // FFT positions and signed indices of the other axes
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
    const T dk0 = (T)it.dk[0], dk1 = (T)it.dk[1], dk2 = (T)it.dk[2];
    const T k2rest = (g.ndim == 3) ? (dk1 * (T)a1) * (dk1 * (T)a1) + (dk2 * (T)al) * (dk2 * (T)al)
                                   : (dk1 * (T)al) * (dk1 * (T)al);

    cx<T> v[8];
    int64_t nstep = 0;
    int hp = 0;
    if (a.mode == MODE_STEP) {
        nstep = it.ctrl->step;
        hp = it.ctrl->have_prev;
    }
    if (a.mode == MODE_SYNC) {
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int i0 = stored_idx(t + q * TPL, N0, kept0, kp0);
            v[q] = (cv && i0 >= 0) ? phi[(size_t)i0 * lstride + poff] : czero<T>();
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; q++) v[q] = cv ? pre0[(size_t)(t + q * TPL) * lstride + poff] : czero<T>();
        fft_line<T, N0, -1>(v, t, L, TILE, tw);
        bool bad = false;
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int j0 = t + q * TPL;
            const int i0 = stored_idx(j0, N0, kept0, kp0);
            if (cv && i0 >= 0) {
                const size_t si = (size_t)i0 * lstride + poff;
                if (a.mode == MODE_IC) {
                    phi[si] = v[q];
                } else {
                    const int a0 = sgn_idx(j0, N0);
                    const T k2 = (dk0 * (T)a0) * (dk0 * (T)a0) + k2rest;
                    const cx<T> F = cmul(nl_pref<T>(it, k2), v[q]);
                    const int key = (g.ndim == 3) ? coef_key(it, a0, a1, al) : coef_key(it, a0, al, 0);
                    const Coef<T> cf = load_coef<T>(it, key);
                    const cx<T> eta = noise_eta<T>(g, it, j0, j1, jl, (uint32_t)nstep);
                    cx<T> nw = cmul(cf.E, phi[si]) + cmul(cf.wa, F) + cf.G * eta;
                    if (it.order == 2) {
                        const cx<T> Fp = hp ? prev[si] : F;
                        nw = nw + cmul(cf.wb, Fp);
                        prev[si] = F;
                    }
                    bad |= !(isfinite(nw.x) && isfinite(nw.y));
                    phi[si] = nw;
                    v[q] = nw;
                }
            } else {
                v[q] = czero<T>();
            }
        }
        if (bad) atomicOr(&it.ctrl->nonfinite, 1);
    }
    cx<T> v2[8];
    const bool kpz = (it.nl == NL_KPZ);
    if (kpz) {
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int j0 = t + q * TPL;
            const T kk = (2 * j0 == N0) ? T(0) : dk0 * (T)sgn_idx(j0, N0);
            v2[q] = {-kk * v[q].y, kk * v[q].x};
        }
    }
    fft_line<T, N0, +1>(v, t, L, TILE, tw);
    if (cv) {
#pragma unroll
        for (int q = 0; q < 8; q++) pre0[(size_t)(t + q * TPL) * lstride + poff] = v[q];
    }
    if (kpz) {
        cx<T>* pre1 = reinterpret_cast<cx<T>*>(it.pre1);
        fft_line<T, N0, +1>(v2, t, L, TILE, tw);
        if (cv) {
#pragma unroll
            for (int q = 0; q < 8; q++) pre1[(size_t)(t + q * TPL) * lstride + poff] = v2[q];
        }
    }
    if (a.mode == MODE_STEP) {
        // the last block of this realization advances its step counter
        __syncthreads();
        if (tid == 0) {
            __threadfence();
            const unsigned prior = atomicAdd(&it.ctrl->done, 1u);
            if (prior == gridDim.x - 1) {
                atomicExch(&it.ctrl->done, 0u);
                atomicExch(reinterpret_cast<unsigned long long*>(&it.ctrl->step), (unsigned long long)(nstep + 1));
                atomicExch(&it.ctrl->have_prev, 1);
                __threadfence();
            }
        }
    }
}

// ---------------------------------------------------------------- axis-1 pass (3D)
// mode +1: stored axis-1 entries of pre -> inverse FFT -> big
// mode -1: big -> forward FFT -> stored axis-1 entries of pre
template <typename T, int N1, int TILE>
__global__ void __launch_bounds__(1024) k_axis1(AxisArgs a)
{
    const Item& it = a.items[blockIdx.y];
    if (a.sub >= it.steps) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    const Geo& g = a.g;
    constexpr int TPL = N1 / 8;
    const int tid = threadIdx.x;
    const int c = tid % TILE, t = tid / TILE;
    const int tile = blockIdx.x % a.ntiles, n0 = blockIdx.x / a.ntiles;
    const int col = tile * TILE + c;
    const bool cv = col < g.kept[2];
    const int pitch = g.pitch, kept1 = g.kept[1], kp1 = g.kp[1];
    cx<T>* small = reinterpret_cast<cx<T>*>(it.pre0) + (size_t)n0 * kept1 * pitch + col;
    cx<T>* big = reinterpret_cast<cx<T>*>(it.big) + (size_t)n0 * N1 * pitch + col;
    const cx<T>* tw = twid<T>(it.tw1);
    cx<T>* L = lds + c;
    cx<T> v[8];
    if (a.mode > 0) {
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int i = stored_idx(t + q * TPL, N1, kept1, kp1);
            v[q] = (cv && i >= 0) ? small[(size_t)i * pitch] : czero<T>();
        }
        fft_line<T, N1, +1>(v, t, L, TILE, tw);
        if (cv) {
#pragma unroll
            for (int q = 0; q < 8; q++) big[(size_t)(t + q * TPL) * pitch] = v[q];
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; q++) v[q] = cv ? big[(size_t)(t + q * TPL) * pitch] : czero<T>();
        fft_line<T, N1, -1>(v, t, L, TILE, tw);
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int i = stored_idx(t + q * TPL, N1, kept1, kp1);
            if (cv && i >= 0) small[(size_t)i * pitch] = v[q];
        }
    }
}

// ---------------------------------------------------------------- linear update (F = 0)
template <typename T>
__global__ void __launch_bounds__(256) k_linear(LinArgs a)
{
    const Item& it = a.items[blockIdx.y];
    if (a.sub >= it.steps) return;
    const Geo& g = a.g;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nstep = it.ctrl->step;
    const int last = g.ndim - 1;
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
            const int key = (g.ndim == 3) ? coef_key(it, a0, a1, al) : coef_key(it, a0, al, 0);
            const Coef<T> cf = load_coef<T>(it, key);
            const cx<T> eta = noise_eta<T>(g, it, j0, j1, jl, (uint32_t)nstep);
            cx<T>* phi = reinterpret_cast<cx<T>*>(it.phi);
            const cx<T> nw = cmul(cf.E, phi[idx]) + cf.G * eta;
            phi[idx] = nw;
            if (!(isfinite(nw.x) && isfinite(nw.y))) atomicOr(&it.ctrl->nonfinite, 1);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned prior = atomicAdd(&it.ctrl->done, 1u);
        if (prior == gridDim.x - 1) {
            atomicExch(&it.ctrl->done, 0u);
            atomicExch(reinterpret_cast<unsigned long long*>(&it.ctrl->step), (unsigned long long)(nstep + 1));
            atomicExch(&it.ctrl->have_prev, 1);
            __threadfence();
        }
    }
}

// ---------------------------------------------------------------- FP64 observables
struct ObsArgs {
    Geo g;
    const Item* items;
    int nitems;
    int kind;       // RED_SK / RED_WIDTH / RED_TWOTIME
    int nbins;
    int total;      // stored elements per realization
    double vol;     // prod L_i / N_i^2
    double* acc;    // [3 * nbins] sums (re, im, weight)
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

}  // namespace setd
