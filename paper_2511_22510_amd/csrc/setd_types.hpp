// setd_types.hpp -- plain structs shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace setd {

// Launch class: everything that fixes the kernels, their grids and the data
// layout.  Realizations of different jobs with the same class share launches.
struct Geo {
    int ndim;         // 2 or 3
    int cplx;         // 0 real field (last axis R2C), 1 complex field
    int prec;         // 32 or 64
    int dealias;      // 0 none, 1 the 2/3 rule, 2 phase shift
    int n[3];         // lattice points per axis (n[ndim..2] = 1)
    int kept[3];      // stored spectral entries per axis
    int kp[3];        // largest stored FFT index on the low side of each axis
    int pitch;        // padded length of the stored last axis (elements)
    int nh_last;      // unpruned spectral length of the last axis (n/2+1 or n)
    int rsn;          // noise drawn in real space and transformed
};

// stored rows of a realization: [kept0][kept1] lines of the last axis (3D),
// kept0 (2D), one (a 1D line)
inline __host__ __device__ int geo_rows(const Geo& g)
{
    return g.ndim == 1 ? 1 : g.kept[0] * (g.ndim == 3 ? g.kept[1] : 1);
}

// Per-realization control block in device memory.
struct Ctrl {
    int64_t step;          // index n of the next transition n -> n+1
    uint32_t done;         // blocks finished in the current update pass
    int32_t have_prev;     // F_{n-1} stored (SETD2)
    int32_t nonfinite;     // a NaN/Inf was produced
    int32_t pad[3];
};

// One realization of one job, as the kernels see it.
struct Item {
    void* phi;        // stored spectral state  [kept0][kept1][pitch] (3D) / [kept0][pitch]
    void* prev;       // F_{n-1}, same layout (SETD2), else null
    void* pre0;       // axis-0 inverse of phi: [n0][kept1][pitch] / [n0][pitch]
    void* pre1;       // KPZ: axis-0 inverse of i k0 phi (2D), else null
    void* big;        // 3D: [n0][n1][pitch] line buffer of the last-axis pass
    void* snap;       // snapshot of phi for two-time correlations
    void* npre;       // real-space noise (2D/3D): its transform over the last axes, laid out as pre0
    void* noise;      // real-space noise (2D/3D): eta_a of the step in the stored layout of phi
    void* preb;       // phase-shift dealiasing: axis-0 inverse of e^{i pi a0/N0} phi, laid out as pre0
    void* pre1b;      // KPZ with phase shifts: axis-0 inverse of e^{i pi a0/N0} i k0 phi, laid out as pre0
    const void* coef; // coefficient table in the state precision
    const void* tw0;  // twiddles exp(-2 pi i k / n_axis), state precision
    const void* tw1;
    const void* tw2;
    Ctrl* ctrl;
    uint64_t seed;
    uint32_t r;       // realization index in the Philox counter
    int32_t nl;       // nonlinearity kind
    int32_t order;    // 1 or 2
    int32_t coef_mode;// COEF_SEPARABLE, COEF_ISO or COEF_PER_MODE
    int32_t coef_cplx;// coefficient table has complex entries
    int32_t steps;    // sub-steps to take in the current scheduler tick
    int32_t keydim[3];// separable key extents (K_i + 1)
    uint32_t coef_bytes;// bytes of the coefficient table (capped at 2^31 - 1)
    double dk[3];     // 2 pi / L_i
    double par0;      // u | lambda | beta
    double inv_vol;   // 1 / prod n_i (inverse DFT scale)
    double ic_sigma;
};

// arguments of the FP64 coefficient-table kernel
struct CoefArgs {
    int nkeys, mode, ndim, order, kpow, cplx_table;
    Geo g;            // lattice (per-mode tables)
    int keydim[3];
    double dk[3];
    double c0[2], c2[2], c4[2];
    double D, h, lat;
    double* out64;
    void* out32;   // float table or null
};

enum { NL_PHI3 = 0, NL_PHI3_CONS = 1, NL_KPZ = 2, NL_CGL = 3, NL_NONE = 4 };

// coefficient table layouts: by (|a0|, |a1|, |a2|), by |a|^2, or one entry
// per stored mode of a 2D lattice in the state layout
enum { COEF_SEPARABLE = 0, COEF_ISO = 1, COEF_PER_MODE = 2 };

// modes of the passes (MODE_RSN: the axis-0 forward transform of the
// real-space noise, npre -> noise)
enum { MODE_STEP = 0, MODE_IC = 1, MODE_SYNC = 2, MODE_RECOVER = 3, MODE_RSN = 4 };
// k_linear: a step of F = 0 in place; the SETD2 carry Y = E phi + G eta_n;
// re-drawing the carry's noise for another step index
enum { LIN_STEP = 0, LIN_CARRY = 1, LIN_RENOISE = 2 };

// arguments of the time-frequency observables of a recorded window (App. C)
struct SpecArgs {
    Geo g;
    const Item* items;
    int nitems, nbins, total;     // total: stored elements per realization
    const char* series;           // sample m of realization r at series + m * slot + r * rstride
    size_t slot, rstride;
    const void* tw;               // exp(-2 pi i k / M), state precision
    int64_t step0;                // step of sample 0 (the kick of the step taken from it)
    double vol, h, D;             // prod L_i / N_i^2, step, D of D(k) = D k^kpow
    int kpow;
    double* acc;                  // [3][nbins][M] sums, then [nbins] mode counts
    double* dacc;                 // null, or [total][M]: the FDT deviation per mode and frequency
};

// arguments of the box-averaged width: class sums of one realization
struct BoxArgs {
    Geo g;
    const Item* items;
    int r;            // realization (item index)
    int total;        // stored elements per realization
    int N, J;         // lattice points per axis (equal axes), log2 N
    double* cls;      // [sum_j (N >> j)^d][re, im] class sums, levels j = 1..J
    double* sums;     // [J + 1]: sums[0] sum_a |h_a|^2, sums[j] sum_c |A_c|^2 of level j (a != 0)
    size_t lds_base;  // first class summed in LDS (the coarse levels at the end)
    int nlds;         // classes summed in LDS, at most 1024
};

// observable reductions
enum { RED_SK = 0, RED_WIDTH = 1, RED_TWOTIME = 2, RED_RESPONSE = 3 };

}  // namespace setd
