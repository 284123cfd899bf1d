/*
 * setd_oracle.c -- plain FP64 CPU oracle for the stochastic exponential-time-
 * differencing (SETD) pseudo-spectral step of Johnsrud & Rana, "Efficient
 * Pseudo-spectral Algorithms for Statistical Field Theories" (arXiv 2511.22510).
 *
 * TEST INFRASTRUCTURE.  This file is the slow, obviously-correct reference that
 * the GPU library is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the product path never does, and
 * it shares no code, header or table with the GPU library.
 *
 * Everything is double precision.  Arrays are full (unpruned) spectra in FFT
 * order: a real field keeps the half spectrum N0 x .. x (N_{d-1}/2+1) of the
 * real-to-complex transform, a complex field the whole N0 x .. x N_{d-1} array.
 * Complex numbers cross the C ABI as interleaved (re, im) doubles.
 *
 * Readings of the paper taken here where it is silent or inconsistent:
 *  - DFT sign and scale (App. A): forward X_a = sum_n x_n e^{-2 pi i a.n/N},
 *    inverse x_n = N^-d sum_a X_a e^{+2 pi i a.n/N}.  The printed discrete pair
 *    has the opposite sign to the continuous one and an inverse without 1/N^d;
 *    the field/lattice mapping of App. A needs the 1/N^d.  The sign does not
 *    change any model here (c(k) even, |grad h|^2 and the noise symmetric).
 *  - Dealiasing (Sec. 4, step 1) is the 2/3 truncation rule: a mode is kept
 *    iff 3|a_i| < N_i on every axis; it masks F and the updated state.
 *  - Noise amplitude (Sec. 4, step 3; Eq. SETD1; App. A):
 *    G_a = prod_i (N_i^2/L_i)^{1/2} sqrt(2 D_a h phi1(2 Re(c_a) h)), which is
 *    the printed (N^2/L)^{d/2} sqrt(D/c (e^{2ch}-1)) written without the 0/0
 *    at c = 0 and with Re(c) for complex c (the variance of int e^{c(h-s)} dW).
 *  - SETD2 weights (Eq. SETD2): [(1+x)e^x-1-2x]/(c^2 h) = h(phi1+phi2) and
 *    [1+x-e^x]/(c^2 h) = -h phi2 with x = c h; phi1, phi2 by Taylor series for
 *    |x| < 1 (replacing the "use Euler-Maruyama for small c" advice of Sec. 4)
 *    and closed forms otherwise.  The first SETD2 step uses F_{-1} = F_0.
 *  - Fourier-space noise (App. B): Philox4x32-10 (Salmon et al., SC'11) keyed
 *    by the seed.  Complex modes get (z1 + i z2)/sqrt2, self-conjugate modes
 *    of a real field get z1, a conjugate pair on the a_d in {0, N_d/2} planes
 *    draws once at the smaller linear index and the partner takes the
 *    conjugate.  Masked modes draw nothing.  The paper fixes the distribution,
 *    not the generator; here one Philox block serves two drawing modes that
 *    differ only in the axis-0 position, j and j' = (j mod M) + (7 - j div M) M
 *    with M = N_0/8 (1 if N_0 < 8): counter (P, step, realization, 0) with P
 *    the linear index of the member with j div M < 4 over an axis-0 extent of
 *    N_0/2; that member takes words (x0, x1), the other (x2, x3), each word a
 *    uniform (x + 1/2) 2^-32, then Box-Muller.  The initial condition draws
 *    per site: counter (site, 0, realization, 1), two 53-bit uniforms.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Problem statement (Sec. 4, Eq. general_fourier; App. A lattice)           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int ndim;              /* 1..3                                          */
    int n[3];              /* points per axis, powers of two                */
    double dx;             /* lattice spacing; L_i = n_i dx                 */
    int complex_field;     /* 0 real order parameter, 1 complex             */
    double c0[2], c2[2], c4[2]; /* c(k) = c0 + c2 k^2 + c4 k^4 (re, im)     */
    int nl;                /* 0 -u phi^3, 1 -u k^2 phi^3, 2 KPZ, 3 CGL, 4 none */
    double nl_par[2];      /* u | lambda | beta                             */
    double noise_D;        /* D in D(k) = D k^kpow                          */
    int noise_kpow;        /* 0 or 2                                        */
    double h;              /* time step                                     */
    int order;             /* 1 SETD1, 2 SETD2                              */
    int realizations;
    uint64_t seed;
    int dealias;           /* 0 none, 1 the 2/3 rule, 2 phase shift         */
    int ic_kind;           /* 0 zero, 1 Gaussian per site                   */
    double ic_sigma;
    int noise_space;       /* 0 Fourier-space draws (App. B), 1 real space  */
} orc_desc;

enum { NL_PHI3 = 0, NL_PHI3_CONS = 1, NL_KPZ = 2, NL_CGL = 3, NL_NONE = 4 };

/* ------------------------------------------------------------------------ */
/* Textbook radix-2 FFT, one line at a time                                 */
/* ------------------------------------------------------------------------ */

/* twiddle tables exp(sign 2 pi i k / n), k < n/2, one per (n, sign) */
typedef struct { int n; int sign; cplx* w; } twtab;
static twtab g_tw[32];
static int g_ntw = 0;

static const cplx* twiddles(int n, int sign)
{
    int i;
    for (i = 0; i < g_ntw; i++)
        if (g_tw[i].n == n && g_tw[i].sign == sign) return g_tw[i].w;
    cplx* w = (cplx*)malloc(sizeof(cplx) * (size_t)(n / 2 + 1));
    for (int k = 0; k <= n / 2; k++) {
        double ang = sign * 2.0 * M_PI * (double)k / (double)n;
        w[k] = cos(ang) + I * sin(ang);
    }
    if (g_ntw < 32) {
        g_tw[g_ntw].n = n; g_tw[g_ntw].sign = sign; g_tw[g_ntw].w = w; g_ntw++;
    }
    return w;
}

/* in place, unscaled: x_k <- sum_m x_m exp(sign 2 pi i k m / n) */
static void fft_line(cplx* x, int n, int sign, const cplx* w)
{
    /* bit-reversal permutation */
    for (int i = 1, j = 0; i < n; i++) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { cplx t = x[i]; x[i] = x[j]; x[j] = t; }
    }
    /* butterflies of growing length */
    for (int len = 2; len <= n; len <<= 1) {
        int half = len / 2, step = n / len;
        for (int i = 0; i < n; i += len)
            for (int k = 0; k < half; k++) {
                cplx u = x[i + k];
                cplx v = x[i + k + half] * w[k * step];
                x[i + k] = u + v;
                x[i + k + half] = u - v;
            }
    }
}

static int is_pow2(int n) { return n >= 1 && (n & (n - 1)) == 0; }

/* N-dimensional complex FFT, row-major shape n[0..ndim).  sign = -1 forward
   (unscaled), sign = +1 inverse (scaled by 1/prod n). */
static void fftn(cplx* x, int ndim, const int* n, int sign)
{
    size_t total = 1;
    for (int d = 0; d < ndim; d++) total *= (size_t)n[d];
    for (int ax = 0; ax < ndim; ax++) {
        size_t inner = 1, outer = 1;
        for (int d = ax + 1; d < ndim; d++) inner *= (size_t)n[d];
        for (int d = 0; d < ax; d++) outer *= (size_t)n[d];
        int len = n[ax];
        const cplx* w = twiddles(len, sign);
        long nlines = (long)(outer * inner);
#pragma omp parallel
        {
            cplx* tmp = (cplx*)malloc(sizeof(cplx) * (size_t)len);
#pragma omp for schedule(static)
            for (long l = 0; l < nlines; l++) {
                size_t o = (size_t)l / inner, i = (size_t)l % inner;
                cplx* base = x + o * (size_t)len * inner + i;
                for (int m = 0; m < len; m++) tmp[m] = base[(size_t)m * inner];
                fft_line(tmp, len, sign, w);
                for (int m = 0; m < len; m++) base[(size_t)m * inner] = tmp[m];
            }
            free(tmp);
        }
    }
    if (sign > 0) {
        double s = 1.0 / (double)total;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < (long)total; i++) x[i] *= s;
    }
}

/* real -> half spectrum: complex FFT of the real data, keep a_d in [0, N_d/2] */
static void rfftn(const double* xr, cplx* out, int ndim, const int* n, cplx* work)
{
    size_t total = 1;
    for (int d = 0; d < ndim; d++) total *= (size_t)n[d];
    for (size_t i = 0; i < total; i++) work[i] = xr[i];
    fftn(work, ndim, n, -1);
    int nl = n[ndim - 1], nh = nl / 2 + 1;
    size_t rows = total / (size_t)nl;
    for (size_t r = 0; r < rows; r++)
        for (int j = 0; j < nh; j++) out[r * nh + j] = work[r * nl + j];
}

/* half spectrum -> real: Hermitian extension X_a = conj(X_{-a}) for the
   missing a_d > N_d/2, complex inverse FFT, real part. */
static void irfftn(const cplx* in, double* xr, int ndim, const int* n, cplx* work)
{
    size_t total = 1;
    for (int d = 0; d < ndim; d++) total *= (size_t)n[d];
    int nl = n[ndim - 1], nh = nl / 2 + 1;
    size_t rows = total / (size_t)nl;
    for (size_t r = 0; r < rows; r++) {
        /* row index r = multi-index (j_0..j_{d-2}); its negation */
        size_t rem = r, neg = 0, mul = 1;
        for (int d = ndim - 2; d >= 0; d--) {
            size_t j = rem % (size_t)n[d]; rem /= (size_t)n[d];
            size_t jn = (j == 0) ? 0 : (size_t)n[d] - j;
            neg += jn * mul; mul *= (size_t)n[d];
        }
        for (int j = 0; j < nl; j++) {
            if (j < nh) work[r * nl + j] = in[r * nh + j];
            else work[r * nl + j] = conj(in[neg * nh + (size_t)(nl - j)]);
        }
    }
    fftn(work, ndim, n, +1);
    for (size_t i = 0; i < total; i++) xr[i] = creal(work[i]);
}

/* exported transforms, interleaved complex */
int orc_fftn(double* data, int ndim, const int* n, int sign)
{
    if (ndim < 1 || ndim > 3) return -1;
    for (int d = 0; d < ndim; d++) if (!is_pow2(n[d])) return -1;
    fftn((cplx*)data, ndim, n, sign < 0 ? -1 : +1);
    return 0;
}

int orc_rfftn(const double* x, double* out, int ndim, const int* n)
{
    if (ndim < 1 || ndim > 3) return -1;
    size_t total = 1;
    for (int d = 0; d < ndim; d++) { if (!is_pow2(n[d]) || n[d] < 2) return -1; total *= (size_t)n[d]; }
    cplx* work = (cplx*)malloc(sizeof(cplx) * total);
    rfftn(x, (cplx*)out, ndim, n, work);
    free(work);
    return 0;
}

int orc_irfftn(const double* in, double* x, int ndim, const int* n)
{
    if (ndim < 1 || ndim > 3) return -1;
    size_t total = 1;
    for (int d = 0; d < ndim; d++) { if (!is_pow2(n[d]) || n[d] < 2) return -1; total *= (size_t)n[d]; }
    cplx* work = (cplx*)malloc(sizeof(cplx) * total);
    irfftn((const cplx*)in, x, ndim, n, work);
    free(work);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller          */
/* ------------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* two standard normals from one Philox block with counter (e, n, r, tag) */
void orc_normal_pair(uint64_t seed, uint32_t e, uint32_t n, uint32_t r, uint32_t tag,
                     double* z1, double* z2)
{
    uint32_t ctr[4] = { e, n, r, tag };
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    uint32_t x[4];
    orc_philox(ctr, key, x);
    /* 53-bit integers from the word pairs, mapped to the open interval (0,1) */
    uint64_t m1 = ((uint64_t)x[0] << 21) | (uint64_t)(x[1] >> 11);
    uint64_t m2 = ((uint64_t)x[2] << 21) | (uint64_t)(x[3] >> 11);
    double u1 = ((double)m1 + 0.5) * 0x1p-53;
    double u2 = ((double)m2 + 0.5) * 0x1p-53;
    double rad = sqrt(-2.0 * log(u1));
    *z1 = rad * cos(2.0 * M_PI * u2);
    *z2 = rad * sin(2.0 * M_PI * u2);
}

/* Box-Muller normals of the Fourier-space noise: words (x0, x1) (half 0) or
   (x2, x3) (half 1) of the Philox block with counter (P, n, r, 0), each word
   a uniform u = (x + 1/2) 2^-32 in (0, 1) */
void orc_noise_normals(uint64_t seed, uint32_t P, uint32_t n, uint32_t r, int half, double* z1, double* z2)
{
    uint32_t ctr[4] = { P, n, r, 0u };
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    uint32_t x[4];
    orc_philox(ctr, key, x);
    double u1 = ((double)x[half ? 2 : 0] + 0.5) * 0x1p-32;
    double u2 = ((double)x[half ? 3 : 1] + 0.5) * 0x1p-32;
    double rad = sqrt(-2.0 * log(u1));
    *z1 = rad * cos(2.0 * M_PI * u2);
    *z2 = rad * sin(2.0 * M_PI * u2);
}

/* ------------------------------------------------------------------------ */
/* ETD functions phi1(x) = (e^x-1)/x, phi2(x) = (e^x-1-x)/x^2  (Eq. SETD1/2) */
/* ------------------------------------------------------------------------ */
static cplx cexpm1_(cplx x)
{
    double a = creal(x), b = cimag(x);
    double s = sin(0.5 * b);
    return (expm1(a) * cos(b) - 2.0 * s * s) + I * (exp(a) * sin(b));
}

static void phi12(cplx x, cplx* p1, cplx* p2)
{
    if (cabs(x) < 1.0) {
        /* Taylor series: phi1 = sum x^k/(k+1)!, phi2 = sum x^k/(k+2)! */
        cplx s1 = 0, s2 = 0, xk = 1;
        double f1 = 1.0, f2 = 2.0;   /* (k+1)!, (k+2)! at k = 0 */
        for (int k = 0; k < 24; k++) {
            s1 += xk / f1;
            s2 += xk / f2;
            xk *= x;
            f1 *= (double)(k + 2);
            f2 *= (double)(k + 3);
        }
        *p1 = s1; *p2 = s2;
    } else {
        cplx em = cexpm1_(x);
        *p1 = em / x;
        *p2 = (em - x) / (x * x);
    }
}

void orc_phi12(double xr, double xi, double* out4)
{
    cplx p1, p2;
    phi12(xr + I * xi, &p1, &p2);
    out4[0] = creal(p1); out4[1] = cimag(p1);
    out4[2] = creal(p2); out4[3] = cimag(p2);
}

/* ------------------------------------------------------------------------ */
/* Simulation state                                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    orc_desc d;
    int r_first, R;            /* realizations [r_first, r_first + R)        */
    int nh[3];                 /* spectral shape                            */
    size_t nspec, nreal;
    cplx* phi;                 /* R x nspec                                 */
    cplx* fprev;               /* R x nspec                                 */
    unsigned char* have_prev;  /* per realization: F_{n-1} exists       */
    int64_t step;
    /* per-mode data (Sec. 4 step 3), computed once */
    double* k2;                /* |k|^2                                     */
    int* kidx;                 /* signed index per axis, 3 per mode         */
    unsigned char* mask;
    cplx* E; cplx* wa; cplx* wb; double* G;
    cplx* pref;                /* prefactor of the transformed nonlinearity */
    /* observables */
    cplx* snap; int64_t snap_step; int have_snap;
    int64_t kick_step; int have_kick;   /* reference step of the response estimator */
    cplx* series; int series_len, series_pos; int64_t series_step0;   /* recorded phi_a(m) */
    double* acc; double acc_count; int nbins;
    /* real-space noise: eta_a of step rs_n, realization rs_r */
    cplx* rs_eta; int64_t rs_n; int64_t rs_r;
    /* scratch */
    cplx* work; cplx* work2; double* rwork; double* rwork2; cplx* F;
} orc_sim;

static size_t prod(const int* n, int d) { size_t p = 1; for (int i = 0; i < d; i++) p *= (size_t)n[i]; return p; }

/* signed wavenumber index for FFT-order position j on an axis of length n */
static int signed_idx(int j, int n) { return (j < n / 2) ? j : j - n; }

/* linear index in the spectral array of FFT-order multi-index j */
static size_t lin_index(const orc_sim* s, const int* j)
{
    size_t e = 0;
    for (int d = 0; d < s->d.ndim; d++) e = e * (size_t)s->nh[d] + (size_t)j[d];
    return e;
}

static void unlin(const orc_sim* s, size_t e, int* j)
{
    for (int d = s->d.ndim - 1; d >= 0; d--) { j[d] = (int)(e % (size_t)s->nh[d]); e /= (size_t)s->nh[d]; }
}

/* ------------------------------------------------------------------------ */
/* Hermitian symmetry of a real field (App. A): phi_{-a} = conj(phi_a).  On the
   planes a_d in {0, N_d/2} of the half spectrum both members of a conjugate
   pair are stored.  Round-off in the transforms breaks the pairing slightly,
   and the anti-Hermitian part is invisible to the real-space nonlinearity, so
   it evolves with e^{c h} alone and grows where Re c > 0.  As for the noise
   (App. B), the member with the smaller linear index is independent and its
   partner is set to its conjugate; self-conjugate modes are made real.       */
/* ------------------------------------------------------------------------ */
static void hermitian_planes(const orc_sim* s, cplx* ph)
{
    const orc_desc* d = &s->d;
    if (d->complex_field) return;
    const int last = d->ndim - 1;
    for (size_t e = 0; e < s->nspec; e++) {
        int j[3] = { 0, 0, 0 };
        unlin(s, e, j);
        if (!(j[last] == 0 || 2 * j[last] == d->n[last])) continue;
        int jp[3] = { 0, 0, 0 };
        for (int i = 0; i < last; i++) jp[i] = (j[i] == 0) ? 0 : d->n[i] - j[i];
        jp[last] = j[last];
        size_t ep = lin_index(s, jp);
        if (ep == e) ph[e] = creal(ph[e]);
        else if (ep < e) ph[e] = conj(ph[ep]);
    }
}


static int isqrt_ceil(long m)
{
    if (m <= 0) return 0;
    long s = (long)floor(sqrt((double)m));
    while (s * s > m) s--;
    while ((s + 1) * (s + 1) <= m) s++;
    return (s * s == m) ? (int)s : (int)(s + 1);
}

void orc_destroy(orc_sim* s);

orc_sim* orc_create_subset(const orc_desc* d, int r_first, int r_count)
{
    if (d->ndim < 1 || d->ndim > 3) return NULL;
    for (int i = 0; i < d->ndim; i++) if (!is_pow2(d->n[i]) || d->n[i] < 4) return NULL;
    if (d->order != 1 && d->order != 2) return NULL;
    if (d->dealias < 0 || d->dealias > 2) return NULL;
    if (!(d->h > 0) || !(d->dx > 0)) return NULL;
    if (d->realizations < 1 || r_first < 0 || r_count < 1 || r_first + r_count > d->realizations) return NULL;
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    s->d = *d;
    s->r_first = r_first; s->R = r_count;
    for (int i = 0; i < d->ndim; i++) s->nh[i] = d->n[i];
    if (!d->complex_field) s->nh[d->ndim - 1] = d->n[d->ndim - 1] / 2 + 1;
    s->nspec = prod(s->nh, d->ndim);
    s->nreal = prod(d->n, d->ndim);
    size_t R = (size_t)r_count;
    s->phi = (cplx*)calloc(R * s->nspec, sizeof(cplx));
    s->fprev = (cplx*)calloc(R * s->nspec, sizeof(cplx));
    s->k2 = (double*)malloc(sizeof(double) * s->nspec);
    s->kidx = (int*)malloc(sizeof(int) * 3 * s->nspec);
    s->mask = (unsigned char*)malloc(s->nspec);
    s->E = (cplx*)malloc(sizeof(cplx) * s->nspec);
    s->wa = (cplx*)malloc(sizeof(cplx) * s->nspec);
    s->wb = (cplx*)malloc(sizeof(cplx) * s->nspec);
    s->G = (double*)malloc(sizeof(double) * s->nspec);
    s->pref = (cplx*)malloc(sizeof(cplx) * s->nspec);
    s->work = (cplx*)malloc(sizeof(cplx) * s->nreal);
    s->work2 = (cplx*)malloc(sizeof(cplx) * s->nreal);
    s->rwork = (double*)malloc(sizeof(double) * s->nreal);
    s->rwork2 = (double*)malloc(sizeof(double) * s->nreal);
    s->F = (cplx*)malloc(sizeof(cplx) * s->nspec);
    s->have_prev = (unsigned char*)calloc(R, 1);
    if (!s->have_prev || !s->phi || !s->fprev || !s->k2 || !s->kidx || !s->mask || !s->E || !s->wa || !s->wb ||
        !s->G || !s->pref || !s->work || !s->work2 || !s->rwork || !s->rwork2 || !s->F) {
        orc_destroy(s);
        return NULL;
    }

    /* lattice (App. A): L_i = N_i dx, dk_i = 2 pi / L_i; noise lattice factor */
    double lat = 1.0;
    for (int i = 0; i < d->ndim; i++) {
        double L = d->n[i] * d->dx;
        lat *= sqrt((double)d->n[i] * (double)d->n[i] / L);
    }
    double h = d->h;
    int maxsq = 0;
    for (int i = 0; i < d->ndim; i++) maxsq += (d->n[i] / 2) * (d->n[i] / 2);
    s->nbins = isqrt_ceil(maxsq) + 1;
    s->acc = (double*)calloc((size_t)2 * (size_t)s->nbins, sizeof(double));

    for (size_t e = 0; e < s->nspec; e++) {
        int j[3] = { 0, 0, 0 };
        unlin(s, e, j);
        double k2 = 0.0;
        int keep = 1;
        for (int i = 0; i < d->ndim; i++) {
            int a = signed_idx(j[i], d->n[i]);
            s->kidx[3 * e + i] = a;
            double dk = 2.0 * M_PI / (d->n[i] * d->dx);
            k2 += (dk * a) * (dk * a);
            if (d->dealias == 1 && 3 * abs(a) >= d->n[i]) keep = 0;
            if (d->dealias == 2 && 2 * abs(a) >= d->n[i]) keep = 0;   /* the Nyquist mode has no shift */
        }
        for (int i = d->ndim; i < 3; i++) s->kidx[3 * e + i] = 0;
        s->k2[e] = k2;
        s->mask[e] = (unsigned char)keep;
        /* c(k) and the coefficients of Sec. 4 step 3 */
        cplx c = (d->c0[0] + I * d->c0[1]) + (d->c2[0] + I * d->c2[1]) * k2 +
                 (d->c4[0] + I * d->c4[1]) * k2 * k2;
        cplx x = c * h, p1, p2;
        phi12(x, &p1, &p2);
        s->E[e] = cexp(x);
        if (d->order == 1) { s->wa[e] = h * p1; s->wb[e] = 0; }
        else { s->wa[e] = h * (p1 + p2); s->wb[e] = -h * p2; }
        double Da = d->noise_D * (d->noise_kpow == 2 ? k2 : 1.0);
        cplx q1, q2;
        phi12(2.0 * creal(x) + 0.0 * I, &q1, &q2);
        double var = 2.0 * Da * h * creal(q1);
        s->G[e] = lat * sqrt(var > 0 ? var : 0.0);
        /* model prefactors of the transformed nonlinearity (Sec. 5) */
        switch (d->nl) {
        case NL_PHI3: s->pref[e] = -d->nl_par[0]; break;
        case NL_PHI3_CONS: s->pref[e] = -d->nl_par[0] * k2; break;
        case NL_KPZ: s->pref[e] = 0.5 * d->nl_par[0]; break;
        case NL_CGL: s->pref[e] = -(1.0 + I * d->nl_par[0]); break;
        default: s->pref[e] = 0; break;
        }
    }

    /* initial condition (per site, Philox tag 1), forward FFT and mask */
    for (int rr = 0; rr < r_count; rr++) {
        uint32_t r = (uint32_t)(r_first + rr);
        cplx* ph = s->phi + (size_t)rr * s->nspec;
        if (d->ic_kind == 1) {
            if (d->complex_field) {
                for (size_t nidx = 0; nidx < s->nreal; nidx++) {
                    double z1, z2;
                    orc_normal_pair(d->seed, (uint32_t)nidx, 0u, r, 1u, &z1, &z2);
                    s->work2[nidx] = d->ic_sigma * (z1 + I * z2);
                }
                fftn(s->work2, d->ndim, d->n, -1);
                for (size_t e = 0; e < s->nspec; e++) ph[e] = s->mask[e] ? s->work2[e] : 0;
            } else {
                for (size_t nidx = 0; nidx < s->nreal; nidx++) {
                    double z1, z2;
                    orc_normal_pair(d->seed, (uint32_t)nidx, 0u, r, 1u, &z1, &z2);
                    s->rwork[nidx] = d->ic_sigma * z1;
                }
                rfftn(s->rwork, ph, d->ndim, d->n, s->work);
                for (size_t e = 0; e < s->nspec; e++) if (!s->mask[e]) ph[e] = 0;
                hermitian_planes(s, ph);
            }
        }
    }
    s->step = 0;
    return s;
}

orc_sim* orc_create(const orc_desc* d) { return orc_create_subset(d, 0, d ? d->realizations : 0); }

void orc_destroy(orc_sim* s)
{
    if (!s) return;
    free(s->phi); free(s->fprev); free(s->k2); free(s->kidx); free(s->mask);
    free(s->E); free(s->wa); free(s->wb); free(s->G); free(s->pref);
    free(s->work); free(s->work2); free(s->rwork); free(s->rwork2); free(s->F);
    free(s->snap); free(s->acc); free(s->have_prev); free(s->series); free(s->rs_eta);
    free(s);
}

size_t orc_nspec(const orc_sim* s) { return s->nspec; }
int64_t orc_step_index(const orc_sim* s) { return s->step; }
int orc_nbins(const orc_sim* s) { return s->nbins; }

/* Number of OpenMP threads the oracle's parallel loops use. */
int orc_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* Step 1 of Sec. 4: F_a = M_a pref_a FFT[N(IFFT[phi])]                      */
/* ------------------------------------------------------------------------ */
static void nonlinear_raw(orc_sim* s, const cplx* ph, cplx* F);

/* Phase-shift dealiasing (Sec. 4; the paper names the method, the rule here
   is this implementation's reading): the nonlinearity is evaluated on the grid
   and on the grids moved by dx/2 along every nonempty set of axes, i.e. from
   e^{i k.s} phi_a with s_i in {0, dx/2}, and each transform is moved back with
   e^{-i k.s}.  In the mean of the 2^d transforms an alias a + m N (m_i in
   {-1, 0, 1} per axis) carries the factor prod_i (1 + (-1)^{m_i}) / 2, which
   vanishes unless m = 0.  With the Nyquist modes dropped, the quadratic and
   cubic products of modes |a_i| < N_i/2 alias at most once per axis, so F is
   alias-free.  On a line: the grid and the grid moved by dx/2. */
static void nonlinear_term(orc_sim* s, const cplx* ph, cplx* F)
{
    const orc_desc* d = &s->d;
    size_t ns = s->nspec;
    if (d->nl == NL_NONE) { for (size_t e = 0; e < ns; e++) F[e] = 0; return; }
    nonlinear_raw(s, ph, F);
    if (d->dealias == 2) {
        const int nsh = 1 << d->ndim;
        cplx* shifted = (cplx*)malloc(sizeof(cplx) * ns);
        cplx* Fs = (cplx*)malloc(sizeof(cplx) * ns);
        for (int m = 1; m < nsh; m++) {   /* m = 0 is the unshifted grid, F already */
            for (size_t e = 0; e < ns; e++) {
                double th = 0.0;
                for (int i = 0; i < d->ndim; i++)
                    if ((m >> i) & 1) th += M_PI * s->kidx[3 * e + i] / d->n[i];
                shifted[e] = cexp(I * th) * ph[e];
            }
            nonlinear_raw(s, shifted, Fs);
            for (size_t e = 0; e < ns; e++) {
                double th = 0.0;
                for (int i = 0; i < d->ndim; i++)
                    if ((m >> i) & 1) th += M_PI * s->kidx[3 * e + i] / d->n[i];
                F[e] += cexp(-I * th) * Fs[e];
            }
        }
        for (size_t e = 0; e < ns; e++) F[e] = F[e] / (double)nsh;
        free(shifted);
        free(Fs);
    }
    for (size_t e = 0; e < ns; e++) F[e] = s->mask[e] ? s->pref[e] * F[e] : 0;
}

/* FFT[N(IFFT[phi])] without mask or prefactor */
static void nonlinear_raw(orc_sim* s, const cplx* ph, cplx* F)
{
    const orc_desc* d = &s->d;
    size_t ns = s->nspec, nr = s->nreal;
    if (d->complex_field) {
        for (size_t e = 0; e < nr; e++) s->work2[e] = ph[e];
        fftn(s->work2, d->ndim, d->n, +1);
        for (size_t e = 0; e < nr; e++) {
            cplx A = s->work2[e];
            if (d->nl == NL_CGL) s->work2[e] = (creal(A) * creal(A) + cimag(A) * cimag(A)) * A;
            else s->work2[e] = A * A * A;   /* phi^3 on a complex field */
        }
        fftn(s->work2, d->ndim, d->n, -1);
        for (size_t e = 0; e < ns; e++) F[e] = s->work2[e];
        return;
    }
    if (d->nl == NL_KPZ) {
        /* |grad h|^2 = sum_j (IFFT[i k_j h_a])^2, Nyquist derivative set to 0 */
        for (size_t e = 0; e < nr; e++) s->rwork2[e] = 0;
        for (int ax = 0; ax < d->ndim; ax++) {
            double dk = 2.0 * M_PI / (d->n[ax] * d->dx);
            for (size_t e = 0; e < ns; e++) {
                int a = s->kidx[3 * e + ax];
                int nyq = (2 * abs(a) == d->n[ax]);
                F[e] = nyq ? 0 : (I * dk * a) * ph[e];
            }
            irfftn(F, s->rwork, d->ndim, d->n, s->work);
            for (size_t e = 0; e < nr; e++) s->rwork2[e] += s->rwork[e] * s->rwork[e];
        }
    } else {
        irfftn(ph, s->rwork, d->ndim, d->n, s->work);
        for (size_t e = 0; e < nr; e++) { double p = s->rwork[e]; s->rwork2[e] = p * p * p; }
    }
    rfftn(s->rwork2, F, d->ndim, d->n, s->work);
}

/* App. B: the mode whose draw gives eta_a of mode e (e itself, or on the
   a_d in {0, N_d/2} planes of a real field the member of the conjugate pair
   with the smaller linear index), how eta_a follows from it (0: (z1 + i z2)
   /sqrt2, 1: z1, 2: the conjugate of kind 0), and its Philox slot */
int orc_noise_slot(const orc_sim* s, size_t e, uint32_t* P, int* half, int* kind)
{
    const orc_desc* d = &s->d;
    int last = d->ndim - 1;
    int j[3] = { 0, 0, 0 };
    unlin(s, e, j);
    size_t ed = e;
    *kind = 0;
    if (!d->complex_field && !(j[last] > 0 && 2 * j[last] < d->n[last])) {
        int jp[3] = { 0, 0, 0 };
        for (int i = 0; i < last; i++) jp[i] = (j[i] == 0) ? 0 : d->n[i] - j[i];
        jp[last] = j[last];
        size_t ep = lin_index(s, jp);
        if (ep == e) *kind = 1;
        else if (ep < e) { *kind = 2; ed = ep; }
    }
    if (d->ndim == 1 && !d->complex_field) {
        /* a real line stores a = 0..N/2: the block of a < N/2 serves a and
           a + 2M (M = N/8, 1 for N < 8), the lower one taking half 0; the
           Nyquist mode a = N/2 draws alone from block 2M */
        size_t M1 = d->n[0] >= 8 ? (size_t)d->n[0] / 8 : 1;
        size_t a = ed;
        if (2 * a == (size_t)d->n[0]) { *P = (uint32_t)(2 * M1); *half = 0; }
        else { size_t q = a / M1; *P = (uint32_t)(a % M1 + (q % 2) * M1); *half = (int)(q / 2); }
        return 0;
    }
    /* pair the drawing mode's axis-0 position j0 with (j0 mod M) + (7 - j0 div M) M */
    size_t S = s->nspec / (size_t)s->nh[0];   /* elements per axis-0 position */
    size_t j0 = ed / S, rest = ed % S;
    size_t M = d->n[0] >= 8 ? (size_t)d->n[0] / 8 : 1;
    size_t q = j0 / M;
    size_t row = j0 % M + (q < 4 ? q : 7 - q) * M;
    *P = (uint32_t)(row * S + rest);
    *half = q >= 4;
    return 0;
}

/* Step 2 of Sec. 4 with App. B: eta_a for realization r at step n */
static cplx noise_eta(const orc_sim* s, size_t e, int64_t n, uint32_t r)
{
    const double rs2 = 0.70710678118654752440;
    double z1, z2;
    uint32_t P;
    int half, kind;
    if (!s->mask[e]) return 0;
    orc_noise_slot(s, e, &P, &half, &kind);
    orc_noise_normals(s->d.seed, P, (uint32_t)n, r, half, &z1, &z2);
    if (kind == 1) return z1;
    if (kind == 2) return conj((z1 + I * z2) * rs2);
    return (z1 + I * z2) * rs2;
}

/* The alternative of Sec. 4 step 2: eta drawn in real space and transformed
   (one more FFT per step; App. B counts one real deviate per site).  Site x
   (linear index over the lattice) takes Box-Muller normals of Philox blocks
   with counter (P, n, r, 3), 32-bit words as for the Fourier noise.  A real
   field: Q = nreal/4 blocks, site x takes normal (x div Q) mod 2 of half
   (x div Q) div 2 of block x mod Q, so eta_x ~ N(0, 1).  A complex field:
   nreal/2 blocks, site x takes (z1 + i z2)/sqrt2 of half x div (nreal/2) of
   block x mod (nreal/2).  Then eta_a = DFT[eta_x]_a / sqrt(nreal), which has
   the statistics of App. B (unit variance, Hermitian for a real field). */
static void noise_block_normals(uint64_t seed, uint32_t P, uint32_t n, uint32_t r, uint32_t tag, int half,
                                double* z1, double* z2)
{
    uint32_t ctr[4] = { P, n, r, tag };
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    uint32_t x[4];
    orc_philox(ctr, key, x);
    double u1 = ((double)x[half ? 2 : 0] + 0.5) * 0x1p-32;
    double u2 = ((double)x[half ? 3 : 1] + 0.5) * 0x1p-32;
    double rad = sqrt(-2.0 * log(u1));
    *z1 = rad * cos(2.0 * M_PI * u2);
    *z2 = rad * sin(2.0 * M_PI * u2);
}

int orc_site_noise(const orc_sim* s, int64_t n, uint32_t r, double* out)
{
    const orc_desc* d = &s->d;
    const size_t nr = s->nreal;
    for (size_t x = 0; x < nr; x++) {
        double z1, z2;
        if (d->complex_field) {
            const size_t Q = nr / 2;
            noise_block_normals(d->seed, (uint32_t)(x % Q), (uint32_t)n, r, 3u, (int)(x / Q), &z1, &z2);
            out[2 * x] = z1 * 0.70710678118654752440;
            out[2 * x + 1] = z2 * 0.70710678118654752440;
        } else {
            const size_t Q = nr / 4, slot = x / Q;
            noise_block_normals(d->seed, (uint32_t)(x % Q), (uint32_t)n, r, 3u, (int)(slot / 2), &z1, &z2);
            out[x] = (slot % 2) ? z2 : z1;
        }
    }
    return 0;
}

static cplx noise_eta_rs(orc_sim* s, size_t e, int64_t n, uint32_t r)
{
    if (!s->mask[e]) return 0;
    if (!s->rs_eta || s->rs_n != n || s->rs_r != (int64_t)r) {
        const orc_desc* d = &s->d;
        const size_t nr = s->nreal;
        if (!s->rs_eta) s->rs_eta = (cplx*)malloc(sizeof(cplx) * s->nspec);
        double* site = (double*)malloc(sizeof(double) * 2 * nr);
        orc_site_noise(s, n, r, site);
        const double sc = 1.0 / sqrt((double)nr);
        if (d->complex_field) {
            for (size_t x = 0; x < nr; x++) s->work2[x] = site[2 * x] + I * site[2 * x + 1];
            fftn(s->work2, d->ndim, d->n, -1);
            for (size_t e2 = 0; e2 < s->nspec; e2++) s->rs_eta[e2] = sc * s->work2[e2];
        } else {
            for (size_t x = 0; x < nr; x++) s->rwork[x] = site[x];
            rfftn(s->rwork, s->rs_eta, d->ndim, d->n, s->work);
            for (size_t e2 = 0; e2 < s->nspec; e2++) s->rs_eta[e2] *= sc;
            hermitian_planes(s, s->rs_eta);
        }
        free(site);
        s->rs_n = n;
        s->rs_r = (int64_t)r;
    }
    return s->rs_eta[e];
}

static cplx step_eta(orc_sim* s, size_t e, int64_t n, uint32_t r)
{
    return s->d.noise_space ? noise_eta_rs(s, e, n, r) : noise_eta(s, e, n, r);
}

/* the additive noise term G_a eta_a of step n for all realizations */
int orc_noise_xi(orc_sim* s, int64_t n, double* xi_out)
{
    cplx* xi = (cplx*)xi_out;
    for (int rr = 0; rr < s->R; rr++)
        for (size_t e = 0; e < s->nspec; e++)
            xi[(size_t)rr * s->nspec + e] = s->G[e] * step_eta(s, e, n, (uint32_t)(s->r_first + rr));
    return 0;
}

/* Steps 3-4 of Sec. 4 (Eq. SETD1 / SETD2) with a given noise term */
static void update(orc_sim* s, int rr, const cplx* xi)
{
    cplx* ph = s->phi + (size_t)rr * s->nspec;
    cplx* fp = s->fprev + (size_t)rr * s->nspec;
    const cplx* F = s->F;
    int first = !s->have_prev[rr];
    for (size_t e = 0; e < s->nspec; e++) {
        if (!s->mask[e]) { ph[e] = 0; fp[e] = 0; continue; }
        cplx Fp = (s->d.order == 2 && !first) ? fp[e] : F[e];
        cplx v = s->E[e] * ph[e] + s->wa[e] * F[e] + xi[e];
        if (s->d.order == 2) v += s->wb[e] * Fp;
        ph[e] = v;
        fp[e] = F[e];
    }
    hermitian_planes(s, ph);
}

static int step_once(orc_sim* s, const cplx* xi_all)
{
    cplx* xi = (cplx*)malloc(sizeof(cplx) * s->nspec);
    for (int rr = 0; rr < s->R; rr++) {
        cplx* ph = s->phi + (size_t)rr * s->nspec;
        nonlinear_term(s, ph, s->F);
        if (xi_all) memcpy(xi, xi_all + (size_t)rr * s->nspec, sizeof(cplx) * s->nspec);
        else
            for (size_t e = 0; e < s->nspec; e++)
                xi[e] = s->G[e] * step_eta(s, e, s->step, (uint32_t)(s->r_first + rr));
        update(s, rr, xi);
        s->have_prev[rr] = 1;
    }
    free(xi);
    s->step += 1;
    return 0;
}

static int shell_of(const orc_sim* s, size_t e);
static double mode_weight(const orc_sim* s, size_t e);

static void series_record(orc_sim* s)
{
    if (!s->series || s->series_pos >= s->series_len) return;
    memcpy(s->series + (size_t)s->series_pos * s->R * s->nspec, s->phi, sizeof(cplx) * (size_t)s->R * s->nspec);
    s->series_pos++;
}

int orc_step(orc_sim* s, int64_t nsteps)
{
    for (int64_t i = 0; i < nsteps; i++) {
        step_once(s, NULL);
        series_record(s);
    }
    return 0;
}

/* Start a time series of M samples (App. C, dynamic correlations): phi_a(m)
   for m = 0 (now) .. M - 1 (after M - 1 further steps). */
int orc_series_start(orc_sim* s, int M)
{
    if (M < 2) return -1;
    free(s->series);
    s->series = (cplx*)malloc(sizeof(cplx) * (size_t)M * s->R * s->nspec);
    if (!s->series) return -1;
    s->series_len = M;
    s->series_pos = 0;
    s->series_step0 = s->step;
    series_record(s);
    return 0;
}

/* Time-frequency observables of App. C from the recorded series, with
   phi_{a,b} = sum_m e^{2 pi i b m / M} phi_a(m) and the same transform xi_{a,b}
   of the kicks xi_a(m) = G_a eta_a(n0 + m) of the steps taken from the samples:
     C(k, w_b)   = (L/N^2)^d (T/M^2) <|phi_{a,b}|^2>,                T = M h,
     chi(k, w_b) = (L/N^2)^d (T/M^2) (1/2D_a) <phi_{a,b} conj[xi_{a,b}/h]>,
   the paper's estimators with the sum over the ensemble taken as its mean
   and [d_t phi - K] over a step taken as the step's kick over h.  Means over
   realizations and over the modes of each shell with G_a > 0 and D_a > 0; an
   interior mode a of a real field also stands for -a, whose transforms at
   w_b are the conjugates of a's at -w_b.  out: C [nbins][M], Re chi
   [nbins][M], Im chi [nbins][M], mode count [nbins]. */
int orc_spectrum(orc_sim* s, double* out, size_t cap, size_t* len)
{
    const orc_desc* d = &s->d;
    const int nb = s->nbins, M = s->series_len;
    /* chi regenerates the kicks' Fourier-space draws */
    if (!s->series || s->series_pos < M || s->d.noise_space || cap < (size_t)3 * nb * M + nb) return -1;
    double vol = 1.0;
    for (int i = 0; i < d->ndim; i++) vol *= (d->n[i] * d->dx) / ((double)d->n[i] * (double)d->n[i]);
    memset(out, 0, sizeof(double) * ((size_t)3 * nb * M + nb));
    double* C = out;
    double* Xr = out + (size_t)nb * M;
    double* Xi = out + (size_t)2 * nb * M;
    double* cnt = out + (size_t)3 * nb * M;
    cplx* ph = (cplx*)malloc(sizeof(cplx) * M);
    cplx* xi = (cplx*)malloc(sizeof(cplx) * M);
    cplx* pbs = (cplx*)malloc(sizeof(cplx) * M);
    cplx* xbs = (cplx*)malloc(sizeof(cplx) * M);
    for (size_t e = 0; e < s->nspec; e++) {
        if (!s->mask[e] || !(s->G[e] > 0)) continue;
        const double Da = d->noise_D * (d->noise_kpow == 2 ? s->k2[e] : 1.0);
        if (!(Da > 0)) continue;
        const int j = shell_of(s, e);
        const double w = mode_weight(s, e);
        cnt[j] += w;
        for (int rr = 0; rr < s->R; rr++) {
            for (int m = 0; m < M; m++) {
                ph[m] = s->series[((size_t)m * s->R + rr) * s->nspec + e];
                xi[m] = s->G[e] * noise_eta(s, e, s->series_step0 + m, (uint32_t)(s->r_first + rr));
            }
            for (int b = 0; b < M; b++) {
                cplx pb = 0, xb = 0;
                for (int m = 0; m < M; m++) {
                    const cplx z = cexp(I * 2.0 * M_PI * (double)(((int64_t)b * m) % M) / (double)M);
                    pb += z * ph[m];
                    xb += z * xi[m];
                }
                pbs[b] = pb;
                xbs[b] = xb;
            }
            for (int b = 0; b < M; b++) {
                const int nbq = (M - b) % M;   /* -b */
                double c2 = creal(pbs[b]) * creal(pbs[b]) + cimag(pbs[b]) * cimag(pbs[b]);
                cplx x = pbs[b] * conj(xbs[b]);
                if (w == 2.0) {
                    c2 += creal(pbs[nbq]) * creal(pbs[nbq]) + cimag(pbs[nbq]) * cimag(pbs[nbq]);
                    x += conj(pbs[nbq] * conj(xbs[nbq]));
                }
                C[(size_t)j * M + b] += vol * d->h / M * c2 / s->R;
                Xr[(size_t)j * M + b] += vol / (2.0 * Da * M) * creal(x) / s->R;
                Xi[(size_t)j * M + b] += vol / (2.0 * Da * M) * cimag(x) / s->R;
            }
        }
    }
    for (int j = 0; j < nb; j++) {
        if (cnt[j] <= 0) continue;
        for (int b = 0; b < M; b++) {
            C[(size_t)j * M + b] /= cnt[j];
            Xr[(size_t)j * M + b] /= cnt[j];
            Xi[(size_t)j * M + b] /= cnt[j];
        }
    }
    free(ph); free(xi); free(pbs); free(xbs);
    *len = (size_t)3 * nb * M + nb;
    return 0;
}

/* FDT check of Sec. 5 (App. C estimators): per mode a and frequency w_b of
   the completed window, the deviation Delta_{a,b} = 2 Im chi - (w_b/D_a) C
   of the ensemble means over the realizations, with C and chi as in
   orc_spectrum (here per mode, not per shell) and w_b = 2 pi b/T, b signed in
   FFT order (b = M/2 taken as -M/2).  With chi normalised by 1/(2 D_a) the
   relation holds with D_a = D k^kpow per mode.  out[0] = the average absolute
   deviation over all N^d modes and M frequencies (an interior mode of a real
   field stands for -a too: Delta_{-a,b} = -Delta_{a,-b}, so it counts twice),
   out[1] = the signed average.  Modes with G_a = 0 or D_a = 0 contribute 0. */
int orc_fdt(orc_sim* s, double* out, size_t cap, size_t* len)
{
    const orc_desc* d = &s->d;
    const int M = s->series_len;
    if (!s->series || s->series_pos < M || s->d.noise_space || cap < 2) return -1;
    double vol = 1.0;
    for (int i = 0; i < d->ndim; i++) vol *= (d->n[i] * d->dx) / ((double)d->n[i] * (double)d->n[i]);
    cplx* ph = (cplx*)malloc(sizeof(cplx) * M);
    cplx* xi = (cplx*)malloc(sizeof(cplx) * M);
    double* dlt = (double*)malloc(sizeof(double) * M);
    double sabs = 0.0, ssgn = 0.0;
    for (size_t e = 0; e < s->nspec; e++) {
        if (!s->mask[e] || !(s->G[e] > 0)) continue;
        const double Da = d->noise_D * (d->noise_kpow == 2 ? s->k2[e] : 1.0);
        if (!(Da > 0)) continue;
        const double w = mode_weight(s, e);
        for (int b = 0; b < M; b++) dlt[b] = 0.0;
        for (int rr = 0; rr < s->R; rr++) {
            for (int m = 0; m < M; m++) {
                ph[m] = s->series[((size_t)m * s->R + rr) * s->nspec + e];
                xi[m] = s->G[e] * noise_eta(s, e, s->series_step0 + m, (uint32_t)(s->r_first + rr));
            }
            for (int b = 0; b < M; b++) {
                cplx pb = 0, xb = 0;
                for (int m = 0; m < M; m++) {
                    const cplx z = cexp(I * 2.0 * M_PI * (double)(((int64_t)b * m) % M) / (double)M);
                    pb += z * ph[m];
                    xb += z * xi[m];
                }
                const int bs = (2 * b < M) ? b : b - M;
                const double wh = 2.0 * M_PI * bs / (double)M;   /* w_b h */
                const double c2 = creal(pb) * creal(pb) + cimag(pb) * cimag(pb);
                const double im = cimag(pb * conj(xb));
                /* 2 Im chi - (w/D_a) C with chi = vol/(2 D_a M) phi conj(xi),
                   C = vol h/M |phi|^2, both means over the realizations */
                dlt[b] += vol / (Da * M) * (im - wh * c2) / s->R;
            }
        }
        for (int b = 0; b < M; b++) {
            sabs += w * fabs(dlt[b]);
            if (w == 1.0) ssgn += dlt[b];
        }
    }
    const double denom = (double)s->nreal * (double)M;
    out[0] = sabs / denom;
    out[1] = ssgn / denom;
    *len = 2;
    free(ph); free(xi); free(dlt);
    return 0;
}

int orc_step_xi(orc_sim* s, const double* xi)
{
    return step_once(s, (const cplx*)xi);
}

/* which: 0 state phi_a, 1 previous nonlinear term F_{n-1} */
int orc_get(const orc_sim* s, int which, int rr, double* out)
{
    if (rr < 0 || rr >= s->R) return -1;
    const cplx* src = (which == 0 ? s->phi : s->fprev) + (size_t)rr * s->nspec;
    memcpy(out, src, sizeof(cplx) * s->nspec);
    return 0;
}

/* setting a realization's state restarts its SETD2 history (F_{-1} = F_0) */
int orc_set(orc_sim* s, int rr, const double* in)
{
    if (rr < 0 || rr >= s->R) return -1;
    cplx* dst = s->phi + (size_t)rr * s->nspec;
    const cplx* src = (const cplx*)in;
    for (size_t e = 0; e < s->nspec; e++) dst[e] = s->mask[e] ? src[e] : 0;
    hermitian_planes(s, dst);
    s->have_prev[rr] = 0;
    return 0;
}

int orc_set_step(orc_sim* s, int64_t n) { s->step = n; return 0; }

/* per-mode coefficient arrays (interleaved complex unless noted)
   which: 0 E, 1 wa, 2 wb, 3 G (real), 4 k^2 (real), 5 mask (real 0/1), 6 pref */
int orc_coef(const orc_sim* s, int which, double* out)
{
    for (size_t e = 0; e < s->nspec; e++) {
        switch (which) {
        case 0: out[2 * e] = creal(s->E[e]); out[2 * e + 1] = cimag(s->E[e]); break;
        case 1: out[2 * e] = creal(s->wa[e]); out[2 * e + 1] = cimag(s->wa[e]); break;
        case 2: out[2 * e] = creal(s->wb[e]); out[2 * e + 1] = cimag(s->wb[e]); break;
        case 3: out[e] = s->G[e]; break;
        case 4: out[e] = s->k2[e]; break;
        case 5: out[e] = s->mask[e]; break;
        case 6: out[2 * e] = creal(s->pref[e]); out[2 * e + 1] = cimag(s->pref[e]); break;
        default: return -1;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Observables (Sec. 5, App. C)                                             */
/* ------------------------------------------------------------------------ */
/* weight of a stored mode in sums over the full spectrum */
static double mode_weight(const orc_sim* s, size_t e)
{
    if (s->d.complex_field) return 1.0;
    int j[3] = { 0, 0, 0 };
    unlin(s, e, j);
    int last = s->d.ndim - 1;
    int ad = j[last];
    return (ad > 0 && 2 * ad < s->d.n[last]) ? 2.0 : 1.0;
}

static int shell_of(const orc_sim* s, size_t e)
{
    long m = 0;
    for (int i = 0; i < s->d.ndim; i++) { long a = s->kidx[3 * e + i]; m += a * a; }
    return isqrt_ceil(m);
}

/* kinds: 0 S(k) by shell, 1 width, 2 snapshot, 3 two-time C(k,n,n_w),
   4 step index, 5 accumulate S(k), 6 mean of accumulated S(k) */
int orc_observe(orc_sim* s, int kind, double* out, size_t cap, size_t* len)
{
    const orc_desc* d = &s->d;
    int nb = s->nbins;
    double vol = 1.0;   /* prod L_i / N_i^2 */
    for (int i = 0; i < d->ndim; i++) vol *= (d->n[i] * d->dx) / ((double)d->n[i] * (double)d->n[i]);
    if (kind == 0 || kind == 5) {
        if (kind == 0 && cap < (size_t)2 * nb) return -1;
        double* sum = (double*)calloc((size_t)nb, sizeof(double));
        double* cnt = (double*)calloc((size_t)nb, sizeof(double));
        for (size_t e = 0; e < s->nspec; e++) {
            if (!s->mask[e]) continue;
            double w = mode_weight(s, e);
            int b = shell_of(s, e);
            double acc = 0;
            for (int rr = 0; rr < s->R; rr++) {
                cplx v = s->phi[(size_t)rr * s->nspec + e];
                acc += creal(v) * creal(v) + cimag(v) * cimag(v);
            }
            sum[b] += w * vol * acc / s->R;
            cnt[b] += w;
        }
        if (kind == 0) {
            for (int b = 0; b < nb; b++) { out[b] = cnt[b] > 0 ? sum[b] / cnt[b] : 0; out[nb + b] = cnt[b]; }
            *len = (size_t)2 * nb;
        } else {
            for (int b = 0; b < nb; b++) { s->acc[b] += cnt[b] > 0 ? sum[b] / cnt[b] : 0; s->acc[nb + b] = cnt[b]; }
            s->acc_count += 1;
            if (cap >= 1) { out[0] = s->acc_count; *len = 1; } else *len = 0;
        }
        free(sum); free(cnt);
        return 0;
    }
    if (kind == 6) {
        if (cap < (size_t)2 * nb) return -1;
        for (int b = 0; b < nb; b++) {
            out[b] = s->acc_count > 0 ? s->acc[b] / s->acc_count : 0;
            out[nb + b] = s->acc[nb + b];
        }
        *len = (size_t)2 * nb;
        return 0;
    }
    if (kind == 1) {
        /* width with l = L via Parseval: var = N^{-2d} sum_{a != 0} |h_a|^2 */
        if (cap < 1) return -1;
        double tot = 0, nn = (double)s->nreal;
        for (int rr = 0; rr < s->R; rr++)
            for (size_t e = 1; e < s->nspec; e++) {
                cplx v = s->phi[(size_t)rr * s->nspec + e];
                tot += mode_weight(s, e) * (creal(v) * creal(v) + cimag(v) * cimag(v));
            }
        out[0] = sqrt(tot / (nn * nn) / s->R);
        *len = 1;
        return 0;
    }
    if (kind == 2) {
        if (!s->snap) s->snap = (cplx*)malloc(sizeof(cplx) * (size_t)s->R * s->nspec);
        memcpy(s->snap, s->phi, sizeof(cplx) * (size_t)s->R * s->nspec);
        s->snap_step = s->step; s->have_snap = 1;
        if (cap >= 1) { out[0] = (double)s->step; *len = 1; } else *len = 0;
        return 0;
    }
    if (kind == 3) {
        if (!s->have_snap || cap < (size_t)3 * nb) return -1;
        double* re = (double*)calloc((size_t)nb, sizeof(double));
        double* im = (double*)calloc((size_t)nb, sizeof(double));
        double* cnt = (double*)calloc((size_t)nb, sizeof(double));
        for (size_t e = 0; e < s->nspec; e++) {
            if (!s->mask[e]) continue;
            double w = mode_weight(s, e);
            int b = shell_of(s, e);
            cplx acc = 0;
            for (int rr = 0; rr < s->R; rr++)
                acc += s->phi[(size_t)rr * s->nspec + e] * conj(s->snap[(size_t)rr * s->nspec + e]);
            acc *= vol / s->R;
            if (w == 2.0) { re[b] += 2.0 * creal(acc); }      /* a and -a: 2 Re */
            else { re[b] += creal(acc); im[b] += cimag(acc); }
            cnt[b] += w;
        }
        for (int b = 0; b < nb; b++) {
            out[b] = cnt[b] > 0 ? re[b] / cnt[b] : 0;
            out[nb + b] = cnt[b] > 0 ? im[b] / cnt[b] : 0;
            out[2 * nb + b] = cnt[b];
        }
        *len = (size_t)3 * nb;
        free(re); free(im); free(cnt);
        return 0;
    }
    if (kind == 4) {
        if (cap < 1) return -1;
        out[0] = (double)s->step;
        *len = 1;
        return 0;
    }
    if (kind == 11) {
        /* box-averaged width (Sec. 5 KPZ): w_l = sqrt of the mean over boxes of
           l^d sites and realizations of [mean_box h^2 - (mean_box h)^2]
           (a complex field: mean_box |A|^2 - |mean_box A|^2), from the
           real-space field, for l = 2, 4, .., N (equal n[i]) */
        int nl = 0;
        for (int l = 2; l <= d->n[0]; l *= 2) nl++;
        if (cap < (size_t)nl) return -1;
        for (int i = 1; i < d->ndim; i++) if (d->n[i] != d->n[0]) return -1;
        const int N = d->n[0], nd = d->ndim;
        double* acc = (double*)calloc((size_t)nl, sizeof(double));
        cplx* x = (cplx*)malloc(sizeof(cplx) * s->nreal);
        for (int rr = 0; rr < s->R; rr++) {
            cplx* src = s->phi + (size_t)rr * s->nspec;
            if (d->complex_field) {
                memcpy(x, src, sizeof(cplx) * s->nreal);
                fftn(x, nd, d->n, +1);                 /* scaled by 1/N^d */
            } else {
                irfftn(src, s->rwork, nd, d->n, s->work);
                for (size_t i = 0; i < s->nreal; i++) x[i] = s->rwork[i];
            }
            int li = 0;
            for (int l = 2; l <= N; l *= 2, li++) {
                const int P = N / l;
                size_t nbox = 1;
                for (int dd = 0; dd < nd; dd++) nbox *= (size_t)P;
                cplx* s1 = (cplx*)calloc(nbox, sizeof(cplx));
                double* s2 = (double*)calloc(nbox, sizeof(double));
                for (size_t i = 0; i < s->nreal; i++) {
                    size_t rem = i, box = 0;
                    int c[3] = { 0, 0, 0 };
                    for (int dd = nd - 1; dd >= 0; dd--) { c[dd] = (int)(rem % (size_t)N); rem /= (size_t)N; }
                    for (int dd = 0; dd < nd; dd++) box = box * (size_t)P + (size_t)(c[dd] / l);
                    s1[box] += x[i];
                    s2[box] += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
                }
                const double per = pow((double)l, nd);
                double v = 0;
                for (size_t b = 0; b < nbox; b++) {
                    const cplx m = s1[b] / per;
                    v += s2[b] / per - (creal(m) * creal(m) + cimag(m) * cimag(m));
                }
                acc[li] += v / (double)nbox;
                free(s1); free(s2);
            }
        }
        for (int i = 0; i < nl; i++) out[i] = sqrt(acc[i] / s->R);
        *len = (size_t)nl;
        free(acc); free(x);
        return 0;
    }
    if (kind == 7) {
        /* the noise of the next step, xi_a(n') = G_a eta_a(n'), is the kick */
        s->kick_step = s->step; s->have_kick = 1;
        if (cap >= 1) { out[0] = (double)s->step; *len = 1; } else *len = 0;
        return 0;
    }
    if (kind == 8) {
        /* Linear response by the noise correlation (the Onsager-Machlup
           estimator of the susceptibility of App. C), in
           discrete time: for the Gaussian kick xi_a(n') of the step taken from
           n', Stein's lemma gives <phi_a(n) conj xi_a(n')> / G_a^2 = the mean
           response of phi_a(n) to an additive kick in that step.  Per shell:
           mean over realizations and modes with G_a > 0 of
           phi_a(n) conj eta_a(n') / G_a, interior modes of a real field as 2 Re. */
        /* the estimator regenerates the kick's Fourier-space draws */
        if (!s->have_kick || s->d.noise_space || cap < (size_t)3 * nb) return -1;
        double* re = (double*)calloc((size_t)nb, sizeof(double));
        double* im = (double*)calloc((size_t)nb, sizeof(double));
        double* cnt = (double*)calloc((size_t)nb, sizeof(double));
        for (size_t e = 0; e < s->nspec; e++) {
            if (!s->mask[e] || !(s->G[e] > 0)) continue;
            double w = mode_weight(s, e);
            int b = shell_of(s, e);
            cplx acc = 0;
            for (int rr = 0; rr < s->R; rr++) {
                cplx eta = noise_eta(s, e, s->kick_step, (uint32_t)(s->r_first + rr));
                acc += s->phi[(size_t)rr * s->nspec + e] * conj(eta);
            }
            acc /= s->G[e] * s->R;
            if (w == 2.0) { re[b] += 2.0 * creal(acc); }
            else { re[b] += creal(acc); im[b] += cimag(acc); }
            cnt[b] += w;
        }
        for (int b = 0; b < nb; b++) {
            out[b] = cnt[b] > 0 ? re[b] / cnt[b] : 0;
            out[nb + b] = cnt[b] > 0 ? im[b] / cnt[b] : 0;
            out[2 * nb + b] = cnt[b];
        }
        *len = (size_t)3 * nb;
        free(re); free(im); free(cnt);
        return 0;
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Scalar SDE schemes (Sec. 2, Eqs. SETD-EM, SETD-Milstein, SETD1)          */
/* ------------------------------------------------------------------------ */
/* du = [c u + F(u)] dt + G(u) dW with F(u) = f1 u + f3 u^3 and
   G(u) = g0 + g1 u: the SAO of Sec. 3 (c = -Gamma, f3 = -Gamma b,
   g0 = sqrt(2 Gamma T)) and GBM (c = lambda - delta, f1 = delta, g1 = mu).
   With x = c h the factors of the schemes are e^x, (e^x - 1)/c = h phi1(x),
   e^{x/2} and sqrt((e^{2x} - 1)/(2c)) = sqrt(h phi1(2x)).  Path p, step n
   draws z = z1 of the Philox block (p, n, 0, 2) (two 53-bit uniforms,
   Box-Muller); dW = sqrt(h) z, and SETD1 takes z as its N(0, 1).
   u_out[p] = u after nsteps steps; w_out[p] (if not NULL) = sum of the dW. */
typedef struct {
    int scheme;           /* 0: SETD-EM, 1: SETD-Milstein, 2: SETD1 */
    double c, f1, f3, g0, g1, h, u0;
    int64_t nsteps;
    int npaths;
    uint64_t seed;
} orc_sde_desc;

int orc_sde_run(const orc_sde_desc* d, double* u_out, double* w_out)
{
    if (!d || d->scheme < 0 || d->scheme > 2 || !(d->h > 0) || d->nsteps < 0 || d->npaths < 0) return -1;
    cplx p1, p2, q1, q2;
    phi12(d->c * d->h, &p1, &p2);
    phi12(2.0 * d->c * d->h, &q1, &q2);
    const double E = exp(d->c * d->h);
    const double fF = d->h * creal(p1);            /* (e^{ch} - 1)/c */
    const double fmid = exp(0.5 * d->c * d->h);    /* e^{ch/2}       */
    const double f4 = sqrt(d->h * creal(q1));      /* sqrt((e^{2ch} - 1)/(2c)) */
    const double sh = sqrt(d->h);
    for (int p = 0; p < d->npaths; p++) {
        double u = d->u0, w = 0.0;
        for (int64_t n = 0; n < d->nsteps; n++) {
            double z1, z2;
            orc_normal_pair(d->seed, (uint32_t)p, (uint32_t)n, 0u, 2u, &z1, &z2);
            const double dW = sh * z1;
            const double F = d->f1 * u + d->f3 * u * u * u;
            const double G = d->g0 + d->g1 * u;
            double noise;
            if (d->scheme == 0) noise = fmid * G * dW;
            else if (d->scheme == 1) noise = fmid * G * (dW + 0.5 * d->g1 * (dW * dW - d->h));
            else noise = f4 * G * z1;
            u = E * u + fF * F + noise;
            w += dW;
        }
        u_out[p] = u;
        if (w_out) w_out[p] = w;
    }
    return 0;
}
