// setd_runtime.hip -- plans and the C ABI of include/setd.h.
#include "setd_runtime.hpp"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <map>
#include <mutex>
#include <new>

#include "setd_launch.hpp"

namespace setd {

static thread_local std::string g_err;

setd_status fail(setd_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

setd_status ok() { return SETD_OK; }

static bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

static int ceil_isqrt_host(long m)
{
    if (m <= 0) return 0;
    long s = (long)std::floor(std::sqrt((double)m));
    while (s * s > m) s--;
    while ((s + 1) * (s + 1) <= m) s++;
    return (int)(s * s == m ? s : s + 1);
}

static size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

setd_status validate(const setd_desc& d)
{
    if (d.ndim < 1 || d.ndim > 3) return fail(SETD_E_INVAL, "ndim must be 1, 2 or 3");
    for (int i = 0; i < d.ndim; i++)
        if (!pow2_in(d.n[i], 8, 1024)) return fail(SETD_E_INVAL, "n[%d] = %d is not a power of two in [8, 1024]", i, d.n[i]);
    if (!(d.dx > 0) || !std::isfinite(d.dx)) return fail(SETD_E_INVAL, "dx must be positive");
    if (!(d.h > 0) || !std::isfinite(d.h)) return fail(SETD_E_INVAL, "h must be positive");
    if (d.order != 1 && d.order != 2) return fail(SETD_E_INVAL, "order must be 1 or 2");
    if (!(d.noise_D >= 0) || !std::isfinite(d.noise_D)) return fail(SETD_E_INVAL, "noise_D must be >= 0");
    if (d.noise_kpow != 0 && d.noise_kpow != 2) return fail(SETD_E_INVAL, "noise_kpow must be 0 or 2");
    if (d.precision != 32 && d.precision != 64) return fail(SETD_E_INVAL, "precision must be 32 or 64");
    if (d.realizations < 1) return fail(SETD_E_INVAL, "realizations must be >= 1");
    if (d.dealias < 0 || d.dealias > 2) return fail(SETD_E_INVAL, "dealias must be 0, 1 or 2");
    if (d.series_len != 0 && !pow2_in(d.series_len, 8, 1024))
        return fail(SETD_E_INVAL, "series_len must be 0 or a power of two in [8, 1024]");
    if (d.ic_kind != 0 && d.ic_kind != 1) return fail(SETD_E_INVAL, "ic_kind must be 0 or 1");
    if (d.complex_field != 0 && d.complex_field != 1) return fail(SETD_E_INVAL, "complex_field must be 0 or 1");
    if (d.noise_space != 0 && d.noise_space != 1) return fail(SETD_E_INVAL, "noise_space must be 0 or 1");
    const bool cimag = d.c0[1] != 0.0 || d.c2[1] != 0.0 || d.c4[1] != 0.0;
    if (cimag && !d.complex_field) return fail(SETD_E_INVAL, "complex c(k) needs a complex field");
    if (d.nl < 0 || d.nl > 4) return fail(SETD_E_INVAL, "unknown nonlinearity %d", d.nl);
    if (d.complex_field && (d.nl == NL_PHI3 || d.nl == NL_PHI3_CONS || d.nl == NL_KPZ))
        return fail(SETD_E_UNSUPPORTED, "complex fields take the CGL nonlinearity or none");
    if (!d.complex_field && d.nl == NL_CGL) return fail(SETD_E_UNSUPPORTED, "the CGL nonlinearity needs a complex field");
    if (d.nl == NL_KPZ && d.ndim == 3) return fail(SETD_E_UNSUPPORTED, "KPZ is built for 1D and 2D lattices");
    const double cs[6] = {d.c0[0], d.c0[1], d.c2[0], d.c2[1], d.c4[0], d.c4[1]};
    for (double v : cs)
        if (!std::isfinite(v)) return fail(SETD_E_INVAL, "c(k) coefficients must be finite");
    if (!std::isfinite(d.nl_par[0]) || !std::isfinite(d.ic_sigma)) return fail(SETD_E_INVAL, "parameters must be finite");
    size_t sites = 1;
    for (int i = 0; i < d.ndim; i++) sites *= (size_t)d.n[i];
    if ((double)sites * d.realizations > 4.0e12) return fail(SETD_E_INVAL, "problem too large");
    return SETD_OK;
}

setd_status Plan::init(const setd_desc& desc)
{
    setd_status st = validate(desc);
    if (st != SETD_OK) return st;
    d = desc;
    R = d.realizations;
    g = Geo{};
    g.ndim = d.ndim;
    g.cplx = d.complex_field;
    g.prec = d.precision;
    g.dealias = d.dealias;
    g.rsn = d.noise_space;
    const int last = d.ndim - 1;
    for (int i = 0; i < 3; i++) {
        if (i >= d.ndim) {
            g.n[i] = 1;
            g.kept[i] = 1;
            g.kp[i] = 0;
            continue;
        }
        const int n = d.n[i];
        g.n[i] = n;
        if (!g.cplx && i == last) {
            // 2/3 rule: 3|a| < n; phase shift: the Nyquist mode dropped
            const int K = d.dealias == 1 ? (n - 1) / 3 : (d.dealias == 2 ? n / 2 - 1 : n / 2);
            g.kept[i] = K + 1;
            g.kp[i] = K;
        } else if (d.dealias) {
            const int K = d.dealias == 1 ? (n - 1) / 3 : n / 2 - 1;
            g.kept[i] = 2 * K + 1;
            g.kp[i] = K;
        } else {
            g.kept[i] = n;
            g.kp[i] = n - 1;
        }
    }
    g.nh_last = g.cplx ? g.n[last] : g.n[last] / 2 + 1;
    const int align = (d.precision == 32) ? 16 : 8;
    g.pitch = (int)round_up((size_t)g.kept[last], (size_t)align);
    elt = (d.precision == 32) ? 8 : 16;

    // lattice (App. A)
    lat = 1.0;
    vol = 1.0;
    nreal = 1;
    nspec = 1;
    for (int i = 0; i < d.ndim; i++) {
        const double L = d.n[i] * d.dx;
        dk[i] = 2.0 * M_PI / L;
        lat *= std::sqrt((double)d.n[i] * (double)d.n[i] / L);
        vol *= L / ((double)d.n[i] * (double)d.n[i]);
        nreal *= (size_t)d.n[i];
        nspec *= (size_t)((i == last) ? g.nh_last : d.n[i]);
    }
    kept_modes = 1;
    for (int i = 0; i < d.ndim; i++) kept_modes *= (size_t)g.kept[i];

    // coefficient keys: |a|^2 when all axes share dk, else separable |a_i|
    iso = 1;
    for (int i = 1; i < d.ndim; i++)
        if (d.n[i] != d.n[0]) iso = 0;
    int kmax[3] = {0, 0, 0};
    for (int i = 0; i < d.ndim; i++)
        kmax[i] = d.dealias == 1 ? (d.n[i] - 1) / 3 : (d.dealias == 2 ? d.n[i] / 2 - 1 : d.n[i] / 2);
    if (d.ndim == 1) {
        coef_mode = COEF_SEPARABLE;  // one entry per |a| of the line
        keydim[0] = kmax[0] + 1;
        keydim[1] = keydim[2] = 1;
        nkeys = keydim[0];
    } else if (d.ndim == 2) {
        coef_mode = COEF_PER_MODE;   // rows |a0| in the state's row layout: coalesced, shared by all realizations
        keydim[0] = keydim[1] = keydim[2] = 1;
    } else if (iso) {
        coef_mode = COEF_ISO;
        long m = 0;
        for (int i = 0; i < d.ndim; i++) m += (long)kmax[i] * kmax[i];
        nkeys = (int)m + 1;
        keydim[0] = keydim[1] = keydim[2] = 1;
    } else {
        coef_mode = COEF_SEPARABLE;
        for (int i = 0; i < 3; i++) keydim[i] = (i < d.ndim) ? kmax[i] + 1 : 1;
        nkeys = keydim[0] * keydim[1] * keydim[2];
    }
    // complex fields always take complex entries (the kernels of a launch class
    // then share one table layout); real fields have real c(k)
    coef_cplx = d.complex_field ? 1 : 0;
    long msq = 0;
    for (int i = 0; i < d.ndim; i++) msq += (long)(d.n[i] / 2) * (d.n[i] / 2);
    nbins = ceil_isqrt_host(msq) + 1;

    // sizes
    // per-mode table of a 2D lattice: rows |a0| = 0..max, the stored columns
    if (coef_mode == COEF_PER_MODE) nkeys = (kmax[0] + 1) * g.pitch;
    const size_t k1 = (d.ndim == 3) ? (size_t)g.kept[1] : 1;
    S = (size_t)geo_rows(g) * g.pitch;
    P = (d.ndim == 1) ? 0 : (size_t)g.n[0] * k1 * g.pitch;   // a line keeps no partial transform
    // 3D: the line buffer of the last-axis pass, four grids of it with phase shifts
    B = (d.ndim == 3) ? (size_t)g.n[0] * g.n[1] * g.pitch * (d.dealias == 2 ? 4 : 1) : 0;
    // Realizations of an array lie an odd multiple of 256 bytes apart: blocks
    // that work on the same columns of different realizations at the same
    // time then reach different HBM channels instead of addresses that agree
    // in all low bits (the unpadded sizes are multiples of 64 KiB).
    auto real_stride = [](size_t bytes) {
        size_t s = round_up(bytes ? bytes : 1, 256);
        if ((s / 256) % 2 == 0) s += 256;
        return s;
    };
    Sb = real_stride(S * elt);
    Pb = real_stride(P * elt);
    Bb = B ? real_stride(B * elt) : 0;
    // SETD2 keeps only the carry unless F_{n-1} must stay readable
    // (real-space noise on 2D/3D lattices is transformed for the step it is
    // used in, so those plans keep phi and F_{n-1})
    lean = d.ndim >= 2 && d.order == 2 && !d.history_readback && d.nl != NL_NONE && !d.noise_space &&
           axis0_register_ok(g, elt / 2);

    // workspace layout, every buffer 256-byte aligned
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += round_up(bytes ? bytes : 1, 256);
        return o;
    };
    const size_t cdbl = coef_cplx ? 8 : 4;
    lay.items = take((size_t)R * sizeof(Item));
    lay.ctrl = take((size_t)R * sizeof(Ctrl));
    lay.coef64 = take((size_t)nkeys * cdbl * 8);
    lay.coef32 = (d.precision == 32) ? take((size_t)nkeys * cdbl * 4) : 0;
    for (int i = 0; i < d.ndim; i++) {
        lay.tw64[i] = take((size_t)d.n[i] * 16);
        lay.tw32[i] = take((size_t)d.n[i] * 8);
    }
    // tables sit below phi: binding clears everything from phi on
    if (d.series_len > 0) {
        lay.twm64 = take((size_t)d.series_len * 16);
        lay.twm32 = take((size_t)d.series_len * 8);
    }
    lay.acc = take((size_t)3 * nbins * 8);
    lay.skacc = take((size_t)(2 * nbins + 1) * 8);
    lay.out = take((size_t)3 * nbins * 8);
    lay.phi = take((size_t)R * Sb);
    lay.prev = (d.order == 2) ? take((size_t)R * Sb) : 0;
    lay.pre0 = take((size_t)R * Pb);
    lay.pre1 = (d.nl == NL_KPZ) ? take((size_t)R * Pb) : 0;
    lay.big = B ? take((size_t)R * Bb) : 0;
    lay.snap = take((size_t)R * Sb);
    if (rsn_grid()) {
        lay.npre = take((size_t)R * Pb);
        lay.noise = take((size_t)R * Sb);
    }
    if (ps_grid()) lay.preb = take((size_t)R * Pb);
    if (ps_grid() && d.nl == NL_KPZ) lay.pre1b = take((size_t)R * Pb);
    if (iso) {
        lay.boxn = 0;
        for (int l = 2; l <= d.n[0]; l *= 2) {
            size_t c = 1;
            for (int i = 0; i < d.ndim; i++) c *= (size_t)(d.n[0] / l);
            lay.boxn += c;
        }
        lay.boxcls = take(lay.boxn * 16);
    }
    if (d.series_len > 0) {
        lay.specacc = take(((size_t)3 * nbins * d.series_len + nbins) * 8);
        lay.fdtacc = take(S * (size_t)d.series_len * 8);
        lay.series = take((size_t)d.series_len * R * Sb);
    }
    lay.total = off;
    return SETD_OK;
}

int Plan::passes_per_step() const
{
    if (d.nl == NL_NONE || d.ndim == 1) return 1;
    return d.ndim == 2 ? 2 : 4;
}

// HBM bytes each pass must move with the stored (2/3-pruned) arrays: one read
// and one write of every array a pass cannot keep in LDS, at the unpadded
// stored sizes.
void Plan::pass_bytes(double* out) const
{
    for (int i = 0; i < 4; i++) out[i] = 0.0;
    const double e = (double)elt * R;
    const double kl = (double)g.kept[g.ndim - 1];
    const double st = (double)kept_modes;                 // stored modes
    const double hist = (d.order == 2 && !lean) ? 2.0 : 0.0;   // read + write F_{n-1} (lean: one carry array)
    if (d.ndim == 1) {
        // a line: state (and F_{n-1}) in and out once per launch, given per step
        // of a one-step launch
        out[0] = (2.0 + hist) * st * e;
        return;
    }
    if (d.nl == NL_NONE) {
        out[0] = 2.0 * st * e;
        return;
    }
    if (d.ndim == 2) {
        const double pre = (double)g.n[0] * kl;
        if (ps_grid()) {
            // phase shifts: pre and its shifted copy in and out of both passes
            // (KPZ: the row pass also reads pre1 and pre1b, which the axis-0
            // pass writes)
            const double g2 = (d.nl == NL_KPZ) ? 2.0 : 0.0;
            out[0] = (4.0 + g2) * pre * e;
            out[1] = (4.0 + g2 + (2.0 + hist) * st / pre) * pre * e;
            return;
        }
        const double npre = (d.nl == NL_KPZ) ? 2.0 : 1.0;
        out[0] = (npre + 1.0) * pre * e;                        // row pass: read pre (and pre1), write pre
        out[1] = ((1.0 + npre) * pre + (2.0 + hist) * st) * e;  // axis 0: pre in/out, state, history
        return;
    }
    const double small = (double)g.n[0] * g.kept[1] * kl;
    const double bigv = (double)g.n[0] * g.n[1] * kl;
    if (ps_grid()) {
        // phase shifts: pre and preb, four grids of the line buffer
        out[0] = (2.0 * small + 4.0 * bigv) * e;
        out[1] = 8.0 * bigv * e;
        out[2] = (4.0 * bigv + 2.0 * small) * e;
        out[3] = (4.0 * small + (2.0 + hist) * st) * e;
        return;
    }
    out[0] = (small + bigv) * e;                                // axis-1 inverse
    out[1] = 2.0 * bigv * e;                                    // row pass
    out[2] = (bigv + small) * e;                                // axis-1 forward
    out[3] = (2.0 * small + (2.0 + hist) * st) * e;             // axis 0
}

double Plan::alg_bytes_per_step() const
{
    double b[4];
    pass_bytes(b);
    double noise = 0.0;
    if (rsn_grid()) {
        // the noise transform: the last-axis pass writes its intermediate
        // (3D: the line buffer, which the axis-1 pass reads and turns into
        // the small intermediate), the axis-0 pass reads that and writes eta_a,
        // and the step reads eta_a
        const double e = (double)elt * R, kl = (double)g.kept[g.ndim - 1];
        const double small = (double)g.n[0] * (g.ndim == 3 ? g.kept[1] : 1) * kl;
        const double bigv = (g.ndim == 3) ? (double)g.n[0] * g.n[1] * kl : 0.0;
        noise = (2.0 * bigv + 2.0 * small + 2.0 * (double)kept_modes) * e;
    }
    return b[0] + b[1] + b[2] + b[3] + noise;
}

template <typename T>
static setd_status launch_pass_t(const Plan& p, int i, const Item* items_dev, int nitems, int sub, hipStream_t s)
{
    const Geo& g = p.g;
    if (g.ndim == 1) {
        SETD_HIP((launch_line1d<T>(g, items_dev, nitems, MODE_STEP, sub, 1, p.d.nl, s)));
        return SETD_OK;
    }
    if (p.d.nl == NL_NONE) {
        SETD_HIP((launch_linear<T>(g, items_dev, nitems, sub, LIN_STEP, 0, s)));
        return SETD_OK;
    }
    if (g.ndim == 2) {
        if (i == 0) SETD_HIP((launch_row<T>(g, items_dev, nitems, MODE_STEP, sub, p.tune.row, p.d.nl == NL_KPZ, s)));
        else SETD_HIP((launch_axis0<T>(g, items_dev, nitems, MODE_STEP, sub, p.tune.ax0, p.d.nl == NL_KPZ, p.lean, s)));
        return SETD_OK;
    }
    // phase shifts: the axis-1 passes carry pre and preb to and from four grids
    const int ps = g.dealias == 2 ? 3 : 1;
    switch (i) {
    case 0: SETD_HIP((launch_axis1<T>(g, items_dev, nitems, +ps, sub, p.tune.ax1, s))); break;
    case 1: SETD_HIP((launch_row<T>(g, items_dev, nitems, MODE_STEP, sub, p.tune.row, p.d.nl == NL_KPZ, s))); break;
    case 2: SETD_HIP((launch_axis1<T>(g, items_dev, nitems, -ps, sub, p.tune.ax1, s))); break;
    default: SETD_HIP((launch_axis0<T>(g, items_dev, nitems, MODE_STEP, sub, p.tune.ax0, p.d.nl == NL_KPZ, p.lean, s))); break;
    }
    return SETD_OK;
}

setd_status Plan::launch_pass(int i, const Item* items_dev, int nitems, int sub, hipStream_t s) const
{
    return d.precision == 32 ? launch_pass_t<float>(*this, i, items_dev, nitems, sub, s)
                             : launch_pass_t<double>(*this, i, items_dev, nitems, sub, s);
}

setd_status Plan::launch_noise(const Item* items_dev, int nitems, int sub, hipStream_t s) const
{
    if (!rsn_grid()) return SETD_OK;
    if (d.precision == 32) SETD_HIP((launch_rsn<float>(g, items_dev, nitems, sub, tune.ax1, tune.ax0, s)));
    else SETD_HIP((launch_rsn<double>(g, items_dev, nitems, sub, tune.ax1, tune.ax0, s)));
    return SETD_OK;
}

setd_status Plan::launch_step(const Item* items_dev, int nitems, int sub, hipStream_t s) const
{
    setd_status st0 = launch_noise(items_dev, nitems, sub, s);
    if (st0 != SETD_OK) return st0;
    for (int i = 0; i < passes_per_step(); i++) {
        setd_status st = launch_pass(i, items_dev, nitems, sub, s);
        if (st != SETD_OK) return st;
    }
    return SETD_OK;
}

template <typename T>
static setd_status launch_ic_t(const Plan& p, const Item* items_dev, int nitems, hipStream_t s)
{
    const Geo& g = p.g;
    if (g.ndim == 1) {
        SETD_HIP((launch_line1d<T>(g, items_dev, nitems, MODE_IC, 0, 0, p.d.nl, s)));
        return SETD_OK;
    }
    SETD_HIP((launch_row<T>(g, items_dev, nitems, MODE_IC, 0, p.tune.row, 0, s)));
    if (g.ndim == 3) SETD_HIP((launch_axis1<T>(g, items_dev, nitems, -1, 0, p.tune.ax1, s)));
    SETD_HIP((launch_axis0<T>(g, items_dev, nitems, MODE_IC, 0, p.tune.ax0, p.d.nl == NL_KPZ, 0, s)));
    return SETD_OK;
}

template <typename T>
static setd_status launch_sync_t(const Plan& p, const Item* items_dev, int nitems, hipStream_t s)
{
    if (p.g.ndim == 1) return SETD_OK;   // a line keeps no partial transform
    SETD_HIP((launch_axis0<T>(p.g, items_dev, nitems, MODE_SYNC, 0, p.tune.ax0, p.d.nl == NL_KPZ, 0, s)));
    return SETD_OK;
}

template <typename T>
static setd_status launch_recover_t(const Plan& p, const Item* items_dev, int nitems, hipStream_t s)
{
    SETD_HIP((launch_axis0<T>(p.g, items_dev, nitems, MODE_RECOVER, 0, p.tune.ax0, p.d.nl == NL_KPZ, 0, s)));
    return SETD_OK;
}

setd_status Plan::ensure_phi()
{
    if (!lean || phi_valid) return SETD_OK;
    const Item* items_dev = reinterpret_cast<const Item*>(ws + lay.items);
    setd_status st = (d.precision == 32) ? launch_recover_t<float>(*this, items_dev, R, stream)
                                         : launch_recover_t<double>(*this, items_dev, R, stream);
    if (st != SETD_OK) return st;
    phi_valid = true;
    return SETD_OK;
}

setd_status Plan::carry_init(const Item* items_dev, int nitems)
{
    if (!lean) return SETD_OK;
    if (d.precision == 32) SETD_HIP((launch_linear<float>(g, items_dev, nitems, 0, LIN_CARRY, 0, stream)));
    else SETD_HIP((launch_linear<double>(g, items_dev, nitems, 0, LIN_CARRY, 0, stream)));
    return SETD_OK;
}

setd_status Plan::bind(void* dev, size_t bytes, hipStream_t s)
{
    if (bound) return fail(SETD_E_STATE, "plan already bound");
    if (!dev) return fail(SETD_E_INVAL, "null workspace");
    if (((uintptr_t)dev) % 256 != 0) return fail(SETD_E_INVAL, "workspace must be 256-byte aligned");
    if (bytes < lay.total) return fail(SETD_E_NOMEM, "workspace of %zu bytes, %zu needed", bytes, lay.total);
    ws = (char*)dev;
    stream = s;
    const int last = d.ndim - 1;
    if (R >= 2 && split_ok && !no_alloc && !aux) {
        SETD_HIP(hipStreamCreateWithFlags(&aux, hipStreamNonBlocking));
        SETD_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
        SETD_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
    }

    items.assign(R, Item{});
    for (int r = 0; r < R; r++) {
        Item& it = items[r];
        it.phi = ws + lay.phi + (size_t)r * Sb;
        it.prev = (d.order == 2) ? ws + lay.prev + (size_t)r * Sb : nullptr;
        it.pre0 = ws + lay.pre0 + (size_t)r * Pb;
        it.pre1 = (d.nl == NL_KPZ) ? ws + lay.pre1 + (size_t)r * Pb : nullptr;
        it.big = B ? ws + lay.big + (size_t)r * Bb : nullptr;
        it.snap = ws + lay.snap + (size_t)r * Sb;
        it.npre = rsn_grid() ? ws + lay.npre + (size_t)r * Pb : nullptr;
        it.noise = rsn_grid() ? ws + lay.noise + (size_t)r * Sb : nullptr;
        it.preb = ps_grid() ? ws + lay.preb + (size_t)r * Pb : nullptr;
        it.pre1b = (ps_grid() && d.nl == NL_KPZ) ? ws + lay.pre1b + (size_t)r * Pb : nullptr;
        it.coef = ws + ((d.precision == 32) ? lay.coef32 : lay.coef64);
        const size_t* tw = (d.precision == 32) ? lay.tw32 : lay.tw64;
        it.tw0 = ws + tw[0];
        it.tw1 = ws + tw[1];
        it.tw2 = (d.ndim == 3) ? ws + tw[2] : nullptr;
        it.ctrl = reinterpret_cast<Ctrl*>(ws + lay.ctrl) + r;
        it.seed = d.seed;
        it.r = (uint32_t)r;
        it.nl = d.nl;
        it.order = d.order;
        it.coef_mode = coef_mode;
        it.coef_cplx = coef_cplx;
        {
            const size_t cb = (size_t)nkeys * (coef_cplx ? 8 : 4) * (d.precision == 32 ? 4 : 8);
            it.coef_bytes = (uint32_t)(cb < 0x7fffffffu ? cb : 0x7fffffffu);
        }
        it.steps = INT_MAX;
        for (int i = 0; i < 3; i++) {
            it.keydim[i] = keydim[i];
            it.dk[i] = dk[i];
        }
        it.par0 = d.nl_par[0];
        it.inv_vol = 1.0 / (double)nreal;
        it.ic_sigma = d.ic_sigma;
    }
    (void)last;
    SETD_HIP(hipMemcpyAsync(ws + lay.items, items.data(), (size_t)R * sizeof(Item), hipMemcpyHostToDevice, s));

    // twiddles and the FP64 coefficient table (Sec. 4 step 3)
    for (int i = 0; i < d.ndim; i++)
        SETD_HIP(launch_twiddle(d.n[i], reinterpret_cast<double*>(ws + lay.tw64[i]),
                                reinterpret_cast<float*>(ws + lay.tw32[i]), s));
    if (d.series_len > 0)
        SETD_HIP(launch_twiddle(d.series_len, reinterpret_cast<double*>(ws + lay.twm64),
                                reinterpret_cast<float*>(ws + lay.twm32), s));
    CoefArgs ca{};
    ca.nkeys = nkeys;
    ca.mode = coef_mode;
    ca.g = g;
    ca.ndim = d.ndim;
    ca.order = d.order;
    ca.kpow = d.noise_kpow;
    ca.cplx_table = coef_cplx;
    for (int i = 0; i < 3; i++) {
        ca.keydim[i] = keydim[i];
        ca.dk[i] = dk[i];
    }
    for (int j = 0; j < 2; j++) {
        ca.c0[j] = d.c0[j];
        ca.c2[j] = d.c2[j];
        ca.c4[j] = d.c4[j];
    }
    ca.D = d.noise_D;
    ca.h = d.h;
    ca.lat = lat;
    ca.out64 = reinterpret_cast<double*>(ws + lay.coef64);
    ca.out32 = (d.precision == 32) ? (void*)(ws + lay.coef32) : nullptr;
    SETD_HIP(launch_coef(ca, s));

    Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws + lay.ctrl);
    SETD_HIP(launch_ctrl_init(ctrl, R, 0, s));
    {
        // variant choice runs real passes on zeroed buffers; everything below
        // resets them again
        SETD_HIP(launch_fill64(reinterpret_cast<double*>(ws + lay.phi), (int64_t)((lay.total - lay.phi) / 8), 0.0, s));
        setd_status tst = autotune();
        if (tst != SETD_OK) return tst;
        // SETD_GRAPH: steps per captured graph (default 0: kernel launches;
        // replaying graphs measured slower than launching on this runtime)
        const char* ge = std::getenv("SETD_GRAPH");
        graph_chunk = (ge && !no_alloc) ? std::max(0, std::min(1024, atoi(ge))) : 0;
        SETD_HIP(launch_ctrl_init(ctrl, R, 0, s));
    }
    SETD_HIP(launch_fill64(reinterpret_cast<double*>(ws + lay.skacc), 2 * nbins + 1, 0.0, s));
    // state buffers start at zero (all of them are multiples of 8 bytes)
    auto zero = [&](size_t off, size_t bytes) -> setd_status {
        if (!bytes) return SETD_OK;
        SETD_HIP(launch_fill64(reinterpret_cast<double*>(ws + off), (int64_t)(bytes / 8), 0.0, s));
        return SETD_OK;
    };
    setd_status st;
    if ((st = zero(lay.phi, (size_t)R * Sb)) != SETD_OK) return st;
    if (d.order == 2 && (st = zero(lay.prev, (size_t)R * Sb)) != SETD_OK) return st;
    if ((st = zero(lay.pre0, (size_t)R * Pb)) != SETD_OK) return st;
    if (d.nl == NL_KPZ && (st = zero(lay.pre1, (size_t)R * Pb)) != SETD_OK) return st;
    // the shifted intermediates of a phase-shift plan: a step reads them
    // before writing them, and a zero initial field writes nothing at bind
    if (ps_grid() && (st = zero(lay.preb, (size_t)R * Pb)) != SETD_OK) return st;
    if (ps_grid() && d.nl == NL_KPZ && (st = zero(lay.pre1b, (size_t)R * Pb)) != SETD_OK) return st;
    if (B && (st = zero(lay.big, (size_t)R * Bb)) != SETD_OK) return st;
    if ((st = zero(lay.snap, (size_t)R * Sb)) != SETD_OK) return st;

    const Item* items_dev = reinterpret_cast<const Item*>(ws + lay.items);
    if (d.ic_kind == 1) {
        st = (d.precision == 32) ? launch_ic_t<float>(*this, items_dev, R, s) : launch_ic_t<double>(*this, items_dev, R, s);
        if (st != SETD_OK) return st;
    }
    phi_valid = true;
    if ((st = carry_init(items_dev, R)) != SETD_OK) return st;
    SETD_HIP(hipStreamSynchronize(s));
    bound = true;
    step_host = 0;
    return SETD_OK;
}

// ---------------------------------------------------------------- autotuner
// Variants are timed per pass with HIP events on the plan's own buffers and
// the fastest kept.  Choices are cached per launch class and realization count
// for the process, and in the text file named by SETD_TUNE_CACHE if set.
// SETD_AUTOTUNE=0 keeps the default variants.
static std::mutex g_tune_mu;
static std::map<std::string, Tune> g_tune_cache;
static bool g_tune_loaded = false;

static std::string tune_key(const Plan& p)
{
    char buf[64];
    snprintf(buf, sizeof buf, "|%d|%d", p.R, p.d.nl);
    return class_key(p) + buf;
}

static void tune_cache_load()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("SETD_TUNE_CACHE");
    if (!path) return;
    // one "key row axis0 axis1 split" per line; lines starting with '#' are comments
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream ls(line);
        std::string key;
        Tune t;
        if (ls >> key >> t.row >> t.ax0 >> t.ax1 >> t.split) g_tune_cache[key] = t;
    }
}

static void tune_cache_store(const std::string& key, const Tune& t)
{
    g_tune_cache[key] = t;
    const char* path = std::getenv("SETD_TUNE_CACHE");
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    f << key << " " << t.row << " " << t.ax0 << " " << t.ax1 << " " << t.split << "\n";
}

setd_status Plan::autotune()
{
    // SETD_VARIANT="row,axis0,axis1" pins the variants (tests, reproducible timing)
    if (const char* pin = std::getenv("SETD_VARIANT")) {
        int r = 0, a0 = 0, a1 = 0;
        if (sscanf(pin, "%d,%d,%d", &r, &a0, &a1) == 3 && r >= 0 && r < 16 && a0 >= 0 && a0 < 16 && a1 >= 0 && a1 < 4) {
            tune.row = r;
            tune.ax0 = (lean && a0 < 4) ? 4 : a0;   // a lean plan steps with the register kernel
            tune.ax1 = a1;
            // SETD_SPLIT=2 pins split steps too
            const char* sp = std::getenv("SETD_SPLIT");
            tune.split = (sp && sp[0] == '2') ? 2 : 1;
            return SETD_OK;
        }
        return fail(SETD_E_INVAL, "SETD_VARIANT must be \"row,axis0,axis1\" with row in 0..15, axis0 in 0..15, axis1 in 0..3");
    }
    const char* env = std::getenv("SETD_AUTOTUNE");
    if ((env && env[0] == '0') || no_alloc) return SETD_OK;
    if (d.nl == NL_NONE || d.ndim == 1) return SETD_OK;   // a line has one kernel
    const std::string key = tune_key(*this);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_cache_load();
        auto itc = g_tune_cache.find(key);
        if (itc != g_tune_cache.end()) {
            tune = itc->second;
            return SETD_OK;
        }
    }
    const Item* items_dev = reinterpret_cast<const Item*>(ws + lay.items);
    hipEvent_t e0, e1;
    SETD_HIP(hipEventCreate(&e0));
    SETD_HIP(hipEventCreate(&e1));
    // pass index in launch order for each tunable knob
    const int row_pass = (d.ndim == 2) ? 0 : 1;
    const int ax0_pass = (d.ndim == 2) ? 1 : 3;
    struct Knob { int* var; int first; int nvar; int pass; int pass2; };
    // row variants 4..15 (several pair groups per workgroup) exist for real
    // fields; axis-0 variants 4 and up (register update) for plans under the
    // 2/3 rule, and are the only ones a plan keeping the SETD2 carry can step
    // with; the item groups of variants 6..11 and 13..15 need 2, 4 or 8 items
    const int ax0_top = g.dealias != 1 ? 4 : 16;
    auto ax0_ok = [&](int v) {
        if (v < 4 || v >= 16) return true;
        const int group = 1 << (v >= 12 ? v - 12 : (v - 4) / 2);
        return group <= R;
    };
    Knob knobs[3] = {{&tune.row, 0, d.complex_field ? 4 : 16, row_pass, -1},
                     {&tune.ax0, lean ? 4 : 0, ax0_top, ax0_pass, -1},
                     {&tune.ax1, 0, 4, 0, 2}};
    const int nknobs = (d.ndim == 3) ? 3 : 2;
    setd_status st = SETD_OK;
    for (int k = 0; k < nknobs && st == SETD_OK; k++) {
        Knob& kb = knobs[k];
        float best = 1e30f;
        int best_v = kb.first;
        // two rounds over the variants, each variant's best kept: a slow
        // outlier of one timing does not decide the choice
        for (int round = 0; round < 2 && st == SETD_OK; round++)
        for (int v = kb.first; v < kb.nvar && st == SETD_OK; v++) {
            if (kb.var == &tune.ax0 && !ax0_ok(v)) continue;
            *kb.var = v;
            auto run = [&]() -> setd_status {
                setd_status s1 = launch_pass(kb.pass, items_dev, R, 0, stream);
                if (s1 == SETD_OK && kb.pass2 >= 0) s1 = launch_pass(kb.pass2, items_dev, R, 0, stream);
                return s1;
            };
            if ((st = run()) != SETD_OK) break;   // warm-up
            if (hipEventRecord(e0, stream) != hipSuccess) { st = fail(SETD_E_DEVICE, "event record failed"); break; }
            for (int rep = 0; rep < 3 && st == SETD_OK; rep++) st = run();
            if (st != SETD_OK) break;
            if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                st = fail(SETD_E_DEVICE, "event wait failed");
                break;
            }
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (const char* vb = std::getenv("SETD_TUNE_VERBOSE"))
                if (vb[0] == '1') fprintf(stderr, "setd tune %s knob %d variant %d: %.1f us\n", key.c_str(), k, v, ms * 1e3f / 3);
            if (ms < best) {
                best = ms;
                best_v = v;
            }
        }
        *kb.var = best_v;
    }
    // whole steps with the realizations in one launch per pass, or split in
    // halves over two streams
    if (st == SETD_OK && aux && R >= 2) {
        // each choice timed three times over 24 steps (a split call pays its
        // fork and join once, and the two halves settle into their overlap
        // over the first steps), interleaved, best of the three
        constexpr int NS = 24;
        float ms_split[2] = {1e30f, 1e30f};
        for (int sp = 1; sp <= 2 && st == SETD_OK; sp++) st = run_steps(2, sp);   // warm-up
        for (int rep = 0; rep < 6 && st == SETD_OK; rep++) {
            const int sp = 1 + rep % 2;
            if (hipEventRecord(e0, stream) != hipSuccess) { st = fail(SETD_E_DEVICE, "event record failed"); break; }
            if ((st = run_steps(NS, sp)) != SETD_OK) break;
            if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                st = fail(SETD_E_DEVICE, "event wait failed");
                break;
            }
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            ms_split[sp - 1] = std::min(ms_split[sp - 1], ms);
            if (const char* vb = std::getenv("SETD_TUNE_VERBOSE"))
                if (vb[0] == '1') fprintf(stderr, "setd tune %s streams %d: %.1f us per step\n", key.c_str(), sp, ms * 1e3f / NS);
        }
        // keep the split only for a clear gain
        tune.split = (st == SETD_OK && ms_split[1] < 0.98f * ms_split[0]) ? 2 : 1;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SETD_OK) return st;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_store(key, tune);
    return SETD_OK;
}


// The realizations of a plan are independent: with split = 2 the first half
// steps on the plan's stream and the second on the auxiliary stream, forked
// from and joined back into the plan's stream with events, so that the passes
// of one half overlap those of the other.  Each realization runs the same
// kernels on the same data either way.
setd_status Plan::run_steps_on(int64_t n, int split, hipStream_t s)
{
    const Item* items_dev = reinterpret_cast<const Item*>(ws + lay.items);
    if (g.ndim == 1) {
        // a line steps in registers: up to 256 steps per launch
        for (int64_t left = n; left > 0;) {
            const int c = (int)std::min<int64_t>(left, 256);
            if (d.precision == 32) SETD_HIP((launch_line1d<float>(g, items_dev, R, MODE_STEP, 0, c, d.nl, s)));
            else SETD_HIP((launch_line1d<double>(g, items_dev, R, MODE_STEP, 0, c, d.nl, s)));
            left -= c;
        }
        return SETD_OK;
    }
    if (split != 2 || !aux || R < 2 || n <= 0) {
        for (int64_t i = 0; i < n; i++) {
            setd_status st = launch_step(items_dev, R, 0, s);
            if (st != SETD_OK) return st;
        }
        return SETD_OK;
    }
    const int h = R / 2;
    SETD_HIP(hipEventRecord(ev_fork, s));
    SETD_HIP(hipStreamWaitEvent(aux, ev_fork, 0));
    setd_status st = SETD_OK;
    for (int64_t i = 0; i < n && st == SETD_OK; i++) {
        st = launch_step(items_dev, h, 0, s);
        if (st == SETD_OK) st = launch_step(items_dev + h, R - h, 0, aux);
    }
    // join even after a failed launch, so that nothing is left running on aux
    SETD_HIP(hipEventRecord(ev_join, aux));
    SETD_HIP(hipStreamWaitEvent(s, ev_join, 0));
    return st;
}

// The launches of graph_chunk steps, captured once on the plan's capture
// stream (the auxiliary stream joins the capture through the fork event) and
// replayed on the bound stream.  Every kernel reads its realization's step
// from device memory and the launch arguments do not change after binding, so
// each replay advances the state exactly as eager launches would.  The steps
// hold only kernel nodes.
setd_status Plan::build_graph()
{
    if (!cap) SETD_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    SETD_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
    const setd_status st = run_steps_on(graph_chunk, graph_chunk >= 4 ? tune.split : 1, cap);
    hipGraph_t g0 = nullptr;
    const hipError_t e = hipStreamEndCapture(cap, &g0);
    if (st != SETD_OK) {
        if (g0) (void)hipGraphDestroy(g0);
        return st;
    }
    if (e != hipSuccess) return fail(SETD_E_DEVICE, "stream capture failed: %s", hipGetErrorString(e));
    graph = g0;
    SETD_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    return SETD_OK;
}

void Plan::release()
{
    for (auto& ev : events) {
        (void)hipEventDestroy(ev.a);
        (void)hipEventDestroy(ev.b);
    }
    events.clear();
    if (aux) {
        (void)hipStreamSynchronize(aux);
        (void)hipStreamDestroy(aux);
        aux = nullptr;
    }
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    ev_fork = ev_join = nullptr;
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    if (cap) (void)hipStreamDestroy(cap);
    cap = nullptr;
}

// Sample series_pos of the window: the stored spectrum of every realization
// (recovered first when the plan keeps the SETD2 carry).
setd_status Plan::series_sample()
{
    const setd_status st = ensure_phi();
    if (st != SETD_OK) return st;
    SETD_HIP(launch_copy(ws + lay.series + (size_t)series_pos * R * Sb, ws + lay.phi, (size_t)R * Sb, stream));
    series_pos++;
    return SETD_OK;
}

setd_status Plan::step(int64_t n)
{
    if (!bound) return fail(SETD_E_STATE, "plan not bound");
    if (n < 0) return fail(SETD_E_INVAL, "negative step count");
    if (step_host + n >= (int64_t)1 << 32) return fail(SETD_E_INVAL, "step index would exceed 2^32");
    const Item* items_dev = reinterpret_cast<const Item*>(ws + lay.items);
    if (n > 0) phi_valid = !lean;
    // an open time-series window takes a sample after every step
    while (n > 0 && series_pos >= 0 && series_pos < d.series_len) {
        setd_status st = run_steps(1, 1);
        if (st != SETD_OK) return st;
        phi_valid = !lean;
        step_host += 1;
        n -= 1;
        if ((st = series_sample()) != SETD_OK) return st;
    }
    if (n > 0) phi_valid = !lean;
    if (!profiling) {
        int64_t left = n;
        if (graph_chunk > 0 && left >= graph_chunk) {
            if (!gexec) {
                setd_status st = build_graph();
                if (st != SETD_OK) return st;
            }
            for (; left >= graph_chunk; left -= graph_chunk) SETD_HIP(hipGraphLaunch(gexec, stream));
        }
        // the two-stream split pays for its fork and join from about four
        // steps per call on (one step per call measured 20% slower split)
        setd_status st = run_steps(left, left >= 4 ? tune.split : 1);
        if (st != SETD_OK) return st;
        step_host += n;
        return SETD_OK;
    }
    for (int64_t i = 0; i < n; i++) {
        // the real-space noise transform of the step is not timed as a pass
        setd_status stn = launch_noise(items_dev, R, 0, stream);
        if (stn != SETD_OK) return stn;
        for (int k = 0; k < passes_per_step(); k++) {
            // timing-only events: no system-scope fence (an L2 writeback)
            // between the passes they bracket
            EvPair ev{k, nullptr, nullptr};
            SETD_HIP(hipEventCreateWithFlags(&ev.a, hipEventDisableSystemFence));
            SETD_HIP(hipEventCreateWithFlags(&ev.b, hipEventDisableSystemFence));
            events.push_back(ev);
            SETD_HIP(hipEventRecord(ev.a, stream));
            setd_status st = launch_pass(k, items_dev, R, 0, stream);
            if (st != SETD_OK) return st;
            SETD_HIP(hipEventRecord(ev.b, stream));
        }
    }
    step_host += n;
    return SETD_OK;
}

setd_status Plan::profile_read(double* out, size_t cap, size_t* len)
{
    if (!out || !len) return fail(SETD_E_INVAL, "null output");
    const int np = passes_per_step();
    if (cap < (size_t)2 * np) return fail(SETD_E_INVAL, "output needs %d doubles", 2 * np);
    if (bound) SETD_HIP(hipStreamSynchronize(stream));
    for (EvPair& ev : events) {
        float ms = 0.0f;
        SETD_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
        prof_ms[ev.pass] += ms;
        prof_cnt[ev.pass] += 1.0;
        (void)hipEventDestroy(ev.a);
        (void)hipEventDestroy(ev.b);
    }
    events.clear();
    for (int k = 0; k < np; k++) {
        out[2 * k] = prof_ms[k];
        out[2 * k + 1] = prof_cnt[k];
        prof_ms[k] = 0.0;
        prof_cnt[k] = 0.0;
    }
    *len = (size_t)2 * np;
    return SETD_OK;
}


setd_status Plan::nonfinite_any(int* flag)
{
    std::vector<Ctrl> c(R);
    SETD_HIP(hipMemcpyAsync(c.data(), ws + lay.ctrl, (size_t)R * sizeof(Ctrl), hipMemcpyDeviceToHost, stream));
    SETD_HIP(hipStreamSynchronize(stream));
    int f = 0;
    for (const Ctrl& x : c) f |= x.nonfinite;
    *flag = f;
    return SETD_OK;
}

setd_status Plan::observe(int kind, double* out, size_t cap, size_t* len)
{
    if (!bound) return fail(SETD_E_STATE, "plan not bound");
    if (!out || !len) return fail(SETD_E_INVAL, "null output");
    const int nb = nbins;
    double* acc = reinterpret_cast<double*>(ws + lay.acc);
    double* skacc = reinterpret_cast<double*>(ws + lay.skacc);
    double* dout = reinterpret_cast<double*>(ws + lay.out);
    const Item* items_dev = reinterpret_cast<const Item*>(ws + lay.items);
    size_t n_out = 0;
    if (kind != SETD_OBS_STEP && kind != SETD_OBS_SK_MEAN && kind != SETD_OBS_KICK) {
        const setd_status st0 = ensure_phi();
        if (st0 != SETD_OK) return st0;
    }
    auto reduce = [&](int red) -> setd_status {
        SETD_HIP(launch_fill64(acc, 3 * nb, 0.0, stream));
        if (d.precision == 32) SETD_HIP((launch_observe<float>(g, items_dev, R, red, nb, vol, acc, kick_step, stream)));
        else SETD_HIP((launch_observe<double>(g, items_dev, R, red, nb, vol, acc, kick_step, stream)));
        return SETD_OK;
    };
    setd_status st;
    switch (kind) {
    case SETD_OBS_SK:
    case SETD_OBS_SK_ACCUM:
        if (!iso) return fail(SETD_E_INVAL, "shell averages need equal n[i]");
        if (kind == SETD_OBS_SK && cap < (size_t)2 * nb) return fail(SETD_E_INVAL, "output needs %d doubles", 2 * nb);
        if (kind == SETD_OBS_SK_ACCUM && cap < 1) return fail(SETD_E_INVAL, "output needs 1 double");
        if ((st = reduce(RED_SK)) != SETD_OK) return st;
        SETD_HIP(launch_obs_final(kind == SETD_OBS_SK ? 0 : 5, nb, acc, dout, skacc, 0.0, stream));
        n_out = (kind == SETD_OBS_SK) ? (size_t)2 * nb : 1;
        break;
    case SETD_OBS_SK_MEAN:
        if (!iso) return fail(SETD_E_INVAL, "shell averages need equal n[i]");
        if (cap < (size_t)2 * nb) return fail(SETD_E_INVAL, "output needs %d doubles", 2 * nb);
        SETD_HIP(launch_obs_mean(nb, skacc, dout, stream));
        n_out = (size_t)2 * nb;
        break;
    case SETD_OBS_WIDTH:
        if (cap < 1) return fail(SETD_E_INVAL, "output needs 1 double");
        if ((st = reduce(RED_WIDTH)) != SETD_OK) return st;
        SETD_HIP(launch_obs_final(1, nb, acc, dout, skacc, 1.0 / ((double)nreal * (double)nreal * R), stream));
        n_out = 1;
        break;
    case SETD_OBS_TWOTIME:
        if (!iso) return fail(SETD_E_INVAL, "shell averages need equal n[i]");
        if (!have_snap) return fail(SETD_E_INVAL, "no snapshot taken");
        if (cap < (size_t)3 * nb) return fail(SETD_E_INVAL, "output needs %d doubles", 3 * nb);
        if ((st = reduce(RED_TWOTIME)) != SETD_OK) return st;
        SETD_HIP(launch_obs_final(3, nb, acc, dout, skacc, 0.0, stream));
        n_out = (size_t)3 * nb;
        break;
    case SETD_OBS_RESPONSE:
        if (!iso) return fail(SETD_E_INVAL, "shell averages need equal n[i]");
        if (!have_kick) return fail(SETD_E_INVAL, "no kick marked");
        if (cap < (size_t)3 * nb) return fail(SETD_E_INVAL, "output needs %d doubles", 3 * nb);
        if ((st = reduce(RED_RESPONSE)) != SETD_OK) return st;
        SETD_HIP(launch_obs_final(3, nb, acc, dout, skacc, 0.0, stream));
        n_out = (size_t)3 * nb;
        break;
    case SETD_OBS_SERIES_START: {
        if (d.series_len <= 0) return fail(SETD_E_INVAL, "the plan has no time series (series_len 0)");
        Ctrl c0;
        SETD_HIP(hipMemcpyAsync(&c0, ws + lay.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, stream));
        SETD_HIP(hipStreamSynchronize(stream));
        series_step0 = c0.step;
        series_pos = 0;
        if ((st = series_sample()) != SETD_OK) return st;
        if (cap >= 1) {
            out[0] = (double)c0.step;
            *len = 1;
        } else {
            *len = 0;
        }
        return SETD_OK;
    }
    case SETD_OBS_SPECTRUM: {
        const int M = d.series_len;
        if (g.rsn) return fail(SETD_E_UNSUPPORTED, "the kick estimators regenerate Fourier-space noise");
        if (!iso) return fail(SETD_E_INVAL, "shell averages need equal n[i]");
        if (M <= 0 || series_pos < M) return fail(SETD_E_INVAL, "no complete time series window");
        const size_t nsum = (size_t)3 * nb * M + nb;
        if (cap < nsum) return fail(SETD_E_INVAL, "output needs %zu doubles", nsum);
        double* sacc = reinterpret_cast<double*>(ws + lay.specacc);
        SETD_HIP(launch_fill64(sacc, (int64_t)nsum, 0.0, stream));
        SpecArgs sa{};
        sa.g = g;
        sa.items = items_dev;
        sa.nitems = R;
        sa.nbins = nb;
        sa.total = (int)(S);
        sa.series = ws + lay.series;
        sa.slot = (size_t)R * Sb;
        sa.rstride = Sb;
        sa.tw = ws + ((d.precision == 32) ? lay.twm32 : lay.twm64);
        sa.step0 = series_step0;
        sa.vol = vol;
        sa.h = d.h;
        sa.D = d.noise_D;
        sa.kpow = d.noise_kpow;
        sa.acc = sacc;
        if (d.precision == 32) SETD_HIP((launch_spectrum<float>(sa, M, stream)));
        else SETD_HIP((launch_spectrum<double>(sa, M, stream)));
        SETD_HIP(hipMemcpyAsync(out, sacc, nsum * sizeof(double), hipMemcpyDeviceToHost, stream));
        SETD_HIP(hipStreamSynchronize(stream));
        // sums to means over each shell's modes
        for (int j = 0; j < nb; j++) {
            const double c = out[(size_t)3 * nb * M + j];
            if (!(c > 0)) continue;
            for (int part = 0; part < 3; part++)
                for (int b = 0; b < M; b++) out[((size_t)part * nb + j) * M + b] /= c;
        }
        *len = nsum;
        int f = 0;
        if ((st = nonfinite_any(&f)) != SETD_OK) return st;
        return f ? fail(SETD_E_NONFINITE, "a realization produced a non-finite value") : SETD_OK;
    }
    case SETD_OBS_BOXWIDTH: {
        if (!iso) return fail(SETD_E_INVAL, "box widths need equal n[i]");
        const int N = d.n[0];
        int J = 0;
        while ((1 << J) < N) J++;
        if (cap < (size_t)J) return fail(SETD_E_INVAL, "output needs %d doubles", J);
        BoxArgs ba{};
        ba.g = g;
        ba.items = items_dev;
        ba.total = (int)S;
        ba.N = N;
        ba.J = J;
        ba.cls = reinterpret_cast<double*>(ws + lay.boxcls);
        ba.sums = acc;
        // whole coarse levels, from l = N down, while they fit the LDS table
        size_t tail = 0;
        for (int j = J; j >= 1; j--) {
            size_t c = 1;
            for (int i = 0; i < d.ndim; i++) c *= (size_t)(N >> j);
            if (tail + c > 1024) break;
            tail += c;
        }
        ba.lds_base = lay.boxn - tail;
        ba.nlds = (int)tail;
        SETD_HIP(launch_fill64(acc, J + 1, 0.0, stream));
        for (int r = 0; r < R; r++) {
            ba.r = r;
            SETD_HIP(launch_fill64(ba.cls, (int64_t)(2 * lay.boxn), 0.0, stream));
            if (d.precision == 32) SETD_HIP((launch_boxwidth<float>(ba, lay.boxn, stream)));
            else SETD_HIP((launch_boxwidth<double>(ba, lay.boxn, stream)));
        }
        double sums[16];
        SETD_HIP(hipMemcpyAsync(sums, acc, (size_t)(J + 1) * sizeof(double), hipMemcpyDeviceToHost, stream));
        SETD_HIP(hipStreamSynchronize(stream));
        // w_l^2 = (sum |h_a|^2 - sum_c |A_c|^2) / N^2d, averaged over realizations
        const double norm = 1.0 / ((double)nreal * (double)nreal * R);
        for (int j = 1; j <= J; j++) {
            const double v = (sums[0] - sums[j]) * norm;
            out[j - 1] = std::sqrt(v > 0.0 ? v : 0.0);
        }
        *len = (size_t)J;
        int f = 0;
        if ((st = nonfinite_any(&f)) != SETD_OK) return st;
        return f ? fail(SETD_E_NONFINITE, "a realization produced a non-finite value") : SETD_OK;
    }
    case SETD_OBS_FDT: {
        const int M = d.series_len;
        if (g.rsn) return fail(SETD_E_UNSUPPORTED, "the kick estimators regenerate Fourier-space noise");
        if (M <= 0 || series_pos < M) return fail(SETD_E_INVAL, "no complete time series window");
        if (cap < 2) return fail(SETD_E_INVAL, "output needs 2 doubles");
        const size_t nsum = (size_t)3 * nb * M + nb;
        double* sacc = reinterpret_cast<double*>(ws + lay.specacc);
        double* dacc = reinterpret_cast<double*>(ws + lay.fdtacc);
        SETD_HIP(launch_fill64(sacc, (int64_t)nsum, 0.0, stream));
        SETD_HIP(launch_fill64(dacc, (int64_t)(S * (size_t)M), 0.0, stream));
        SETD_HIP(launch_fill64(acc, 2, 0.0, stream));
        SpecArgs sa{};
        sa.g = g;
        sa.items = items_dev;
        sa.nitems = R;
        sa.nbins = nb;
        sa.total = (int)(S);
        sa.series = ws + lay.series;
        sa.slot = (size_t)R * Sb;
        sa.rstride = Sb;
        sa.tw = ws + ((d.precision == 32) ? lay.twm32 : lay.twm64);
        sa.step0 = series_step0;
        sa.vol = vol;
        sa.h = d.h;
        sa.D = d.noise_D;
        sa.kpow = d.noise_kpow;
        sa.acc = sacc;
        sa.dacc = dacc;
        if (d.precision == 32) {
            SETD_HIP((launch_spectrum<float>(sa, M, stream)));
            SETD_HIP((launch_fdt_reduce<float>(g, dacc, (int)S, M, acc, stream)));
        } else {
            SETD_HIP((launch_spectrum<double>(sa, M, stream)));
            SETD_HIP((launch_fdt_reduce<double>(g, dacc, (int)S, M, acc, stream)));
        }
        double sums[2];
        SETD_HIP(hipMemcpyAsync(sums, acc, sizeof sums, hipMemcpyDeviceToHost, stream));
        SETD_HIP(hipStreamSynchronize(stream));
        // averages over all prod n_i modes and M frequencies
        const double denom = (double)nreal * (double)M;
        out[0] = sums[0] / denom;
        out[1] = sums[1] / denom;
        *len = 2;
        int f = 0;
        if ((st = nonfinite_any(&f)) != SETD_OK) return st;
        return f ? fail(SETD_E_NONFINITE, "a realization produced a non-finite value") : SETD_OK;
    }
    case SETD_OBS_KICK: {
        if (g.rsn) return fail(SETD_E_UNSUPPORTED, "the kick estimators regenerate Fourier-space noise");
        Ctrl c0;
        SETD_HIP(hipMemcpyAsync(&c0, ws + lay.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, stream));
        SETD_HIP(hipStreamSynchronize(stream));
        kick_step = c0.step;
        have_kick = true;
        if (cap >= 1) {
            out[0] = (double)c0.step;
            *len = 1;
        } else {
            *len = 0;
        }
        return SETD_OK;
    }
    case SETD_OBS_SNAPSHOT: {
        SETD_HIP(launch_copy(ws + lay.snap, ws + lay.phi, (size_t)R * Sb, stream));
        have_snap = true;
        Ctrl c0;
        SETD_HIP(hipMemcpyAsync(&c0, ws + lay.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, stream));
        SETD_HIP(hipStreamSynchronize(stream));
        if (cap >= 1) {
            out[0] = (double)c0.step;
            *len = 1;
        } else {
            *len = 0;
        }
        int f = 0;
        if ((st = nonfinite_any(&f)) != SETD_OK) return st;
        return f ? fail(SETD_E_NONFINITE, "a realization produced a non-finite value") : SETD_OK;
    }
    case SETD_OBS_STEP: {
        if (cap < 2) return fail(SETD_E_INVAL, "output needs 2 doubles");
        Ctrl c0;
        SETD_HIP(hipMemcpyAsync(&c0, ws + lay.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, stream));
        int f = 0;
        if ((st = nonfinite_any(&f)) != SETD_OK) return st;
        out[0] = (double)c0.step;
        out[1] = (double)f;
        *len = 2;
        return f ? fail(SETD_E_NONFINITE, "a realization produced a non-finite value") : SETD_OK;
    }
    default:
        return fail(SETD_E_INVAL, "unknown observable kind %d", kind);
    }
    SETD_HIP(hipMemcpyAsync(out, dout, n_out * sizeof(double), hipMemcpyDeviceToHost, stream));
    SETD_HIP(hipStreamSynchronize(stream));
    *len = n_out;
    int f = 0;
    if ((st = nonfinite_any(&f)) != SETD_OK) return st;
    return f ? fail(SETD_E_NONFINITE, "a realization produced a non-finite value") : SETD_OK;
}

// Scatter a stored block (phi or F_{n-1}) of realization r into the unpruned
// FFT-order layout of the ABI, as interleaved doubles.
setd_status Plan::get_block(size_t off, int r, double* out, size_t cap)
{
    if (!bound) return fail(SETD_E_STATE, "plan not bound");
    if (r < 0 || r >= R) return fail(SETD_E_INVAL, "realization %d out of range", r);
    if (!out || cap < 2 * nspec) return fail(SETD_E_INVAL, "output needs %zu doubles", 2 * nspec);
    std::vector<char> host(S * elt);
    SETD_HIP(hipMemcpyAsync(host.data(), ws + off + (size_t)r * Sb, S * elt, hipMemcpyDeviceToHost, stream));
    SETD_HIP(hipStreamSynchronize(stream));
    scatter(host.data(), out);
    return SETD_OK;
}

// Stored block of one realization (state precision, padded last axis) ->
// unpruned FFT-order spectrum as interleaved doubles.
void Plan::scatter(const char* raw, double* out) const
{
    std::memset(out, 0, 2 * nspec * sizeof(double));
    const int last = d.ndim - 1;
    const int k1 = (d.ndim == 3) ? g.kept[1] : 1;
    for (int i0 = 0; i0 < (d.ndim == 1 ? 1 : g.kept[0]); i0++) {
        const int j0 = (i0 <= g.kp[0]) ? i0 : i0 + g.n[0] - g.kept[0];
        for (int i1 = 0; i1 < k1; i1++) {
            const int j1 = (d.ndim == 3) ? ((i1 <= g.kp[1]) ? i1 : i1 + g.n[1] - g.kept[1]) : 0;
            for (int c = 0; c < g.kept[last]; c++) {
                const int jl = g.cplx ? ((c <= g.kp[last]) ? c : c + g.n[last] - g.kept[last]) : c;
                const size_t src = ((size_t)i0 * k1 + i1) * g.pitch + c;
                const size_t dst = (d.ndim == 3) ? ((size_t)j0 * g.n[1] + j1) * g.nh_last + jl
                                                 : (size_t)j0 * g.nh_last + jl;
                double re, im;
                if (d.precision == 32) {
                    const float* f = reinterpret_cast<const float*>(raw) + 2 * src;
                    re = f[0];
                    im = f[1];
                } else {
                    const double* f = reinterpret_cast<const double*>(raw) + 2 * src;
                    re = f[0];
                    im = f[1];
                }
                out[2 * dst] = re;
                out[2 * dst + 1] = im;
            }
        }
    }
}

setd_status Plan::set_field(int r, const double* in, size_t len)
{
    if (!bound) return fail(SETD_E_STATE, "plan not bound");
    if (r < 0 || r >= R) return fail(SETD_E_INVAL, "realization %d out of range", r);
    if (!in || len < 2 * nspec) return fail(SETD_E_INVAL, "input needs %zu doubles", 2 * nspec);
    std::vector<char> host(S * elt, 0);
    const int last = d.ndim - 1;
    const int k1 = (d.ndim == 3) ? g.kept[1] : 1;
    for (int i0 = 0; i0 < (d.ndim == 1 ? 1 : g.kept[0]); i0++) {
        const int j0 = (i0 <= g.kp[0]) ? i0 : i0 + g.n[0] - g.kept[0];
        for (int i1 = 0; i1 < k1; i1++) {
            const int j1 = (d.ndim == 3) ? ((i1 <= g.kp[1]) ? i1 : i1 + g.n[1] - g.kept[1]) : 0;
            for (int c = 0; c < g.kept[last]; c++) {
                const int jl = g.cplx ? ((c <= g.kp[last]) ? c : c + g.n[last] - g.kept[last]) : c;
                const size_t dst = ((size_t)i0 * k1 + i1) * g.pitch + c;
                const size_t src = (d.ndim == 3) ? ((size_t)j0 * g.n[1] + j1) * g.nh_last + jl
                                                 : (size_t)j0 * g.nh_last + jl;
                if (d.precision == 32) {
                    float* f = reinterpret_cast<float*>(host.data()) + 2 * dst;
                    f[0] = (float)in[2 * src];
                    f[1] = (float)in[2 * src + 1];
                } else {
                    double* f = reinterpret_cast<double*>(host.data()) + 2 * dst;
                    f[0] = in[2 * src];
                    f[1] = in[2 * src + 1];
                }
            }
        }
    }
    SETD_HIP(hipMemcpyAsync(ws + lay.phi + (size_t)r * Sb, host.data(), S * elt, hipMemcpyHostToDevice, stream));
    const Item* items_dev = reinterpret_cast<const Item*>(ws + lay.items) + r;
    // a real field's spectrum is Hermitian on the a_last = 0 (and N/2) planes
    if (d.precision == 32) SETD_HIP((launch_hermitian<float>(g, items_dev, 1, 0, stream)));
    else SETD_HIP((launch_hermitian<double>(g, items_dev, 1, 0, stream)));
    setd_status st = (d.precision == 32) ? launch_sync_t<float>(*this, items_dev, 1, stream)
                                         : launch_sync_t<double>(*this, items_dev, 1, stream);
    if (st != SETD_OK) return st;
    SETD_HIP(launch_ctrl_set(reinterpret_cast<Ctrl*>(ws + lay.ctrl) + r, 1, 0, 1, stream));
    // a fresh state has no F_{n-1}: the carry restarts as E phi + G eta_n
    if ((st = carry_init(items_dev, 1)) != SETD_OK) return st;
    SETD_HIP(hipStreamSynchronize(stream));
    return SETD_OK;
}

setd_status Plan::set_step(int64_t s)
{
    if (!bound) return fail(SETD_E_STATE, "plan not bound");
    if (s < 0 || s >= ((int64_t)1 << 32)) return fail(SETD_E_INVAL, "step index out of range");
    if (lean) {
        // the carry holds G eta of the old step index: re-draw it for step s
        const Item* items_dev = reinterpret_cast<const Item*>(ws + lay.items);
        if (d.precision == 32) SETD_HIP((launch_linear<float>(g, items_dev, R, 0, LIN_RENOISE, s, stream)));
        else SETD_HIP((launch_linear<double>(g, items_dev, R, 0, LIN_RENOISE, s, stream)));
    }
    SETD_HIP(launch_ctrl_set(reinterpret_cast<Ctrl*>(ws + lay.ctrl), R, s, 0, stream));
    SETD_HIP(hipStreamSynchronize(stream));
    step_host = s;
    return SETD_OK;
}

std::string class_key(const Plan& p)
{
    char buf[160];
    const int kind = p.d.nl == NL_NONE ? 1 : (p.d.nl == NL_KPZ ? 2 : 0);
    snprintf(buf, sizeof buf, "%d|%d|%d|%d|%d|%d|%d|%d|%d|%d", p.g.ndim, p.g.cplx, p.g.prec, p.g.dealias, p.g.n[0],
             p.g.n[1], p.g.n[2], kind, p.lean ? 1 : 0, p.g.rsn);
    return buf;
}

}  // namespace setd

// ====================================================================== C ABI
using setd::Plan;

struct setd_plan {
    Plan p;
};

extern "C" {

setd_status setd_plan_create(const setd_desc* desc, setd_plan** out)
{
    if (!desc || !out) return setd::fail(SETD_E_INVAL, "null argument");
    *out = nullptr;
    setd_plan* h = new (std::nothrow) setd_plan();
    if (!h) return setd::fail(SETD_E_NOMEM, "host allocation failed");
    setd_status st = h->p.init(*desc);
    if (st != SETD_OK) {
        delete h;
        return st;
    }
    *out = h;
    return SETD_OK;
}

setd_status setd_plan_workspace(const setd_plan* plan, size_t* bytes)
{
    if (!plan || !bytes) return setd::fail(SETD_E_INVAL, "null argument");
    *bytes = plan->p.lay.total;
    return SETD_OK;
}

setd_status setd_plan_info(const setd_plan* plan, setd_plan_info_t* info)
{
    if (!plan || !info) return setd::fail(SETD_E_INVAL, "null argument");
    const Plan& p = plan->p;
    info->workspace_bytes = p.lay.total;
    info->spectral_len = p.nspec;
    info->kept_modes = p.kept_modes;
    info->nbins = p.nbins;
    info->passes_per_step = p.passes_per_step();
    info->alg_bytes_per_step = p.alg_bytes_per_step();
    info->site_updates_per_step = (double)p.nreal * p.R;
    p.pass_bytes(info->pass_bytes);
    info->variants[0] = p.tune.row;
    info->variants[1] = p.tune.ax0;
    info->variants[2] = p.tune.ax1;
    info->streams = (p.tune.split == 2 && p.aux) ? 2 : 1;
    info->graph_steps = p.graph_chunk;
    setd::axis_shape(p.d.precision, p.g.n[0], p.tune.ax0, &info->axis_tile[0], &info->axis_tile[1]);
    return SETD_OK;
}

setd_status setd_profile(setd_plan* plan, int enable)
{
    if (!plan) return setd::fail(SETD_E_INVAL, "null plan");
    plan->p.profiling = enable != 0;
    return SETD_OK;
}

setd_status setd_profile_read(setd_plan* plan, double* out, size_t cap, size_t* len)
{
    if (!plan) return setd::fail(SETD_E_INVAL, "null plan");
    return plan->p.profile_read(out, cap, len);
}


setd_status setd_plan_bind(setd_plan* plan, void* dev_ws, size_t bytes, void* hip_stream)
{
    if (!plan) return setd::fail(SETD_E_INVAL, "null plan");
    return plan->p.bind(dev_ws, bytes, (hipStream_t)hip_stream);
}

setd_status setd_step(setd_plan* plan, int64_t nsteps)
{
    if (!plan) return setd::fail(SETD_E_INVAL, "null plan");
    return plan->p.step(nsteps);
}

setd_status setd_observe(setd_plan* plan, int kind, double* host_out, size_t cap, size_t* len)
{
    if (!plan) return setd::fail(SETD_E_INVAL, "null plan");
    return plan->p.observe(kind, host_out, cap, len);
}

setd_status setd_get_field(setd_plan* plan, int realization, double* host_out, size_t cap)
{
    if (!plan) return setd::fail(SETD_E_INVAL, "null plan");
    if (plan->p.bound) {
        const setd_status st = plan->p.ensure_phi();
        if (st != SETD_OK) return st;
    }
    return plan->p.get_block(plan->p.lay.phi, realization, host_out, cap);
}

setd_status setd_get_history(setd_plan* plan, int realization, double* host_out, size_t cap)
{
    if (!plan) return setd::fail(SETD_E_INVAL, "null plan");
    if (plan->p.d.order != 2) return setd::fail(SETD_E_INVAL, "SETD1 keeps no history");
    if (plan->p.lean)
        return setd::fail(SETD_E_UNSUPPORTED, "the plan keeps the SETD2 carry, not F_{n-1} (history_readback 0)");
    return plan->p.get_block(plan->p.lay.prev, realization, host_out, cap);
}

setd_status setd_set_field(setd_plan* plan, int realization, const double* host_in, size_t len)
{
    if (!plan) return setd::fail(SETD_E_INVAL, "null plan");
    return plan->p.set_field(realization, host_in, len);
}

setd_status setd_set_step(setd_plan* plan, int64_t step)
{
    if (!plan) return setd::fail(SETD_E_INVAL, "null plan");
    return plan->p.set_step(step);
}

setd_status setd_plan_destroy(setd_plan* plan)
{
    if (plan) plan->p.release();
    delete plan;
    return SETD_OK;
}

const char* setd_last_error(void) { return setd::g_err.c_str(); }

}  // extern "C"
