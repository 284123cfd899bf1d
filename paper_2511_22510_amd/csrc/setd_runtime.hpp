// setd_runtime.hpp -- host-side plan object shared by the C ABI and the server.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <string>
#include <vector>

#include "setd.h"
#include "setd_types.hpp"

namespace setd {

setd_status fail(setd_status s, const char* fmt, ...);
setd_status ok();

#define SETD_HIP(call)                                                                                       \
    do {                                                                                                     \
        hipError_t e_ = (call);                                                                              \
        if (e_ != hipSuccess) return ::setd::fail(SETD_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Byte offsets of every buffer of a plan's workspace.
struct Layout {
    size_t items = 0, ctrl = 0, coef64 = 0, coef32 = 0;
    size_t tw64[3] = {0, 0, 0}, tw32[3] = {0, 0, 0};
    size_t acc = 0, skacc = 0, out = 0;
    size_t phi = 0, prev = 0, pre0 = 0, pre1 = 0, big = 0, snap = 0;
    size_t twm64 = 0, twm32 = 0, specacc = 0, series = 0, fdtacc = 0;   // time series (series_len > 0)
    size_t boxcls = 0, boxn = 0;  // box-width class sums and their count (equal n[i])
    size_t npre = 0, noise = 0;   // real-space noise on 2D/3D lattices: intermediate, eta_a
    size_t preb = 0;              // phase-shift dealiasing: the shifted intermediate
    size_t pre1b = 0;             // KPZ with phase shifts: the shifted gradient intermediate
    size_t total = 0;
};

// Kernel variants of a plan's passes (see setd_launch_impl.hpp).
struct Tune {
    int row = 0;   // 0..15 (0..3 for complex fields)
    int ax0 = 0;   // 0..5
    int ax1 = 0;   // 0..3
    int split = 1; // 1, or 2: the halves of the realizations on two streams
};

struct Plan {
    setd_desc d{};
    Tune tune{};
    Geo g{};
    int R = 0;
    int nkeys = 0, iso = 0, coef_mode = 0, coef_cplx = 0, nbins = 0;
    int keydim[3] = {1, 1, 1};
    double dk[3] = {0, 0, 0};
    double lat = 1.0, vol = 1.0;
    size_t S = 0, P = 0, B = 0;   // complex elements per realization: state, pre, big
    size_t Sb = 0, Pb = 0, Bb = 0;// bytes from one realization's array to the next
    size_t elt = 0;               // bytes per complex element
    size_t nspec = 0;             // unpruned spectral length per realization
    size_t nreal = 0;             // lattice sites per realization
    size_t kept_modes = 0;
    Layout lay;
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    // second stream and fork/join events for split steps (Tune::split)
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool split_ok = true;         // whether bind may create the auxiliary stream
    // bind creates no stream, event or graph and times no variant (the
    // default variants, or those pinned by SETD_VARIANT, are used)
    bool no_alloc = false;
    // setd_step replays a captured graph of graph_chunk steps (0: eager
    // launches only), captured on a stream of the plan at the first use
    int graph_chunk = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool bound = false;
    bool have_snap = false;
    bool have_kick = false;       // SETD_OBS_KICK taken: the response's reference step
    int64_t kick_step = 0;
    // time series window: samples taken so far (series_len when complete, -1
    // before SETD_OBS_SERIES_START) and the step of sample 0
    int series_pos = -1;
    int64_t series_step0 = 0;
    setd_status series_sample();
    // SETD2 storage: the carry Y_n = E phi_n + w_b F_{n-1} + G eta_n in the
    // F_{n-1} array, phi recovered from pre when read (phi_valid tracks it)
    bool lean = false;
    bool phi_valid = true;
    int64_t step_host = 0;        // steps queued so far (mirror of the device counter)
    std::vector<Item> items;      // host copy of the device item table
    // kernel timing (setd_profile)
    bool profiling = false;
    struct EvPair { int pass; hipEvent_t a, b; };
    std::vector<EvPair> events;
    double prof_ms[4] = {0, 0, 0, 0};
    double prof_cnt[4] = {0, 0, 0, 0};

    ~Plan() { release(); }
    setd_status init(const setd_desc& desc);
    setd_status bind(void* dev, size_t bytes, hipStream_t s);
    // queue the passes of one step for nitems items starting at items_dev
    // (after the transform of the step's real-space noise, if the plan draws it)
    setd_status launch_step(const Item* items_dev, int nitems, int sub, hipStream_t s) const;
    // 2D/3D plans with real-space noise: its transform for the current step
    setd_status launch_noise(const Item* items_dev, int nitems, int sub, hipStream_t s) const;
    bool rsn_grid() const { return d.noise_space == 1 && d.ndim >= 2; }
    // 2D/3D plans with phase-shift dealiasing keep a shifted copy of pre
    // (3D: and four grids in the line buffer)
    bool ps_grid() const { return d.dealias == 2 && d.ndim >= 2; }
    // queue pass i (launch order) of one step
    setd_status launch_pass(int i, const Item* items_dev, int nitems, int sub, hipStream_t s) const;
    setd_status profile_read(double* out, size_t cap, size_t* len);
    void pass_bytes(double* out4) const;
    setd_status step(int64_t n);
    // n steps of every realization without per-pass events, split over two
    // streams when `split` is 2
    setd_status run_steps(int64_t n, int split) { return run_steps_on(n, split, stream); }
    setd_status run_steps_on(int64_t n, int split, hipStream_t s);
    setd_status build_graph();
    void release();
    // time every variant of every pass on the bound buffers and keep the fastest
    setd_status autotune();
    setd_status observe(int kind, double* out, size_t cap, size_t* len);
    setd_status get_block(size_t off, int r, double* out, size_t cap);
    void scatter(const char* raw, double* out) const;
    setd_status set_field(int r, const double* in, size_t len);
    setd_status set_step(int64_t step);
    setd_status nonfinite_any(int* flag);
    // lean plans: recover phi from pre for every realization if a step has
    // run since the last recovery (other plans: nothing to do)
    setd_status ensure_phi();
    // lean plans: carry Y = E phi + G eta_n of nitems items from items_dev,
    // n each realization's step index
    setd_status carry_init(const Item* items_dev, int nitems);
    double alg_bytes_per_step() const;
    int passes_per_step() const;
};

// descriptor validation shared by plans and the server
setd_status validate(const setd_desc& d);
// launch class key: jobs with equal keys can share launches
std::string class_key(const Plan& p);

}  // namespace setd
