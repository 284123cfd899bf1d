/*
 * setd.h -- C ABI of the MI355X (gfx950) SETD pseudo-spectral integrator.
 *
 * The library advances stochastic field theories written in Fourier space as
 *     d phi_a/dt = c(k_a) phi_a + F_a[phi] + sqrt(2 D(k_a)) eta_a(t)
 * (Johnsrud & Rana, arXiv 2511.22510, Sec. 4 Eq. general_fourier) with the
 * stochastic exponential-time-differencing schemes SETD1 (Sec. 2 Eq. SETD1) and
 * SETD2 (Sec. 2 Eq. SETD2), evaluating F_a pseudo-spectrally (Sec. 4, the
 * algorithm box), drawing the noise directly in Fourier space (App. B) with the
 * lattice normalisation of App. A, or per site in real space and transformed
 * (Sec. 4 step 2), and dealiasing by the 2/3 truncation rule or by phase
 * shifts (Sec. 4 step 1), on 1D, 2D and 3D periodic lattices.
 *
 * Conventions shared by every entry point:
 *  - Every call returns a setd_status.  No call aborts; setd_last_error()
 *    gives a text for the last failing call of the calling thread.
 *  - Device memory and HIP streams belong to the caller.  The library only
 *    borrows the workspace and stream handed to setd_plan_bind /
 *    setd_server_create and never frees them.  Work it queues on streams of
 *    its own (a plan's second stream, a server's class streams) is forked
 *    from and joined back into the caller's stream with events, so ordering
 *    against the caller's stream is as if all of it ran there.
 *  - Fields cross the boundary as host arrays of interleaved (re, im) doubles
 *    in FFT order: a real field as its real-to-complex half spectrum
 *    n[0] x .. x (n[d-1]/2 + 1), a complex field as the full n[0] x .. x n[d-1]
 *    spectrum.  Modes removed by dealiasing are zero on output and ignored on
 *    input.
 *  - DFT convention: forward X_a = sum_n x_n e^{-2 pi i a.n/N} (unscaled),
 *    inverse x_n = N^-d sum_a X_a e^{+2 pi i a.n/N}.
 *  - Work is queued on the bound stream; setd_step returns before the GPU has
 *    finished.  setd_observe, setd_get_field and setd_set_field synchronise
 *    the stream.
 */
#ifndef SETD_H
#define SETD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SETD_OK = 0,
    SETD_E_INVAL = -1,        /* bad argument or descriptor                      */
    SETD_E_NOMEM = -2,        /* workspace / arena too small                     */
    SETD_E_DEVICE = -3,       /* a HIP call failed                               */
    SETD_E_NONFINITE = -4,    /* a realization produced NaN/Inf (Sec. 2 warns of
                                 blow-up of explicit schemes); data still returned */
    SETD_E_BUSY = -5,         /* job not finished yet                            */
    SETD_E_UNSUPPORTED = -6,  /* valid physics the library does not run           */
    SETD_E_STATE = -7         /* call out of order (e.g. step before bind)       */
} setd_status;

/* Nonlinear term F_a (Sec. 5).  The prefactor acts in Fourier space. */
typedef enum {
    SETD_NL_PHI3 = 0,         /* Model A, Eq. modelA:   F = -u FFT[phi^3]             */
    SETD_NL_PHI3_CONS = 1,    /* Model B, Eq. modelB:   F = -u k^2 FFT[phi^3]         */
    SETD_NL_KPZ = 2,          /* KPZ, Eq. kpz_fourier:  F = lambda/2 FFT[|grad h|^2],
                                 gradient taken spectrally (1D and 2D real fields)   */
    SETD_NL_CGL = 3,          /* CGL, Eq. cgle:         F = -(1 + i beta) FFT[|A|^2 A] */
    SETD_NL_NONE = 4          /* linear theory, F = 0                                */
} setd_nonlin;

/* Observables (Sec. 5 and App. C), accumulated in FP64 on the device. */
typedef enum {
    SETD_OBS_SK = 0,          /* equal-time S(k, t) = (L/N^2)^d <|phi_a|^2> over
                                 realizations, averaged over shells ceil|a| = j
                                 (App. C shells k - dk < |q| <= k; needs equal
                                 n[i]).  out: [mean_j (nbins), count_j (nbins)]     */
    SETD_OBS_WIDTH = 1,       /* interface width w(t) with l = L (Sec. 5 KPZ),
                                 sqrt of the ensemble mean real-space variance.
                                 out: [w]                                           */
    SETD_OBS_SNAPSHOT = 2,    /* store the current state as the reference time t'
                                 of the two-time correlation.  out: [step]          */
    SETD_OBS_TWOTIME = 3,     /* C(k, t, t') = (L/N^2)^d <phi_a(t) conj phi_a(t')>,
                                 shell averaged.  out: [Re (nbins), Im (nbins),
                                 count (nbins)]                                     */
    SETD_OBS_STEP = 4,        /* out: [step index n, non-finite flag]               */
    SETD_OBS_SK_ACCUM = 5,    /* add the current shell S(k) to a running FP64 sum.
                                 out: [number of samples accumulated]               */
    SETD_OBS_SK_MEAN = 6,     /* time mean of the accumulated S(k).
                                 out: [mean_j (nbins), count_j (nbins)]             */
    SETD_OBS_KICK = 7,        /* mark the noise of the next step, xi_a(n') =
                                 G_a eta_a(n'), as the kick of the response
                                 estimator.  out: [n']                              */
    SETD_OBS_RESPONSE = 8,    /* linear response by the noise correlation (App. C
                                 susceptibility, Onsager-Machlup): per shell the
                                 mean over realizations and modes with G_a > 0 of
                                 phi_a(n) conj eta_a(n') / G_a, i.e. (Stein) the
                                 mean response of phi_a(n) to an additive kick
                                 in the step taken from n'; interior modes of a
                                 real field as 2 Re.  Needs SETD_OBS_KICK first.
                                 out: [Re (nbins), Im (nbins), count (nbins)]      */
    SETD_OBS_SERIES_START = 9,/* start a window of series_len samples: phi_a now
                                 (m = 0) and after each of the next M - 1 steps.
                                 out: [n0]                                         */
    SETD_OBS_SPECTRUM = 10,   /* App. C dynamic correlation and susceptibility
                                 of the completed window, with
                                 phi_{a,b} = sum_m e^{2 pi i b m/M} phi_a(m) and
                                 xi_{a,b} the same of the kicks of the steps
                                 taken from the samples (T = M h):
                                   C(k, w_b)   = (L/N^2)^d (T/M^2) <|phi_{a,b}|^2>
                                   chi(k, w_b) = (L/N^2)^d (T/M^2) (1/2D_a)
                                                 <phi_{a,b} conj xi_{a,b}> / h,
                                 means over realizations and over the modes of
                                 each shell with G_a, D_a > 0 (an interior mode
                                 of a real field stands for -a too; its
                                 transforms at w_b are the conjugates of a's at
                                 -w_b); b in FFT order, w_b = 2 pi b / T.
                                 out: [C (nbins x M), Re chi (nbins x M),
                                 Im chi (nbins x M), count (nbins)]              */
    SETD_OBS_BOXWIDTH = 11,   /* box-averaged width (Sec. 5 KPZ): for l = 2, 4, ..
                                 N (equal n[i] = N) the sqrt of the ensemble mean,
                                 over the N^d/l^d boxes of l^d sites, of the
                                 variance of the field within the box (complex
                                 field: of |phi - box mean|^2).  Computed from the
                                 spectrum without a transform.
                                 out: [w_2, w_4, .., w_N] (log2 N values)        */
    SETD_OBS_FDT = 12         /* FDT check of Sec. 5 on the completed window: per
                                 mode a and frequency w_b the deviation
                                 Delta = 2 Im chi - (w_b / D_a) C of the ensemble
                                 means (chi with 1/(2 D_a), as for
                                 SETD_OBS_SPECTRUM; b signed, M/2 taken as -M/2),
                                 averaged over all prod n_i modes (an interior
                                 mode of a real field also stands for -a) and
                                 the M frequencies.
                                 out: [mean |Delta|, mean Delta]                  */
} setd_obs_kind;

/*
 * Problem statement (Sec. 4 Eq. general_fourier; lattice of App. A):
 *   lattice n[0..ndim) points, spacing dx, L_i = n[i] dx, k_i = 2 pi a_i / L_i;
 *   c(k) = c0 + c2 k^2 + c4 k^4 (complex, {re, im}); D(k) = noise_D k^noise_kpow.
 * Model A: c0 = -r, c2 = -1, kpow 0, nl PHI3, nl_par[0] = u.
 * Model B: c2 = -r, c4 = -1, kpow 2, nl PHI3_CONS, nl_par[0] = u.
 * KPZ:     c2 = -nu, kpow 0, nl KPZ, nl_par[0] = lambda.
 * CGL:     c0 = 1, c2 = -(1 + i alpha), complex_field 1, nl CGL, nl_par[0] = beta.
 */
typedef struct {
    int ndim;                 /* 1, 2 or 3 (a 1D line steps up to 256 steps per
                                 kernel launch with its state in registers)       */
    int n[3];                 /* points per axis, powers of two in [8, 1024]       */
    double dx;                /* lattice spacing (> 0)                             */
    int complex_field;        /* 0: real order parameter (R2C); 1: complex (C2C)   */
    double c0[2], c2[2], c4[2];
    int nl;                   /* setd_nonlin                                       */
    double nl_par[2];         /* u | lambda | beta                                 */
    double noise_D;           /* >= 0                                              */
    int noise_kpow;           /* 0 or 2                                            */
    double h;                 /* time step (> 0)                                   */
    int order;                /* 1 = SETD1, 2 = SETD2                              */
    int precision;            /* 32: complex64 state and transforms, coefficients
                                 evaluated in FP64 and rounded; 64: complex128     */
    int realizations;         /* independent noise realizations in one plan (>= 1) */
    uint64_t seed;            /* Philox4x32-10 key                                 */
    int dealias;              /* 0: none; 1: 2/3 rule, keep 3|a_i| < n[i]; 2:
                                 phase shift, the
                                 nonlinearity averaged over the grid and the
                                 2^d - 1 grids moved by dx/2 along each
                                 nonempty set of axes, keeping 2|a_i| < n[i]
                                 (alias-free for the quadratic and cubic terms).
                                 2D/3D plans with dealias 2 keep phi and
                                 F_{n-1} (no carry) and take 2^(d-1) times the
                                 transforms of a 2/3 step (3D: four copies of
                                 the n0 n1 (n2/2+1) line buffer)             */
    int ic_kind;              /* 0: phi = 0; 1: i.i.d. N(0, ic_sigma^2) per site
                                 (complex fields: ic_sigma (z1 + i z2))             */
    double ic_sigma;
    int history_readback;     /* SETD2 storage.  0 (default): each realization
                                 keeps, beside pre, only the carry
                                 Y_n = E phi_n + w_b F_{n-1} + G eta_n (Eq. SETD2
                                 regrouped, the noise of step n drawn one step
                                 early), so a step moves one stored array less;
                                 phi is recovered from pre when read, and
                                 setd_get_history returns SETD_E_UNSUPPORTED.
                                 1: phi and F_{n-1} are stored separately and
                                 setd_get_history works.  Plans without the 2/3
                                 rule, SETD1 plans, and plans whose per-
                                 realization arrays reach 2 GiB always use the
                                 separate storage.                                 */
    int series_len;           /* 0 (default), or M, a power of two in [8, 1024]:
                                 the workspace holds a window of M samples of
                                 the stored spectrum per realization for
                                 SETD_OBS_SERIES_START / SETD_OBS_SPECTRUM      */
    int noise_space;          /* 0 (default): eta_a drawn in Fourier space (App. B);
                                 1: eta drawn per site in real space and
                                 transformed, eta_a = DFT[eta_x]_a / sqrt(prod n)
                                 (Sec. 4 step 2's alternative, one more transform
                                 per step).  On 2D/3D lattices each step first
                                 transforms its site noise into a noise array
                                 (more workspace, more bytes per step) and the
                                 plan keeps phi and F_{n-1} (no carry).  The
                                 kick estimators (SETD_OBS_KICK / RESPONSE /
                                 SPECTRUM) need 0.                               */
} setd_desc;

/* Derived sizes of a plan (filled by setd_plan_info). */
typedef struct {
    size_t workspace_bytes;   /* device bytes setd_plan_bind needs                 */
    size_t spectral_len;      /* complex values per realization crossing the ABI   */
    size_t kept_modes;        /* stored (non-dealiased) modes per realization      */
    int nbins;                /* shell bins of the S(k) and two-time observables   */
    int passes_per_step;      /* kernel launches per time step                     */
    double alg_bytes_per_step;/* HBM bytes one step must move (all realizations)   */
    double site_updates_per_step; /* prod n[i] * realizations                      */
    double pass_bytes[4];     /* HBM bytes each kernel launch of a step must move,
                                 in launch order (unused entries 0); with real-
                                 space noise on a 2D/3D lattice the launches of
                                 its transform come first and are counted in
                                 alg_bytes_per_step only                         */
    int variants[3];          /* kernel variants in use (row, axis 0, axis 1) after
                                 the autotuner; meaningful once bound; row
                                 variant bits: 0 LDS padding, 1 256-thread
                                 workgroups, 2-3 log2 of the row-pair groups a
                                 workgroup takes in turn (real fields); axis-0
                                 variants 4 and up update in registers: 4 + 2j,
                                 5 + 2j and 12 + j at three tile widths, the
                                 items interleaved per column tile in groups of
                                 2^j                                             */
    int axis_tile[2];         /* axis-0 pass: column tile width, columns per thread */
    int streams;              /* 2 when setd_step runs the two halves of the
                                 realizations on the bound stream and an
                                 auxiliary one of the plan (joined again before
                                 setd_step returns; calls of four or more
                                 steps), else 1                                  */
    int graph_steps;          /* setd_step runs whole chunks of this many steps
                                 as one HIP graph captured at the first such
                                 call (environment SETD_GRAPH at bind time;
                                 default 0: kernel launches only)                */
} setd_plan_info_t;

typedef struct setd_plan setd_plan;
typedef struct setd_server setd_server;
typedef int64_t setd_job;

/*
 * Validate *desc and prepare a plan (host work only, no device memory).
 * Errors: SETD_E_INVAL for ndim not in {1,2,3}, n[i] not a power of two in
 * [8, 1024], order not in {1,2}, h <= 0, dx <= 0, noise_D < 0, noise_kpow not
 * in {0,2}, precision not in {32,64}, realizations < 1, a complex c(k) on a
 * real field, ic_kind not in {0,1}; SETD_E_UNSUPPORTED for KPZ outside 1D/2D
 * real fields, PHI3/PHI3_CONS on complex fields or CGL on real fields.
 * *out is owned by the caller and released with setd_plan_destroy.
 */
setd_status setd_plan_create(const setd_desc* desc, setd_plan** out);

/* Device bytes the plan needs (state, SETD2 history, transform intermediates,
   coefficient and twiddle tables, FP64 observable accumulators). */
setd_status setd_plan_workspace(const setd_plan* plan, size_t* bytes);

setd_status setd_plan_info(const setd_plan* plan, setd_plan_info_t* info);

/*
 * Bind caller-owned device memory dev_ws[0, bytes) (bytes >= the workspace
 * size, 256-byte aligned) and a hipStream_t (NULL = the null stream).  Queues
 * the FP64 coefficient table (Sec. 4 step 3), twiddle tables and the initial
 * condition on the stream.  May be called once per plan.
 * Errors: SETD_E_INVAL (null/misaligned pointer), SETD_E_NOMEM (too small),
 * SETD_E_STATE (already bound), SETD_E_DEVICE.
 */
setd_status setd_plan_bind(setd_plan* plan, void* dev_ws, size_t bytes, void* hip_stream);

/*
 * Queue nsteps time steps (Sec. 4 algorithm box with Eq. SETD1/SETD2) of every
 * realization on the bound stream; asynchronous.  Step n draws its noise with
 * Philox counter (mode, n, realization, 0).  nsteps >= 0; the step index must
 * stay below 2^32.  Errors: SETD_E_STATE (not bound), SETD_E_INVAL.
 */
setd_status setd_step(setd_plan* plan, int64_t nsteps);

/*
 * Compute observable `kind` (setd_obs_kind) in FP64 on the device and copy
 * it to host_out[0, cap); *len receives the number of doubles written.
 * Synchronises the stream.  Returns SETD_E_NONFINITE (after writing the
 * output) if any realization has produced a non-finite value.
 * Errors: SETD_E_INVAL (cap too small, unknown kind, SETD_OBS_TWOTIME before
 * a snapshot, SETD_OBS_RESPONSE before a kick, SETD_OBS_SPECTRUM before a full
 * window or without series_len, shells on unequal n[i]),
 * SETD_E_STATE, SETD_E_DEVICE.
 */
setd_status setd_observe(setd_plan* plan, int kind, double* host_out, size_t cap, size_t* len);

/* Copy realization r's spectral state phi_a (layout above) into host_out,
   cap >= 2 * spectral_len doubles.  Synchronises the stream. */
setd_status setd_get_field(setd_plan* plan, int realization, double* host_out, size_t cap);

/* Overwrite realization r's spectral state from host_in (len >= 2 *
   spectral_len doubles); dealiased modes are dropped.  Restarts that
   realization's SETD2 history (its next step uses F_{n-1} = F_n).
   Synchronises the stream. */
setd_status setd_set_field(setd_plan* plan, int realization, const double* host_in, size_t len);

/* Copy realization r's previous nonlinear term F_{n-1} (SETD2 history, layout
   above, already multiplied by the model prefactor) into host_out.
   SETD_E_UNSUPPORTED when the plan keeps only the combined carry
   (history_readback 0, see setd_desc). */
setd_status setd_get_history(setd_plan* plan, int realization, double* host_out, size_t cap);

/* Set the step index n of every realization (checkpoint restart); the next
   step draws noise for step n. */
setd_status setd_set_step(setd_plan* plan, int64_t step);

/* Kernel timing: while enabled, setd_step records a pair of HIP events on
   the bound stream around every pass launch. */
setd_status setd_profile(setd_plan* plan, int enable);

/* Synchronise and return, per pass of a step in launch order, the summed
   duration in milliseconds and the number of launches timed since the last
   read: out = [ms_0, count_0, ms_1, count_1, ...]; resets the sums. */
setd_status setd_profile_read(setd_plan* plan, double* out, size_t cap, size_t* len);

/* Release a plan (not the caller's device memory or stream). */
setd_status setd_plan_destroy(setd_plan* plan);

/*
 * Serving.  A server owns a scheduler thread that admits submitted jobs into
 * the caller's device arena dev_arena[0, bytes) by their workspace footprint,
 * keeps their fields resident, and advances all admitted jobs together:
 * realizations of jobs with the same lattice class share one launch per pass,
 * the classes of a tick run side by side on up to four streams of the server
 * (SETD_SERVER_LANES, default 4; 0 or 1 keeps everything on hip_stream), and
 * newly admitted jobs join the next scheduler tick (continuous batching).
 * A job's trajectory does not depend on what else is running.
 */
setd_status setd_server_create(void* dev_arena, size_t bytes, void* hip_stream, setd_server** out);

/* Queue a job: a copy of *desc advanced nsteps steps.  *out receives its id.
   Errors: SETD_E_INVAL/UNSUPPORTED as setd_plan_create, SETD_E_NOMEM if the job
   could never fit the arena. */
setd_status setd_submit(setd_server* server, const setd_desc* desc, int64_t nsteps, setd_job* out);

/* *done = 1 once the job has finished; *job_status is its outcome
   (SETD_OK, SETD_E_NONFINITE, ...). */
setd_status setd_poll(setd_server* server, setd_job job, int* done, setd_status* job_status);

/* Block until every submitted job has finished. */
setd_status setd_server_drain(setd_server* server);

/* Observable of a finished job, computed when it finished (kinds SETD_OBS_SK,
   SETD_OBS_WIDTH, SETD_OBS_STEP).  SETD_E_BUSY while it runs. */
setd_status setd_job_observe(setd_server* server, setd_job job, int kind, double* out, size_t cap, size_t* len);

/* Final spectral state of a finished job's realization r (layout above). */
setd_status setd_job_get_field(setd_server* server, setd_job job, int realization, double* host_out, size_t cap);

/* Host timestamps of a job in seconds on a monotonic clock:
   out[0] submit, out[1] admit, out[2] finish; out[3] steps done. */
setd_status setd_job_times(setd_server* server, setd_job job, double* out4);

/* Counters of the server since its creation: out[0] scheduler ticks that ran
   steps, out[1] pass launches those ticks queued (per launch unit and
   sub-step), out[2] the launches among them that several lattice classes
   shared (2D real fields of square lattices N = 64..512, complex64, 2/3 rule,
   SETD2, phi^3 nonlinearities: one launch per pass for all of them;
   environment SETD_SERVER_MULTI=0 at creation keeps one launch per class).
   cap >= 3; *len receives 3. */
setd_status setd_server_stats(setd_server* server, double* out, size_t cap, size_t* len);

/* Stop the scheduler thread and release the server (jobs still queued are
   dropped; the arena itself is the caller's). */
setd_status setd_server_destroy(setd_server* server);

/*
 * Scalar SDEs (Sec. 2, Eqs. SETD-EM, SETD-Milstein and SETD1; the examples of
 * Sec. 3): npaths independent paths of
 *   du = [c u + F(u)] dt + G(u) dW,  F(u) = f1 u + f3 u^3,  G(u) = g0 + g1 u,
 * in FP64 (the SAO: c = -Gamma, f3 = -Gamma b, g0 = sqrt(2 Gamma T); GBM:
 * c = lambda - delta, f1 = delta, g1 = mu).  With x = c h the schemes use
 * e^x, (e^x - 1)/c and either e^{x/2} G dW (SETD-EM),
 * e^{x/2} G [dW + g1 (dW^2 - h)/2] (SETD-Milstein) or
 * sqrt((e^{2x} - 1)/(2c)) G z (SETD1).  Step n of path p draws z, the first
 * Box-Muller normal of the Philox4x32-10 block with counter (p, n, 0, 2) keyed
 * by seed (two 53-bit uniforms), and dW = sqrt(h) z.
 */
typedef enum { SETD_SDE_EM = 0, SETD_SDE_MILSTEIN = 1, SETD_SDE_SETD1 = 2 } setd_sde_scheme;

typedef struct {
    int scheme;               /* setd_sde_scheme                                  */
    double c, f1, f3, g0, g1; /* the SDE above                                    */
    double h, u0;             /* step, initial value of every path                */
    int64_t nsteps;           /* steps, < 2^32                                    */
    int npaths;               /* paths (0: nothing to do)                         */
    uint64_t seed;
} setd_sde_desc;

/* Queue nsteps steps of every path on hip_stream (asynchronous; NULL is the
   default stream).  dev_u[p] receives u after nsteps steps from u0, dev_w[p]
   (may be NULL) the sum of the path's dW: npaths doubles each, device memory
   of the caller.  Errors: SETD_E_INVAL (unknown scheme, h <= 0, negative or
   too large counts, null dev_u with npaths > 0), SETD_E_DEVICE. */
setd_status setd_sde_run(const setd_sde_desc* desc, double* dev_u, double* dev_w, void* hip_stream);

/*
 * For callers that cannot allocate device memory (code running under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * work of setd_plan_create + setd_plan_bind + setd_step + setd_get_field for
 * every realization, in one call that calls no hipMalloc / hipFree and
 * creates no stream, event or graph.
 *
 * The plan's workspace is a fixed device array of SETD_NOALLOC_MAX_WORKSPACE
 * bytes inside the library, one per GPU, held from the first call on that GPU
 * until the process ends.  Every call on a GPU reuses that GPU's array and
 * rewrites all of it that the plan uses, so nothing carries over between
 * calls; calls that overlap on one GPU (from several host threads, or on
 * streams not ordered against each other) race on it.  Variants are the
 * defaults (no autotuning) and the realizations step in one launch per pass,
 * with the same kernels as a bound plan.
 *
 * desc:    as setd_plan_create; the plan's workspace (setd_plan_workspace)
 *          must not exceed SETD_NOALLOC_MAX_WORKSPACE.
 * nsteps:  time steps from the initial condition (>= 0, < 2^32).
 * dev_out: caller-owned device memory of cap doubles, cap >= 2 * spectral_len
 *          * realizations; receives the spectra after nsteps steps in the
 *          layout of setd_get_field, realization r at dev_out + 2 r
 *          spectral_len (dealiased modes written as zero).
 * hip_stream: the work is queued on it and the call returns before the
 *          steps have finished (the set-up synchronises the stream once).
 * Errors: SETD_E_INVAL / SETD_E_UNSUPPORTED as setd_plan_create, or a null
 * pointer, negative nsteps, cap too small; SETD_E_NOMEM when the plan needs
 * more than SETD_NOALLOC_MAX_WORKSPACE bytes; SETD_E_DEVICE.
 */
#define SETD_NOALLOC_MAX_WORKSPACE (64u << 20)
setd_status setd_run_noalloc(const setd_desc* desc, int64_t nsteps, double* dev_out, size_t cap, void* hip_stream);

/* Seconds on the clock used by setd_job_times. */
double setd_clock(void);

/* Text of the calling thread's last error. */
const char* setd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SETD_H */
