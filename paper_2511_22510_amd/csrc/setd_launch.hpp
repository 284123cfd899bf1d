// setd_launch.hpp -- host launchers of the SETD kernels (one instantiation per
// state precision lives in setd_k32.hip / setd_k64.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "setd_types.hpp"

namespace setd {

// padding of the stored last axis, in elements (128 bytes)
template <typename T>
constexpr int pitch_align() { return sizeof(T) == 4 ? 16 : 8; }

// `var` selects a kernel variant (see setd_launch_impl.hpp); 0..3 for the row
// and axis-1 passes, 0..5 for the axis-0 pass
template <typename T>
hipError_t launch_row(const Geo& g, const Item* items, int nitems, int mode, int sub, int var, int kpz,
                      hipStream_t s);
// whether the register-update axis-0 kernel (buffer accesses into arrays of
// under 2 GiB per realization, 2/3 rule on) can run a plan's time step
inline bool axis0_register_ok(const Geo& g, size_t real_bytes)
{
    const size_t pre_bytes = (size_t)g.n[0] * (g.ndim == 3 ? g.kept[1] : 1) * g.pitch * 2 * real_bytes;
    return g.dealias == 1 && pre_bytes < ((size_t)1 << 31);
}

// lean: the plan keeps the SETD2 carry instead of phi and F_{n-1} (needs
// axis0_register_ok)
template <typename T>
hipError_t launch_axis0(const Geo& g, const Item* items, int nitems, int mode, int sub, int var, int kpz,
                        int lean, hipStream_t s);
template <typename T>
hipError_t launch_axis1(const Geo& g, const Item* items, int nitems, int dir, int sub, int var, hipStream_t s);
// keep the stored a_last = 0 (and N_last/2) planes of a real field Hermitian
// (which: 0 phi, 1 the F_{n-1} array / SETD2 carry); no-op for complex fields
template <typename T>
hipError_t launch_hermitian(const Geo& g, const Item* items, int nitems, int which, hipStream_t s);
// mode LIN_STEP / LIN_CARRY / LIN_RENOISE (new_step: the re-drawn step index)
template <typename T>
hipError_t launch_linear(const Geo& g, const Item* items, int nitems, int sub, int mode, int64_t new_step,
                         hipStream_t s);
template <typename T>
hipError_t launch_observe(const Geo& g, const Item* items, int nitems, int kind, int nbins, double vol,
                          double* acc, int64_t kick, hipStream_t s);
// time-frequency observables of a recorded window (M a power of two in [8, 1024])
template <typename T>
hipError_t launch_spectrum(const SpecArgs& a, int M, hipStream_t s);
// sums of |Delta| and Delta of the per-mode FDT deviations
template <typename T>
hipError_t launch_fdt_reduce(const Geo& g, const double* dacc, int total, int M, double* out, hipStream_t s);
// the noise of the current step of plans that draw it in real space (2D/3D):
// site draws and transforms into each item's noise array (var1, var0: the
// axis-1 and axis-0 pass variants)
template <typename T>
hipError_t launch_rsn(const Geo& g, const Item* items, int nitems, int sub, int var1, int var0, hipStream_t s);
// Lattice classes that share one launch per pass (k_row_multi, k_axis0_multi):
// 2D real fields on square lattices of N = 64, 128, 256 or 512 points, complex64,
// 2/3 rule, SETD2 with the carry storage, a phi^3 nonlinearity, Fourier-space
// noise.  Slot s of launch_multi2d takes the class of N = 64 << s (nitems 0:
// none); pass 0 is the row pass, 1 the axis-0 pass with the update.
struct MultiClass {
    Geo g;
    const Item* items;
    int nitems;
};
inline bool multi2d_ok(const Geo& g, bool lean, int nl)
{
    const int n = g.n[0];
    return g.ndim == 2 && !g.cplx && g.prec == 32 && g.dealias == 1 && !g.rsn && lean && n == g.n[1] &&
           (n == 64 || n == 128 || n == 256 || n == 512) && (nl == NL_PHI3 || nl == NL_PHI3_CONS);
}
inline int multi2d_slot(int n) { return n == 64 ? 0 : n == 128 ? 1 : n == 256 ? 2 : 3; }
template <typename T>
hipError_t launch_multi2d(const MultiClass (&cls)[4], int pass, int sub, hipStream_t s);
// 1D lattices: nsteps steps per launch// 1D lattices: nsteps steps per launch (MODE_STEP) or the initial condition (MODE_IC)
template <typename T>
hipError_t launch_line1d(const Geo& g, const Item* items, int nitems, int mode, int sub, int nsteps, int nl,
                         hipStream_t s);
// box-averaged width: class sums of one realization, then sum_c |A_c|^2 per level
template <typename T>
hipError_t launch_boxwidth(const BoxArgs& a, size_t ncls, hipStream_t s);

// (tile width, columns per thread) of axis-pass variant `var` for line length n
void axis_shape(int precision, int n, int var, int* tile, int* lpt);

struct CoefArgs;
hipError_t launch_coef(const CoefArgs& a, hipStream_t s);
hipError_t launch_twiddle(int n, double* out64, float* out32, hipStream_t s);
hipError_t launch_ctrl_init(Ctrl* ctrl, int n, int64_t step, hipStream_t s);
hipError_t launch_ctrl_set(Ctrl* ctrl, int n, int64_t step, int which, hipStream_t s);
hipError_t launch_fill64(double* p, int64_t n, double v, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
// stored state of R realizations (rstride bytes apart) -> unpruned FFT-order
// spectra as interleaved doubles in device memory, nspec values each
hipError_t launch_unpack(const Geo& g, const void* phi, size_t rstride, int R, int64_t nspec, double* out,
                         hipStream_t s);
hipError_t launch_obs_final(int kind, int nb, const double* acc, double* out, double* skacc, double wscale,
                            hipStream_t s);
hipError_t launch_obs_mean(int nb, const double* skacc, double* out, hipStream_t s);

}  // namespace setd
