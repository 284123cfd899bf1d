"""ctypes binding of the FP64 CPU oracle (oracle/setd_oracle.c).

TEST INFRASTRUCTURE: only the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this module.  The GPU library never imports it and it
never imports the GPU library.

A problem is given as a plain dict (the fields of the paper's problem statement,
Sec. 4 Eq. general_fourier with the lattice of App. A):
    ndim, n, dx, complex_field, c0, c2, c4, nl, nl_par, noise_D, noise_kpow,
    h, order, realizations, seed, dealias, ic_kind, ic_sigma
Extra keys (e.g. precision) are ignored here.
"""
import ctypes
import os

import numpy as np

from . import build as _build

NL_CODES = {"phi3": 0, "phi3_cons": 1, "kpz": 2, "cgl": 3, "none": 4}

OBS_SK, OBS_WIDTH, OBS_SNAPSHOT, OBS_TWOTIME, OBS_STEP, OBS_SK_ACCUM, OBS_SK_MEAN, OBS_KICK, OBS_RESPONSE, \
    OBS_SERIES_START, OBS_SPECTRUM, OBS_BOXWIDTH = range(12)


class _Desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("dx", ctypes.c_double),
        ("complex_field", ctypes.c_int),
        ("c0", ctypes.c_double * 2), ("c2", ctypes.c_double * 2), ("c4", ctypes.c_double * 2),
        ("nl", ctypes.c_int), ("nl_par", ctypes.c_double * 2),
        ("noise_D", ctypes.c_double), ("noise_kpow", ctypes.c_int),
        ("h", ctypes.c_double), ("order", ctypes.c_int),
        ("realizations", ctypes.c_int), ("seed", ctypes.c_uint64), ("dealias", ctypes.c_int),
        ("ic_kind", ctypes.c_int), ("ic_sigma", ctypes.c_double), ("noise_space", ctypes.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        vp = ctypes.c_void_p
        L.orc_fftn.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int]
        L.orc_rfftn.argtypes = [dp, dp, ctypes.c_int, ip]
        L.orc_irfftn.argtypes = [dp, dp, ctypes.c_int, ip]
        L.orc_philox.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.orc_philox.restype = None
        L.orc_normal_pair.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_uint32, ctypes.c_uint32, dp, dp]
        L.orc_normal_pair.restype = None
        L.orc_noise_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_uint32, ctypes.c_int, dp, dp]
        L.orc_noise_normals.restype = None
        L.orc_noise_slot.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint32), ip, ip]
        L.orc_sde_run.argtypes = [ctypes.POINTER(_SdeDesc), dp, dp]
        L.orc_series_start.argtypes = [vp, ctypes.c_int]
        L.orc_spectrum.argtypes = [vp, dp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
        L.orc_fdt.argtypes = [vp, dp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
        L.orc_phi12.argtypes = [ctypes.c_double, ctypes.c_double, dp]
        L.orc_phi12.restype = None
        L.orc_create_subset.argtypes = [ctypes.POINTER(_Desc), ctypes.c_int, ctypes.c_int]
        L.orc_create_subset.restype = vp
        L.orc_destroy.argtypes = [vp]
        L.orc_destroy.restype = None
        L.orc_nspec.argtypes = [vp]
        L.orc_nspec.restype = ctypes.c_size_t
        L.orc_step_index.argtypes = [vp]
        L.orc_step_index.restype = ctypes.c_int64
        L.orc_nbins.argtypes = [vp]
        L.orc_threads.argtypes = []
        L.orc_step.argtypes = [vp, ctypes.c_int64]
        L.orc_step_xi.argtypes = [vp, dp]
        L.orc_noise_xi.argtypes = [vp, ctypes.c_int64, dp]
        L.orc_site_noise.argtypes = [vp, ctypes.c_int64, ctypes.c_uint32, dp]
        L.orc_get.argtypes = [vp, ctypes.c_int, ctypes.c_int, dp]
        L.orc_set.argtypes = [vp, ctypes.c_int, dp]
        L.orc_set_step.argtypes = [vp, ctypes.c_int64]
        L.orc_coef.argtypes = [vp, ctypes.c_int, dp]
        L.orc_observe.argtypes = [vp, ctypes.c_int, dp, ctypes.c_size_t,
                                  ctypes.POINTER(ctypes.c_size_t)]
        _lib = L
    return _lib


def threads():
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().orc_threads())


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _shape_arg(shape):
    arr = (ctypes.c_int * 3)(*(list(shape) + [1] * (3 - len(shape))))
    return arr


# ---------------------------------------------------------------- transforms
def fftn(x, inverse=False):
    """Complex N-D DFT: forward e^{-}, unscaled; inverse e^{+}, scaled 1/N^d."""
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    rc = lib().orc_fftn(_dptr(a.view(np.float64)), a.ndim, _shape_arg(a.shape), 1 if inverse else -1)
    assert rc == 0
    return a


def rfftn(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    shp = list(x.shape)
    out = np.zeros(shp[:-1] + [shp[-1] // 2 + 1], dtype=np.complex128)
    rc = lib().orc_rfftn(_dptr(x), _dptr(out.view(np.float64)), x.ndim, _shape_arg(shp))
    assert rc == 0
    return out


def irfftn(X, shape):
    X = np.ascontiguousarray(X, dtype=np.complex128)
    out = np.zeros(shape, dtype=np.float64)
    rc = lib().orc_irfftn(_dptr(X.view(np.float64)), _dptr(out), len(shape), _shape_arg(shape))
    assert rc == 0
    return out


# ---------------------------------------------------------------- noise
def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox(c, k, o)
    return [int(v) for v in o]


def normal_pair(seed, e, n, r, tag):
    z1 = ctypes.c_double()
    z2 = ctypes.c_double()
    lib().orc_normal_pair(ctypes.c_uint64(seed), e, n, r, tag, ctypes.byref(z1), ctypes.byref(z2))
    return z1.value, z2.value


def noise_normals(seed, P, n, r, half):
    """Box-Muller normals of the Fourier-space noise from words (x0, x1)
    (half 0) or (x2, x3) (half 1) of the Philox block (P, n, r, 0)."""
    z1 = ctypes.c_double()
    z2 = ctypes.c_double()
    lib().orc_noise_normals(ctypes.c_uint64(seed), P, n, r, int(half), ctypes.byref(z1), ctypes.byref(z2))
    return z1.value, z2.value


class _SdeDesc(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int), ("c", ctypes.c_double), ("f1", ctypes.c_double),
                ("f3", ctypes.c_double), ("g0", ctypes.c_double), ("g1", ctypes.c_double),
                ("h", ctypes.c_double), ("u0", ctypes.c_double), ("nsteps", ctypes.c_int64),
                ("npaths", ctypes.c_int), ("seed", ctypes.c_uint64)]


SDE_EM, SDE_MILSTEIN, SDE_SETD1 = 0, 1, 2


def sde_run(scheme, c, h, nsteps, npaths, seed, u0=1.0, f1=0.0, f3=0.0, g0=0.0, g1=0.0):
    """Scalar SETD schemes (Sec. 2) for du = (c u + f1 u + f3 u^3) dt +
    (g0 + g1 u) dW: (u after nsteps, sum of the dW) per path."""
    d = _SdeDesc(scheme, c, f1, f3, g0, g1, h, u0, nsteps, npaths, seed)
    u = np.zeros(max(npaths, 1))
    w = np.zeros(max(npaths, 1))
    if lib().orc_sde_run(ctypes.byref(d), _dptr(u), _dptr(w)) != 0:
        raise RuntimeError("oracle sde_run failed")
    return u[:npaths], w[:npaths]


def phi12(x):
    out = (ctypes.c_double * 4)()
    x = complex(x)
    lib().orc_phi12(x.real, x.imag, out)
    return complex(out[0], out[1]), complex(out[2], out[3])


# ---------------------------------------------------------------- simulation
def make_desc(p):
    d = _Desc()
    d.ndim = int(p["ndim"])
    n = list(p["n"]) + [1] * (3 - len(p["n"]))
    for i in range(3):
        d.n[i] = int(n[i])
    d.dx = float(p.get("dx", 1.0))
    d.complex_field = int(p.get("complex_field", 0))
    for name in ("c0", "c2", "c4"):
        v = p.get(name, (0.0, 0.0))
        if not hasattr(v, "__len__"):
            v = (float(v), 0.0)
        getattr(d, name)[0] = float(v[0])
        getattr(d, name)[1] = float(v[1])
    nl = p.get("nl", "none")
    d.nl = NL_CODES[nl] if isinstance(nl, str) else int(nl)
    par = list(p.get("nl_par", (0.0, 0.0))) + [0.0, 0.0]
    d.nl_par[0] = float(par[0])
    d.nl_par[1] = float(par[1])
    d.noise_D = float(p.get("noise_D", 0.0))
    d.noise_kpow = int(p.get("noise_kpow", 0))
    d.h = float(p["h"])
    d.order = int(p.get("order", 1))
    d.realizations = int(p.get("realizations", 1))
    d.seed = int(p.get("seed", 0))
    d.dealias = int(p.get("dealias", 1))
    d.ic_kind = int(p.get("ic_kind", 0))
    d.ic_sigma = float(p.get("ic_sigma", 0.0))
    d.noise_space = int(p.get("noise_space", 0))
    return d


class Sim:
    """One oracle simulation over realizations [r_first, r_first + r_count)."""

    def __init__(self, params, r_first=0, r_count=None):
        self.p = dict(params)
        self.desc = make_desc(self.p)
        R = self.desc.realizations
        if r_count is None:
            r_count = R - r_first
        self.r_first, self.R = r_first, r_count
        self._h = lib().orc_create_subset(ctypes.byref(self.desc), r_first, r_count)
        if not self._h:
            raise ValueError("oracle rejected the problem description")
        ndim = self.desc.ndim
        self.shape = tuple(self.desc.n[i] for i in range(ndim))
        spec = list(self.shape)
        if not self.desc.complex_field:
            spec[-1] = spec[-1] // 2 + 1
        self.spec_shape = tuple(spec)
        self.nspec = int(lib().orc_nspec(self._h))
        self.nbins = int(lib().orc_nbins(self._h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    @property
    def step_index(self):
        return int(lib().orc_step_index(self._h))

    def step(self, n=1):
        assert lib().orc_step(self._h, int(n)) == 0

    def get(self, r=0, which=0):
        out = np.zeros(self.spec_shape, dtype=np.complex128)
        assert lib().orc_get(self._h, which, r, _dptr(out.view(np.float64))) == 0
        return out

    def get_all(self, which=0):
        return np.stack([self.get(r, which) for r in range(self.R)])

    def set(self, r, arr):
        a = np.ascontiguousarray(arr, dtype=np.complex128).reshape(self.spec_shape)
        assert lib().orc_set(self._h, r, _dptr(a.view(np.float64))) == 0

    def set_step(self, n):
        lib().orc_set_step(self._h, int(n))

    def noise_xi(self, n):
        out = np.zeros((self.R,) + self.spec_shape, dtype=np.complex128)
        lib().orc_noise_xi(self._h, int(n), _dptr(out.view(np.float64)))
        return out

    def site_noise(self, n, r):
        """The real-space draws eta_x of step n, realization r (noise_space 1),
        in lattice shape (complex for a complex field)."""
        cplx = bool(self.p.get("complex_field", 0))
        shape = tuple(int(v) for v in self.p["n"])
        out = np.zeros(int(np.prod(shape)) * (2 if cplx else 1))
        lib().orc_site_noise(self._h, int(n), int(r), _dptr(out))
        return (out.view(np.complex128) if cplx else out).reshape(shape)

    def noise_slot(self, e):
        """(P, half, kind) of stored element e: the Philox slot its noise is
        drawn from and how eta follows from the normals (App. B)."""
        P = ctypes.c_uint32()
        half = ctypes.c_int()
        kind = ctypes.c_int()
        lib().orc_noise_slot(self._h, int(e), ctypes.byref(P), ctypes.byref(half), ctypes.byref(kind))
        return P.value, half.value, kind.value

    def series_start(self, M):
        """Record phi_a(m), m = 0 (now) .. M - 1, over the next M - 1 steps."""
        assert lib().orc_series_start(self._h, int(M)) == 0
        self.series_len = int(M)

    def spectrum(self):
        """(C, Re chi, Im chi) as [nbins, M] arrays and the shell counts, from
        the recorded series (App. C dynamic correlations and susceptibility)."""
        nb, M = self.nbins, self.series_len
        out = np.zeros(3 * nb * M + nb)
        ln = ctypes.c_size_t(0)
        if lib().orc_spectrum(self._h, _dptr(out), out.size, ctypes.byref(ln)) != 0:
            raise RuntimeError("oracle spectrum failed")
        return (out[:nb * M].reshape(nb, M), out[nb * M:2 * nb * M].reshape(nb, M),
                out[2 * nb * M:3 * nb * M].reshape(nb, M), out[3 * nb * M:])

    def fdt(self):
        """(average absolute, signed average) FDT deviation of the recorded
        window over all modes and frequencies (Sec. 5)."""
        out = np.zeros(2)
        ln = ctypes.c_size_t(0)
        if lib().orc_fdt(self._h, _dptr(out), out.size, ctypes.byref(ln)) != 0:
            raise RuntimeError("oracle FDT failed")
        return float(out[0]), float(out[1])

    def step_xi(self, xi):
        a = np.ascontiguousarray(xi, dtype=np.complex128).reshape((self.R,) + self.spec_shape)
        assert lib().orc_step_xi(self._h, _dptr(a.view(np.float64))) == 0

    def coef(self, which):
        cplx = which in (0, 1, 2, 6)
        out = np.zeros(self.spec_shape, dtype=np.complex128 if cplx else np.float64)
        buf = out.view(np.float64) if cplx else out
        assert lib().orc_coef(self._h, which, _dptr(buf)) == 0
        return out

    def observe(self, kind):
        cap = 3 * self.nbins + 8
        out = np.zeros(cap, dtype=np.float64)
        ln = ctypes.c_size_t(0)
        rc = lib().orc_observe(self._h, kind, _dptr(out), cap, ctypes.byref(ln))
        if rc != 0:
            raise RuntimeError("oracle observe failed")
        return out[: ln.value].copy()
