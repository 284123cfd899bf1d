"""ctypes binding of libsetd.so, the gfx950 SETD library behind include/setd.h.

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch provides device memory (a uint8 tensor as the workspace or
arena) and the HIP stream.  The library is loaded from this package directory;
if it has not been built the first call raises instead of falling back to
anything else.

The module exposes the C entry points under their C names (setd_plan_create,
setd_step, setd_observe, setd_submit, ...) plus two conveniences, :class:`Plan`
and :class:`Server`, that own the torch allocations.
"""
import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsetd.so")

SETD_OK = 0
SETD_E_INVAL = -1
SETD_E_NOMEM = -2
SETD_E_DEVICE = -3
SETD_E_NONFINITE = -4
SETD_E_BUSY = -5
SETD_E_UNSUPPORTED = -6
SETD_E_STATE = -7
STATUS_NAMES = {0: "SETD_OK", -1: "SETD_E_INVAL", -2: "SETD_E_NOMEM", -3: "SETD_E_DEVICE",
                -4: "SETD_E_NONFINITE", -5: "SETD_E_BUSY", -6: "SETD_E_UNSUPPORTED", -7: "SETD_E_STATE"}

NL = {"phi3": 0, "phi3_cons": 1, "kpz": 2, "cgl": 3, "none": 4}

OBS_SK, OBS_WIDTH, OBS_SNAPSHOT, OBS_TWOTIME, OBS_STEP, OBS_SK_ACCUM, OBS_SK_MEAN, OBS_KICK, OBS_RESPONSE, \
    OBS_SERIES_START, OBS_SPECTRUM, OBS_BOXWIDTH, OBS_FDT = range(13)


class setd_desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("dx", ctypes.c_double),
        ("complex_field", ctypes.c_int),
        ("c0", ctypes.c_double * 2), ("c2", ctypes.c_double * 2), ("c4", ctypes.c_double * 2),
        ("nl", ctypes.c_int), ("nl_par", ctypes.c_double * 2),
        ("noise_D", ctypes.c_double), ("noise_kpow", ctypes.c_int),
        ("h", ctypes.c_double), ("order", ctypes.c_int), ("precision", ctypes.c_int),
        ("realizations", ctypes.c_int), ("seed", ctypes.c_uint64), ("dealias", ctypes.c_int),
        ("ic_kind", ctypes.c_int), ("ic_sigma", ctypes.c_double),
        ("history_readback", ctypes.c_int), ("series_len", ctypes.c_int), ("noise_space", ctypes.c_int),
    ]


class setd_plan_info_t(ctypes.Structure):
    _fields_ = [
        ("workspace_bytes", ctypes.c_size_t), ("spectral_len", ctypes.c_size_t),
        ("kept_modes", ctypes.c_size_t), ("nbins", ctypes.c_int), ("passes_per_step", ctypes.c_int),
        ("alg_bytes_per_step", ctypes.c_double), ("site_updates_per_step", ctypes.c_double),
        ("pass_bytes", ctypes.c_double * 4), ("variants", ctypes.c_int * 3),
        ("axis_tile", ctypes.c_int * 2), ("streams", ctypes.c_int), ("graph_steps", ctypes.c_int),
    ]


class setd_sde_desc(ctypes.Structure):
    _fields_ = [
        ("scheme", ctypes.c_int), ("c", ctypes.c_double), ("f1", ctypes.c_double), ("f3", ctypes.c_double),
        ("g0", ctypes.c_double), ("g1", ctypes.c_double), ("h", ctypes.c_double), ("u0", ctypes.c_double),
        ("nsteps", ctypes.c_int64), ("npaths", ctypes.c_int), ("seed", ctypes.c_uint64),
    ]


SDE_EM, SDE_MILSTEIN, SDE_SETD1 = 0, 1, 2


class SetdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


# every symbol declared in include/setd.h, with its ctypes signature
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_SZ = ctypes.c_size_t
_I64 = ctypes.c_int64
SIGNATURES = {
    "setd_plan_create": (ctypes.c_int, [ctypes.POINTER(setd_desc), ctypes.POINTER(_P)]),
    "setd_plan_workspace": (ctypes.c_int, [_P, ctypes.POINTER(_SZ)]),
    "setd_plan_info": (ctypes.c_int, [_P, ctypes.POINTER(setd_plan_info_t)]),
    "setd_plan_bind": (ctypes.c_int, [_P, _P, _SZ, _P]),
    "setd_step": (ctypes.c_int, [_P, _I64]),
    "setd_observe": (ctypes.c_int, [_P, ctypes.c_int, _D, _SZ, ctypes.POINTER(_SZ)]),
    "setd_get_field": (ctypes.c_int, [_P, ctypes.c_int, _D, _SZ]),
    "setd_set_field": (ctypes.c_int, [_P, ctypes.c_int, _D, _SZ]),
    "setd_get_history": (ctypes.c_int, [_P, ctypes.c_int, _D, _SZ]),
    "setd_set_step": (ctypes.c_int, [_P, _I64]),
    "setd_profile": (ctypes.c_int, [_P, ctypes.c_int]),
    "setd_profile_read": (ctypes.c_int, [_P, _D, _SZ, ctypes.POINTER(_SZ)]),
    "setd_plan_destroy": (ctypes.c_int, [_P]),
    "setd_server_create": (ctypes.c_int, [_P, _SZ, _P, ctypes.POINTER(_P)]),
    "setd_submit": (ctypes.c_int, [_P, ctypes.POINTER(setd_desc), _I64, ctypes.POINTER(_I64)]),
    "setd_poll": (ctypes.c_int, [_P, _I64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "setd_server_drain": (ctypes.c_int, [_P]),
    "setd_job_observe": (ctypes.c_int, [_P, _I64, ctypes.c_int, _D, _SZ, ctypes.POINTER(_SZ)]),
    "setd_job_get_field": (ctypes.c_int, [_P, _I64, ctypes.c_int, _D, _SZ]),
    "setd_job_times": (ctypes.c_int, [_P, _I64, _D]),
    "setd_server_stats": (ctypes.c_int, [_P, _D, _SZ, ctypes.POINTER(_SZ)]),
    "setd_server_destroy": (ctypes.c_int, [_P]),
    "setd_sde_run": (ctypes.c_int, [ctypes.POINTER(setd_sde_desc), _P, _P, _P]),
    "setd_run_noalloc": (ctypes.c_int, [ctypes.POINTER(setd_desc), _I64, _P, _SZ, _P]),
    "setd_clock": (ctypes.c_double, []),
    "setd_last_error": (ctypes.c_char_p, []),
}

_libs = {}


def load(path=None):
    """Load libsetd.so (the in-tree build unless a path is given)."""
    path = os.path.abspath(path or LIB_PATH)
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path):
        raise RuntimeError("%s is missing: build it with __graft_entry__.build()" % path)
    if path == os.path.abspath(LIB_PATH):
        # the library runs on the HIP runtime torch has loaded
        import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue   # calling it raises AttributeError; the ABI test lists it
        fn.restype = res
        fn.argtypes = args
    _libs[path] = lib
    return lib


def _check(lib, st):
    if st != SETD_OK:
        raise SetdError(st, lib.setd_last_error().decode())
    return st


def make_desc(p):
    """setd_desc from a problem dict (see paper_2511_22510_amd.workloads)."""
    d = setd_desc()
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
    d.nl = NL[nl] if isinstance(nl, str) else int(nl)
    par = list(p.get("nl_par", (0.0, 0.0))) + [0.0, 0.0]
    d.nl_par[0] = float(par[0])
    d.nl_par[1] = float(par[1])
    d.noise_D = float(p.get("noise_D", 0.0))
    d.noise_kpow = int(p.get("noise_kpow", 0))
    d.h = float(p["h"])
    d.order = int(p.get("order", 1))
    d.precision = int(p.get("precision", 64))
    d.realizations = int(p.get("realizations", 1))
    d.seed = int(p.get("seed", 0))
    d.dealias = int(p.get("dealias", 1))
    d.ic_kind = int(p.get("ic_kind", 0))
    d.ic_sigma = float(p.get("ic_sigma", 0.0))
    d.history_readback = int(p.get("history_readback", 0))
    d.noise_space = int(p.get("noise_space", 0))
    d.series_len = int(p.get("series_len", 0))
    return d


def spectral_shape(p):
    shp = list(p["n"][: p["ndim"]])
    if not p.get("complex_field", 0):
        shp[-1] = shp[-1] // 2 + 1
    return tuple(shp)


# ---------------------------------------------------------------- C names
def setd_plan_create(desc, lib=None):
    lib = lib or load()
    h = _P()
    _check(lib, lib.setd_plan_create(ctypes.byref(desc), ctypes.byref(h)))
    return h


def setd_plan_workspace(plan, lib=None):
    lib = lib or load()
    b = _SZ()
    _check(lib, lib.setd_plan_workspace(plan, ctypes.byref(b)))
    return b.value


def setd_plan_info(plan, lib=None):
    lib = lib or load()
    info = setd_plan_info_t()
    _check(lib, lib.setd_plan_info(plan, ctypes.byref(info)))
    return info


def setd_plan_bind(plan, dev_ptr, nbytes, stream_ptr, lib=None):
    lib = lib or load()
    _check(lib, lib.setd_plan_bind(plan, _P(dev_ptr), nbytes, _P(stream_ptr or 0)))


def setd_step(plan, nsteps, lib=None):
    lib = lib or load()
    _check(lib, lib.setd_step(plan, int(nsteps)))


def setd_observe(plan, kind, cap, lib=None, allow_nonfinite=False):
    lib = lib or load()
    out = np.zeros(cap, dtype=np.float64)
    ln = _SZ()
    st = lib.setd_observe(plan, int(kind), out.ctypes.data_as(_D), cap, ctypes.byref(ln))
    if not (allow_nonfinite and st == SETD_E_NONFINITE):
        _check(lib, st)
    return out[: ln.value].copy(), st


def setd_get_field(plan, r, nspec, lib=None):
    lib = lib or load()
    out = np.zeros(2 * nspec, dtype=np.float64)
    _check(lib, lib.setd_get_field(plan, int(r), out.ctypes.data_as(_D), out.size))
    return out.view(np.complex128)


def setd_set_field(plan, r, arr, lib=None):
    lib = lib or load()
    a = np.ascontiguousarray(arr, dtype=np.complex128).reshape(-1)
    buf = a.view(np.float64)
    _check(lib, lib.setd_set_field(plan, int(r), buf.ctypes.data_as(_D), buf.size))


def setd_get_history(plan, r, nspec, lib=None):
    lib = lib or load()
    out = np.zeros(2 * nspec, dtype=np.float64)
    _check(lib, lib.setd_get_history(plan, int(r), out.ctypes.data_as(_D), out.size))
    return out.view(np.complex128)


def setd_set_step(plan, step, lib=None):
    lib = lib or load()
    _check(lib, lib.setd_set_step(plan, int(step)))


def setd_profile(plan, enable, lib=None):
    lib = lib or load()
    _check(lib, lib.setd_profile(plan, int(enable)))


def setd_profile_read(plan, lib=None):
    lib = lib or load()
    out = np.zeros(8, dtype=np.float64)
    ln = _SZ()
    _check(lib, lib.setd_profile_read(plan, out.ctypes.data_as(_D), out.size, ctypes.byref(ln)))
    return out[: ln.value].reshape(-1, 2)


def setd_plan_destroy(plan, lib=None):
    lib = lib or load()
    lib.setd_plan_destroy(plan)


def setd_server_create(arena_ptr, nbytes, stream_ptr, lib=None):
    lib = lib or load()
    h = _P()
    _check(lib, lib.setd_server_create(_P(arena_ptr), nbytes, _P(stream_ptr or 0), ctypes.byref(h)))
    return h


def setd_submit(server, desc, nsteps, lib=None):
    lib = lib or load()
    job = _I64()
    _check(lib, lib.setd_submit(server, ctypes.byref(desc), int(nsteps), ctypes.byref(job)))
    return job.value


def setd_poll(server, job, lib=None):
    lib = lib or load()
    done = ctypes.c_int()
    js = ctypes.c_int()
    _check(lib, lib.setd_poll(server, int(job), ctypes.byref(done), ctypes.byref(js)))
    return bool(done.value), js.value


def setd_server_drain(server, lib=None):
    lib = lib or load()
    _check(lib, lib.setd_server_drain(server))


def setd_job_observe(server, job, kind, cap, lib=None, allow_nonfinite=False):
    lib = lib or load()
    out = np.zeros(cap, dtype=np.float64)
    ln = _SZ()
    st = lib.setd_job_observe(server, int(job), int(kind), out.ctypes.data_as(_D), cap, ctypes.byref(ln))
    if not (allow_nonfinite and st == SETD_E_NONFINITE):
        _check(lib, st)
    return out[: ln.value].copy(), st


def setd_job_get_field(server, job, r, nspec, lib=None):
    lib = lib or load()
    out = np.zeros(2 * nspec, dtype=np.float64)
    _check(lib, lib.setd_job_get_field(server, int(job), int(r), out.ctypes.data_as(_D), out.size))
    return out.view(np.complex128)


def setd_job_times(server, job, lib=None):
    lib = lib or load()
    out = np.zeros(4, dtype=np.float64)
    _check(lib, lib.setd_job_times(server, int(job), out.ctypes.data_as(_D)))
    return out


def setd_server_stats(server, lib=None):
    lib = lib or load()
    out = np.zeros(3, dtype=np.float64)
    ln = _SZ()
    _check(lib, lib.setd_server_stats(server, out.ctypes.data_as(_D), out.size, ctypes.byref(ln)))
    return out[: ln.value].copy()


def setd_server_destroy(server, lib=None):
    lib = lib or load()
    lib.setd_server_destroy(server)


def setd_run_noalloc(desc, nsteps, dev_out_ptr, cap, stream_ptr, lib=None):
    lib = lib or load()
    _check(lib, lib.setd_run_noalloc(ctypes.byref(desc), int(nsteps), _P(dev_out_ptr), int(cap),
                                     _P(stream_ptr or 0)))


def setd_clock(lib=None):
    lib = lib or load()
    return lib.setd_clock()


def setd_last_error(lib=None):
    lib = lib or load()
    return lib.setd_last_error().decode()


# ---------------------------------------------------------------- conveniences
def _torch_workspace(nbytes):
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device: the SETD library runs on the GPU only")
    buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    return buf, buf.data_ptr(), stream


class Server:
    """A continuous-batching job server over a device arena from torch."""

    def __init__(self, arena_bytes, lib=None, workspace=None):
        self.lib = lib or load()
        if workspace is None:
            self._buf, ptr, stream = _torch_workspace(arena_bytes)
        else:
            self._buf, ptr, stream = workspace(arena_bytes)
        self.stream = stream
        self.h = setd_server_create(ptr, int(arena_bytes), stream, self.lib)
        self._shape = {}

    def submit(self, params, nsteps):
        jid = setd_submit(self.h, make_desc(params), nsteps, self.lib)
        shp = spectral_shape(params)
        self._shape[jid] = (shp, int(np.prod(shp)))
        return jid

    def poll(self, jid):
        return setd_poll(self.h, jid, self.lib)

    def drain(self):
        setd_server_drain(self.h, self.lib)

    def times(self, jid):
        return setd_job_times(self.h, jid, self.lib)

    def observe(self, jid, kind, allow_nonfinite=False):
        out, _ = setd_job_observe(self.h, jid, kind, 4096, self.lib, allow_nonfinite)
        return out

    def get(self, jid, r=0):
        shp, n = self._shape[jid]
        return setd_job_get_field(self.h, jid, r, n, self.lib).reshape(shp)

    def stats(self):
        """[ticks, pass launches, shared launches] (setd_server_stats)."""
        return setd_server_stats(self.h, self.lib)

    def close(self):
        if getattr(self, "h", None):
            setd_server_destroy(self.h, self.lib)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """A bound plan: problem dict -> workspace on the current torch device."""

    def __init__(self, params, lib=None, workspace=None):
        self.lib = lib or load()
        self.p = dict(params)
        self.desc = make_desc(self.p)
        self.h = setd_plan_create(self.desc, self.lib)
        self.info = setd_plan_info(self.h, self.lib)
        self.nbytes = int(self.info.workspace_bytes)
        if workspace is None:
            self._buf, ptr, stream = _torch_workspace(self.nbytes)
        else:
            self._buf, ptr, stream = workspace(self.nbytes)
        self.stream = stream
        setd_plan_bind(self.h, ptr, max(self.nbytes, 256), stream, self.lib)
        self.info = setd_plan_info(self.h, self.lib)
        self.spec_shape = spectral_shape(self.p)
        self.nspec = int(self.info.spectral_len)
        self.nbins = int(self.info.nbins)
        self.R = self.desc.realizations

    def step(self, n=1):
        setd_step(self.h, n, self.lib)

    def observe(self, kind, allow_nonfinite=False):
        M = int(self.p.get("series_len", 0)) if isinstance(getattr(self, "p", None), dict) else 0
        cap = 3 * self.nbins * max(M, 1) + self.nbins + 8
        out, _ = setd_observe(self.h, kind, cap, self.lib, allow_nonfinite)
        return out

    def spectrum(self):
        """(C, Re chi, Im chi) as [nbins, M] arrays and the shell counts of the
        completed window (SETD_OBS_SPECTRUM)."""
        nb, M = self.nbins, int(self.p["series_len"])
        out = self.observe(OBS_SPECTRUM)
        return (out[:nb * M].reshape(nb, M), out[nb * M:2 * nb * M].reshape(nb, M),
                out[2 * nb * M:3 * nb * M].reshape(nb, M), out[3 * nb * M:3 * nb * M + nb])

    def fdt(self):
        """(mean |Delta|, mean Delta): the FDT deviation of the completed
        window over all modes and frequencies (SETD_OBS_FDT)."""
        out = self.observe(OBS_FDT)
        return float(out[0]), float(out[1])

    def box_width(self):
        """[w_2, w_4, .., w_N]: the box-averaged widths (SETD_OBS_BOXWIDTH)."""
        return self.observe(OBS_BOXWIDTH)[:int(self.p["n"][0]).bit_length() - 1]

    def status_observe(self, kind):
        cap = 3 * self.nbins + 8
        return setd_observe(self.h, kind, cap, self.lib, True)

    def get(self, r=0):
        return setd_get_field(self.h, r, self.nspec, self.lib).reshape(self.spec_shape)

    def get_all(self):
        return np.stack([self.get(r) for r in range(self.R)])

    def history(self, r=0):
        return setd_get_history(self.h, r, self.nspec, self.lib).reshape(self.spec_shape)

    def set(self, r, arr):
        setd_set_field(self.h, r, arr, self.lib)

    def set_step(self, n):
        setd_set_step(self.h, n, self.lib)

    def close(self):
        if getattr(self, "h", None):
            setd_plan_destroy(self.h, self.lib)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_noalloc(params, nsteps, lib=None):
    """Spectra of every realization after nsteps steps from the initial
    condition, computed by setd_run_noalloc (no device allocation inside the
    library; the output buffer is a torch tensor): [R, *spectral shape]."""
    import torch
    lib = lib or load()
    desc = make_desc(params)
    shp = spectral_shape(params)
    nspec = int(np.prod(shp))
    R = int(desc.realizations)
    out = torch.empty(2 * nspec * R, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    setd_run_noalloc(desc, nsteps, out.data_ptr(), out.numel(), stream.cuda_stream, lib)
    stream.synchronize()
    return out.cpu().numpy().view(np.complex128).reshape((R,) + tuple(shp))


def sde_run(scheme, c, h, nsteps, npaths, seed, u0=1.0, f1=0.0, f3=0.0, g0=0.0, g1=0.0, lib=None):
    """Scalar SETD schemes (Sec. 2) on the GPU for du = (c u + f1 u + f3 u^3) dt
    + (g0 + g1 u) dW: returns (u after nsteps, sum of the dW) per path as host
    arrays; the paths run in device memory on torch's current stream."""
    import torch
    lib = lib or load()
    u = torch.empty(max(npaths, 1), dtype=torch.float64, device="cuda")
    w = torch.empty(max(npaths, 1), dtype=torch.float64, device="cuda")
    d = setd_sde_desc(scheme, c, f1, f3, g0, g1, h, u0, nsteps, npaths, seed)
    _check(lib, lib.setd_sde_run(ctypes.byref(d), u.data_ptr(), w.data_ptr(),
                                 torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return u[:npaths].cpu().numpy(), w[:npaths].cpu().numpy()
