"""Problem descriptions and seeded synthetic inputs.

This module holds parameters and random inputs only -- none of the method's
arithmetic -- so that the GPU tests, the oracle tests and the benchmark build
their problems from one place.

A problem is a plain dict with the fields of the paper's problem statement
(Sec. 4, Eq. general_fourier; lattice of App. A):
    ndim, n, dx, complex_field, c0, c2, c4 (complex as (re, im)), nl, nl_par,
    noise_D, noise_kpow, h, order, realizations, seed, dealias, ic_kind,
    ic_sigma, precision, and optionally history_readback (SETD2 storage: 0,
    the default, keeps only the combined carry; 1 keeps F_{n-1} readable).
c(k) = c0 + c2 k^2 + c4 k^4 and D(k) = noise_D k^noise_kpow.

The models of Sec. 5 map onto it as
    Model A  (Eq. modelA):  c = -(r + k^2),        D(k) = T,     F = -u FFT[phi^3]
    Model B  (Eq. modelB):  c = -k^2 (r + k^2),    D(k) = T k^2, F = -u k^2 FFT[phi^3]
    KPZ      (Eq. kpz):     c = -nu k^2,           D(k) = D,     F = lambda/2 FFT[|grad h|^2]
    CGL      (Eq. cgle):    c = 1 - (1 + i alpha) k^2, D = T,    F = -(1 + i beta) FFT[|A|^2 A]
(alpha, beta are the paper's b, c of the CGL equation.)
"""
import numpy as np


def model_a(n, r=-1.0, u=1.0, T=0.1, **kw):
    p = dict(ndim=len(n), n=list(n), dx=1.0, complex_field=0,
             c0=(-r, 0.0), c2=(-1.0, 0.0), c4=(0.0, 0.0),
             nl="phi3", nl_par=(u, 0.0), noise_D=T, noise_kpow=0,
             h=0.01, order=1, realizations=1, seed=0, dealias=1,
             ic_kind=1, ic_sigma=0.1, precision=64)
    p.update(kw)
    return p


def model_b(n, r=-1.0, u=1.0, T=0.05, **kw):
    p = dict(ndim=len(n), n=list(n), dx=1.0, complex_field=0,
             c0=(0.0, 0.0), c2=(-r, 0.0), c4=(-1.0, 0.0),
             nl="phi3_cons", nl_par=(u, 0.0), noise_D=T, noise_kpow=2,
             h=0.005, order=2, realizations=1, seed=1, dealias=1,
             ic_kind=1, ic_sigma=0.05, precision=32)
    p.update(kw)
    return p


def kpz(n, nu=1.0, lam=3.0, D=1.0, **kw):
    p = dict(ndim=len(n), n=list(n), dx=1.0, complex_field=0,
             c0=(0.0, 0.0), c2=(-nu, 0.0), c4=(0.0, 0.0),
             nl="kpz", nl_par=(lam, 0.0), noise_D=D, noise_kpow=0,
             h=0.01, order=2, realizations=1, seed=2, dealias=1,
             ic_kind=0, ic_sigma=0.0, precision=32)
    p.update(kw)
    return p


def cgl(n, alpha=0.5, beta=-1.2, T=0.01, **kw):
    p = dict(ndim=len(n), n=list(n), dx=0.5, complex_field=1,
             c0=(1.0, 0.0), c2=(-1.0, -alpha), c4=(0.0, 0.0),
             nl="cgl", nl_par=(beta, 0.0), noise_D=T, noise_kpow=0,
             h=0.002, order=2, realizations=1, seed=3, dealias=1,
             ic_kind=1, ic_sigma=0.01, precision=32)
    p.update(kw)
    return p


# The four simulation workloads and their run lengths.
CONFIG_A = dict(model_a([64, 64], order=1, precision=64, realizations=1, seed=0), steps=1000)
CONFIG_B = dict(model_b([512, 512], order=2, precision=32, realizations=64, seed=1), steps=10000)
CONFIG_KPZ = dict(kpz([1024, 1024], order=2, precision=32, realizations=16, seed=2), steps=50000)
CONFIG_CGL = dict(cgl([256, 256, 256], order=2, precision=32, realizations=4, seed=3), steps=20000)
# the lines of Sec. 5's 1D figures, batched over realizations: Model A
# (u = 0, N = 256, L = 64, D = 0.1, h = 0.01, r = 1) and KPZ (N = 1024, L = 512,
# lambda = 50, nu = 1, D = 0.01, h = 2e-3)
LINE_MODEL_A = dict(model_a([256], r=1.0, u=0.0, T=0.1, dx=0.25, h=0.01, order=1, precision=32,
                            realizations=16384, ic_kind=0, seed=4), steps=100000)
LINE_KPZ = dict(kpz([1024], nu=1.0, lam=50.0, D=0.01, dx=0.5, h=2e-3, order=2, precision=32,
                    realizations=4096, ic_kind=0, seed=5), steps=100000)


def problem(cfg, **over):
    """The problem dict of a workload (without its run length), with overrides."""
    p = {k: v for k, v in cfg.items() if k != "steps"}
    p.update(over)
    return p


def spectral_shape(p):
    shp = list(p["n"][: p["ndim"]])
    if not p.get("complex_field", 0):
        shp[-1] = shp[-1] // 2 + 1
    return tuple(shp)


def random_spectrum(p, seed, scale=1.0):
    """A seeded random spectral state of the problem's shape (complex128).

    It is not Hermitian-consistent on the a_d = 0 plane on purpose: both
    implementations must treat the stored half spectrum the same way.
    """
    rng = np.random.default_rng(seed)
    shp = spectral_shape(p)
    return scale * (rng.standard_normal(shp) + 1j * rng.standard_normal(shp))


def random_real_field(p, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal(tuple(p["n"][: p["ndim"]]))


# ---------------------------------------------------------------- serving trace
SERVING_TYPES = (
    ("A", [128, 128]), ("A", [256, 256]), ("A", [512, 512]),
    ("B", [256, 256]), ("B", [512, 512]),
    ("KPZ", [512, 512]),
    ("CGL", [128, 128, 128]),
)


def serving_trace(n_jobs=200, rate=20.0, seed=2024, precision=32, steps_range=(1000, 10000),
                  kinds=None):
    """A Poisson stream of SETD2 jobs: type uniform over the four models, then the
    size uniform within the model, realizations in {1, 4, 16}, steps uniform in
    steps_range, and a seed of its own per job."""
    rng = np.random.default_rng(seed)
    models = {}
    for name, n in SERVING_TYPES:
        models.setdefault(name, []).append(n)
    names = sorted(models) if kinds is None else list(kinds)
    t = 0.0
    jobs = []
    for j in range(n_jobs):
        t += float(rng.exponential(1.0 / rate))
        name = names[int(rng.integers(len(names)))]
        n = models[name][int(rng.integers(len(models[name])))]
        R = int(rng.choice([1, 4, 16]))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        jseed = int(rng.integers(1, 2**63 - 1))
        maker = {"A": model_a, "B": model_b, "KPZ": kpz, "CGL": cgl}[name]
        p = maker(n, order=2, precision=precision, realizations=R, seed=jseed)
        jobs.append(dict(id=j, arrival=t, model=name, problem=p, steps=steps))
    return jobs


def site_updates(p, steps):
    return int(np.prod(p["n"][: p["ndim"]])) * int(p.get("realizations", 1)) * int(steps)

