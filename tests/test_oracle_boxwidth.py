"""Pins of the oracle's box-averaged width w_l (Sec. 5 KPZ): the mean over
boxes of l^d sites of the variance within the box, for l = 2, 4, .., N."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2511_22510_amd import workloads as W


def _sim(n, **kw):
    kw.setdefault("ic_kind", 0)
    p = W.kpz(list(n), dealias=0, realizations=kw.pop("R", 1), precision=64, **kw)
    return O.Sim(p), p


@pytest.mark.parametrize("a", [(0, 1), (0, 3), (2, 0), (1, 2), (3, 5)])
def test_plane_wave_box_variance(a):
    """h = A cos(2 pi (a0 x0 + a1 x1)/N) set through its spectrum: the widths
    equal the box variances of the cosine evaluated on the grid (brute force,
    no transform), and where a and -a fall in different classes mod N/l they
    equal the closed form A^2/2 (1 - |D_l(a)|^2),
    D_l(a) = prod_i sin(pi a_i l/N)/(l sin(pi a_i/N)) (1 for a_i = 0)."""
    N, A = 16, 0.7
    s, p = _sim((N, N))
    spec = np.zeros(s.spec_shape, dtype=complex)
    a0, a1 = a
    if a1 > 0:
        spec[a0 % N, a1] = N * N * A / 2
    else:   # a1 = 0: both a and -a are stored
        spec[a0 % N, 0] += N * N * A / 2
        spec[(-a0) % N, 0] += N * N * A / 2
    s.set(0, spec)
    w = s.observe(O.OBS_BOXWIDTH)
    x0, x1 = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    h = A * np.cos(2 * np.pi * (a0 * x0 + a1 * x1) / N)

    def D1(ai, l):
        return 1.0 if ai % N == 0 else np.sin(np.pi * ai * l / N) / (l * np.sin(np.pi * ai / N))

    for wl, l in zip(w, [2, 4, 8, 16]):
        P = N // l
        b = h.reshape(P, l, P, l)
        brute = np.mean(np.mean(b ** 2, axis=(1, 3)) - np.mean(b, axis=(1, 3)) ** 2)
        assert wl ** 2 == pytest.approx(brute, rel=1e-12, abs=1e-15)
        if (2 * a0) % P or (2 * a1) % P:
            D = D1(a0, l) * D1(a1, l)
            assert wl ** 2 == pytest.approx(A * A / 2 * (1 - D * D), rel=1e-12, abs=1e-15)


def test_largest_box_is_the_global_width():
    s, p = _sim((32, 32), ic_kind=1, ic_sigma=0.4, R=3, seed=3)
    s.step(2)
    assert s.observe(O.OBS_BOXWIDTH)[-1] == pytest.approx(s.observe(O.OBS_WIDTH)[0], rel=1e-12)


def test_white_noise_box_variance():
    """i.i.d. N(0, s^2) sites: E w_l^2 = s^2 (1 - 1/l^d) (the box mean of l^d
    independent sites has variance s^2/l^d)."""
    sig, R = 0.3, 64
    s, p = _sim((32, 32), ic_kind=1, ic_sigma=sig, R=R, seed=8)
    w = s.observe(O.OBS_BOXWIDTH)
    for wl, l in zip(w, [2, 4, 8, 16, 32]):
        want = sig * sig * (1 - 1.0 / l ** 2)
        # relative SE of a sample variance over R 32^2 sites: ~ sqrt(2 / (R 32^2))
        assert abs(wl ** 2 - want) < 6 * want * np.sqrt(2.0 / (R * 1024)) + 1e-15


def test_white_noise_box_variance_on_a_line():
    """1D (the line of the KPZ scaling figure): i.i.d. sites give
    E w_l^2 = s^2 (1 - 1/l), and a plane wave's box variances equal the brute
    force over the grid."""
    sig, R, N = 0.3, 64, 256
    p = W.kpz([N], dealias=0, realizations=R, precision=64, ic_kind=1, ic_sigma=sig, seed=4)
    s = O.Sim(p)
    w = s.observe(O.OBS_BOXWIDTH)
    assert len(w) == 8
    for wl, l in zip(w, [2 ** j for j in range(1, 9)]):
        want = sig * sig * (1 - 1.0 / l)
        assert abs(wl ** 2 - want) < 6 * want * np.sqrt(2.0 / (R * N)) + 1e-15
    p = W.kpz([16], dealias=0, realizations=1, precision=64, ic_kind=0)
    s = O.Sim(p)
    A, m = 0.7, 3
    spec = np.zeros(s.spec_shape, dtype=complex)
    spec[m] = 16 * A / 2
    s.set(0, spec)
    h = A * np.cos(2 * np.pi * m * np.arange(16) / 16)
    for wl, l in zip(s.observe(O.OBS_BOXWIDTH), [2, 4, 8, 16]):
        b = h.reshape(16 // l, l)
        brute = np.mean(np.mean(b ** 2, axis=1) - np.mean(b, axis=1) ** 2)
        assert wl ** 2 == pytest.approx(brute, rel=1e-12, abs=1e-15)
