"""Pins of the ETD coefficients (Eq. SETD1, Eq. SETD2, Sec. 4 step 3) against
50-digit mpmath evaluations of the defining closed forms."""
import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O
from paper_2511_22510_amd import workloads as W

mp.mp.dps = 50


def mp_phi1(x):
    x = mp.mpc(x)
    return mp.expm1(x) / x if x != 0 else mp.mpf(1)


def mp_phi2(x):
    x = mp.mpc(x)
    return (mp.expm1(x) - x) / x**2 if x != 0 else mp.mpf(1) / 2


def _grid():
    pts = []
    for mag in [1e-12, 1e-8, 1e-4, 1e-2, 0.3, 0.999, 1.0, 1.001, 3.0, 30.0, 700.0]:
        for ang in [0.0, np.pi, np.pi / 2, 2.0, -0.7]:
            pts.append(complex(mag * np.cos(ang), mag * np.sin(ang)))
    return pts


@pytest.mark.parametrize("x", _grid())
def test_phi_functions_against_mpmath(x):
    p1, p2 = O.phi12(x)
    r1 = complex(mp_phi1(x))
    r2 = complex(mp_phi2(x))
    # relative to the value, with a floor for the e^{-700}-sized imaginary noise
    assert abs(p1 - r1) <= 4e-15 * abs(r1) + 1e-300
    assert abs(p2 - r2) <= 4e-15 * abs(r2) + 1e-300


def test_limits_and_continuity():
    p1, p2 = O.phi12(0.0)
    assert p1 == 1.0 and p2 == 0.5
    # both branches (series inside |x| < 1, closed form outside) stay accurate
    # right at the switch, so the coefficients have no jump there
    for ang in np.linspace(0, 2 * np.pi, 13):
        for scale in (1 - 1e-12, 1 + 1e-12):
            x = complex(np.cos(ang), np.sin(ang)) * scale
            a = O.phi12(x)
            assert abs(a[0] - complex(mp_phi1(x))) <= 4e-15 * abs(complex(mp_phi1(x)))
            assert abs(a[1] - complex(mp_phi2(x))) <= 4e-15 * abs(complex(mp_phi2(x)))


@pytest.mark.parametrize("x", [0.37, -2.5, 1e-3, complex(0.2, -0.9), complex(-3.0, 4.0)])
def test_setd2_weights_are_the_printed_ones(x):
    """Eq. SETD2 prints [(1+ch)e^{ch}-1-2ch]/(c^2 h) and [1+ch-e^{ch}]/(c^2 h);
    the oracle uses h(phi1+phi2) and -h phi2.  Equal at 50 digits."""
    h = mp.mpf("0.01")
    c = mp.mpc(x) / h
    ch = c * h
    w_now = ((1 + ch) * mp.exp(ch) - 1 - 2 * ch) / (c**2 * h)
    w_prev = (1 + ch - mp.exp(ch)) / (c**2 * h)
    p1, p2 = mp_phi1(ch), mp_phi2(ch)
    assert abs(w_now - h * (p1 + p2)) < mp.mpf(10) ** -40
    assert abs(w_prev + h * p2) < mp.mpf(10) ** -40
    # and the oracle's double-precision phi's reproduce them
    q1, q2 = O.phi12(complex(ch))
    assert abs(0.01 * (q1 + q2) - complex(w_now)) <= 1e-16 * 10
    assert abs(-0.01 * q2 - complex(w_prev)) <= 1e-16 * 10


def test_per_mode_coefficients_of_a_problem():
    """E = e^{ch}, noise amplitude G = (N^2/L)^{d/2} sqrt(D/c (e^{2ch}-1)) of Sec. 4
    step 3, for Model B (c = -k^2(r+k^2), D(k) = T k^2) on a 16 x 32 lattice."""
    p = W.model_b([16, 32], dx=0.7, h=0.05, order=2, dealias=0, ic_kind=0)
    s = O.Sim(p)
    E, wa, wb, G, k2 = (s.coef(i) for i in range(5))
    r, T, h = -1.0, 0.05, 0.05
    L = np.array([16 * 0.7, 32 * 0.7])
    lat = np.sqrt(16**2 / L[0]) * np.sqrt(32**2 / L[1])
    it = np.nditer(k2, flags=["multi_index"])
    for kk in it:
        kk = float(kk)
        c = mp.mpf(-kk * (r + kk))
        ch = c * h
        assert abs(E[it.multi_index] - complex(mp.exp(ch))) < 1e-15 * 4
        if kk == 0:
            assert G[it.multi_index] == 0.0
            continue
        if c == 0:
            var = 2 * T * kk * h
        else:
            var = (T * kk) / c * (mp.exp(2 * ch) - 1)
        g = lat * float(mp.sqrt(var))
        assert abs(G[it.multi_index] - g) <= 1e-14 * g
        ra = complex(h * (mp_phi1(ch) + mp_phi2(ch)))
        rb = complex(-h * mp_phi2(ch))
        assert abs(wa[it.multi_index] - ra) <= 4e-16 * abs(ra)
        assert abs(wb[it.multi_index] - rb) <= 4e-16 * abs(rb)
