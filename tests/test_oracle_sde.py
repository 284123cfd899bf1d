"""Pins of the oracle's scalar SETD schemes (Sec. 2; tests of Sec. 3):
du = (c u + f1 u + f3 u^3) dt + (g0 + g1 u) dW."""
import numpy as np
import pytest

from oracle import oracle as O


def _gbm_strong_error(scheme, lam, mu, delta, h, paths=20000, seed=5):
    n = int(round(1.0 / h))
    u, w = O.sde_run(scheme, lam - delta, h, n, paths, seed, u0=1.0, f1=delta, g1=mu)
    U = np.exp((lam - 0.5 * mu * mu) * 1.0 + mu * w)   # exact GBM on the same path
    return np.mean(np.abs(u - U))


@pytest.mark.parametrize("delta", [0.0, 2.0])
def test_gbm_strong_orders(delta):
    """Against GBM's exact solution on the same Brownian path (Eq. gbm-analytical):
    SETD-Milstein converges with strong order 1, SETD-EM with 1/2 (Sec. 3)."""
    lam, mu = 2.0, 1.0
    for scheme, lo, hi in [(O.SDE_MILSTEIN, 1.7, 2.3), (O.SDE_EM, 1.2, 1.65)]:
        e = [_gbm_strong_error(scheme, lam, mu, delta, 2.0 ** -k) for k in (5, 6, 7)]
        r = [e[0] / e[1], e[1] / e[2]]
        assert all(lo < x < hi for x in r), (scheme, delta, e)


def test_setd1_is_exact_in_distribution_for_ou_at_any_step():
    """Additive noise, F = 0 (SAO with b = 0): SETD1 draws the exact transition,
    u_n ~ N(u0 e^{c t}, g0^2 (e^{2 c t} - 1)/(2c)) even for h = 0.5."""
    c, g0, u0, h, n, P = -2.0, 1.5, 3.0, 0.5, 3, 200000
    u, _ = O.sde_run(O.SDE_SETD1, c, h, n, P, 9, u0=u0, g0=g0)
    t = n * h
    m, v = u0 * np.exp(c * t), g0 * g0 * (np.exp(2 * c * t) - 1) / (2 * c)
    assert abs(u.mean() - m) < 5 * np.sqrt(v / P)
    assert abs(u.var() - v) < 5 * v * np.sqrt(2.0 / P)


def test_setd_em_stationary_variance_is_the_midpoint_variance():
    """SETD-EM with additive noise takes the kick e^{ch/2} G dW: its stationary
    variance is e^{ch} h g0^2 / (1 - e^{2ch}) (the midpoint rule of Sec. 2),
    not the exact g0^2 / (2|c|); at h = 0.8 the two differ by 10%."""
    c, g0, h, P = -1.0, 1.0, 0.8, 200000
    u, _ = O.sde_run(O.SDE_EM, c, h, 30, P, 11, u0=0.0, g0=g0)
    v = np.exp(c * h) * h * g0 * g0 / (1 - np.exp(2 * c * h))
    assert abs(u.var() - v) < 5 * v * np.sqrt(2.0 / P)
    assert abs(v - g0 * g0 / (2 * abs(c))) > 10 * v * np.sqrt(2.0 / P)


@pytest.mark.parametrize("z", [0.0, 0.5, 1.0])
def test_one_step_mean_square_matches_the_stability_table(z):
    """GBM, c = z lambda, delta = (1 - z) lambda: the one-step mean square
    <S(h)^2> of each scheme is the expression of the paper's stability table."""
    lam, mu, h, P = -1.5, 1.2, 0.3, 400000
    c, delta = z * lam, (1 - z) * lam
    f1 = np.exp(c * h)
    f2 = (np.exp(c * h) - 1) / c if c != 0 else h
    f3 = np.exp(c * h / 2)
    f4 = np.sqrt((np.exp(2 * c * h) - 1) / (2 * c)) if c != 0 else np.sqrt(h)
    a = f1 + f2 * delta
    want = {O.SDE_EM: a * a + h * (f3 * mu) ** 2,
            O.SDE_MILSTEIN: a * a + h * (f3 * mu) ** 2 + 0.5 * h * h * (f3 * mu * mu) ** 2,
            O.SDE_SETD1: a * a + (f4 * mu) ** 2}
    for scheme, w in want.items():
        u, _ = O.sde_run(scheme, c, h, 1, P, 13, u0=1.0, f1=delta, g1=mu)
        s2 = u * u
        assert abs(s2.mean() - w) < 5 * s2.std() / np.sqrt(P), (scheme, z, s2.mean(), w)


def test_sao_reaches_the_boltzmann_distribution():
    """SAO (Eq. sao) with Gamma = 5, T = 6, b = 0.01: SETD1 at h = 0.01 samples
    P(u) ~ exp(-V(u)/T), V = u^2/2 + b u^4/4; <u^2> and <u^4> by quadrature."""
    G, T, b, h, P = 5.0, 6.0, 0.01, 0.01, 40000
    u, _ = O.sde_run(O.SDE_SETD1, -G, h, 600, P, 17, u0=0.0, f3=-G * b, g0=np.sqrt(2 * G * T))
    x = np.linspace(-40, 40, 400001)
    wgt = np.exp(-(0.5 * x * x + 0.25 * b * x ** 4) / T)
    m2 = np.trapezoid(x * x * wgt, x) / np.trapezoid(wgt, x)
    m4 = np.trapezoid(x ** 4 * wgt, x) / np.trapezoid(wgt, x)
    assert abs(np.mean(u * u) - m2) < 5 * np.sqrt((m4 - m2 * m2) / P)
    assert abs(np.mean(u ** 4) - m4) < 0.05 * m4


def test_invalid_descriptors_are_rejected():
    with pytest.raises(RuntimeError):
        O.sde_run(3, -1.0, 0.1, 1, 1, 0)
    with pytest.raises(RuntimeError):
        O.sde_run(0, -1.0, 0.0, 1, 1, 0)
