"""Pins of the oracle's time-frequency observables (App. C dynamic correlations
C(k, w) and susceptibility chi(k, w), the quantities of the FDT check of Sec. 5)
recorded over a window of M steps."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2511_22510_amd import workloads as W


def _linear(R, seed, order=1):
    return W.model_a([16, 16], dealias=0, ic_kind=0, T=1.0, r=1.0, u=0.0, h=0.05, realizations=R,
                     precision=64, order=order, seed=seed)


def _record(s, M, with_sk=False):
    s.series_start(M)
    sk = []
    for m in range(M):
        if with_sk:
            sk.append(s.observe(O.OBS_SK)[:s.nbins])
        if m < M - 1:
            s.step(1)
    return sk


def test_frequency_sum_of_c_is_the_time_sum_of_s():
    """Parseval over the window, exact: sum_b C(k, w_b) = h sum_m S(k, t_m)
    (shell means with the same mode weights)."""
    p = W.model_a([16, 16], ic_kind=1, ic_sigma=0.5, r=-1.0, u=1.0, h=0.02, realizations=3, precision=64, seed=5)
    s = O.Sim(p)
    s.step(10)
    sk = _record(s, 16, with_sk=True)
    C, Xr, Xi, cnt = s.spectrum()
    assert np.allclose(C.sum(axis=1), p["h"] * np.sum(sk, axis=0), rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("order", [1, 2])
def test_linear_theory_matches_the_exact_window_expectations(order):
    """F = 0, stationary: phi_a(m+1) = E phi_a(m) + xi_a(m) with <|xi|^2> = G^2,
    so over a window of M samples
      <|phi_b|^2>           = C0 [M + 2 Re sum_d (M - d)(E e^{i th})^d],  C0 = G^2/(1 - E^2),
      <phi_b conj xi_b>     = G^2 sum_d (M - d) e^{i th d} E^{d - 1},        th = 2 pi b / M,
    the finite-window forms of the paper's C(k, w) and chi(k, w) (their FDT
    2 Im chi = (w/D) C is reached as M -> infinity and h -> 0).  z-tests per
    shell and frequency with standard errors from 16 realization groups."""
    M, groups, per = 16, 16, 16
    res = []
    for g in range(groups):
        s = O.Sim(_linear(groups * per, 7, order), r_first=g * per, r_count=per)
        s.step(300)   # E^300 < 1e-6 for every mode: stationary
        _record(s, M)
        res.append(s.spectrum())
    C = np.array([r[0] for r in res])
    X = np.array([r[1] + 1j * r[2] for r in res])
    cnt = res[0][3]
    s = O.Sim(_linear(1, 7, order))
    E = np.real(s.coef(0)).reshape(-1)
    G = s.coef(3).reshape(-1)
    p = _linear(1, 7, order)
    vol = (p["n"][0] * p["dx"] / p["n"][0] ** 2) ** 2 if "dx" in p else (1.0 / 16) ** 2
    h, D = p["h"], p["noise_D"]
    th = 2 * np.pi * np.arange(M) / M
    d = np.arange(1, M)
    # shell of every stored mode and its weight (interior modes of the real field: 2)
    shape = s.spec_shape
    i0, i1 = np.indices(shape).reshape(2, -1)
    a0 = np.where(i0 < 8, i0, i0 - 16)
    shell = np.ceil(np.sqrt(a0 ** 2 + i1 ** 2) - 1e-12).astype(int)
    w = np.where((i1 > 0) & (2 * i1 < 16), 2.0, 1.0)
    EC = np.zeros((s.nbins, M))
    EX = np.zeros((s.nbins, M), dtype=complex)
    for e in range(E.size):
        if not G[e] > 0:
            continue
        C0 = G[e] ** 2 / (1 - E[e] ** 2)
        ec = np.array([C0 * (M + 2 * np.real(np.sum((M - d) * (E[e] * np.exp(1j * t)) ** d))) for t in th])
        ex = np.array([G[e] ** 2 * np.sum((M - d) * np.exp(1j * t * d) * E[e] ** (d - 1)) for t in th])
        EC[shell[e]] += w[e] * vol * h / M * ec
        EX[shell[e]] += w[e] * vol / (2 * D * M) * ex
    sel = cnt > 0
    EC[sel] /= cnt[sel, None]
    EX[sel] /= cnt[sel, None]
    z = []
    for est, want in [(C, EC), (X.real, EX.real), (X.imag, EX.imag)]:
        mean, se = est.mean(axis=0)[sel], est.std(axis=0, ddof=1)[sel] / np.sqrt(groups)
        # entries that vanish by symmetry (Im chi at w = 0 and the Nyquist
        # frequency) have a standard error at rounding level
        floor = 1e-12 * np.max(np.abs(want[sel]))
        z.append((mean - want[sel]) / np.sqrt(se * se + floor * floor))
    z = np.concatenate([v.reshape(-1) for v in z])
    assert np.max(np.abs(z)) < 6.0
    assert 0.5 < np.mean(z * z) < 1.8


def test_spectrum_needs_a_full_window():
    s = O.Sim(_linear(2, 1))
    s.series_start(8)
    s.step(3)
    with pytest.raises(RuntimeError):
        s.spectrum()


def _exact_fdt(N, dx, r, D, h, M):
    """Average |E Delta_{a,b}| and signed average E Delta of linear Model A in
    the stationary state, from the exact window expectations of |phi_b|^2 and
    phi_b conj xi_b (SETD1 is the exact OU transition)."""
    L = N * dx
    vol, lat = L / (N * N), N * N / L
    d = np.arange(1, M)
    sabs = ssgn = 0.0
    for a in range(-N // 2, N // 2):
        k = 2 * np.pi * a / L
        c = -(r + k * k)
        E = np.exp(c * h)
        G2 = lat * D * np.expm1(2 * c * h) / c
        C0 = G2 / (1 - E * E)
        for b in range(M):
            bs = b if 2 * b < M else b - M
            th = 2 * np.pi * b / M
            phib2 = C0 * (M + 2 * np.real(np.sum((M - d) * (E * np.exp(1j * th)) ** d)))
            cross = G2 * np.sum((M - d) * np.exp(1j * th * d) * E ** (d - 1))
            delta = vol / (D * M) * (cross.imag - 2 * np.pi * bs / M * phib2)
            sabs += abs(delta)
            ssgn += delta
    return sabs / (N * M), ssgn / (N * M)


def test_fdt_deviation_matches_the_exact_window_expectation():
    """FDT check (Sec. 5): per mode and frequency Delta = 2 Im chi - (w/D) C of
    the ensemble means.  For linear Model A the estimators' exact window
    expectations give E Delta (the finite window and step bias); with 96
    realizations the statistical part is small beside it, so the average
    |Delta| over all modes and frequencies lands on the average |E Delta|."""
    N, dx, r, D, h, M, R = 32, 1.0, 1.0, 0.5, 0.1, 128, 96
    p = W.model_a([N], r=r, u=0.0, T=D, nl="none", h=h, order=1, ic_kind=0, realizations=R, dealias=0,
                  seed=5, dx=dx)
    s = O.Sim(p)
    s.step(100)   # t = 10 >> 1/|c|: stationary
    s.series_start(M)
    s.step(M - 1)
    got_abs, got_sgn = s.fdt()
    want_abs, want_sgn = _exact_fdt(N, dx, r, D, h, M)
    assert got_abs == pytest.approx(want_abs, rel=0.03)
    # the signed average is a sum of cancelling terms: compare on the scale of |Delta|
    assert abs(got_sgn - want_sgn) < 0.03 * want_abs
