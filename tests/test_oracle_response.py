"""Pins of the oracle's linear-response observable: the susceptibility by the
noise correlation (App. C, Onsager-Machlup), in the discrete form
R_a(n, n') = <phi_a(n) conj xi_a(n')> / G_a^2 with xi_a(n') = G_a eta_a(n') the
kick of the step taken from n' (Stein's lemma: the mean response of phi_a(n) to
an additive kick in that step)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2511_22510_amd import workloads as W


def _shell_mean(s, vals):
    """Weighted shell means of a per-mode array, weights as the observables use
    (interior modes of a real field count twice)."""
    nb = s.nbins
    shape = s.spec_shape
    n = s.p["n"][: s.p["ndim"]]
    dk = [2 * np.pi / (ni * s.p.get("dx", 1.0)) for ni in n]
    idx = np.indices(shape).reshape(len(shape), -1)
    a = [np.where(idx[i] < n[i] // 2, idx[i], idx[i] - n[i]) if (i < len(n) - 1 or s.p.get("complex_field")) else idx[i]
         for i in range(len(shape))]
    a2 = sum(ai.astype(np.int64) ** 2 for ai in a)
    shell = np.ceil(np.sqrt(a2) - 1e-12).astype(int)
    last = idx[-1]
    w = np.where((not s.p.get("complex_field")) & (last > 0) & (2 * last < n[-1]), 2.0, 1.0)
    v = np.asarray(vals).reshape(-1)
    num = np.bincount(shell, weights=w * v, minlength=nb)[:nb]
    den = np.bincount(shell, weights=w, minlength=nb)[:nb]
    return num / np.where(den > 0, den, 1), den


@pytest.mark.parametrize("order", [1, 2])
def test_linear_theory_response_is_causal_greens_function(order):
    """F = 0: phi_a(n) = E_a^(n-n') phi_a(n') + sum_m E_a^(n-1-m) xi_a(m), so the
    estimator has mean 0 for n = n' and E_a^(n-n'-1) after; z-tests per shell."""
    R = 512
    p = W.model_a([16, 16], dealias=0, ic_kind=0, T=1.0, r=1.0, u=0.0, h=0.1, realizations=R,
                  precision=64, order=order, seed=31)
    s = O.Sim(p)
    s.p = p
    s.step(3)
    assert s.observe(O.OBS_KICK)[0] == 3
    E = np.real(s.coef(0)).reshape(-1)
    nb = s.nbins
    worst = 0.0
    for m in range(0, 5):
        out = s.observe(O.OBS_RESPONSE)
        got, cnt = out[:nb], out[2 * nb:]
        want, den = _shell_mean(s, E ** (m - 1) if m >= 1 else np.zeros_like(E))
        assert np.allclose(cnt, den)
        # per mode and realization the estimator's variance is at most
        # 1/(1 - E^2) + 1 (the stationary |phi|^2/G^2 plus the kick itself)
        var = 1.0 / (1.0 - np.max(E) ** 2) + 1.0
        se = np.sqrt(2.0 * var / (R * np.maximum(cnt, 1)))
        z = np.abs(got - want) / se
        worst = max(worst, float(np.max(z[cnt > 0])))
        assert np.all(np.abs(out[nb:2 * nb]) < 5 * se)
        s.step(1)
    assert worst < 5.0


@pytest.mark.parametrize("p", [
    W.model_a([16, 16], ic_kind=1, ic_sigma=0.5, T=1.0, r=-1.0, u=1.0, h=0.05, realizations=256, precision=64,
              order=2, seed=41),
    W.kpz([16, 16], ic_kind=1, ic_sigma=0.3, realizations=256, precision=64, seed=42),
    W.cgl([16, 16], ic_kind=1, ic_sigma=0.3, realizations=256, precision=64, seed=43),
])
def test_response_one_step_after_the_kick_is_one_for_any_model(p):
    """The kick enters phi(n'+1) additively next to E phi(n') and the
    nonlinear terms of earlier states, which it does not affect: the mean
    response one step later is exactly 1, whatever the nonlinearity.  The
    standard error comes from 16 independent groups of realizations."""
    groups = []
    for g in range(16):
        s = O.Sim(p, r_first=16 * g, r_count=16)
        s.step(4)
        s.observe(O.OBS_KICK)
        s.step(1)
        nb = s.nbins
        out = s.observe(O.OBS_RESPONSE)
        groups.append(out[:nb])
        cnt = out[2 * nb:]
    x = np.array(groups)
    sel = cnt > 0
    mean, se = x.mean(axis=0)[sel], x.std(axis=0, ddof=1)[sel] / 4.0
    z = np.abs(mean - 1.0) / se
    assert np.max(z) < 5.0
    # and the same for all shells together (weights cnt)
    tot = (x[:, sel] * cnt[sel]).sum(axis=1) / cnt[sel].sum()
    assert abs(tot.mean() - 1.0) < 5.0 * tot.std(ddof=1) / 4.0


def test_response_needs_a_kick():
    s = O.Sim(W.model_a([8, 8], dealias=0, ic_kind=0, realizations=1, precision=64))
    with pytest.raises(RuntimeError):
        s.observe(O.OBS_RESPONSE)
