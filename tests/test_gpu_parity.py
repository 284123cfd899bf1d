"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Relative error metric: ||phi_gpu - phi_oracle||_2 /
||phi_oracle||_2 over the whole batched spectral state, maximum over the
compared steps.  Bars: 1e-10 in FP64, 2e-4 in FP32 over 100-step trajectories.
"""
import sys
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2511_22510_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {64: 1e-10, 32: 2e-4}


def _setd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_22510_amd import setd
    return setd


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def run_pair(p, steps, every=1, r_sample=None, progress=False):
    """Advance GPU (all realizations, one launch per pass) and oracle (the
    sampled realizations) side by side, comparing the sampled states after
    every `every` steps; returns the largest relative error seen (steps 1 to
    `steps`)."""
    S = _setd()
    rs = list(range(p["realizations"])) if r_sample is None else list(r_sample)
    say("case", p["nl"], p["n"], "prec", p["precision"], "R", p["realizations"], "order", p["order"],
        "dealias", p["dealias"], "steps", steps, "compared every", every, "realizations", rs)
    t0 = time.time()
    g = S.Plan(p)
    oracles = [O.Sim(p, r_first=r, r_count=1) for r in rs]
    t_orc = time.time() - t0
    worst = 0.0
    done = 0
    while done < steps:
        k = min(every, steps - done)
        g.step(k)
        t1 = time.time()
        for o in oracles:
            o.step(k)
        t_orc += time.time() - t1
        done += k
        num = sum(np.linalg.norm(g.get(r) - o.get(0)) ** 2 for r, o in zip(rs, oracles))
        den = sum(np.linalg.norm(o.get(0)) ** 2 for o in oracles)
        err = float(np.sqrt(num / max(den, 1e-300)))
        worst = max(worst, err)
        if progress:
            say("  step %d rel err %.3g (oracle %.1f s so far, %d threads)" % (done, err, t_orc, O.threads()))
    g.close()
    say("  oracle wall time %.1f s for %d realization(s) x %d steps" % (t_orc, len(rs), steps))
    return worst


SMALL = [
    W.model_a([64, 64], precision=64, order=1, realizations=2),
    W.model_a([64, 64], precision=32, order=2, realizations=3),
    W.model_b([64, 128], precision=64, realizations=2),
    W.model_b([128, 128], precision=32, realizations=2),
    W.kpz([128, 128], precision=64, realizations=2, ic_kind=1, ic_sigma=0.2),
    W.kpz([64, 64], precision=32, realizations=2),
    W.cgl([32, 32, 32], precision=64, realizations=2),
    W.cgl([16, 32, 64], precision=32, realizations=1),
    W.cgl([64, 64], precision=32, realizations=2, dx=0.5),
    W.model_a([16, 16, 32], precision=64, order=2, realizations=2),
    W.model_a([8, 8], precision=64, order=2, realizations=1),
    W.model_b([32, 32], precision=64, dealias=0, realizations=2),
    W.cgl([16, 16], precision=64, dealias=0, realizations=1),
    W.model_a([32, 32], precision=64, nl="none", u=0.0, r=0.5, realizations=2),
]


@pytest.mark.parametrize("p", SMALL, ids=lambda p: "%s-%s-f%d-o%d-d%d" % (
    p["nl"], "x".join(map(str, p["n"])), p["precision"], p["order"], p["dealias"]))
def test_trajectory_parity_small(p):
    err = run_pair(p, steps=100, every=1)
    say("max rel err", err)
    assert err <= TOL[p["precision"]]


def test_config_a_full_trajectory():
    """Model A, plain SETD1, FP64, one realization, 64^2, h = 0.01, all 1000 steps."""
    p = W.problem(W.CONFIG_A)
    err = run_pair(p, steps=1000, every=1)
    say("config A max rel err", err)
    assert err <= 1e-10


def test_config_b_full_size_sampled():
    """Model B, SETD2, complex64, 64 realizations of 512^2 in one launch: the
    first and last realizations against the oracle after each of 100 steps."""
    p = W.problem(W.CONFIG_B)
    err = run_pair(p, steps=100, every=1, r_sample=[0, 63])
    say("config B max rel err", err)
    assert err <= 2e-4


@pytest.mark.timeout(900)
def test_config_kpz_full_size_100_steps():
    """KPZ, SETD2, FP32, 16 realizations of 1024^2 in one launch (the 1024-point
    transforms, two gradient inverses): realizations 0 and 15 against the
    oracle after each of 100 steps."""
    p = W.problem(W.CONFIG_KPZ)
    err = run_pair(p, steps=100, every=1, r_sample=[0, 15], progress=True)
    say("config KPZ max rel err", err)
    assert err <= 2e-4


@pytest.mark.timeout(1200)
def test_config_cgl_full_size_100_steps():
    """CGL, SETD2, complex64, 4 realizations of 256^3 in one launch per pass
    (the four 3D passes at N = 256): realization 3 against the oracle every 5
    steps over 100 steps."""
    p = W.problem(W.CONFIG_CGL)
    err = run_pair(p, steps=100, every=5, r_sample=[3], progress=True)
    say("config CGL max rel err", err)
    assert err <= 2e-4


# noise drawn per site in real space and transformed (Sec. 4 step 2's
# alternative) on 2D and 3D lattices: real and complex fields, SETD1/SETD2,
# both precisions, anisotropic lattices, the register and tile-sweep axis-0
# kernels (2/3 rule on / off) and the linear kernel
RSN_CASES = [
    W.model_a([64, 64], precision=64, order=2, realizations=2, noise_space=1),
    W.model_b([128, 64], precision=32, realizations=3, noise_space=1),
    W.kpz([128, 128], precision=32, realizations=2, noise_space=1),
    W.kpz([64, 64], precision=64, order=1, realizations=1, ic_kind=1, ic_sigma=0.2, noise_space=1),
    W.cgl([32, 32, 32], precision=64, realizations=2, noise_space=1),
    W.cgl([16, 32, 64], precision=32, realizations=1, noise_space=1),
    W.cgl([64, 64], precision=32, order=1, realizations=2, dx=0.5, noise_space=1),
    W.model_a([16, 16, 32], precision=64, order=2, realizations=2, noise_space=1),
    W.model_a([8, 8, 8], precision=32, order=1, realizations=3, noise_space=1),
    W.model_b([32, 32], precision=64, dealias=0, realizations=2, noise_space=1),
    W.cgl([16, 16], precision=64, dealias=0, realizations=1, noise_space=1),
    W.model_a([32, 32], precision=64, nl="none", u=0.0, r=0.5, realizations=2, noise_space=1),
]


@pytest.mark.parametrize("p", RSN_CASES, ids=lambda p: "rs-%s-%s-f%d-o%d-d%d" % (
    p["nl"], "x".join(map(str, p["n"])), p["precision"], p["order"], p["dealias"]))
def test_real_space_noise_parity(p):
    """The GPU draws the site noise of each step (Philox blocks (x mod Q, n,
    r, 3)), transforms it over every axis and scales by 1/sqrt(prod n); the
    oracle draws the same sites and transforms them with its own FFT."""
    err = run_pair(p, steps=100, every=1)
    say("max rel err", err)
    assert err <= TOL[p["precision"]]


def test_real_space_noise_full_size_model_b():
    """Real-space noise at the Model B workload's size (512^2 x 64, FP32): the
    first and last realizations against the oracle over 30 steps."""
    p = W.problem(W.CONFIG_B, noise_space=1)
    err = run_pair(p, steps=30, every=1, r_sample=[0, 63])
    say("model B real-space noise max rel err", err)
    assert err <= 2e-4


# phase-shift dealiasing on 2D lattices (reading 25: the mean over the four
# grids moved by dx/2 along no axis, either axis or both): real and complex
# fields, both precisions and orders, anisotropic lattices, the largest axis-0
# tile (64 KiB of LDS at N0 = 1024 in FP32 and N0 = 512 in FP64)
PS_CASES = [
    W.model_a([64, 64], precision=64, order=2, realizations=2, dealias=2),
    W.model_a([32, 64], precision=32, order=1, realizations=3, dealias=2),
    W.model_b([64, 64], precision=32, realizations=2, dealias=2),
    W.cgl([32, 32], precision=64, realizations=2, dealias=2),
    W.cgl([64, 32], precision=32, order=1, realizations=1, dx=0.5, dealias=2),
    W.model_a([16, 16], precision=64, order=2, realizations=1, ic_sigma=0.4, dealias=2),
    W.model_a([8, 8], precision=32, order=2, realizations=2, dealias=2),
    W.model_a([1024, 32], precision=32, order=2, realizations=1, dealias=2),
    W.model_b([512, 16], precision=64, realizations=1, dealias=2),
    W.model_a([32, 32], precision=64, nl="none", u=0.0, r=0.5, realizations=1, dealias=2),
    # 3D: eight grids
    W.model_a([16, 16, 16], precision=64, order=2, realizations=2, dealias=2),
    W.model_a([32, 16, 16], precision=32, order=1, realizations=2, dealias=2),
    W.model_b([16, 32, 16], precision=32, realizations=1, dealias=2),
    W.model_b([16, 16, 16], precision=64, realizations=1, ic_kind=1, ic_sigma=0.3, dealias=2),
    W.cgl([16, 16, 16], precision=64, realizations=2, dealias=2),
    W.cgl([32, 16, 32], precision=32, order=1, realizations=1, dealias=2),
    W.model_a([8, 8, 8], precision=32, order=2, realizations=3, dealias=2),
    # KPZ: four axis-0 inverses, four lines per row pair
    W.kpz([64, 64], precision=64, order=2, realizations=2, ic_kind=1, ic_sigma=0.2, dealias=2),
    W.kpz([32, 128], precision=32, realizations=2, ic_kind=1, ic_sigma=0.2, dealias=2),
    W.kpz([16, 1024], precision=64, realizations=1, ic_kind=1, ic_sigma=0.1, dealias=2),
    W.kpz([8, 8], precision=32, order=1, realizations=3, dealias=2),
    W.kpz([64, 32], precision=32, realizations=1, ic_kind=1, ic_sigma=0.2, dealias=2, noise_space=1),
    # with the noise drawn in real space
    W.model_b([32, 64], precision=64, realizations=2, dealias=2, noise_space=1),
    W.cgl([32, 32], precision=32, realizations=1, dealias=2, noise_space=1),
    W.model_a([16, 16, 32], precision=32, order=1, realizations=2, dealias=2, noise_space=1),
    W.cgl([16, 16, 16], precision=64, realizations=1, dealias=2, noise_space=1),
]


@pytest.mark.parametrize("p", PS_CASES, ids=lambda p: "ps-%s-%s-f%d-o%d-n%d" % (
    p["nl"], "x".join(map(str, p["n"])), p["precision"], p["order"], p.get("noise_space", 0)))
def test_phase_shift_lattice_parity(p):
    """The row pass evaluates the nonlinearity on the rows and on the rows
    moved by dx/2, for pre and for its axis-0-shifted copy (3D: for the four
    grids the axis-1 pass makes of them, moved or not along axis 1); the
    passes after it fold the grids back, and the axis-0 pass combines the last
    two; the oracle averages its 2^d shifted evaluations directly."""
    err = run_pair(p, steps=100, every=1)
    say("max rel err", err)
    assert err <= TOL[p["precision"]]


def _nan_workspace(nbytes):
    """A workspace whose every byte pattern is a NaN (0xff), as memory left by
    earlier work may hold anything."""
    import torch
    buf = torch.full((max(int(nbytes), 256),), 0xff, dtype=torch.uint8, device="cuda")
    return buf, buf.data_ptr(), torch.cuda.current_stream().cuda_stream


@pytest.mark.parametrize("p", [W.model_b([32, 32], precision=64, realizations=2, ic_kind=0, dealias=2),
                               W.cgl([16, 16, 16], precision=32, realizations=1, ic_kind=0, dealias=2),
                               W.kpz([32, 64], precision=64, realizations=2, dealias=2)],
                         ids=["model_b-2d", "cgl-3d", "kpz-2d"])
def test_phase_shift_plans_start_from_a_dirty_workspace(p):
    """Binding clears every array a step reads before writing it, also the
    shifted intermediates of a phase-shift plan whose initial field is zero
    (no initial-condition pass writes them): the trajectory in a workspace
    filled with NaN bytes matches the oracle."""
    S = _setd()
    g = S.Plan(p, workspace=_nan_workspace)
    o = O.Sim(p)
    for _ in range(3):
        g.step(4)
        o.step(4)
        err = max(relerr(g.get(r), o.get(r)) for r in range(p["realizations"]))
        say("dirty workspace", p["nl"], p["n"], "err", err)
        assert err <= TOL[p["precision"]]
    g.close()


@pytest.mark.parametrize("history", [0, 1])
@pytest.mark.parametrize("prec", [32, 64])
def test_long_model_a_stays_on_the_oracle(prec, history):
    """Model A with r < 0 has Re c > 0 near k = 0, where an anti-Hermitian part
    of the a_last = 0 plane (transform round-off, invisible in real space)
    would grow like e^{c t}: without keeping the plane Hermitian the FP32 run
    blows up near step 2000 (t = 20).  3000 steps stay within the bars."""
    p = W.model_a([128, 128], order=2, precision=prec, realizations=1, seed=7373773241406430705,
                  history_readback=history)
    err = run_pair(p, steps=3000, every=1000)
    say("long model A f%d history %d err %.3g" % (prec, history, err))
    assert err <= TOL[prec]


def test_long_model_a_3d_stays_on_the_oracle():
    """The same for a 3D real field, whose a_last = 0 plane pairs span blocks
    of the axis-0 pass (a separate Hermitian pass after each step)."""
    p = W.model_a([32, 32, 32], order=2, precision=32, realizations=1, seed=11, h=0.02)
    err = run_pair(p, steps=1500, every=500)
    say("long model A 3D err %.3g" % err)
    assert err <= 2e-4


@pytest.mark.timeout(600)
def test_fp64_plain_model_b_full_size():
    """The plain FP64 per-realization run the batched FP32 path is measured
    against: 512^2, SETD2, compared after each of 100 steps."""
    p = W.problem(W.CONFIG_B, precision=64, realizations=1)
    err = run_pair(p, steps=100, every=1, progress=False)
    say("model B fp64 max rel err", err)
    assert err <= 1e-10


def test_set_field_history_and_restart():
    S = _setd()
    p = W.model_b([64, 64], precision=64, realizations=2, history_readback=1)
    g = S.Plan(p)
    o = O.Sim(p)
    x = W.random_spectrum(p, 11, 0.05)
    g.set(1, x)
    o.set(1, x)
    g.step(7)
    o.step(7)
    for r in range(2):
        assert relerr(g.get(r), o.get(r)) <= 1e-10
        assert relerr(g.history(r), o.get(r, which=1)) <= 1e-10
    g.set_step(1000)
    o.set_step(1000)
    g.step(3)
    o.step(3)
    assert max(relerr(g.get(r), o.get(r)) for r in range(2)) <= 1e-10
    out = g.observe(S.OBS_STEP)
    assert out[0] == 1003 and out[1] == 0


def test_lean_set_field_and_set_step_match_oracle():
    """SETD2 keeping only the carry E phi_n + w_b F_{n-1} + G eta_n: a state set
    mid-run restarts the carry (F_{-1} = F_0), a new step index re-draws the
    carry's noise, and F_{n-1} is not readable."""
    S = _setd()
    for prec, tol in ((64, 1e-10), (32, 2e-4)):
        p = W.model_b([64, 64], precision=prec, realizations=2)
        g = S.Plan(p)
        o = O.Sim(p)
        g.step(4)
        o.step(4)
        x = W.random_spectrum(p, 11, 0.05)
        g.set(1, x)
        o.set(1, x)
        g.step(7)
        o.step(7)
        assert max(relerr(g.get(r), o.get(r)) for r in range(2)) <= tol
        g.set_step(1000)
        o.set_step(1000)
        g.step(3)
        o.step(3)
        assert max(relerr(g.get(r), o.get(r)) for r in range(2)) <= tol
        with pytest.raises(S.SetdError) as e:
            g.history(0)
        assert e.value.status == S.SETD_E_UNSUPPORTED
        g.close()


@pytest.mark.parametrize("prec", [64, 32])
def test_lean_and_separate_storage_agree(prec):
    """The two SETD2 storages compute Eq. SETD2 with different groupings: the
    trajectories agree to rounding, and reading phi from the carry plan (a
    recovery from pre) leaves its trajectory bitwise unchanged."""
    S = _setd()
    base = W.kpz([64, 64], precision=prec, realizations=2, ic_kind=1, ic_sigma=0.2)
    lean = S.Plan(dict(base, history_readback=0))
    sep = S.Plan(dict(base, history_readback=1))
    quiet = S.Plan(dict(base, history_readback=0))
    worst = 0.0
    for _ in range(5):
        lean.step(6)
        sep.step(6)
        quiet.step(6)
        for r in range(2):
            worst = max(worst, relerr(lean.get(r), sep.get(r)))
    say("lean vs separate storage, f%d: %.3g" % (prec, worst))
    assert worst <= (1e-12 if prec == 64 else 2e-5)
    for r in range(2):
        assert np.array_equal(quiet.get(r), lean.get(r))
    for g in (lean, sep, quiet):
        g.close()


@pytest.mark.parametrize("p", [W.model_b([64, 64], precision=32, realizations=5),
                               W.cgl([32, 32, 32], precision=64, realizations=3),
                               W.kpz([64, 64], precision=32, realizations=2, ic_kind=1, ic_sigma=0.2)])
def test_split_streams_match_one_stream(p, monkeypatch):
    """Stepping the two halves of the realizations on two streams runs the same
    kernels on the same data: bitwise the trajectory of one stream, and the
    observables after it agree (to the rounding of their FP64 atomic sums,
    whose order depends on block timing)."""
    S = _setd()
    monkeypatch.setenv("SETD_VARIANT", "1,4,1")
    one = S.Plan(p)
    monkeypatch.setenv("SETD_SPLIT", "2")
    two = S.Plan(p)
    assert int(one.info.streams) == 1 and int(two.info.streams) == 2
    for _ in range(3):
        one.step(7)
        two.step(7)
        for r in range(p["realizations"]):
            assert np.array_equal(one.get(r), two.get(r))
    assert np.allclose(one.observe(S.OBS_SK), two.observe(S.OBS_SK), rtol=1e-12, atol=0)
    one.close()
    two.close()


@pytest.mark.parametrize("split", ["1", "2"])
@pytest.mark.parametrize("p", [W.model_b([64, 64], precision=32, realizations=5),
                               W.cgl([32, 32, 32], precision=64, realizations=3),
                               W.kpz([256], precision=32, order=2, realizations=3)])
def test_graph_replays_match_eager_launches(p, split, monkeypatch):
    """setd_step replays a captured graph of 4 steps: every replay, with eager
    steps, field reads and observables between replays, gives bitwise the
    trajectory of kernel launches alone (one stream or two)."""
    S = _setd()
    monkeypatch.setenv("SETD_VARIANT", "1,4,1")
    monkeypatch.setenv("SETD_SPLIT", split)
    monkeypatch.setenv("SETD_GRAPH", "0")
    eager = S.Plan(p)
    monkeypatch.setenv("SETD_GRAPH", "4")
    graph = S.Plan(p)
    assert int(eager.info.graph_steps) == 0 and int(graph.info.graph_steps) == 4
    for n in [8, 3, 4, 13, 1]:   # replays, eager remainders, both
        eager.step(n)
        graph.step(n)
        for r in range(p["realizations"]):
            assert np.array_equal(eager.get(r), graph.get(r)), (n, r)
        assert np.allclose(eager.observe(S.OBS_SK), graph.observe(S.OBS_SK), rtol=1e-12, atol=0)
    eager.close()
    graph.close()


@pytest.mark.parametrize("p", [W.model_a([64, 64], precision=64, realizations=3, order=2),
                               W.model_b([64, 64], precision=32, realizations=4),
                               W.kpz([64, 64], precision=32, realizations=2, ic_kind=1, ic_sigma=0.2),
                               W.cgl([32, 32], precision=32, realizations=2),
                               W.cgl([32, 32, 32], precision=64, realizations=2),
                               W.model_a([16, 16, 16], precision=32, realizations=2, order=2),
                               # phase-shift dealiasing: |a_i| < N_i/2 kept
                               W.model_b([32, 32], precision=64, realizations=2, dealias=2),
                               W.cgl([16, 16, 16], precision=64, realizations=2, dealias=2)])
def test_response_matches_oracle(p):
    """Linear response by the noise correlation (App. C): the device regenerates
    the kick's noise with the step's own generator and precision, divides by the
    table's G, and reduces in FP64; the oracle does the same from its own parts."""
    S = _setd()
    g = S.Plan(p)
    o = O.Sim(p)
    g.step(5)
    o.step(5)
    assert g.observe(S.OBS_KICK)[0] == o.observe(O.OBS_KICK)[0] == 5
    for m, then in ((0, 1), (1, 2), (3, 0)):   # steps since the kick, steps to the next look
        a, b = g.observe(S.OBS_RESPONSE), o.observe(O.OBS_RESPONSE)
        nb = g.nbins
        assert np.array_equal(a[2 * nb:], b[2 * nb:])
        tol = 1e-10 if p["precision"] == 64 else 2e-4
        scale = max(1.0, float(np.max(np.abs(b[:2 * nb]))))
        err = float(np.max(np.abs(a[:2 * nb] - b[:2 * nb]))) / scale
        say("response", p["nl"], p["n"], "f%d" % p["precision"], "m", m, "err", err)
        assert err <= tol
        g.step(then)
        o.step(then)
    g.close()


@pytest.mark.parametrize("p,M", [(W.model_a([32, 32], precision=64, realizations=3, order=2), 16),
                                 (W.model_b([32, 32], precision=32, realizations=2), 32),
                                 (W.kpz([32, 32], precision=32, realizations=2, ic_kind=1, ic_sigma=0.2), 16),
                                 (W.cgl([16, 16, 16], precision=64, realizations=2), 8),
                                 (W.model_a([32, 32], precision=64, realizations=2, order=2, dealias=2), 16)])
def test_spectrum_matches_oracle(p, M):
    """App. C time-frequency observables of a window of M steps: the device
    records the stored spectrum after every step, transforms each mode's
    window and the regenerated kicks along time and reduces per shell and
    frequency in FP64; the oracle transforms by direct sums."""
    S = _setd()
    g = S.Plan(dict(p, series_len=M))
    o = O.Sim(p)
    g.step(5)
    o.step(5)
    assert g.observe(S.OBS_SERIES_START)[0] == 5
    o.series_start(M)
    g.step(M - 2)
    o.step(M - 2)
    with pytest.raises(S.SetdError):
        g.spectrum()   # one sample short
    g.step(1)
    o.step(1)
    a, b = g.spectrum(), o.spectrum()
    assert np.array_equal(a[3], b[3])
    tol = 1e-10 if p["precision"] == 64 else 2e-4
    for x, y, name in zip(a[:3], b[:3], ["C", "Re chi", "Im chi"]):
        err = float(np.max(np.abs(x - y))) / max(float(np.max(np.abs(y))), 1e-300)
        say("spectrum", p["nl"], p["n"], "f%d" % p["precision"], name, "err", err)
        assert err <= tol
    # the window leaves the trajectory alone
    g.step(2)
    o.step(2)
    assert relerr(g.get(0), o.get(0)) <= (1e-10 if p["precision"] == 64 else 2e-4)
    g.close()


@pytest.mark.parametrize("p,M", [(W.model_a([32], r=1.0, u=0.0, T=0.5, nl="none", h=0.1, realizations=24,
                                          dealias=0, ic_kind=0, seed=5), 128),
                                 (W.model_a([32, 32], precision=64, realizations=3, order=2), 16),
                                 (W.model_b([32, 32], precision=32, realizations=2), 32),
                                 (W.cgl([16, 16, 16], precision=64, realizations=2), 8)])
def test_fdt_deviation_matches_oracle(p, M):
    """FDT check of Sec. 5 on a window: the device adds each realization's
    per-mode deviation in FP64 and sums |Delta| over modes and frequencies;
    the oracle forms the per-mode ensemble means directly."""
    S = _setd()
    g = S.Plan(dict(p, series_len=M))
    o = O.Sim(p)
    g.step(6)
    o.step(6)
    with pytest.raises(S.SetdError):
        g.fdt()   # no window yet
    g.observe(S.OBS_SERIES_START)
    o.series_start(M)
    g.step(M - 2)
    o.step(M - 2)
    with pytest.raises(S.SetdError):
        g.fdt()   # one sample short
    g.step(1)
    o.step(1)
    a, b = g.fdt(), o.fdt()
    tol = 1e-10 if p["precision"] == 64 else 1e-3
    say("fdt", p["nl"], p["n"], "f%d" % p["precision"], a, b)
    assert a[0] == pytest.approx(b[0], rel=tol)
    assert abs(a[1] - b[1]) <= tol * b[0]
    g.close()


@pytest.mark.parametrize("p", [W.model_a([64, 64], precision=64, realizations=3, order=2),
                               W.kpz([32, 32], precision=32, realizations=2, dealias=0, ic_kind=1, ic_sigma=0.2),
                               W.kpz([64, 64], precision=64, realizations=2, ic_kind=1, ic_sigma=0.3),
                               W.model_a([16, 16, 16], precision=32, realizations=2),
                               W.cgl([16, 16, 16], precision=64, realizations=2),
                               W.model_a([32, 32], precision=64, realizations=2, dealias=2)])
def test_box_width_matches_oracle(p):
    """Box-averaged width w_l (Sec. 5 KPZ): the device sums the spectrum into
    the alias classes of each box size (no transform); the oracle takes box
    means of the real-space field."""
    S = _setd()
    g = S.Plan(p)
    o = O.Sim(p)
    tol = 1e-10 if p["precision"] == 64 else 2e-4
    for steps in (0, 6):
        g.step(steps)
        o.step(steps)
        a, b = g.box_width(), o.observe(O.OBS_BOXWIDTH)
        assert len(a) == len(b) == int(p["n"][0]).bit_length() - 1
        err = float(np.max(np.abs(a - b) / np.maximum(b, 1e-300)))
        say("boxwidth", p["nl"], p["n"], "f%d" % p["precision"], "steps", steps, "err", err)
        assert err <= tol
    # the largest box is the whole lattice: the global width
    assert a[-1] == pytest.approx(g.observe(S.OBS_WIDTH)[0], rel=1e-9)
    g.close()


@pytest.mark.parametrize("prec", [32, 64])
def test_box_width_full_size_set_state(prec):
    """512^2 Model B, the same seeded spectrum set on both sides."""
    S = _setd()
    p = W.model_b([512, 512], precision=prec, realizations=2, dealias=1)
    g = S.Plan(p)
    o = O.Sim(p)
    for r in range(2):
        x = W.random_spectrum(p, 40 + r, 0.05)
        g.set(r, x)
        o.set(r, x)
    a, b = g.box_width(), o.observe(O.OBS_BOXWIDTH)
    err = float(np.max(np.abs(a - b) / b))
    say("boxwidth 512^2 f%d err" % prec, err)
    assert err <= (1e-10 if prec == 64 else 1e-5)
    g.close()


def test_box_width_needs_equal_axes():
    S = _setd()
    g = S.Plan(W.model_a([32, 64], precision=64, realizations=1))
    with pytest.raises(S.SetdError):
        g.box_width()
    g.close()


def test_observables_match_oracle():
    S = _setd()
    for p in [W.model_a([64, 64], precision=64, realizations=3, order=2),
              W.cgl([32, 32, 32], precision=64, realizations=2),
              W.model_b([32, 32], precision=64, realizations=2, dealias=2),
              W.model_a([16, 16, 16], precision=64, realizations=2, dealias=2)]:
        g = S.Plan(p)
        o = O.Sim(p)
        g.step(5)
        o.step(5)
        nb = g.nbins
        a, b = g.observe(S.OBS_SK), o.observe(O.OBS_SK)
        assert np.allclose(a[nb:], b[nb:])
        assert np.allclose(a[:nb], b[:nb], rtol=1e-11, atol=1e-300)
        a, b = g.observe(S.OBS_WIDTH), o.observe(O.OBS_WIDTH)
        assert a[0] == pytest.approx(b[0], rel=1e-11)
        g.observe(S.OBS_SNAPSHOT)
        o.observe(O.OBS_SNAPSHOT)
        g.step(4)
        o.step(4)
        a, b = g.observe(S.OBS_TWOTIME), o.observe(O.OBS_TWOTIME)
        scale = np.max(np.abs(b[:2 * nb]))
        assert np.max(np.abs(a[:2 * nb] - b[:2 * nb])) <= 1e-11 * scale
        for _ in range(3):
            g.observe(S.OBS_SK_ACCUM)
            o.observe(O.OBS_SK_ACCUM)
            g.step(1)
            o.step(1)
        a, b = g.observe(S.OBS_SK_MEAN), o.observe(O.OBS_SK_MEAN)
        assert np.allclose(a[:nb], b[:nb], rtol=1e-11, atol=1e-300)
        g.close()


def test_fp32_observables_accumulate_in_fp64():
    S = _setd()
    p = W.kpz([128, 128], precision=32, realizations=4, ic_kind=1, ic_sigma=0.5)
    g = S.Plan(p)
    o = O.Sim(p)
    g.step(10)
    o.step(10)
    assert g.observe(S.OBS_WIDTH)[0] == pytest.approx(o.observe(O.OBS_WIDTH)[0], rel=2e-4)


def test_nonfinite_is_flagged_not_faulted():
    """An explicit nonlinearity with a huge step blows up (Sec. 2 warns of this);
    the library reports it and keeps running."""
    S = _setd()
    p = W.model_a([32, 32], precision=32, order=1, h=5.0, ic_kind=1, ic_sigma=3.0, u=50.0)
    g = S.Plan(p)
    g.step(40)
    out, st = g.status_observe(S.OBS_STEP)
    assert st == S.SETD_E_NONFINITE and out[1] == 1


def test_linear_theory_variance_full_size():
    """u = 0 Model A at 512^2 (any size): the stationary variance per shell is
    D/(r + k^2) times (N^2/L)^2, checked statistically after relaxation."""
    S = _setd()
    r, T = 1.0, 0.2
    p = W.model_a([512, 512], r=r, u=0.0, T=T, nl="none", h=0.5, order=1, ic_kind=0,
                  realizations=8, precision=32, dealias=1, seed=77)
    g = S.Plan(p)
    g.step(40)
    out = g.observe(S.OBS_SK)
    nb = g.nbins
    zs = []
    dk = 2 * np.pi / 512
    for b in (1, 5, 20, 60, 120, 170):
        cnt = out[nb + b]
        a = np.arange(-170, 171)
        aa = a[:, None] ** 2 + a[None, :] ** 2
        sel = (np.ceil(np.sqrt(aa) - 1e-12) == b)
        th = np.mean(T / (r + dk**2 * aa[sel]))
        zs.append((out[b] / th - 1) / np.sqrt(2.0 / (cnt * 8)))
    say("z-scores", zs)
    assert np.max(np.abs(zs)) < 4.5


VARIANT_CASES = [
    W.model_b([64, 64], precision=32, realizations=2),
    W.kpz([64, 32], precision=64, realizations=1, ic_kind=1, ic_sigma=0.2),
    W.cgl([32, 32], precision=32, realizations=1),
    W.cgl([16, 32, 32], precision=64, realizations=1),
    W.model_a([8, 16], precision=32, order=2, realizations=3),
    W.kpz([128, 64], precision=32, realizations=2, ic_kind=1, ic_sigma=0.2),
    # five items: groups of 2, 4 and 8 end in a partial group
    W.model_b([64, 64], precision=32, realizations=5),
]


@pytest.mark.parametrize("variant", ["0,0,0", "1,1,1", "2,2,2", "3,3,3", "1,2,3", "3,0,1", "0,4,0", "2,5,3",
                                     "5,4,0", "14,1,1", "11,5,2", "15,0,3", "1,6,1", "0,9,2", "3,11,0",
                                     "1,12,1", "2,15,0"])
@pytest.mark.parametrize("history", [0, 1])
def test_every_kernel_variant_matches_oracle(variant, history, monkeypatch):
    """Each autotuner choice (row: LDS padding x block size x row-pair groups
    per workgroup; axis passes: tile width x columns per thread; axis-0
    variants 4 and up: the register-update kernel at three tile widths, items
    interleaved per tile in groups of 1, 2, 4 or 8) gives the same
    trajectory, with either SETD2 storage (the carry-only storage always
    steps with the register kernel)."""
    monkeypatch.setenv("SETD_VARIANT", variant)
    for p in VARIANT_CASES:
        p = dict(p, history_readback=history)
        err = run_pair(p, steps=12, every=6)
        say("variant", variant, "history", history, p["nl"], p["n"], "err", err)
        assert err <= TOL[p["precision"]]


def test_full_configurations_run_to_completion():
    """The 2D/3D workloads at their full sizes and step counts: Model B 512^2 x 64
    for 10^4 steps keeps every realization's conserved a = 0 mode (c(0) = 0,
    D(0) = 0 and F_0 = 0 by the k^2 factor; the carry storage takes the state
    through an FP32 transform pair every step, so the mode random-walks by
    rounding: within 1e-4 of its column's rms after 10^4 steps, where a
    systematic drift of one rounding per step would reach 6e-4); KPZ 1024^2 x 16 for
    5 10^4 steps stays finite with a growing width; CGL 256^3 x 4 for 2 10^4
    steps stays finite and reaches |A|^2 of order 1 (Parseval over the
    spectrum)."""
    S = _setd()
    p = W.problem(W.CONFIG_B)
    g = S.Plan(p)
    a0 = [g.get(r)[0, 0] for r in range(p["realizations"])]
    g.step(W.CONFIG_B["steps"])
    st = g.observe(S.OBS_STEP)
    assert st[0] == W.CONFIG_B["steps"] and st[1] == 0
    for r in range(p["realizations"]):
        x = g.get(r)
        col = float(np.sqrt(np.mean(np.abs(x[:, 0]) ** 2)))   # scale of the rounding in its transforms
        assert abs(x[0, 0] - a0[r]) <= 1e-4 * col
    g.close()
    p = W.problem(W.CONFIG_KPZ)
    g = S.Plan(p)
    g.step(1000)
    w1 = g.observe(S.OBS_WIDTH)[0]
    g.step(W.CONFIG_KPZ["steps"] - 1000)
    w2 = g.observe(S.OBS_WIDTH)[0]
    say("KPZ 1024^2 width after 1e3 and 5e4 steps", w1, w2)
    assert np.isfinite(w2) and w2 > w1 > 0
    g.close()
    p = W.problem(W.CONFIG_CGL)
    g = S.Plan(p)
    g.step(W.CONFIG_CGL["steps"])
    assert g.observe(S.OBS_STEP)[1] == 0
    spec = g.get(0)
    n3 = float(np.prod(p["n"]))
    a2 = float(np.sum(np.abs(spec) ** 2)) / n3 ** 2
    say("CGL 256^3 mean |A|^2 after 2e4 steps", a2)
    assert 0.3 < a2 < 1.2
    g.close()


@pytest.mark.parametrize("variant", ["1,4,1", "1,6,1", "1,9,1", "1,11,1", "1,13,1", "1,15,1"])
def test_item_groups_are_bitwise_the_same(variant, monkeypatch):
    """The item interleaving of the register axis-0 kernel changes only which
    block runs when: every realization's trajectory is bitwise that of the
    item-after-item order (variant 4 / 5 / 12 at the same tile width)."""
    S = _setd()
    p = W.model_b([128, 128], precision=32, realizations=7)
    v = int(variant.split(",")[1])
    base = "1,%d,1" % (12 if v >= 12 else 4 + (v - 4) % 2)
    monkeypatch.setenv("SETD_VARIANT", base)
    ref = S.Plan(p)
    monkeypatch.setenv("SETD_VARIANT", variant)
    g = S.Plan(p)
    for _ in range(3):
        ref.step(5)
        g.step(5)
        for r in range(p["realizations"]):
            assert np.array_equal(ref.get(r), g.get(r))
    ref.close()
    g.close()
