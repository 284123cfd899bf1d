"""GPU tests of the continuous-batching server: jobs of several models, sizes
and precisions arriving while others run are batched into shared launches,
and every job's result equals its solo run (bitwise: the kernels do the same
arithmetic for any batch) and the oracle within the precision's bar."""
import sys
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2511_22510_amd import workloads as W

pytestmark = pytest.mark.gpu


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


MIX = [
    (W.model_b([64, 64], precision=32, realizations=4, seed=101), 40),
    (W.model_a([128, 128], precision=32, order=2, realizations=2, seed=102), 25),
    (W.kpz([64, 64], precision=32, realizations=3, seed=103, ic_kind=1, ic_sigma=0.2), 30),
    (W.cgl([16, 16, 16], precision=32, realizations=2, seed=104), 20),
    (W.model_b([64, 64], precision=32, realizations=1, seed=105), 12),
    (W.model_a([64, 32], precision=64, order=1, realizations=1, seed=106), 33),
    (W.model_b([64, 64], precision=32, realizations=2, seed=107), 50),
    (W.cgl([32, 32], precision=32, realizations=1, seed=108), 18),
    # 1D lines: two jobs of one launch class share a line pair across the job
    # boundary (3 + 1 realizations)
    (W.model_a([256], precision=32, realizations=3, seed=109, dx=0.25), 27),
    (W.model_a([256], precision=32, realizations=1, seed=110, dx=0.25), 19),
    (W.kpz([128], precision=32, order=2, realizations=2, seed=111, ic_kind=1, ic_sigma=0.2), 21),
    (W.cgl([64], precision=64, realizations=1, seed=112), 15),
    # line options: their own launch classes
    (W.model_a([256], precision=32, realizations=2, seed=113, dx=0.25, dealias=2), 17),
    (W.model_a([256], precision=32, realizations=1, seed=114, dx=0.25, noise_space=1), 23),
    # 2D options: phase shifts, real-space noise
    (W.model_a([64, 64], precision=32, order=2, realizations=2, seed=115, dealias=2), 21),
    (W.model_b([64, 64], precision=32, realizations=2, seed=116, noise_space=1), 17),
    (W.cgl([16, 16, 16], precision=32, realizations=1, seed=117, dealias=2), 15),
]


@pytest.mark.parametrize("lanes", [4, 0])
def test_mix_equals_solo_and_oracle(lanes, monkeypatch):
    """Each served job equals the same job run alone, bitwise, and the oracle
    within the bars; with the launch classes of a tick on four streams of the
    server and with everything on one stream."""
    monkeypatch.setenv("SETD_SERVER_LANES", str(lanes))
    S = _setd()
    say("server mix of", len(MIX), "jobs, lanes", lanes)
    srv = S.Server(256 << 20)
    ids = []
    for k, (p, n) in enumerate(MIX):
        ids.append(srv.submit(p, n))
        if k % 3 == 2:
            time.sleep(0.002)   # later jobs arrive while earlier ones run
    srv.drain()
    for jid, (p, n) in zip(ids, MIX):
        done, st = srv.poll(jid)
        assert done and st == S.SETD_OK
        times = srv.times(jid)
        assert times[3] == n and times[0] <= times[1] <= times[2]
        solo = S.Plan(p)
        solo.step(n)
        for r in range(p["realizations"]):
            assert np.array_equal(srv.get(jid, r), solo.get(r)), (jid, r)
        solo.close()
        o = O.Sim(p, r_first=0, r_count=1)
        o.step(n)
        err = relerr(srv.get(jid, 0), o.get(0))
        say("job", jid, p["nl"], p["n"], "f%d" % p["precision"], "oracle err", err)
        assert err <= (1e-10 if p["precision"] == 64 else 2e-4)
    srv.close()


def test_admission_by_footprint_queues_instead_of_failing():
    """An arena that holds about two jobs: the rest wait in the queue and are
    admitted as blocks free up; nothing runs out of memory."""
    S = _setd()
    p = W.model_b([128, 128], precision=32, realizations=8, seed=7)
    info = S.Plan(p).info
    need = int(info.workspace_bytes)
    srv = S.Server(2 * need + (4 << 20))
    ids = [srv.submit(dict(p, seed=7 + k), 30) for k in range(6)]
    srv.drain()
    admits = []
    for jid in ids:
        done, st = srv.poll(jid)
        assert done and st == S.SETD_OK
        t = srv.times(jid)
        admits.append(t[1] - t[0])
    say("admission waits", ["%.4f" % a for a in admits])
    assert max(admits) > 0.0 and sorted(admits)[-1] > sorted(admits)[0]
    solo = S.Plan(dict(p, seed=7 + 5))
    solo.step(30)
    assert np.array_equal(srv.get(ids[5], 3), solo.get(3))
    srv.close()


def test_failing_job_is_retired_alone():
    """A job that blows up (explicit nonlinearity, huge step) ends with
    SETD_E_NONFINITE; its neighbours in the same launches are unaffected."""
    S = _setd()
    good = W.model_a([64, 64], precision=32, order=1, realizations=2, seed=31)
    bad = W.model_a([64, 64], precision=32, order=1, realizations=2, seed=32, h=5.0, u=50.0,
                    ic_sigma=3.0)
    srv = S.Server(128 << 20)
    j1 = srv.submit(good, 40)
    j2 = srv.submit(bad, 40)
    srv.drain()
    assert srv.poll(j1) == (True, S.SETD_OK)
    assert srv.poll(j2) == (True, S.SETD_E_NONFINITE)
    solo = S.Plan(good)
    solo.step(40)
    for r in range(2):
        assert np.array_equal(srv.get(j1, r), solo.get(r))
    srv.close()


def test_oversized_job_is_rejected_at_submit():
    S = _setd()
    srv = S.Server(8 << 20)
    with pytest.raises(S.SetdError) as e:
        srv.submit(W.model_b([512, 512], precision=32, realizations=64), 10)
    assert e.value.status == S.SETD_E_NOMEM
    srv.close()


def test_serving_trace_small():
    """A short Poisson trace of the mixed workload types at reduced sizes and
    step counts; reports latency percentiles and checks every job finished."""
    S = _setd()
    trace = W.serving_trace(n_jobs=16, rate=200.0, seed=5, steps_range=(20, 60))
    srv = S.Server(8 << 30)
    t0 = S.setd_clock(srv.lib)
    ids = []
    for job in trace:
        while S.setd_clock(srv.lib) - t0 < job["arrival"]:
            time.sleep(0.0002)
        ids.append(srv.submit(job["problem"], job["steps"]))
    srv.drain()
    lat = []
    for jid in ids:
        done, st = srv.poll(jid)
        assert done and st == S.SETD_OK
        t = srv.times(jid)
        lat.append(t[2] - t[0])
    say("p50 %.4f s  p99 %.4f s" % (np.percentile(lat, 50), np.percentile(lat, 99)))
    srv.close()


def test_admission_keeps_item_entries_within_the_table(monkeypatch):
    """Admission counts the per-tick item-table entries (a realization each,
    plus one padding entry for a real 1D line with an odd count): jobs whose
    realizations together exceed the table wait instead of failing the tick,
    and each finishes with its solo result."""
    monkeypatch.setenv("SETD_SERVER_ITEMS", "48")
    S = _setd()
    jobs = [(W.model_a([16, 16], precision=32, order=2, realizations=32, seed=201), 20),
            (W.model_a([16, 16], precision=32, order=2, realizations=32, seed=202), 20),
            (W.model_b([16, 16], precision=32, realizations=20, seed=203), 15),
            # 47 realizations + 1 padding entry fill the table exactly
            (W.model_a([32], precision=32, order=2, realizations=47, seed=204), 30)]
    srv = S.Server(64 << 20)
    ids = [srv.submit(p, n) for p, n in jobs]
    with pytest.raises(S.SetdError) as e:
        srv.submit(W.model_a([16, 16], precision=32, order=2, realizations=49, seed=205), 5)
    assert e.value.status == S.SETD_E_INVAL   # 49 entries never fit
    srv.drain()
    for jid, (p, n) in zip(ids, jobs):
        assert srv.poll(jid) == (True, S.SETD_OK)
        solo = S.Plan(p)
        solo.step(n)
        for r in (0, p["realizations"] - 1):
            assert np.array_equal(srv.get(jid, r), solo.get(r)), (jid, r)
        solo.close()
    srv.close()


SHARED = [
    (W.model_a([64, 64], precision=32, order=2, realizations=3, seed=301), 37),
    (W.model_a([128, 128], precision=32, order=2, realizations=2, seed=302), 41),
    (W.model_b([256, 256], precision=32, realizations=4, seed=303), 29),
    (W.model_a([512, 512], precision=32, order=2, realizations=1, seed=304), 33),
    # the same class as the 128^2 Model A job: both fill one slot
    (W.model_b([128, 128], precision=32, realizations=1, seed=305), 45),
    # classes that keep launches of their own
    (W.kpz([128, 128], precision=32, realizations=2, seed=306), 23),
    (W.cgl([32, 32, 32], precision=32, realizations=1, seed=307), 19),
]


@pytest.mark.parametrize("multi", ["1", "0"])
def test_uneven_lattices_share_launches(multi, monkeypatch):
    """2D real-field jobs on 64^2 to 512^2 lattices advance in one launch per
    pass per tick (each lattice size a slot of the shared kernels); every job
    equals its solo run bitwise and the oracle within the bar.  With
    SETD_SERVER_MULTI=0 the same jobs run one launch per class."""
    monkeypatch.setenv("SETD_SERVER_MULTI", multi)
    S = _setd()
    srv = S.Server(512 << 20)
    ids = [srv.submit(p, n) for p, n in SHARED]
    srv.drain()
    ticks, launches, shared = srv.stats()
    say("multi", multi, "ticks", ticks, "pass launches", launches, "shared", shared)
    assert ticks > 0 and launches > 0
    assert (shared > 0) if multi == "1" else (shared == 0)
    for jid, (p, n) in zip(ids, SHARED):
        assert srv.poll(jid) == (True, S.SETD_OK)
        solo = S.Plan(p)
        solo.step(n)
        for r in range(p["realizations"]):
            assert np.array_equal(srv.get(jid, r), solo.get(r)), (jid, r)
        solo.close()
        o = O.Sim(p, r_first=0, r_count=1)
        o.step(n)
        err = relerr(srv.get(jid, 0), o.get(0))
        say("job", jid, p["nl"], p["n"], "oracle err", err)
        assert err <= 2e-4
    srv.close()
