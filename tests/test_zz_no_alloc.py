"""setd_run_noalloc (the entry point for callers that cannot allocate device
memory) against the bound-plan path (setd_plan_create / bind / step /
get_field) on the same problems: two and more calls in a row on the one static
scratch array, each later call with a smaller workspace than the one before,
so that anything an earlier call left behind would show.  Bars: 1e-10 relative
in FP64, 2e-4 in FP32 (the kernels are the same, so the two usually agree
bitwise)."""
import sys

import numpy as np
import pytest

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


# descending workspace sizes: 3D complex, KPZ (two intermediates), Model B
# (SETD2 carry), Model A FP64 SETD1, a 1D line
CASES = [
    (W.cgl([32, 32, 64], precision=32, realizations=3, seed=91), 40),
    (W.kpz([256, 256], precision=32, realizations=3, seed=92), 60),
    (W.model_b([128, 128], precision=32, realizations=4, seed=93), 70),
    (W.model_a([64, 64], precision=64, order=1, realizations=2, seed=94), 50),
    (W.model_a([256], precision=32, order=2, realizations=5, seed=95), 300),
]


def _workspace(S, p):
    plan = S.setd_plan_create(S.make_desc(p))
    try:
        return S.setd_plan_workspace(plan)
    finally:
        S.setd_plan_destroy(plan)


def test_noalloc_matches_bound_plan_calls_in_a_row():
    S = _setd()
    sizes = [_workspace(S, p) for p, _ in CASES]
    assert sizes == sorted(sizes, reverse=True), sizes
    assert sizes[0] <= (64 << 20)
    for p, steps in CASES:
        say("noalloc case", p["nl"], p["n"], "f%d" % p["precision"], "R", p["realizations"], "steps", steps)
        got = S.run_noalloc(p, steps)
        g = S.Plan(p)
        g.step(steps)
        ref = g.get_all()
        g.close()
        err = relerr(got, ref)
        say("  rel err %.3g bitwise %s" % (err, bool(np.array_equal(got, ref))))
        assert got.shape == ref.shape
        assert err <= TOL[p["precision"]]


def test_noalloc_repeat_call_is_reproducible_and_smaller_call_follows():
    """The same call twice gives the same result; a smaller call after a
    larger one matches its own bound plan."""
    S = _setd()
    big = W.model_b([256, 256], precision=32, realizations=8, seed=3)
    small = W.model_b([64, 64], precision=64, realizations=1, seed=4)
    a = S.run_noalloc(big, 25)
    b = S.run_noalloc(big, 25)
    assert np.array_equal(a, b)
    c = S.run_noalloc(small, 25)
    g = S.Plan(small)
    g.step(25)
    ref = g.get_all()
    g.close()
    assert relerr(c, ref) <= 1e-10
    # zero steps: the initial condition itself
    z = S.run_noalloc(small, 0)
    g = S.Plan(small)
    ref0 = g.get_all()
    g.close()
    assert relerr(z, ref0) <= 1e-10


def test_noalloc_rejects_a_plan_beyond_its_scratch():
    S = _setd()
    import torch
    p = W.model_b([1024, 1024], precision=32, realizations=16)
    assert _workspace(S, p) > (64 << 20)
    out = torch.empty(16, dtype=torch.float64, device="cuda")
    with pytest.raises(S.SetdError) as e:
        S.setd_run_noalloc(S.make_desc(p), 1, out.data_ptr(), out.numel(), torch.cuda.current_stream().cuda_stream)
    assert e.value.status == S.SETD_E_NOMEM
    small = W.model_b([64, 64], precision=32, realizations=2)
    with pytest.raises(S.SetdError) as e:
        S.setd_run_noalloc(S.make_desc(small), 1, out.data_ptr(), out.numel(),
                           torch.cuda.current_stream().cuda_stream)
    assert e.value.status == S.SETD_E_INVAL


def test_noalloc_phase_shift_plan_after_another_call():
    """A phase-shift plan whose initial field is zero (no initial-condition
    pass writes its shifted intermediates), run right after a call that left
    other data in the scratch: binding clears them, so each matches its
    bound plan."""
    S = _setd()
    S.run_noalloc(W.cgl([32, 32, 64], precision=32, realizations=3, seed=91), 5)   # fills the scratch
    for p in (W.model_b([64, 64], precision=64, realizations=2, ic_kind=0, dealias=2, seed=5),
              W.kpz([64, 64], precision=64, realizations=2, dealias=2, seed=6),
              W.cgl([16, 16, 16], precision=64, realizations=1, ic_kind=0, dealias=2, seed=7)):
        say("noalloc phase-shift case", p["nl"], p["n"])
        got = S.run_noalloc(p, 20)
        g = S.Plan(p)
        g.step(20)
        ref = g.get_all()
        g.close()
        err = relerr(got, ref)
        say("  rel err %.3g" % err)
        assert err <= 1e-10
