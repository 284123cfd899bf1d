"""Host logic of the C ABI without a GPU: setd_plan_create validates the
descriptor (status codes of include/setd.h) and sizes the plan; nothing here
touches the device (plan creation, info and destruction are host work)."""
import os

import pytest

from paper_2511_22510_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2511_22510_amd", "libsetd.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libsetd.so not built")


def _status(p):
    from paper_2511_22510_amd import setd
    try:
        h = setd.setd_plan_create(setd.make_desc(p))
    except setd.SetdError as e:
        return e.status, None
    info = setd.setd_plan_info(h)
    setd.setd_plan_destroy(h)
    return setd.SETD_OK, info


@pytest.mark.parametrize("bad,code", [
    (dict(ndim=4), "SETD_E_INVAL"),
    (dict(n=[48, 64]), "SETD_E_INVAL"),
    (dict(n=[2048, 64]), "SETD_E_INVAL"),
    (dict(n=[4, 64]), "SETD_E_INVAL"),
    (dict(order=3), "SETD_E_INVAL"),
    (dict(h=0.0), "SETD_E_INVAL"),
    (dict(dx=-1.0), "SETD_E_INVAL"),
    (dict(realizations=0), "SETD_E_INVAL"),
    (dict(dealias=3), "SETD_E_INVAL"),
    (dict(precision=16), "SETD_E_INVAL"),
    (dict(noise_kpow=1), "SETD_E_INVAL"),
    (dict(series_len=12), "SETD_E_INVAL"),
    (dict(c2=(-1.0, 0.5)), "SETD_E_INVAL"),          # complex c(k) on a real field
    (dict(noise_space=2), "SETD_E_INVAL"),
    (dict(nl="cgl"), "SETD_E_UNSUPPORTED"),          # CGL needs a complex field
])
def test_invalid_descriptors_are_refused(bad, code):
    from paper_2511_22510_amd import setd
    p = dict(W.model_a([64, 64], precision=32), **bad)
    if "n" in bad:
        p["ndim"] = len(bad["n"])
    st, _ = _status(p)
    assert st == getattr(setd, code)


def test_unsupported_combinations():
    from paper_2511_22510_amd import setd
    assert _status(W.kpz([32, 32, 32]))[0] == setd.SETD_E_UNSUPPORTED
    assert _status(W.kpz([32, 32], dealias=2))[0] == setd.SETD_OK
    assert _status(W.model_a([32, 32], dealias=2))[0] == setd.SETD_OK
    assert _status(W.cgl([32, 32], dealias=2))[0] == setd.SETD_OK
    assert _status(W.model_b([16, 16, 16], dealias=2))[0] == setd.SETD_OK
    assert _status(W.cgl([16, 16, 16], dealias=2))[0] == setd.SETD_OK
    assert _status(W.model_a([16, 16, 16], dealias=2, noise_space=1))[0] == setd.SETD_OK
    assert _status(W.cgl([32, 32], dealias=2, noise_space=1))[0] == setd.SETD_OK
    assert _status(W.model_a([64], dealias=2, noise_space=1))[0] == setd.SETD_OK
    assert _status(dict(W.cgl([32, 32]), nl="phi3"))[0] == setd.SETD_E_UNSUPPORTED


@pytest.mark.parametrize("p,kept,nb,passes", [
    (W.model_b([512, 512]), 58311, 364, 2),              # (2K+1)(K+1), K = 170
    (W.kpz([1024, 1024]), 233586, 726, 2),
    (W.cgl([256, 256, 256]), 171 ** 3, 223, 4),             # (2K+1)^3 = 5,000,211
    (W.model_a([256]), 86, 129, 1),                      # a line: K + 1
    (W.model_a([256], dealias=2), 128, 129, 1),          # phase shift: |a| < N/2
    (W.cgl([64], dealias=0), 64, 33, 1),
    (W.model_a([64, 64], dealias=2), 63 * 32, 47, 2),  # phase shifts: |a_i| < N_i/2
    (W.cgl([16, 16, 16], dealias=2), 15 ** 3, 15, 4),
    (W.model_a([16, 32, 16], dealias=2), 15 * 31 * 8, 21, 4),
])
def test_plan_sizes(p, kept, nb, passes):
    from paper_2511_22510_amd import setd
    st, info = _status(p)
    assert st == setd.SETD_OK
    assert info.kept_modes == kept and info.nbins == nb and info.passes_per_step == passes
    assert info.workspace_bytes > 0
    assert info.site_updates_per_step == float(p["realizations"]) * float(__import__("numpy").prod(p["n"]))
