"""Pins of the oracle's Philox4x32-10 and Box-Muller normals."""
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        a, b = line.split("|")
        ins = [int(v, 16) for v in a.split()]
        outs = [int(v, 16) for v in b.split()]
        rows.append((ins[:4], ins[4:6], outs))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(ctr, key, out):
    assert O.philox(ctr, key) == out


def test_normal_pair_is_box_muller_of_philox_words():
    # the 53-bit uniforms and Box-Muller, rebuilt from the raw words in numpy
    seed, e, n, r, tag = 0x0123456789ABCDEF, 17, 3, 5, 0
    x = O.philox([e, n, r, tag], [seed & 0xFFFFFFFF, seed >> 32])
    m1 = (x[0] << 21) | (x[1] >> 11)
    m2 = (x[2] << 21) | (x[3] >> 11)
    u1 = (m1 + 0.5) / 2.0**53
    u2 = (m2 + 0.5) / 2.0**53
    z1, z2 = O.normal_pair(seed, e, n, r, tag)
    assert z1 == pytest.approx(np.sqrt(-2 * np.log(u1)) * np.cos(2 * np.pi * u2), rel=1e-15, abs=1e-15)
    assert z2 == pytest.approx(np.sqrt(-2 * np.log(u1)) * np.sin(2 * np.pi * u2), rel=1e-15, abs=1e-15)


def test_normals_moments():
    zs = np.array([O.normal_pair(99, e, 0, 0, 0) for e in range(40000)]).reshape(-1)
    nz = zs.size
    assert abs(zs.mean()) < 5 / np.sqrt(nz)
    assert abs(zs.var() - 1) < 5 * np.sqrt(2 / nz)
    # fourth moment of a normal is 3
    assert abs(np.mean(zs**4) - 3) < 5 * np.sqrt(96 / nz)
    # neighbouring counters are uncorrelated
    a = np.array([O.normal_pair(99, e, 1, 0, 0)[0] for e in range(20000)])
    assert abs(np.corrcoef(a[:-1], a[1:])[0, 1]) < 5 / np.sqrt(a.size)


def test_noise_normals_are_box_muller_of_32bit_words():
    # the Fourier-space noise: words (x0, x1) for half 0 and (x2, x3) for
    # half 1, each a uniform (x + 1/2) 2^-32, rebuilt in numpy
    seed, P, n, r = 0x0123456789ABCDEF, 41, 7, 2
    x = O.philox([P, n, r, 0], [seed & 0xFFFFFFFF, seed >> 32])
    for half in (0, 1):
        u1 = (x[2 * half] + 0.5) / 2.0**32
        u2 = (x[2 * half + 1] + 0.5) / 2.0**32
        z1, z2 = O.noise_normals(seed, P, n, r, half)
        assert z1 == pytest.approx(np.sqrt(-2 * np.log(u1)) * np.cos(2 * np.pi * u2), rel=1e-15, abs=1e-15)
        assert z2 == pytest.approx(np.sqrt(-2 * np.log(u1)) * np.sin(2 * np.pi * u2), rel=1e-15, abs=1e-15)


def test_noise_normals_moments_and_independent_halves():
    z = np.array([[O.noise_normals(7, P, 3, 1, h) for h in (0, 1)] for P in range(20000)])   # P x half x 2
    zs = z.reshape(-1)
    nz = zs.size
    assert abs(zs.mean()) < 5 / np.sqrt(nz)
    assert abs(zs.var() - 1) < 5 * np.sqrt(2 / nz)
    assert abs(np.mean(zs**4) - 3) < 5 * np.sqrt(96 / nz)
    m = z.shape[0]
    # the two halves of one block, and z1 against z2, are uncorrelated
    for a, b in [(z[:, 0, 0], z[:, 1, 0]), (z[:, 0, 1], z[:, 1, 1]), (z[:, 0, 0], z[:, 0, 1])]:
        assert abs(np.corrcoef(a, b)[0, 1]) < 5 / np.sqrt(m)
