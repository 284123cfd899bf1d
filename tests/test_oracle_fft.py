"""Pins of the oracle's own FFT (App. A conventions, reading: forward e^{-},
inverse scaled by 1/N^d) against numpy's pocketfft, brute-force DFT sums,
round trips and Parseval."""
import numpy as np
import pytest

from oracle import oracle as O

RNG = np.random.default_rng(7)


def brute_dft(x, sign):
    """Plain O(N^2d) sum over all sites, for tiny lattices."""
    shp = x.shape
    idx = np.indices(shp).reshape(len(shp), -1).T
    out = np.zeros(x.size, dtype=np.complex128)
    xf = x.reshape(-1)
    for a_i, a in enumerate(idx):
        ph = sum(a[d] * idx[:, d] / shp[d] for d in range(len(shp)))
        out[a_i] = np.sum(xf * np.exp(sign * 2j * np.pi * ph))
    return out.reshape(shp)


@pytest.mark.parametrize("shape", [(8,), (16,), (4, 8), (8, 4, 2), (16, 16)])
def test_fft_matches_brute_force(shape):
    x = RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)
    got = O.fftn(x)
    ref = brute_dft(x, -1)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    inv = O.fftn(x, inverse=True)
    ref_inv = brute_dft(x, +1) / x.size
    assert np.max(np.abs(inv - ref_inv)) <= 1e-12 * np.max(np.abs(ref_inv))


@pytest.mark.parametrize("shape", [(1024,), (64, 128), (32, 16, 64), (512, 512)])
def test_fft_matches_numpy(shape):
    x = RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)
    got = O.fftn(x)
    ref = np.fft.fftn(x)
    assert np.linalg.norm(got - ref) <= 1e-14 * np.sqrt(np.log2(x.size)) * np.linalg.norm(ref) * 4
    back = O.fftn(got, inverse=True)
    assert np.linalg.norm(back - x) <= 1e-14 * np.linalg.norm(x) * 8


@pytest.mark.parametrize("shape", [(16,), (8, 16), (64, 32), (8, 8, 16)])
def test_rfft_irfft_match_numpy(shape):
    x = RNG.standard_normal(shape)
    X = O.rfftn(x)
    ref = np.fft.rfftn(x)
    assert X.shape == ref.shape
    assert np.max(np.abs(X - ref)) <= 1e-13 * np.max(np.abs(ref))
    y = O.irfftn(X, shape)
    assert np.max(np.abs(y - x)) <= 1e-13
    # a Hermitian half spectrum from numpy goes back to the same real field
    assert np.max(np.abs(O.irfftn(ref, shape) - np.fft.irfftn(ref, shape, axes=list(range(len(shape)))))) <= 1e-13


def test_parseval_and_delta():
    x = RNG.standard_normal((32, 64)) + 1j * RNG.standard_normal((32, 64))
    X = O.fftn(x)
    assert abs(np.sum(np.abs(X) ** 2) / x.size - np.sum(np.abs(x) ** 2)) <= 1e-11 * np.sum(np.abs(x) ** 2)
    d = np.zeros((16, 16), dtype=np.complex128)
    d[0, 0] = 1.0
    assert np.allclose(O.fftn(d), 1.0, atol=1e-15)
    # a shifted delta is a pure phase ramp e^{-2 pi i a.n/N}
    d = np.zeros((8, 16), dtype=np.complex128)
    d[3, 5] = 1.0
    a0, a1 = np.indices((8, 16))
    assert np.allclose(O.fftn(d), np.exp(-2j * np.pi * (3 * a0 / 8 + 5 * a1 / 16)), atol=1e-14)


def test_plane_wave_lands_on_one_mode():
    n = 32
    xs = np.arange(n)
    w = np.exp(2j * np.pi * 5 * xs / n)
    X = O.fftn(w)
    expect = np.zeros(n, dtype=complex)
    expect[5] = n
    assert np.allclose(X, expect, atol=1e-12)
