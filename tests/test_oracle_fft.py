"""Pins for the oracle's Fourier transforms (Sec. 1.3 notation; the DFT normalisation
||F_2D||^2 = N^2 is the one used by the matrix amplitude-flow step, Sec. 3.4)."""
import numpy as np
import pytest


def _rand(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


def _dft_matrix(n, sign=-1):
    k = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(k, k) / n)


@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_fft1d_matches_brute_force_dft(orc, n):
    x = _rand(n, n)
    ref = orc.dft1d(x)
    got = orc.fft1d(x)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-13
    # the brute-force DFT itself equals the DFT matrix written out from its definition
    assert np.allclose(ref, _dft_matrix(n) @ x, rtol=0, atol=1e-12)


def test_fft2d_8x8_matches_brute_force(orc):
    x = _rand((8, 8), 3)
    f = _dft_matrix(8)
    ref = f @ x @ f.T          # 2D DFT = 1D DFT along both axes
    got = orc.fft2d(x)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-13


@pytest.mark.parametrize("n", [64, 128, 256])
def test_fft2d_matches_numpy(orc, n):
    x = _rand((n, n), n)
    got = orc.fft2d(x)
    ref = np.fft.fft2(x)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-13
    inv = orc.fft2d(x, +1)
    assert np.linalg.norm(inv - np.fft.ifft2(x) * n * n) / np.linalg.norm(inv) < 1e-13


@pytest.mark.parametrize("n", [8, 64])
def test_parseval_and_inverse(orc, n):
    x = _rand((n, n), 7)
    fx = orc.fft2d(x)
    assert abs(np.vdot(fx, fx).real - n * n * np.vdot(x, x).real) < 1e-10 * n * n * np.vdot(x, x).real
    back = orc.fft2d(fx, +1) / (n * n)
    assert np.abs(back - x).max() < 1e-12


def test_closed_forms(orc):
    n = 16
    delta = np.zeros((n, n), complex)
    delta[0, 0] = 1.0
    assert np.allclose(orc.fft2d(delta), 1.0, atol=1e-15)
    ones = np.ones((n, n), complex)
    f = orc.fft2d(ones)
    assert abs(f[0, 0] - n * n) < 1e-12
    f[0, 0] = 0.0
    assert np.abs(f).max() < 1e-12
    # a plane wave of frequency (ky, kx) lands in exactly one bin
    ky, kx = 3, 13
    y, x = np.mgrid[0:n, 0:n]
    pw = np.exp(2j * np.pi * (ky * y + kx * x) / n)
    f = orc.fft2d(pw)
    assert abs(f[ky, kx] - n * n) < 1e-10
    f[ky, kx] = 0
    assert np.abs(f).max() < 1e-10


def test_fftfreq_matches_numpy(orc):
    for n in (8, 64, 128):
        assert np.array_equal(orc.fftfreq(n, 0.2), np.fft.fftfreq(n, 0.2))


def test_non_power_of_two_rejected(orc):
    with pytest.raises(ValueError):
        orc.fft1d(np.ones(12))
