"""Pins for the oracle's DFT: the definition written as a dense matrix, NumPy's
FFT as the library routine, and closed forms (impulse, tone, Parseval)."""
import numpy as np
import pytest

SMOOTH = sorted({2 ** a * 3 ** b * 5 ** c for a in range(7) for b in range(4) for c in range(3)
                 if 2 ** a * 3 ** b * 5 ** c <= 64})


def dft_matrix(n, sign=-1):
    k = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(k, k) / n)


@pytest.mark.parametrize("n", SMOOTH + [7, 11, 13, 49])
def test_fft_matches_dense_definition(O, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = dft_matrix(n) @ x
    got = O.fft(x)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    inv = O.fft(x, inverse=True)
    ref_inv = dft_matrix(n, +1) @ x / n
    assert np.max(np.abs(inv - ref_inv)) <= 1e-13 * max(1.0, np.max(np.abs(ref_inv)))


@pytest.mark.parametrize("n", [512, 2160, 3840])
def test_fft_workload_lengths_against_library(O, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    got = O.fft(x)
    ref = np.fft.fft(x)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
    assert np.linalg.norm(O.fft(got, inverse=True) - x) <= 1e-13 * np.linalg.norm(x)


def test_fft_impulse_tone_parseval(O):
    n = 60
    x = np.zeros(n, complex)
    x[0] = 1.0
    assert np.allclose(O.fft(x), np.ones(n), atol=1e-15)
    k0 = 7
    tone = np.exp(2j * np.pi * k0 * np.arange(n) / n)
    X = O.fft(tone)
    expect = np.zeros(n, complex)
    expect[k0] = n
    assert np.max(np.abs(X - expect)) < 1e-12
    rng = np.random.default_rng(3)
    y = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    Y = O.fft(y)
    assert abs(np.sum(abs(Y) ** 2) / n - np.sum(abs(y) ** 2)) < 1e-12 * np.sum(abs(y) ** 2)


@pytest.mark.parametrize("shape", [(6, 10), (16, 15), (45, 32)])
def test_fft2_against_library(O, shape):
    rng = np.random.default_rng(sum(shape))
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    assert np.allclose(O.fft2(x), np.fft.fft2(x), rtol=0, atol=1e-12)
    assert np.allclose(O.fft2(x, inverse=True), np.fft.ifft2(x), rtol=0, atol=1e-14)
