"""Pins of the oracle's orthonormal 2-D DFT (Sec. II: F is the 2D orthonormal
Fourier transform; forward kernel exp(-2 pi i (km + ln)/Np)/Np, DC at [0, 0])."""
import numpy as np
import pytest

from oracle import pmace_oracle as O


def brute_dft2(a):
    """O(N^4) definition, written out as sums."""
    n1, n2 = a.shape
    out = np.zeros((n1, n2), dtype=np.complex128)
    for k in range(n1):
        for l in range(n2):
            acc = 0j
            for m in range(n1):
                for n in range(n2):
                    acc += a[m, n] * np.exp(-2j * np.pi * (k * m / n1 + l * n / n2))
            out[k, l] = acc / np.sqrt(n1 * n2)
    return out


@pytest.mark.parametrize("np_", [1, 2, 3, 4, 8, 16])
def test_dft_matches_definition(np_):
    rng = np.random.default_rng(np_)
    a = rng.standard_normal((np_, np_)) + 1j * rng.standard_normal((np_, np_))
    assert np.allclose(O.dft2(a), brute_dft2(a), atol=1e-12, rtol=0)


@pytest.mark.parametrize("np_", [4, 32, 64])
def test_parseval_and_inverse(np_):
    rng = np.random.default_rng(7)
    a = rng.standard_normal((3, np_, np_)) + 1j * rng.standard_normal((3, np_, np_))
    A = O.dft2(a)
    assert np.allclose(np.linalg.norm(A), np.linalg.norm(a), rtol=1e-13)
    assert np.allclose(O.idft2(A), a, atol=1e-12)


@pytest.mark.parametrize("np_", [2, 8, 32])
def test_delta_and_constant(np_):
    delta = np.zeros((np_, np_), complex)
    delta[0, 0] = 1
    assert np.allclose(O.dft2(delta), np.full((np_, np_), 1.0 / np_))
    ones = np.ones((np_, np_), complex)
    expect = np.zeros((np_, np_), complex)
    expect[0, 0] = np_
    assert np.allclose(O.dft2(ones), expect, atol=1e-12)


def test_sign_convention_single_mode():
    # exp(+2 pi i m/N) along rows lands in frequency bin k = 1 under the
    # e^{-2 pi i} forward kernel (bin N-1 under the opposite sign).
    n = 8
    m = np.arange(n)
    a = np.exp(2j * np.pi * m / n)[:, None] * np.ones((1, n))
    A = O.dft2(a)
    assert abs(A[1, 0]) == pytest.approx(n, rel=1e-12)
    assert abs(A[n - 1, 0]) < 1e-10
