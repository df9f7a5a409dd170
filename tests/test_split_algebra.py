"""The coset-block (split) form of the agent, checked index by index on the
CPU with NumPy FFTs (no GPU, no oracle): the identities the split kernels are
built on.  For Np = 2M, block ab (a, b in {0, 1}) of a patch f is

    Z_ab[m] = W_Np^(a m1 + b m2) sum_q (-1)^(a q1 + b q2) f[m + M q],   m in [0, M)^2, q in {0, 1}^2,

(one radix-2 x 2 decimation-in-frequency step of the 2-D DFT)."""
import numpy as np
import pytest


def _w(np_, m):
    return np.exp(-2j * np.pi * np.asarray(m) / np_)


def split(f):
    np_ = f.shape[-1]
    M = np_ // 2
    m1 = np.arange(M)[:, None]
    m2 = np.arange(M)[None, :]
    q = {(q1, q2): f[q1 * M:(q1 + 1) * M, q2 * M:(q2 + 1) * M] for q1 in (0, 1) for q2 in (0, 1)}
    out = np.zeros((4, M, M), complex)
    for ab in range(4):
        a, b = ab >> 1, ab & 1
        h = sum(((-1) ** (a * q1 + b * q2)) * q[(q1, q2)] for (q1, q2) in q)
        out[ab] = h * _w(np_, a * m1 + b * m2)
    return out


def unsplit(Z):
    """s[m + M q] = 1/4 sum_ab (-1)^(a q1 + b q2) W_Np^-(a m1 + b m2) Z_ab[m] (the consensus's read)."""
    M = Z.shape[-1]
    np_ = 2 * M
    m1 = np.arange(M)[:, None]
    m2 = np.arange(M)[None, :]
    out = np.zeros((np_, np_), complex)
    for q1 in (0, 1):
        for q2 in (0, 1):
            acc = 0
            for ab in range(4):
                a, b = ab >> 1, ab & 1
                acc = acc + ((-1) ** (a * q1 + b * q2)) * np.conj(_w(np_, a * m1 + b * m2)) * Z[ab]
            out[q1 * M:(q1 + 1) * M, q2 * M:(q2 + 1) * M] = acc / 4
    return out


@pytest.fixture(params=[4, 8, 12, 16])
def data(request):
    np_ = request.param
    rng = np.random.default_rng(np_)
    c = lambda: rng.standard_normal((np_, np_)) + 1j * rng.standard_normal((np_, np_))
    return np_, c(), c(), c()


def test_block_dft_is_the_coset_spectrum(data):
    np_, s, _, _ = data
    X = np.fft.fft2(s)
    Z = split(s)
    for ab in range(4):
        a, b = ab >> 1, ab & 1
        assert np.allclose(np.fft.fft2(Z[ab]), X[a::2, b::2], atol=1e-9 * np.abs(X).max())


def test_four_times_block_inverse_is_the_split_of_the_inverse(data):
    """The new state's blocks come from the state spectrum coset by coset:
    4 x the unnormalised M x M inverse of coset ab = block ab of the
    unnormalised Np x Np inverse."""
    np_, _, S, _ = data
    M = np_ // 2
    full = np.fft.ifft2(S) * np_ * np_
    Zn = np.stack([4 * np.fft.ifft2(S[(ab >> 1)::2, (ab & 1)::2]) * M * M for ab in range(4)])
    assert np.allclose(Zn, split(full), atol=1e-9 * np.abs(full).max())


def test_unsplit_inverts_split(data):
    np_, s, _, _ = data
    assert np.allclose(unsplit(split(s)), s)


def test_window_term_adds_blockwise(data):
    """The frame block is the stored state's block plus the same butterfly of
    2 rho d P_j xbar, formed from the four quadrant products."""
    np_, s, d, win = data
    rho = 0.37
    assert np.allclose(split(s) + split(2 * rho * d * win), split(s + 2 * rho * d * win))


def test_amplitude_coset_order(data):
    """Element m of amplitude block ab holds frequency (2 m1 + a, 2 m2 + b)."""
    np_, _, _, _ = data
    M = np_ // 2
    y = np.arange(np_ * np_, dtype=float).reshape(np_, np_)
    ys = np.zeros(4 * M * M)
    for i in range(4 * M * M):
        ab, m = divmod(i, M * M)
        k, l = 2 * (m // M) + (ab >> 1), 2 * (m % M) + (ab & 1)
        ys[i] = y[k, l]
    for ab in range(4):
        assert np.array_equal(ys[ab * M * M:(ab + 1) * M * M].reshape(M, M), y[(ab >> 1)::2, (ab & 1)::2])


def test_symmetric_probe_has_exact_nyquist_zeros_in_fp64():
    """The flat-start case behind the split agent's first-pass deviation: a
    probe symmetric about its half-pixel centre has an exactly zero spectrum
    on its Nyquist row and column in exact arithmetic; NumPy's FP64 FFT
    returns those zeros exactly."""
    np_ = 16
    r = np.arange(np_) - (np_ - 1) / 2
    f = np.exp(-r ** 2 / (2 * (np_ / 4) ** 2)) * np.exp(1j * np.pi * (2 * r / np_) ** 2)
    d = np.outer(f, f)
    assert np.array_equal(d, d[::-1, ::-1])
    W = np.fft.fft2(d)
    assert np.all(W[:, np_ // 2] == 0) and np.all(W[np_ // 2, :] == 0)
