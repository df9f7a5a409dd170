"""The row-spectrum form of the agent, checked on the CPU with NumPy FFTs (no
GPU): the identities the row-spectrum kernels are built on, and one agent
step taken that way against the oracle's eq. (9).

Transforms are unnormalised, F = F_c F_r (column DFTs of the row DFTs), and
F_r F_r* = Np I for the unnormalised inverse F_r*.  A PMACE state t_j is
kept as H_j = F_r(d t_j)/Np, the row DFTs of the probe-weighted state; the
frame is v_j = t_j + 2 rho P_j xbar (the Mann update of Alg. 1)."""
import numpy as np
import pytest

from oracle import pmace_oracle as O


def Fr(a):
    return np.fft.fft(a, axis=-1)


def Fr_inv(a):
    return np.fft.ifft(a, axis=-1) * a.shape[-1]


def Fc(a):
    return np.fft.fft(a, axis=-2)


def Fc_inv(a):
    return np.fft.ifft(a, axis=-2) * a.shape[-2]


@pytest.fixture(params=[8, 12, 20])   # radix 2, and sides with factors 3 and 5
def case(request):
    np_ = request.param
    rng = np.random.default_rng(100 + np_)
    c = lambda: rng.standard_normal((np_, np_)) + 1j * rng.standard_normal((np_, np_))
    d = c() + 3.0                 # a probe with no exact zeros
    assert np.all(np.abs(d) > 0)
    t, xw = c(), c()              # a state and its window P_j xbar
    y = np.abs(c()) * 2.0         # amplitudes, orthonormal scaling as in eq. (1)
    return np_, d, t, xw, y


def test_unnormalised_pair(case):
    np_, _, t, _, _ = case
    assert np.allclose(Fr(Fr_inv(t)), np_ * t)
    assert np.allclose(Fc(Fr(t)), np.fft.fft2(t))


def test_row_pass_frame_spectrum(case):
    """F_r(d v) = Np H + F_r(2 rho d P xbar): only the window term needs a
    row transform in the row pass."""
    np_, d, t, xw, _ = case
    rho = 0.5
    H = Fr(d * t) / np_
    v = t + 2 * rho * xw
    assert np.allclose(np_ * H + Fr(2 * rho * d * xw), Fr(d * v), rtol=1e-12, atol=1e-11)


@pytest.mark.parametrize("alpha,rho", [(0.5, 0.5), (0.0, 0.5), (2.0, 0.3)])
def test_column_pass_output_is_the_next_state(case, alpha, rho):
    """One agent step the row-spectrum way equals the oracle's: with
    W = F_c(Np H + F_r(2 rho d P xbar)) and the data step in unnormalised
    scaling U = (alpha W + Np y W/|W|)/(1 + alpha), the column pass's output
    F_c*(W - 2 rho U)/Np^2 is F_r(d t+)/Np for t+ = v - 2 rho F_j(v)."""
    np_, d, t, xw, y = case
    H = Fr(d * t) / np_
    W = Fc(np_ * H + Fr(2 * rho * d * xw))
    U = (alpha * W + np_ * y * W / np.abs(W)) / (1 + alpha)
    H_new = Fc_inv(W - 2 * rho * U) / np_ ** 2
    v = t + 2 * rho * xw
    t_new = v - 2 * rho * O.agent(v, d, y, alpha)
    ref = Fr(d * t_new) / np_
    assert np.allclose(H_new, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_dropped_data_scale_is_caught(case):
    """The Np on the amplitudes is what ties the unnormalised route to eq. (9):
    without it the step above no longer matches the oracle."""
    np_, d, t, xw, y = case
    alpha, rho = 0.5, 0.5
    W = Fc(Fr(d * t) + Fr(2 * rho * d * xw))
    U = (alpha * W + y * W / np.abs(W)) / (1 + alpha)
    v = t + 2 * rho * xw
    ref = Fr(d * (v - 2 * rho * O.agent(v, d, y, alpha))) / np_
    assert not np.allclose(Fc_inv(W - 2 * rho * U) / np_ ** 2, ref, rtol=1e-6, atol=1e-9)


def test_consensus_recovers_the_weighted_state(case):
    """The consensus inverts each stored row: F_r*(H) = d t, and the weights
    |d|^kappa / d on it give the eq. (11) numerator term |d|^kappa t."""
    np_, d, t, _, _ = case
    H = Fr(d * t) / np_
    s = Fr_inv(H)
    assert np.allclose(s, d * t, rtol=1e-12, atol=1e-12)
    kappa = 1.25
    assert np.allclose(np.abs(d) ** kappa / d * s, O.consensus_weights(d, kappa) * t,
                       rtol=1e-12, atol=1e-12)


def test_sharp_plus_state_update_in_row_spectra(case):
    """SHARP+ with T = F_r(t)/Np and frame s = t + 2 beta d P xbar: for the
    magnitude projection's column inverse C (so P_a s = F_r*(C)/Np^2, the
    oracle's eq. (14) projection), the next state
    t' = (1 - 2 beta) P_a s + beta (s - d P xbar) has row spectrum
    F_r(t')/Np = (1 - 2 beta)/Np^2 C + (2 beta - 1)/(2 Np) F_r(s) + T/2."""
    np_, d, t, xw, y = case
    beta = 0.8
    T = Fr(t) / np_
    s = t + 2 * beta * d * xw
    Rs = np_ * T + Fr(2 * beta * d * xw)
    assert np.allclose(Rs, Fr(s), rtol=1e-12, atol=1e-11)
    W = Fc(Rs)
    C = Fc_inv(np_ * y * W / np.abs(W))
    pa = O.sharp_magnitude_projection(s, y)
    assert np.allclose(Fr_inv(C) / np_ ** 2, pa, rtol=1e-12, atol=1e-12 * np.abs(pa).max())
    t_next = (1 - 2 * beta) * pa + beta * (s - d * xw)
    T_next = (1 - 2 * beta) / np_ ** 2 * C + (2 * beta - 1) / (2 * np_) * Rs + T / 2
    ref = Fr(t_next) / np_
    assert np.allclose(T_next, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
