"""The pins above must catch plausible mistakes: each case plants one mistake
in the oracle (on the CPU, by patching a module attribute) and checks that at
least one pin fails."""
import numpy as np
import pytest

from oracle import pmace_oracle as O
import test_oracle_agent as TA
import test_oracle_consensus as TC
import test_oracle_dft as TD
import test_oracle_iteration as TI
import test_oracle_nrmse as TN
import test_oracle_sharp as TS


def _small():
    rng = np.random.default_rng(11)
    from paper_2111_14240_amd import synth
    d = synth.make_probe(16) * 3.0
    x = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    y = np.abs(rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))) * 2.0
    return d, x, y


PINS = [
    lambda: TD.test_dft_matches_definition(8),
    lambda: TD.test_parseval_and_inverse(32),
    lambda: TD.test_sign_convention_single_mode(),
    lambda: TA.test_golden_2x2_cases(),
    lambda: TA.test_magnitude_step_exact_zero(),
    lambda: TA.test_fourier_magnitude_is_r_star(_small(), 0.3),
    lambda: TA.test_noise_free_truth_is_fixed_point(0.7),
    lambda: TA.test_scale_covariance_of_probe(_small()),
    lambda: TC.test_golden_hand_example(),
    lambda: TC.test_reproduces_consistent_patches(),
    lambda: TI.test_golden_worked_two_iterations(),
    lambda: TI.test_noise_free_truth_is_fixed_point(0.8, 2.0, 0.3),
    lambda: TI.test_step_equals_mann_update_of_T(),
    lambda: TN.test_nrmse_special_values(),
    lambda: TN.test_nrmse_theta_is_grid_minimiser(),
    lambda: TS.test_init_golden_hand_example(),
    lambda: TS.test_reconstruct_inverts_init_on_covered_pixels(3),
]


def _count_failures():
    bad = 0
    with np.errstate(all="ignore"):
        for pin in PINS:
            try:
                pin()
            except Exception:
                bad += 1
    return bad


def _step_wrong_reflection(v, d, y, pos, shape, alpha, kappa, rho):
    w = O.agent_stack(v, d, y, alpha)
    z = O.consensus(2.0 * w + v, d, pos, shape, kappa)
    return v + 2.0 * rho * (z - w), w, z


def _step_wrong_sign(v, d, y, pos, shape, alpha, kappa, rho):
    w = O.agent_stack(v, d, y, alpha)
    z = O.consensus(2.0 * w - v, d, pos, shape, kappa)
    return v + 2.0 * rho * (w - z), w, z


def _agent_conj_probe(xj, d, yj, alpha):
    W = O.dft2(d * xj)
    back = O.idft2(O.fourier_magnitude_step(W, yj))
    return (alpha * xj + back / np.conj(d)) / (1 + alpha)


def _agent_swapped_blend(xj, d, yj, alpha):
    W = O.dft2(d * xj)
    back = O.idft2(O.fourier_magnitude_step(W, yj)) / d
    return (xj + alpha * back) / (1 + alpha)


def _mag_no_zero_rule(W, y):
    return y * W / np.abs(W)


def _weights_squared(d, kappa):
    return np.abs(d) ** 2


def _inv_weight_identity(lam):
    return np.ones_like(lam)


def _nrmse_conj_theta(xhat, x, mask=None):
    c = np.vdot(xhat, x)
    th = np.angle(c)
    return float(np.linalg.norm(xhat - np.exp(1j * th) * x) / np.linalg.norm(x))


def _sharp_init_conj_probe(x0, d, pos):
    return np.conj(np.asarray(d, complex)) * O.extract(np.asarray(x0, complex), pos, np.asarray(d).shape[0])


def _sharp_init_transposed_probe(x0, d, pos):
    return np.asarray(d, complex).T * O.extract(np.asarray(x0, complex), pos, np.asarray(d).shape[0])


def _sharp_init_magnitude(x0, d, pos):
    return np.abs(np.asarray(d, complex)) * O.extract(np.asarray(x0, complex), pos, np.asarray(d).shape[0])


MUTATIONS = {
    "dft_sign": ("dft2", lambda a: np.fft.ifft2(np.asarray(a, complex), norm="ortho")),
    "dft_unnormalised": ("dft2", lambda a: np.fft.fft2(np.asarray(a, complex))),
    "agent_conj_probe": ("agent", _agent_conj_probe),
    "agent_swapped_blend": ("agent", _agent_swapped_blend),
    "no_zero_fraction_rule": ("fourier_magnitude_step", _mag_no_zero_rule),
    "weights_squared": ("consensus_weights", _weights_squared),
    "no_lambda_normalisation": ("inv_weight_image", _inv_weight_identity),
    "reflection_sign": ("pmace_step", _step_wrong_reflection),
    "mann_sign": ("pmace_step", _step_wrong_sign),
    "nrmse_theta_conj": ("nrmse", _nrmse_conj_theta),
    "sharp_init_conj_probe": ("sharp_plus_init", _sharp_init_conj_probe),
    "sharp_init_transposed_probe": ("sharp_plus_init", _sharp_init_transposed_probe),
    "sharp_init_probe_magnitude": ("sharp_plus_init", _sharp_init_magnitude),
}


def test_pins_pass_unmutated():
    assert _count_failures() == 0


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(O, attr, fn)
    assert _count_failures() >= 1, f"planted mistake '{name}' passed every pin"
