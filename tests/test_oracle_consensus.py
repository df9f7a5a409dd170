"""Pins of the oracle's consensus operator G (Sec. III-A, eqs. (10)-(11))."""
import numpy as np
import pytest

from conftest import cplx, load_golden
from oracle import pmace_oracle as O
from paper_2111_14240_amd import synth


def _setup(seed=2, n=40, np_=16, scan=4, step=8, kappa=1.25):
    rng = np.random.default_rng(seed)
    d = synth.make_probe(np_)
    pos = synth.make_positions(n, np_, scan, step, rng)
    J = len(pos)
    u = rng.standard_normal((J, np_, np_)) + 1j * rng.standard_normal((J, np_, np_))
    return d, pos, (n, n), u, kappa, rng


def test_golden_hand_example():
    g = load_golden("consensus_worked.json")
    d = cplx(g["probe"])
    u = cplx(g["u"])
    pos = np.asarray(g["pos"])
    shape = (g["n1"], g["n2"])
    lam = O.weight_image(d, pos, shape, g["kappa"])
    assert np.allclose(lam, np.asarray(g["lambda"], float))
    xbar = O.weighted_average(u, d, pos, shape, g["kappa"])
    assert np.allclose(xbar, cplx(g["xbar"]), atol=1e-14)
    z = O.consensus(u, d, pos, shape, g["kappa"])
    assert np.allclose(z[1], cplx(g["xbar"])[:, 1:3])


def test_reproduces_consistent_patches():
    d, pos, shape, u, kappa, rng = _setup()
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    lam = O.weight_image(d, pos, shape, kappa)
    x = np.where(lam > 0, x, 0)
    patches = O.extract(x, pos, d.shape[0])
    assert np.allclose(O.consensus(patches, d, pos, shape, kappa), patches, atol=1e-12)


def test_idempotent_and_reflection_involution():
    d, pos, shape, u, kappa, _ = _setup()
    g1 = O.consensus(u, d, pos, shape, kappa)
    assert np.allclose(O.consensus(g1, d, pos, shape, kappa), g1, atol=1e-12)
    r = 2 * g1 - u
    assert np.allclose(2 * O.consensus(r, d, pos, shape, kappa) - r, u, atol=1e-12)


def test_self_adjoint_in_weighted_inner_product():
    d, pos, shape, u, kappa, rng = _setup()
    b = rng.standard_normal(u.shape) + 1j * rng.standard_normal(u.shape)
    w = O.consensus_weights(d, kappa)

    def ip(a, c):
        return np.sum(w * np.conj(a) * c)

    lhs = ip(u, O.consensus(b, d, pos, shape, kappa))
    rhs = ip(O.consensus(u, d, pos, shape, kappa), b)
    assert np.allclose(lhs, rhs, rtol=1e-12)


def test_non_overlapping_scan_is_identity():
    np_ = 8
    d = synth.make_probe(np_)
    pos = np.array([[0, 0], [0, 8], [8, 0], [8, 8]])
    rng = np.random.default_rng(1)
    u = rng.standard_normal((4, np_, np_)) + 1j * rng.standard_normal((4, np_, np_))
    assert np.allclose(O.consensus(u, d, pos, (16, 16), 1.25), u, atol=1e-14)


def test_permutation_invariance_and_weights():
    d, pos, shape, u, kappa, rng = _setup()
    perm = rng.permutation(len(pos))
    a = O.weighted_average(u, d, pos, shape, kappa)
    b = O.weighted_average(u[perm], d, pos[perm], shape, kappa)
    assert np.allclose(a, b, atol=1e-13)
    # The weights are |d|^kappa: two patches on the same pixel average with
    # weights |d1|^kappa and |d2|^kappa.
    dsq = np.array([[1.0, 0.0], [0.0, 2.0j]])
    pos2 = np.array([[0, 0], [0, 0]])
    uu = np.zeros((2, 2, 2), complex)
    uu[0, 1, 1] = 3.0
    uu[1, 1, 1] = 7.0
    xb = O.weighted_average(uu, dsq, pos2, (2, 2), 2.0)
    assert xb[1, 1] == pytest.approx((4 * 3 + 4 * 7) / 8)
    assert xb[0, 1] == 0 and xb[1, 0] == 0             # zero probe => Lambda = 0 => 0
