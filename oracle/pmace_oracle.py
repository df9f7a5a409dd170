"""FP64 CPU oracle for PMACE (Projected Multi-Agent Consensus Equilibrium).

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow reference that the
HIP path is checked against.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import it; the product path never does.
It shares no code with the HIP library: every step below is written directly
from the paper's equations in complex128 with NumPy, with no blocking, fusion
or reordering beyond what the equations state.

Notation (Sec. II and III-A): x is the N1 x N2 complex object, d the Np x Np
known probe with D = Diag(d), P_j extracts the Np x Np patch whose top-left
corner is pos[j] = (row, col), P_j^t back-projects (zero-filled) a patch into
the object grid, F is the 2-D orthonormal DFT and y_j = sqrt(z_j) are the
measured amplitudes.

Readings of points the paper leaves open (each is repeated in the design
notes of the repository):
  * DFT convention (Sec. II, "2D orthonormal"): forward kernel
    exp(-2 pi i (k m + l n)/Np) / Np, DC at index [0, 0] (numpy 'ortho').
  * Where the probe vanishes, eq. (6) does not constrain v; the tie is broken
    with v = x_j there, so the agent returns its input at those pixels.
  * Where Lambda = 0 (pixel seen by no patch, or only by zero-probe pixels)
    Lambda^{-1} is taken as 0, so the consensus image is 0 there.
  * Back-projections are summed in ascending j.
  * The "fraction is 0 where w_j is 0" rule (Sec. III-A, below eq. (7)) is
    applied with an exact == 0 test.
  * NRMSE (eq. (17)): theta = arg sum(conj(x) * xhat) minimises the
    numerator in closed form (theta := 0 when the sum is 0); the norms are
    taken over an optional boolean region.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "dft2", "idft2", "extract", "back_project", "amplitudes",
    "consensus_weights", "weight_image", "inv_weight_image",
    "fourier_magnitude_step", "agent", "agent_stack", "consensus",
    "weighted_average", "T_operator", "pmace_step", "PMACEState",
    "pmace_init", "pmace_iterate", "pmace_solve", "reconstruct", "nrmse",
    "data_fit_cost", "sharp_magnitude_projection", "sharp_overlap_projection",
    "sharp_plus_init", "sharp_plus_step", "sharp_plus_reconstruct",
]


# --------------------------------------------------------------------------
# Operators of Sec. II: F, P_j, P_j^t, y_j
# --------------------------------------------------------------------------

def dft2(a: np.ndarray) -> np.ndarray:
    """F: 2-D orthonormal DFT over the last two axes (Sec. II, eq. (1))."""
    return np.fft.fft2(np.asarray(a, dtype=np.complex128), norm="ortho")


def idft2(a: np.ndarray) -> np.ndarray:
    """F^* = F^{-1}: adjoint of the orthonormal DFT (Sec. III-A, eq. (9))."""
    return np.fft.ifft2(np.asarray(a, dtype=np.complex128), norm="ortho")


def extract(x: np.ndarray, pos: np.ndarray, np_: int) -> np.ndarray:
    """Stacked patches [P_j x]_j, shape (J, Np, Np) (Sec. II; Alg. 1 initialisation)."""
    out = np.empty((len(pos), np_, np_), dtype=np.complex128)
    for j, (r, c) in enumerate(pos):
        out[j] = x[r:r + np_, c:c + np_]
    return out


def back_project(patches: np.ndarray, pos: np.ndarray, shape) -> np.ndarray:
    """sum_j P_j^t patches[j] into an image of `shape`, summed in ascending j."""
    np_ = patches.shape[-1]
    img = np.zeros(shape, dtype=np.result_type(patches.dtype, np.float64))
    for j, (r, c) in enumerate(pos):
        img[r:r + np_, c:c + np_] += patches[j]
    return img


def amplitudes(z: np.ndarray) -> np.ndarray:
    """y_j = sqrt(z_j): measured amplitudes (Sec. II, eq. (2))."""
    return np.sqrt(np.asarray(z, dtype=np.float64))


# --------------------------------------------------------------------------
# Consensus weights of Sec. III-A, eq. (11)
# --------------------------------------------------------------------------

def consensus_weights(d: np.ndarray, kappa: float) -> np.ndarray:
    """|D|^kappa as an Np x Np real array (eq. (11))."""
    return np.abs(np.asarray(d, dtype=np.complex128)) ** kappa


def weight_image(d: np.ndarray, pos: np.ndarray, shape, kappa: float) -> np.ndarray:
    """Lambda = sum_j P_j^t |D|^kappa (eq. (11))."""
    w = consensus_weights(d, kappa)
    return back_project(np.broadcast_to(w, (len(pos),) + w.shape), pos, shape)


def inv_weight_image(lam: np.ndarray) -> np.ndarray:
    """Lambda^{-1}, with 0 where Lambda = 0 (uncovered pixels)."""
    out = np.zeros_like(lam)
    nz = lam != 0
    out[nz] = 1.0 / lam[nz]
    return out


# --------------------------------------------------------------------------
# The data agent F_j of Sec. III-A, eqs. (6)-(9)
# --------------------------------------------------------------------------

def fourier_magnitude_step(W: np.ndarray, y: np.ndarray) -> np.ndarray:
    """y * W / |W| with the fraction taken as 0 where W is 0 (Sec. III-A,
    the phase argument below eq. (7)).  This is the alpha = 0 minimiser u* of
    eq. (7)."""
    W = np.asarray(W, dtype=np.complex128)
    mag = np.abs(W)
    frac = np.zeros_like(W)
    nz = mag != 0
    frac[nz] = W[nz] / mag[nz]
    return y * frac


def agent(xj: np.ndarray, d: np.ndarray, yj: np.ndarray, alpha: float) -> np.ndarray:
    """Probe-weighted proximal map F_j(x_j), closed form eq. (9):

        F_j(x_j) = (alpha x_j + D^{-1} F^* ( y_j (F D x_j)/|F D x_j| )) / (1 + alpha)

    Where d = 0 the data term is replaced by x_j (tie-break of eq. (6))."""
    xj = np.asarray(xj, dtype=np.complex128)
    d = np.asarray(d, dtype=np.complex128)
    W = dft2(d * xj)                              # F D x_j
    back = idft2(fourier_magnitude_step(W, yj))   # F^*( y_j W/|W| )
    data_point = xj.copy()
    nz = d != 0
    data_point[..., nz] = back[..., nz] / d[nz]   # D^{-1}( . )
    return (alpha * xj + data_point) / (1.0 + alpha)


def agent_stack(v: np.ndarray, d: np.ndarray, y: np.ndarray, alpha: float) -> np.ndarray:
    """Stacked operator F(v) = [F_j(v_j)]_j (eq. (10))."""
    return np.stack([agent(v[j], d, y[j], alpha) for j in range(v.shape[0])])


# --------------------------------------------------------------------------
# The consensus operator G of Sec. III-A, eqs. (10)-(11)
# --------------------------------------------------------------------------

def weighted_average(u: np.ndarray, d: np.ndarray, pos: np.ndarray, shape,
                     kappa: float) -> np.ndarray:
    """Lambda^{-1} sum_i P_i^t |D|^kappa u_i: the full-image weighted average of
    eq. (11), also the reconstruction returned by Alg. 1."""
    w = consensus_weights(d, kappa)
    num = back_project(w * u, pos, shape)
    lam = weight_image(d, pos, shape, kappa)
    return inv_weight_image(lam) * num


def consensus(u: np.ndarray, d: np.ndarray, pos: np.ndarray, shape,
              kappa: float) -> np.ndarray:
    """G(u) = [P_j xbar]_j with xbar the weighted average above (eq. (11))."""
    xbar = weighted_average(u, d, pos, shape, kappa)
    return extract(xbar, pos, u.shape[-1])


def T_operator(v, d, y, pos, shape, alpha, kappa):
    """T = (2G - I)(2F - I) (eq. (12))."""
    r = 2.0 * agent_stack(v, d, y, alpha) - v
    return 2.0 * consensus(r, d, pos, shape, kappa) - r


# --------------------------------------------------------------------------
# Algorithm 1 (Mann iteration for the PMACE solution)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class PMACEState:
    v: np.ndarray          # stacked agent states, (J, Np, Np) complex128
    w: np.ndarray          # last agent output F(v) (equals v after initialisation)
    z: Optional[np.ndarray]  # last consensus output G(2w - v)
    k: int                 # iterations taken


def pmace_init(x0: np.ndarray, pos: np.ndarray, np_: int) -> PMACEState:
    """Alg. 1 initialisation: w = v = [P_j x^(0)]_j."""
    v = extract(np.asarray(x0, dtype=np.complex128), pos, np_)
    return PMACEState(v=v, w=v.copy(), z=None, k=0)


def pmace_step(v, d, y, pos, shape, alpha, kappa, rho):
    """One pass of the Alg. 1 loop body; returns (v_new, w, z)."""
    w = agent_stack(v, d, y, alpha)                        # w <- F(v)
    z = consensus(2.0 * w - v, d, pos, shape, kappa)       # z <- G(2w - v)
    v_new = v + 2.0 * rho * (z - w)                        # v <- v + 2 rho (z - w)
    return v_new, w, z


def pmace_iterate(state: PMACEState, d, y, pos, shape, alpha, kappa, rho,
                  n_iter: int) -> PMACEState:
    v = state.v
    w, z = state.w, state.z
    for _ in range(n_iter):
        v, w, z = pmace_step(v, d, y, pos, shape, alpha, kappa, rho)
    return PMACEState(v=v, w=w, z=z, k=state.k + n_iter)


def reconstruct(state: PMACEState, d, pos, shape, kappa) -> np.ndarray:
    """Alg. 1 output: xhat = Lambda^{-1} sum_j P_j^t |D|^kappa v_j."""
    return weighted_average(state.v, d, pos, shape, kappa)


def pmace_solve(x0, d, z, pos, alpha, kappa, rho, n_iter: int,
                x_true: Optional[np.ndarray] = None,
                mask: Optional[np.ndarray] = None,
                record: bool = False):
    """Run Alg. 1 for n_iter iterations from x0.

    Returns (xhat, state, history) where history holds, per iteration, the
    reconstruction (if record) and the NRMSE against x_true (if given)."""
    d = np.asarray(d, dtype=np.complex128)
    y = amplitudes(z)
    shape = np.asarray(x0).shape
    np_ = d.shape[0]
    st = pmace_init(x0, pos, np_)
    hist = {"xhat": [], "v": [], "nrmse": []}
    for _ in range(n_iter):
        st = pmace_iterate(st, d, y, pos, shape, alpha, kappa, rho, 1)
        if record or x_true is not None:
            xh = reconstruct(st, d, pos, shape, kappa)
            if record:
                hist["xhat"].append(xh)
                hist["v"].append(st.v.copy())
            if x_true is not None:
                hist["nrmse"].append(nrmse(xh, x_true, mask))
    return reconstruct(st, d, pos, shape, kappa), st, hist


# --------------------------------------------------------------------------
# Evaluation: eq. (17) and the data-fit cost of eq. (4)
# --------------------------------------------------------------------------

def nrmse(xhat: np.ndarray, x: np.ndarray, mask: Optional[np.ndarray] = None) -> float:
    """e = ||xhat - e^{i theta} x|| / ||x|| with theta minimising the numerator
    (eq. (17)).  theta = arg sum conj(x) xhat is the closed-form minimiser."""
    xhat = np.asarray(xhat, dtype=np.complex128)
    x = np.asarray(x, dtype=np.complex128)
    if mask is not None:
        xhat = xhat[mask]
        x = x[mask]
    c = np.vdot(x, xhat)                  # sum conj(x) * xhat
    theta = np.angle(c) if c != 0 else 0.0
    num = np.linalg.norm(xhat - np.exp(1j * theta) * x)
    return float(num / np.linalg.norm(x))


def data_fit_cost(v: np.ndarray, d: np.ndarray, y: np.ndarray,
                  sigma_n2: float = 1.0) -> float:
    """sum_j f_j(v_j) = sum_j ||y_j - |F D v_j|||^2 / (2 sigma_n^2) (eq. (4))."""
    W = dft2(np.asarray(d, dtype=np.complex128) * v)
    return float(np.sum((y - np.abs(W)) ** 2) / (2.0 * sigma_n2))


# --------------------------------------------------------------------------
# SHARP+ (Sec. III-B, eqs. (14)-(15), Alg. 2), the paper's comparison method
# built from the same operators.  It acts on frames s_j = D P_j x.
# --------------------------------------------------------------------------

def sharp_magnitude_projection(s, y):
    """P_a: F^*( y F s / |F s| ) per frame (eq. (14)); 0 where F s = 0."""
    return idft2(fourier_magnitude_step(dft2(s), y))


def sharp_overlap_projection(s, d, pos, shape):
    """P_Q: D P_j (sum_k P_k^t |D|^2)^{-1} sum_i P_i^t D^* s_i (eq. (15))."""
    d = np.asarray(d, dtype=np.complex128)
    num = back_project(np.conj(d) * s, pos, shape)
    lam = back_project(np.broadcast_to(np.abs(d) ** 2, s.shape), pos, shape)
    img = inv_weight_image(lam.real) * num
    return d * extract(img, pos, d.shape[0])


def sharp_plus_init(x0, d, pos):
    """Alg. 2 initialisation: s_j = D P_j x^(0)."""
    return np.asarray(d, dtype=np.complex128) * extract(np.asarray(x0, dtype=np.complex128), pos,
                                                         np.asarray(d).shape[0])


def sharp_plus_step(s, d, y, pos, shape, beta):
    """s <- [2 beta P_Q P_a + (1 - 2 beta) P_a - beta (P_Q - I)] s  (Alg. 2 loop body)."""
    pa = sharp_magnitude_projection(s, y)
    return (2.0 * beta * sharp_overlap_projection(pa, d, pos, shape) + (1.0 - 2.0 * beta) * pa
            - beta * (sharp_overlap_projection(s, d, pos, shape) - s))


def sharp_plus_reconstruct(s, d, pos, shape):
    """Alg. 2 output: (sum_k P_k^t |D|^2)^{-1} sum_j P_j^t D^* s_j."""
    d = np.asarray(d, dtype=np.complex128)
    num = back_project(np.conj(d) * s, pos, shape)
    lam = back_project(np.broadcast_to(np.abs(d) ** 2, s.shape), pos, shape)
    return inv_weight_image(lam.real) * num
