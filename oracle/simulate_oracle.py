"""Reference for simulated measurements (FP64, CPU).

TEST INFRASTRUCTURE ONLY: used by the test suite to check the device
simulator; never imported by the product path.  Written from the
definitions, sharing no code with the HIP library.

* Forward model, Sec. II eq. (1) without the detector noise:
  I_j = |F D P_j x|^2 with F the 2-D orthonormal DFT.
* Noisy data, Sec. IV eq. (16): z_j = Pois(I_j * r_p / max I), the maximum
  over every position and pixel.
* Random numbers: the counter-based generator Philox4x32-10 (Salmon, Moraes,
  Dror, Shaw, SC 2011).  The stream of element i under a seed is block n =
  Philox(counter = (i mod 2^32, i >> 32, n, 0x50495853), key = (seed mod 2^32,
  seed >> 32)); each block gives two uniforms from (word0, word1) and
  (word2, word3) as (a >> 5, b >> 6) -> ((a>>5) * 2^26 + (b>>6) + 0.5) / 2^53.
* Poisson variates: product of uniforms below mean 10; Hormann's transformed
  rejection with squeeze (PTRS, 1993) from mean 10 up.
"""
from __future__ import annotations

import math

import numpy as np

_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = 0xFFFFFFFF


def forward_intensities(x, d, pos) -> np.ndarray:
    """|F D P_j x|^2 for every position (eq. (1)), FP64."""
    x = np.asarray(x, np.complex128)
    d = np.asarray(d, np.complex128)
    np_ = d.shape[0]
    out = np.empty((len(pos), np_, np_))
    for j, (r, c) in enumerate(pos):
        W = np.fft.fft2(d * x[r:r + np_, c:c + np_], norm="ortho")
        out[j] = W.real ** 2 + W.imag ** 2
    return out


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on a 4-word counter and a 2-word key."""
    c0, c1, c2, c3 = (int(v) & _MASK for v in ctr)
    k0, k1 = (int(v) & _MASK for v in key)
    for _ in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        c0, c1, c2, c3 = (p1 >> 32) ^ c1 ^ k0, p1 & _MASK, (p0 >> 32) ^ c3 ^ k1, p0 & _MASK
        k0, k1 = (k0 + _W0) & _MASK, (k1 + _W1) & _MASK
    return c0, c1, c2, c3


class Uniforms:
    """Uniform variates in (0, 1) of element `idx` under `seed` (see module doc)."""

    def __init__(self, seed: int, idx: int):
        self.key = (seed & _MASK, (seed >> 32) & _MASK)
        self.i0, self.i1 = idx & _MASK, (idx >> 32) & _MASK
        self.n = 0
        self.buf = []

    def next(self) -> float:
        if not self.buf:
            w = philox4x32_10((self.i0, self.i1, self.n, 0x50495853), self.key)
            self.n += 1
            self.buf = [(w[0], w[1]), (w[2], w[3])]
        a, b = self.buf.pop(0)
        return ((a >> 5) * 67108864.0 + (b >> 6) + 0.5) / 9007199254740992.0


def poisson_draw(lam: float, u: Uniforms) -> float:
    if not lam > 0.0:
        return 0.0
    if lam < 10.0:
        L = math.exp(-lam)
        p, k = 1.0, 0
        while True:
            k += 1
            p *= u.next()
            if not (p > L and k < 1000):
                break
        return float(k - 1)
    slam, loglam = math.sqrt(lam), math.log(lam)
    b = 0.931 + 2.53 * slam
    a = -0.059 + 0.02483 * b
    invalpha = 1.1239 + 1.1328 / (b - 3.4)
    vr = 0.9277 - 3.6224 / (b - 2.0)
    for _ in range(1000):
        U = u.next() - 0.5
        V = u.next()
        us = 0.5 - abs(U)
        k = math.floor((2.0 * a / us + b) * U + lam + 0.43)
        if us >= 0.07 and V <= vr:
            return float(k)
        if k < 0 or (us < 0.013 and V > us):
            continue
        if (math.log(V) + math.log(invalpha) - math.log(a / (us * us) + b)
                <= -lam + k * loglam - math.lgamma(k + 1.0)):
            return float(k)
    return float(math.floor(lam + 0.5))


def poisson(lams, seed: int) -> np.ndarray:
    """Element i of the flattened means draws from the stream of index i."""
    lams = np.asarray(lams, np.float64).ravel()
    return np.array([poisson_draw(float(l), Uniforms(seed, i)) for i, l in enumerate(lams)])


def simulate(x, d, pos, peak, seed: int):
    """(z, scale): noise-free intensities, or Poisson counts at peak rate `peak`
    with the global-max scaling of eq. (16)."""
    inten = forward_intensities(x, d, pos)
    if not peak or peak <= 0:
        return inten, 1.0
    scale = peak / inten.max()
    return poisson(inten * scale, seed).reshape(inten.shape), scale
