"""Seeded synthetic ptychography problems shaped like the paper's experiments.

This module only *makes inputs*: an object, a probe, a raster of scan
positions and simulated diffraction intensities.  It holds none of the
reconstruction method's arithmetic (no agent, no consensus, no Mann update);
the HIP path and the FP64 oracle both consume what it returns and share
nothing else.

Data model (Sec. II, eq. (1)): the detector records z_j = Pois(|F D P_j x|^2)
where F is the 2-D orthonormal DFT, D = Diag(d) the known probe and P_j the
patch extractor.  Noisy data follow eq. (16): the noiseless intensities are
scaled so that the brightest detector pixel has mean r_p photons before the
Poisson draw.  The paper's max(.) is read as the maximum over *all* positions
and pixels (one scale per experiment); the scale is folded into the returned
probe so that the object keeps its units.

The paper's own test object and probe (a 660x660 image and a 256x256 probe,
Sec. IV) are not public; these seeded stand-ins have the shapes, overlaps and
noise levels of the paper's experiments:

* object: magnitude and phase are two independent white Gaussian fields,
  periodically low-passed with a Gaussian of 4 px standard deviation and
  min-max mapped to magnitude [0.5, 1] and phase [-pi/2, pi/2];
* probe: Gaussian amplitude (sigma = Np/4, centred at ((Np-1)/2, (Np-1)/2))
  times a quadratic phase exp(i*pi*(2r/Np)^2), peak amplitude 1 before the
  photon scaling;
* scan: an n x n raster with step s, centred in the object, integer jitter
  uniform in {-2..2} per axis, clamped so every patch lies inside the object,
  ordered row-major;
* intensities: DC at index [0, 0] (unshifted DFT layout), float32.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np
from scipy import ndimage

__all__ = [
    "Problem", "CONFIGS", "make_object", "make_probe", "make_positions", "make_positions_rect",
    "simulate_intensities", "make_problem", "make_config_problem",
    "draw_mix_specs", "roi_mask",
]


@dataclasses.dataclass
class Problem:
    """One reconstruction problem (all arrays on the host)."""
    x_true: np.ndarray          # (N1, N2) complex128 ground-truth transmittance
    probe: np.ndarray           # (Np, Np) complex128 probe d (photon-scaled)
    pos: np.ndarray             # (J, 2) int32 top-left (row, col) of each patch
    z: np.ndarray               # (J, Np, Np) float32 intensities, DC at [0, 0]
    peak_photons: Optional[float]  # r_p of eq. (16); None = noiseless
    name: str = ""

    @property
    def n1(self) -> int:
        return self.x_true.shape[0]

    @property
    def n2(self) -> int:
        return self.x_true.shape[1]

    @property
    def np_(self) -> int:
        return self.probe.shape[0]

    @property
    def num_pos(self) -> int:
        return self.pos.shape[0]

    @property
    def patch_pixels(self) -> int:
        return self.num_pos * self.np_ * self.np_


# The three single-reconstruction workloads (object side n, probe side np_,
# scan side, raster step in px, Poisson peak r_p or None, iteration budget).
CONFIGS: Dict[str, dict] = {
    "c1": dict(n=128, np_=32, scan=6, step=16, peak=None, iters=50, seed=1),
    "c2": dict(n=512, np_=128, scan=15, step=24, peak=1e5, iters=100, seed=2),
    "c3": dict(n=1024, np_=256, scan=40, step=20, peak=1e6, iters=100, seed=3),
}
KAPPA = 1.25   # probe exponent of the consensus weights (Sec. IV)
RHO = 0.5      # Mann averaging parameter (Sec. IV)


def make_object(n1: int, n2: int, rng: np.random.Generator,
                sigma_px: float = 4.0) -> np.ndarray:
    """Smooth random complex transmittance with |x| in [0.5,1], arg x in [-pi/2,pi/2]."""
    def field():
        g = rng.standard_normal((n1, n2))
        g = ndimage.gaussian_filter(g, sigma=sigma_px, mode="wrap")
        lo, hi = g.min(), g.max()
        return (g - lo) / (hi - lo) if hi > lo else np.zeros_like(g)
    mag = 0.5 + 0.5 * field()
    phase = -0.5 * math.pi + math.pi * field()
    return mag * np.exp(1j * phase)


def make_probe(np_: int) -> np.ndarray:
    """Gaussian probe with quadratic phase, sigma = Np/4, centred between pixels."""
    c = (np_ - 1) / 2.0
    ii, jj = np.meshgrid(np.arange(np_), np.arange(np_), indexing="ij")
    r2 = (ii - c) ** 2 + (jj - c) ** 2
    sigma = np_ / 4.0
    amp = np.exp(-r2 / (2.0 * sigma * sigma))
    phase = math.pi * (4.0 * r2 / (np_ * np_))   # pi * (2 r / Np)^2
    return amp * np.exp(1j * phase)


def make_positions(n_obj: int, np_: int, scan: int, step: int,
                   rng: np.random.Generator, jitter: int = 2) -> np.ndarray:
    """Centred, jittered, clamped n x n raster of top-left patch offsets (row-major)."""
    span = (scan - 1) * step + np_
    off = (n_obj - span) // 2
    base = off + step * np.arange(scan)
    rows = np.repeat(base, scan)
    cols = np.tile(base, scan)
    jit = rng.integers(-jitter, jitter + 1, size=(scan * scan, 2))
    pos = np.stack([rows, cols], axis=1) + jit
    pos = np.clip(pos, 0, n_obj - np_)
    return pos.astype(np.int32)


def make_positions_rect(n1: int, n2: int, np_: int, scan1: int, scan2: int, step: int,
                        rng: np.random.Generator, jitter: int = 2) -> np.ndarray:
    """As make_positions for a rectangular object: a centred scan1 x scan2
    raster (row-major, jittered, clamped)."""
    def axis(n, scan):
        return (n - ((scan - 1) * step + np_)) // 2 + step * np.arange(scan)
    rows = np.repeat(axis(n1, scan1), scan2)
    cols = np.tile(axis(n2, scan2), scan1)
    jit = rng.integers(-jitter, jitter + 1, size=(scan1 * scan2, 2))
    pos = np.stack([rows, cols], axis=1) + jit
    pos[:, 0] = np.clip(pos[:, 0], 0, n1 - np_)
    pos[:, 1] = np.clip(pos[:, 1], 0, n2 - np_)
    return pos.astype(np.int32)


def _patch_intensities(x: np.ndarray, d: np.ndarray, pos: np.ndarray) -> np.ndarray:
    """|F D P_j x|^2 for every position (eq. (1) without the Poisson draw), float64."""
    np_ = d.shape[0]
    out = np.empty((pos.shape[0], np_, np_), dtype=np.float64)
    chunk = 64
    for a in range(0, pos.shape[0], chunk):
        b = min(a + chunk, pos.shape[0])
        frames = np.stack([d * x[r:r + np_, c:c + np_] for r, c in pos[a:b]])
        spec = np.fft.fft2(frames, norm="ortho")
        out[a:b] = spec.real ** 2 + spec.imag ** 2
    return out


def simulate_intensities(x: np.ndarray, d: np.ndarray, pos: np.ndarray,
                         peak: Optional[float], rng: np.random.Generator):
    """Return (z float32, probe actually illuminating) per eq. (1)/(16)."""
    inten = _patch_intensities(x, d, pos)
    if peak is None:
        return inten.astype(np.float32), d
    scale = peak / inten.max()
    lam = inten * scale
    z = rng.poisson(lam).astype(np.float32)
    return z, d * math.sqrt(scale)


def make_problem(n: int, np_: int, scan: int, step: int, peak: Optional[float],
                 seed: int, name: str = "", n2: Optional[int] = None,
                 scan2: Optional[int] = None) -> Problem:
    """Build one seeded problem.  RNG draw order: object, jitter, Poisson.
    With scan2 the raster is scan x scan2 (rows x columns) on an n x n2 object."""
    n2 = n if n2 is None else n2
    rng = np.random.default_rng(seed)
    x = make_object(n, n2, rng)
    d = make_probe(np_)
    if scan2 is not None:
        pos = make_positions_rect(n, n2, np_, scan, scan2, step, rng)
    elif n2 != n:
        pr = make_positions(n, np_, scan, step, rng)
        pc = make_positions(n2, np_, scan, step, rng)
        pos = np.stack([pr[:, 0], pc[:, 1]], axis=1).astype(np.int32)
    else:
        pos = make_positions(n, np_, scan, step, rng)
    z, d_eff = simulate_intensities(x, d, pos, peak, rng)
    return Problem(x_true=x, probe=d_eff, pos=pos, z=z, peak_photons=peak, name=name)


def make_config_problem(cfg: str) -> Problem:
    c = CONFIGS[cfg]
    return make_problem(c["n"], c["np_"], c["scan"], c["step"], c["peak"], c["seed"], name=cfg)


def draw_mix_specs(count: int = 64, seed: int = 4, peak: float = 1e5) -> List[dict]:
    """Sizes of the mixed-size batch: object side {256,512,1024}, probe side
    {64,128,256} (redrawn while Np > N/2), scan side uniform in 7..30, step
    chosen so the raster fits and overlap is at least 50%.  Item i is seeded
    with 1000*seed + i."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        while True:
            n = int(rng.choice([256, 512, 1024]))
            np_ = int(rng.choice([64, 128, 256]))
            if np_ <= n // 2:
                break
        scan = int(rng.integers(7, 31))
        step = max(1, min((n - np_ - 4) // (scan - 1), np_ // 2))
        specs.append(dict(n=n, np_=np_, scan=scan, step=step, peak=peak,
                          seed=1000 * seed + i, name=f"mix{i}"))
    return specs


def roi_mask(probe: np.ndarray, pos: np.ndarray, n1: int, n2: int,
             frac: float = 0.01) -> np.ndarray:
    """Evaluation region for NRMSE: the union over positions of the probe
    footprint where |d|^2 >= frac * max |d|^2 (the well-illuminated pixels)."""
    np_ = probe.shape[0]
    p2 = np.abs(probe) ** 2
    lit = p2 >= frac * p2.max()
    mask = np.zeros((n1, n2), dtype=bool)
    for r, c in pos:
        mask[r:r + np_, c:c + np_] |= lit
    return mask
