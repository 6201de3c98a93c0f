"""Seeded synthetic inputs for Cartesian dynamic parallel MRI.

This module draws phantoms, coil sensitivity maps, phase-encode sampling masks
and k-space noise.  It holds none of the reconstruction's arithmetic: no
Fourier transform, no measurement operator, no solver step.  Both the FP64
oracle tests and the GPU path take their inputs from here, so the two sides
always see identical data.

The paper's experiment (Sec. V) uses a measured cardiac cine series (32-coil
body array, 128x128, 22 frames) that is not available; the generators below
stand in for it with the same structure:

* images are normalised so that the largest magnitude over the series is 1,
  as the paper normalises its fully sampled reconstruction (Sec. V);
* only phase-encode (vertical, ky) lines are subsampled, a fresh variable
  density random pattern per frame, with a fully sampled centre band
  (Sec. II-A, eq. mri_csmcoill2 and Fig. 1; Sec. V);
* coil maps are smooth complex profiles normalised to sum-of-squares 1;
* noise is circular complex Gaussian with E|n|^2 = sigma^2, drawn only where
  k-space is sampled.

Array layouts (C order, last index fastest):
  image  x    : (nt, nv, nh)       complex128
  coil   s    : (nc, nv, nh)       complex128
  mask        : (nt, nv)           uint8, 1 = phase-encode line acquired
  noise       : (nt, nc, nv, nh)   complex128, zero on unsampled lines
Index j runs over the vertical (phase-encode) axis and i over the horizontal
(readout) axis, as in eq. x_def.  Frequency index 0 is DC (no fftshift).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Problem",
    "phantom",
    "coil_maps",
    "vd_mask",
    "kspace_noise",
    "make_problem",
    "CONFIGS",
    "batch_slice_spec",
]


def _grid(nv: int, nh: int):
    """Normalised field-of-view coordinates in [-1, 1) (row = vertical)."""
    yy = (np.arange(nv) - nv / 2) / (nv / 2)
    xx = (np.arange(nh) - nh / 2) / (nh / 2)
    return np.meshgrid(yy, xx, indexing="ij")


def _ellipse(Y, X, cy, cx, ay, ax, angle):
    ca, sa = math.cos(angle), math.sin(angle)
    yr = (Y - cy) * ca - (X - cx) * sa
    xr = (Y - cy) * sa + (X - cx) * ca
    return ((yr / ay) ** 2 + (xr / ax) ** 2) <= 1.0


def phantom(nt: int, nv: int, nh: int, family: str, rng: np.random.Generator,
            period: float | None = None) -> np.ndarray:
    """Dynamic complex phantom, normalised to max |x| = 1.

    family:
      "ellipses3" -- 3 complex ellipses, centres U[-0.4,0.4]^2, semi-axes
                     U[0.15,0.4], amplitude U[0.3,1]*exp(i U[0,2pi)), radii
                     scaled by (1 + 0.2 sin(2 pi t / period + psi_k)).
      "cardiac"   -- body ellipse, 3 static organs and 2 pulsating ellipses
                     whose radii scale by (1 + 0.25 sin(2 pi t / period)).
      "periodic"  -- ellipses whose intensity is 1 + 0.5 cos(2 pi f_k t / nt
                     + psi_k), f_k in {1,2,3} (sparse in temporal frequency),
                     plus 2 ellipses whose radius varies with the given period.
    """
    Y, X = _grid(nv, nh)
    x = np.zeros((nt, nv, nh), dtype=np.complex128)
    if family == "ellipses3":
        period = period or 8.0
        for _ in range(3):
            cy, cx = rng.uniform(-0.4, 0.4, 2)
            ay, ax = rng.uniform(0.15, 0.4, 2)
            ang = rng.uniform(0, math.pi)
            amp = rng.uniform(0.3, 1.0) * np.exp(1j * rng.uniform(0, 2 * math.pi))
            psi = rng.uniform(0, 2 * math.pi)
            for t in range(nt):
                sc = 1.0 + 0.2 * math.sin(2 * math.pi * t / period + psi)
                x[t][_ellipse(Y, X, cy, cx, ay * sc, ax * sc, ang)] += amp
    elif family == "cardiac":
        period = period or 16.0
        body_phase = np.exp(1j * rng.uniform(0, 2 * math.pi))
        body = _ellipse(Y, X, 0.0, 0.0, 0.85, 0.7, 0.0)
        organs = []
        for _ in range(3):
            cy, cx = rng.uniform(-0.45, 0.45, 2)
            ay, ax = rng.uniform(0.08, 0.2, 2)
            amp = rng.uniform(0.2, 0.6) * np.exp(1j * rng.uniform(-0.5, 0.5))
            organs.append((_ellipse(Y, X, cy, cx, ay, ax, rng.uniform(0, math.pi)), amp))
        pulsing = []
        for _ in range(2):
            cy, cx = rng.uniform(-0.3, 0.3, 2)
            ay, ax = rng.uniform(0.1, 0.2, 2)
            amp = rng.uniform(0.4, 0.8) * np.exp(1j * rng.uniform(-0.5, 0.5))
            pulsing.append((cy, cx, ay, ax, rng.uniform(0, math.pi), amp))
        for t in range(nt):
            frame = 0.3 * body_phase * body.astype(np.complex128)
            for msk, amp in organs:
                frame[msk] += amp
            sc = 1.0 + 0.25 * math.sin(2 * math.pi * t / period)
            for cy, cx, ay, ax, ang, amp in pulsing:
                frame[_ellipse(Y, X, cy, cx, ay * sc, ax * sc, ang)] += amp
            x[t] = frame
    elif family == "periodic":
        period = period or 20.0
        shapes = []
        for _ in range(4):
            cy, cx = rng.uniform(-0.45, 0.45, 2)
            ay, ax = rng.uniform(0.1, 0.3, 2)
            f = int(rng.integers(1, 4))
            psi = rng.uniform(0, 2 * math.pi)
            amp = rng.uniform(0.3, 0.8) * np.exp(1j * rng.uniform(0, 2 * math.pi))
            shapes.append((_ellipse(Y, X, cy, cx, ay, ax, rng.uniform(0, math.pi)), f, psi, amp))
        moving = []
        for _ in range(2):
            cy, cx = rng.uniform(-0.3, 0.3, 2)
            ay, ax = rng.uniform(0.08, 0.18, 2)
            amp = rng.uniform(0.3, 0.6) * np.exp(1j * rng.uniform(0, 2 * math.pi))
            moving.append((cy, cx, ay, ax, rng.uniform(0, math.pi), amp))
        for t in range(nt):
            for msk, f, psi, amp in shapes:
                x[t][msk] += amp * (1.0 + 0.5 * math.cos(2 * math.pi * f * t / nt + psi))
            sc = 1.0 + 0.2 * math.sin(2 * math.pi * t / period)
            for cy, cx, ay, ax, ang, amp in moving:
                x[t][_ellipse(Y, X, cy, cx, ay * sc, ax * sc, ang)] += amp
    else:
        raise ValueError(f"unknown phantom family {family!r}")
    peak = np.abs(x).max()
    if peak > 0:
        x /= peak
    return x


def coil_maps(nc: int, nv: int, nh: int, rng: np.random.Generator,
              radius: float = 1.5, sigma: float = 1.0) -> np.ndarray:
    """Smooth complex coil sensitivities, sum-of-squares normalised to 1.

    Coil c has a Gaussian magnitude profile centred on a circle of the given
    radius (normalised coordinates), a constant phase and a small linear phase
    ramp.  Normalisation makes sum_c |s_c|^2 = 1 at every pixel.
    """
    Y, X = _grid(nv, nh)
    s = np.empty((nc, nv, nh), dtype=np.complex128)
    for c in range(nc):
        ang = 2 * math.pi * c / nc
        cy, cx = radius * math.sin(ang), radius * math.cos(ang)
        mag = np.exp(-((Y - cy) ** 2 + (X - cx) ** 2) / (2 * sigma ** 2))
        ph0 = rng.uniform(0, 2 * math.pi)
        gy, gx = rng.uniform(-0.5, 0.5, 2)
        s[c] = mag * np.exp(1j * (ph0 + gy * Y + gx * X))
    sos = np.sqrt((np.abs(s) ** 2).sum(axis=0))
    return s / sos


def vd_mask(nt: int, nv: int, accel: float, ncenter: int,
            rng: np.random.Generator) -> np.ndarray:
    """Variable-density random phase-encode mask, a fresh draw per frame.

    Each frame keeps m = round(nv / accel) lines: the ncenter lines of lowest
    |ky| (indices wrap, DC at 0), plus lines drawn without replacement from
    the rest with probability proportional to (1 - |k|)^2, k = ky / (nv/2).
    """
    m = int(round(nv / accel))
    m = max(min(m, nv), 0)
    ky = np.fft.fftfreq(nv, d=1.0 / nv)          # 0, 1, ..., -1 (integer ky)
    order = np.argsort(np.abs(ky), kind="stable")
    nctr = min(ncenter, m)
    centre = order[:nctr]
    rest = np.setdiff1d(np.arange(nv), centre)
    kn = np.abs(ky[rest]) / (nv / 2)
    p = (1.0 - kn) ** 2
    mask = np.zeros((nt, nv), dtype=np.uint8)
    for t in range(nt):
        mask[t, centre] = 1
        extra = m - nctr
        if extra > 0:
            pos = np.flatnonzero(p > 0)
            k = min(extra, pos.size)
            pick = rng.choice(rest[pos], size=k, replace=False, p=p[pos] / p[pos].sum())
            mask[t, pick] = 1
    return mask


def kspace_noise(mask: np.ndarray, nc: int, nh: int, sigma: float,
                 rng: np.random.Generator) -> np.ndarray:
    """Circular complex Gaussian noise, E|n|^2 = sigma^2, on sampled lines only."""
    nt, nv = mask.shape
    g = rng.standard_normal((nt, nc, nv, nh)) + 1j * rng.standard_normal((nt, nc, nv, nh))
    n = sigma / math.sqrt(2.0) * g
    return n * mask[:, None, :, None]


@dataclasses.dataclass
class Problem:
    """One synthetic dynamic slice: ground truth, coils, mask and noise.

    The measured data are y = A(x_true) + noise; forming them needs the
    measurement operator, which lives on each side (oracle or GPU), not here.
    """
    x_true: np.ndarray
    coil: np.ndarray
    mask: np.ndarray
    noise: np.ndarray
    prior: str            # "tv" or "dft"
    lam: float
    mu: float
    rho: float
    iters: int
    name: str = ""

    @property
    def shape(self):
        nt, nv, nh = self.x_true.shape
        return nt, nv, nh, self.coil.shape[0]


def make_problem(nv, nh, nt, nc, accel, ncenter, prior, family, seed,
                 lam=0.01, mu=0.1, rho=0.5, sigma=0.005, iters=100,
                 period=None, name=""):
    rng = np.random.default_rng(seed)
    x = phantom(nt, nv, nh, family, rng, period)
    s = coil_maps(nc, nv, nh, rng)
    m = vd_mask(nt, nv, accel, ncenter, rng)
    n = kspace_noise(m, nc, nh, sigma, rng)
    return Problem(x, s, m, n, prior, lam, mu, rho, iters, name)


def batch_slice_spec(s: int) -> dict:
    """Shape and prior of slice s (0..23) of the 24-slice uneven batch."""
    sizes = [(128, 96), (128, 128), (192, 128), (192, 192), (256, 192), (256, 256)]
    nv, nh = sizes[s // 4]
    nt = [16, 24, 32, 40][s % 4]
    nc = [8, 12, 16][s % 3]
    accel = [4, 6, 8, 10][(s // 2) % 4]
    prior = "tv" if s % 2 == 0 else "dft"
    return dict(nv=nv, nh=nh, nt=nt, nc=nc, accel=accel,
                ncenter=8 if nv == 128 else 12, prior=prior,
                family="cardiac" if prior == "tv" else "periodic",
                period=nt / 2, seed=2000 + s)


def _cfg1():
    return make_problem(64, 64, 8, 4, 4, 8, "tv", "ellipses3", 1001,
                        lam=0.01, mu=0.1, rho=0.5, sigma=0.01, iters=50, period=8.0,
                        name="tv-64x64x8-4c")


def _cfg2():
    return make_problem(256, 256, 32, 8, 8, 12, "tv", "cardiac", 1002,
                        sigma=0.005, iters=100, period=16.0, name="tv-256x256x32-8c")


def _cfg3():
    return make_problem(192, 192, 40, 12, 10, 8, "dft", "periodic", 1003,
                        sigma=0.005, iters=100, period=20.0, name="dft-192x192x40-12c")


def _cfg5():
    return make_problem(192, 192, 24, 12, 8, 12, "tv", "cardiac", 1005,
                        sigma=0.005, iters=20, period=12.0, name="tv-192x192x24-12c-unrolled")


def _paper(prior: str):
    """The shape of the paper's own experiment (Sec. V): 128x128 pixels, 22
    frames, 32 coils, R = 8 variable-density random lines per frame, with the
    paper's lambda = 0.002 and mu (= mu2) = 0.06, mu2 / mu1 = 0.5, 200
    iterations; a synthetic phantom stands in for its cardiac cine data."""
    fam = "cardiac" if prior == "tv" else "periodic"
    return make_problem(128, 128, 22, 32, 8, 8, prior, fam, 1006 if prior == "tv" else 1007,
                        lam=0.002, mu=0.06, rho=0.5, sigma=0.005, iters=200, period=11.0,
                        name=f"paper-{prior}-128x128x22-32c")


def batch_slice(s: int):
    """The seeded problem of slice s (0..23) of the 24-slice uneven batch."""
    sp = batch_slice_spec(s)
    return make_problem(sp["nv"], sp["nh"], sp["nt"], sp["nc"], sp["accel"], sp["ncenter"],
                        sp["prior"], sp["family"], sp["seed"], sigma=0.005, iters=100,
                        period=sp["period"], name=f"batch{s}")


# Named workloads.  Values are factories (drawing a large problem is not free).
CONFIGS = {
    "tv64": _cfg1,
    "tv256": _cfg2,
    "dft192": _cfg3,
    "tv192_unrolled": _cfg5,
    "paper128tv": lambda: _paper("tv"),
    "paper128dft": lambda: _paper("dft"),
}
