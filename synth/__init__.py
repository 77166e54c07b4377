"""Seeded synthetic 4D-STEM inputs for the live WDD per-frame update.

This module simulates the microscope, not the reconstruction: it draws a
weak-phase object, forms a probe from a circular Fourier-space aperture and
produces far-field diffraction intensities (the forward model of Section 2,
equation "forward"), optionally with Poisson counting noise at a fixed dose
per frame (Section 8).  It holds none of the reconstruction's arithmetic and
serves the oracle, the tests and the benchmark alike.

Conventions (shared by every consumer of these inputs):
  * object O is an M x M complex array, periodic;
  * the probe window is N x N; patch_s[i, j] = O[(y_s*step + i) % M, (x_s*step + j) % M];
  * frames are fftshifted far-field intensities: DC at (N//2, N//2);
  * scan positions are integer raster indices (y, x), 0 <= y < Sy, 0 <= x < Sx.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence, Tuple, Union

import numpy as np

Range = Union[float, Tuple[float, float]]


def _draw(rng: np.random.Generator, spec: Range, n: int) -> np.ndarray:
    if isinstance(spec, (tuple, list)):
        return rng.uniform(spec[0], spec[1], size=n)
    return np.full(n, float(spec))


def phase_map(m: int, n_gauss: int, sigma: Range, amp: Range, seed: int) -> np.ndarray:
    """Sum of periodic Gaussians on an m x m grid (minimum-image distance), float64 radians."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cy = rng.uniform(0, m, size=n_gauss)
    cx = rng.uniform(0, m, size=n_gauss)
    sg = _draw(rng, sigma, n_gauss)
    am = _draw(rng, amp, n_gauss)
    yy = np.arange(m, dtype=np.float64)
    phi = np.zeros((m, m), dtype=np.float64)
    for j in range(n_gauss):
        dy = (yy - cy[j] + m / 2) % m - m / 2
        dx = (yy - cx[j] + m / 2) % m - m / 2
        gy = np.exp(-dy * dy / (2 * sg[j] ** 2))
        gx = np.exp(-dx * dx / (2 * sg[j] ** 2))
        phi += am[j] * np.outer(gy, gx)
    return phi


def phase_object(m: int, n_gauss: int, sigma: Range, amp: Range, seed: int) -> np.ndarray:
    """Pure phase object exp(i*phi), complex128."""
    return np.exp(1j * phase_map(m, n_gauss, sigma, amp, seed))


def fourier_aperture(n: int, radius: float, defocus_edge: float = 0.0, amplitude: float = 1.0) -> np.ndarray:
    """Circular aperture on the n x n detector grid, centred at (n//2, n//2), with an
    optional quadratic (defocus) phase of `defocus_edge` radians at the rim."""
    u = np.arange(n, dtype=np.float64) - n // 2
    r2 = u[:, None] ** 2 + u[None, :] ** 2
    inside = r2 <= radius * radius
    return amplitude * inside * np.exp(-1j * defocus_edge * r2 / (radius * radius))


def real_space_probe(aperture: np.ndarray, unit_intensity: bool = True) -> np.ndarray:
    """Probe in the sample plane, centred in the window: fftshift(ifft2(ifftshift(aperture)))."""
    p = np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(aperture)))
    if unit_intensity:
        p = p / np.sqrt(np.sum(np.abs(p) ** 2))
    return p


def unit_intensity_amplitude(n: int, radius: float) -> float:
    """Aperture value a for which the real-space probe has unit total intensity."""
    count = int(np.count_nonzero(np.abs(fourier_aperture(n, radius)) > 0))
    return float(n) / np.sqrt(count)


def raster_positions(sy: int, sx: int) -> np.ndarray:
    """All (y, x) scan indices in raster (row-major) order, int32 [Sy*Sx, 2]."""
    yy, xx = np.meshgrid(np.arange(sy, dtype=np.int32), np.arange(sx, dtype=np.int32), indexing="ij")
    return np.stack([yy.ravel(), xx.ravel()], axis=1)


def intensities(obj: np.ndarray, probe: np.ndarray, positions: np.ndarray, step: int = 1,
                chunk: int = 256) -> np.ndarray:
    """Noiseless fftshifted far-field intensities, float64 [n, N, N]."""
    m = obj.shape[0]
    n = probe.shape[0]
    out = np.empty((len(positions), n, n), dtype=np.float64)
    ii = np.arange(n)
    for c0 in range(0, len(positions), chunk):
        pos = positions[c0:c0 + chunk]
        rows = (pos[:, 0:1] * step + ii[None, :]) % m          # [c, n]
        cols = (pos[:, 1:2] * step + ii[None, :]) % m
        patch = obj[rows[:, :, None], cols[:, None, :]]          # [c, n, n]
        wave = np.fft.fft2(probe[None] * patch)
        out[c0:c0 + chunk] = np.fft.fftshift(np.abs(wave) ** 2, axes=(-2, -1))
    return out


def poisson_counts(intens: np.ndarray, positions: np.ndarray, sx: int, dose: float, seed: int) -> np.ndarray:
    """Poisson(dose * I_s / sum(I_s)) per frame, uint16 (saturating).  Each frame draws from
    its own stream keyed by (seed, linear scan index), so data do not depend on batching."""
    out = np.empty(intens.shape, dtype=np.uint16)
    for i in range(len(positions)):
        lin = int(positions[i, 0]) * sx + int(positions[i, 1])
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, lin])))
        lam = intens[i] * (dose / intens[i].sum())
        out[i] = np.minimum(rng.poisson(lam), 65535).astype(np.uint16)
    return out


@dataclasses.dataclass
class Workload:
    """Geometry and data recipe of one synthetic acquisition."""
    name: str
    sy: int
    sx: int
    n: int                 # detector is n x n
    radius: float          # aperture radius, detector pixels
    k: int                 # reduced basis size
    batch: int             # frames per push
    m: int                 # object is m x m (periodic)
    n_gauss: int
    sigma: Range
    amp: Range
    dose: Optional[float]  # electrons per frame; None -> noiseless float32 frames
    defocus_edge: float = 0.0
    step: int = 1
    seed: int = 0
    snapshot_every: Optional[int] = None

    @property
    def frames_total(self) -> int:
        return self.sy * self.sx

    def aperture_amplitude(self) -> float:
        return unit_intensity_amplitude(self.n, self.radius)

    def probe(self) -> np.ndarray:
        ap = fourier_aperture(self.n, self.radius, self.defocus_edge, self.aperture_amplitude())
        return real_space_probe(ap, unit_intensity=True)

    def object(self) -> np.ndarray:
        return phase_object(self.m, self.n_gauss, self.sigma, self.amp, self.seed)

    def frames(self, positions: Optional[np.ndarray] = None, obj: Optional[np.ndarray] = None) -> np.ndarray:
        """Frames for `positions` (default: full raster): uint16 counts or float32 intensities."""
        if positions is None:
            positions = raster_positions(self.sy, self.sx)
        if obj is None:
            obj = self.object()
        inten = intensities(obj, self.probe(), positions, self.step)
        if self.dose is None:
            return inten.astype(np.float32)
        return poisson_counts(inten, positions, self.sx, self.dose, 1000 + self.seed)


# The acquisitions used throughout: shapes follow the paper's timing workloads
# (square scans and detectors, Section 9) at sizes one GPU holds.
WORKLOADS = {
    # 32x32 scan over a 64x64 object, 32x32 detector, noiseless float32 frames.
    "small": Workload("small", 32, 32, 32, 8.0, 64, 32, 64, 12, 1.5, 0.3, None, seed=1),
    # 128x128 scan, 64x64 detector, 1e4 e/frame, uint16, pushed 128 frames at a time.
    "medium": Workload("medium", 128, 128, 64, 16.0, 256, 128, 256, 60, (1.0, 3.0), (0.2, 0.5), 1e4, seed=2),
    # 256x256 scan, 128x128 detector, defocus pi rad at the rim, 1e3 e/frame, K = 64.
    "defocus": Workload("defocus", 256, 256, 128, 32.0, 64, 256, 512, 240, (1.0, 3.0), (0.2, 0.5), 1e3,
                        defocus_edge=np.pi, seed=3),
    # 512x512 scan, 256x256 detector, 5e3 e/frame, K = 128, snapshot every 16384 frames.
    "large": Workload("large", 512, 512, 256, 48.0, 128, 256, 1024, 960, (1.0, 3.0), (0.2, 0.5), 5e3,
                      seed=4, snapshot_every=16384),
}


def periodic_workload(s: int = 32, n: int = 32, radius: float = 8.0, k: int = 64, seed: int = 11) -> Workload:
    """Scan = object = detector grid (periodic), the geometry of the paper's validation."""
    return Workload(f"periodic{s}", s, s, n, radius, k, s, s, 12, 1.5, 0.3, None, seed=seed)
