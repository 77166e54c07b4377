"""FP64 CPU oracle of Wigner Distribution Deconvolution, offline and live.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow reference that the
GPU path is checked against.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import it; the product path never does.
It shares no code with the HIP library.

Every quantity is float64 / complex128.  Where the paper is silent, the readings
below are used (each is a numbered reading in the design notes):

  R1  K counts 2D basis functions.  Pairs (n_y, n_x) are ordered by
      (max(n_y, n_x), n_y + n_x, n_y) and the first K are kept; L = ceil(sqrt(K)).
  R2  Normalised Hermite functions, t = (i - c) / sigma with c the aperture centre,
      sigma = R / sqrt(2L - 1) unless given; each sampled 1D column is L2-normalised
      on the grid.
  R3  Aperture value a * 1[|u| <= R] * exp(-i phi_edge |u|^2 / R^2), u = q - c, with the
      aperture centre c in detector pixels; c = (N_y/2, N_x/2) unless given.
  R4  Y_v(q) = P(q - c) * conj(P(q - c + d_v)), d_v = v_signed * N / (S * step).
  R5  v is kept iff some detector pixel lies inside both discs (exact test).
  R6  eps_abs = eps_rel * max over kept v and k of |Y^B_v[k]|^2.
  R7  Unitary scan DFT, 0-based indices, phases from (v*s) mod S into FP64 tables.
  R9  The Wiener filter may be applied after accumulating the spectrum (order "N")
      or per frame (order "P", as written in the modified-WDD algorithm); both
      are computed and must agree.
  R10 D[v] = sum_k W[v,k] A[v,k]  (the q = 0 value of the object Wigner function).
  R11 O~ = conj(IDFT2_unitary(D)) / sqrt(|D[0]|), zero when D[0] = 0.

Parity status: every function here is pinned by a test in tests/test_oracle_*.py
against a property fixed by the paper or by the mathematics (see each test module),
except the shape of patch_window: the paper names no merge window for field-of-view
patches, so its trapezoid is a choice of this reading (parity unpinned); the properties
the merge relies on (weights normalised, merge linear and independent of patch order,
one patch = the full scan) are pinned.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterable, Optional, Sequence, Tuple

import numpy as np

# ----------------------------------------------------------------------------
# Probe, frequencies and the probe's Wigner function (Section 2, Algorithm
# "pre-computed Wiener filter")
# ----------------------------------------------------------------------------


def default_center(ny: int, nx: int) -> Tuple[float, float]:
    """The detector's zero frequency for fftshifted frames, (ny//2, nx//2)."""
    return float(ny // 2), float(nx // 2)


def aperture(ny: int, nx: int, radius: float, amplitude: float = 1.0, defocus_edge: float = 0.0,
             shift: Tuple[float, float] = (0.0, 0.0), center: Optional[Tuple[float, float]] = None) -> np.ndarray:
    """Fourier-space probe P(q - c + shift) on the ny x nx detector grid, c the aperture
    centre (default (ny//2, nx//2)).

    The initial probe is a circular aperture generated from its radius
    (pre-computed Wiener filter algorithm, initialisation step 1); `shift`
    evaluates it at q + q_v for the Wigner function (Section 2).
    """
    cy, cx = default_center(ny, nx) if center is None else center
    uy = np.arange(ny, dtype=np.float64) - cy + shift[0]
    ux = np.arange(nx, dtype=np.float64) - cx + shift[1]
    r2 = uy[:, None] ** 2 + ux[None, :] ** 2
    inside = r2 <= radius * radius
    phase = np.exp(-1j * defocus_edge * r2 / (radius * radius))
    return amplitude * inside * phase


def signed_index(v: np.ndarray, s: int) -> np.ndarray:
    """0-based DFT index -> signed frequency (indices >= s/2 are negative)."""
    v = np.asarray(v)
    return v - s * (2 * v >= s)


def detector_shift(vy, vx, sy: int, sx: int, ny: int, nx: int, step: float = 1.0):
    """Shift of the aperture on the detector, in pixels, for scan frequency (vy, vx).

    A scan frequency of v cycles over the S-position scan (step `step` object
    pixels) is v / (S * step) cycles per pixel, i.e. v * N / (S * step) detector
    pixels (Section 6.2, transformation to physical coordinates).
    """
    dy = signed_index(np.asarray(vy), sy) * ny / (sy * step)
    dx = signed_index(np.asarray(vx), sx) * nx / (sx * step)
    return dy, dx


def probe_wigner(vy: int, vx: int, sy: int, sx: int, ny: int, nx: int, radius: float,
                 amplitude: float = 1.0, defocus_edge: float = 0.0, step: float = 1.0,
                 center: Optional[Tuple[float, float]] = None) -> np.ndarray:
    """Y_v(q) = P(q) conj(P(q + q_v)) on the detector grid (pre-computed Wiener filter algorithm)."""
    dy, dx = detector_shift(vy, vx, sy, sx, ny, nx, step)
    p0 = aperture(ny, nx, radius, amplitude, defocus_edge, center=center)
    pv = aperture(ny, nx, radius, amplitude, defocus_edge, shift=(float(dy), float(dx)), center=center)
    return p0 * np.conj(pv)


def nonzero_frequencies(sy: int, sx: int, ny: int, nx: int, radius: float, step: float = 1.0,
                        chunk: int = 4096, center: Optional[Tuple[float, float]] = None) -> np.ndarray:
    """All (vy, vx) whose shifted aperture overlaps the unshifted one on at least one
    detector pixel (Section 6.2, omitting frequencies without intersection).

    Brute force over the aperture's pixels: a pixel u (relative to the centre) is in
    both discs iff |u|^2 <= R^2 and |u + d_v|^2 <= R^2.  All shifts are dyadic
    rationals for power-of-two sizes (and half-pixel centres), so the comparisons are
    exact in FP64.  Returned as int32 [n, 2], sorted by (vy, vx); (0, 0) is always first.
    """
    cy, cx = default_center(ny, nx) if center is None else center
    uy = np.arange(ny, dtype=np.float64) - cy
    ux = np.arange(nx, dtype=np.float64) - cx
    UY, UX = np.meshgrid(uy, ux, indexing="ij")
    inside = UY ** 2 + UX ** 2 <= radius * radius
    py, px = UY[inside], UX[inside]
    vy, vx = np.meshgrid(np.arange(sy), np.arange(sx), indexing="ij")
    vy, vx = vy.ravel(), vx.ravel()
    dy, dx = detector_shift(vy, vx, sy, sx, ny, nx, step)
    # centres farther apart than 2R (+ margin) cannot share a pixel: skip them
    cand = np.nonzero((np.abs(dy) <= 2 * radius + 2) & (np.abs(dx) <= 2 * radius + 2))[0]
    keep = np.zeros(vy.shape, dtype=bool)
    r2 = radius * radius
    for c0 in range(0, len(cand), chunk):
        idx = cand[c0:c0 + chunk]
        sy2 = (py[None, :] + dy[idx, None]) ** 2
        sx2 = (px[None, :] + dx[idx, None]) ** 2
        keep[idx] = np.any(sy2 + sx2 <= r2, axis=1)
    out = np.stack([vy[keep], vx[keep]], axis=1).astype(np.int32)
    return out


# ----------------------------------------------------------------------------
# Hermite-Gauss basis (Sections 4 and 5)
# ----------------------------------------------------------------------------


def hermite_functions(nmax: int, t: np.ndarray) -> np.ndarray:
    """psi_n(t) for n < nmax: L2-normalised Hermite functions H_n(t) exp(-t^2/2) / sqrt(2^n n! sqrt(pi)),
    by the three-term recurrence (equation HO-eigenfunction with the normalisation of Section 4)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros((nmax,) + t.shape, dtype=np.float64)
    out[0] = np.pi ** -0.25 * np.exp(-0.5 * t * t)
    if nmax > 1:
        out[1] = math.sqrt(2.0) * t * out[0]
    for n in range(1, nmax - 1):
        out[n + 1] = math.sqrt(2.0 / (n + 1)) * t * out[n] - math.sqrt(n / (n + 1.0)) * out[n - 1]
    return out


def basis_order(k: int) -> np.ndarray:
    """First k pairs (n_y, n_x) in shell order (reading R1), int [k, 2]."""
    lsz = int(math.ceil(math.sqrt(k)))
    pairs = [(ny, nx) for ny in range(lsz) for nx in range(lsz)]
    pairs.sort(key=lambda p: (max(p), p[0] + p[1], p[0]))
    return np.array(pairs[:k], dtype=np.int64)


def basis_size_1d(k: int) -> int:
    return int(math.ceil(math.sqrt(k)))


def default_sigma(radius: float, k: int) -> float:
    """sigma = R / sqrt(2L - 1): the highest order's classical turning point sits on the rim."""
    return radius / math.sqrt(2 * basis_size_1d(k) - 1)


def sampled_hermite(n: int, nmax: int, sigma: float, center: Optional[float] = None) -> np.ndarray:
    """psi_x in R^{n x nmax} (Section 5): Hermite functions sampled on the grid centred
    at `center` (default n//2, the aperture centre), each column L2-normalised on the grid."""
    c = float(n // 2) if center is None else float(center)
    t = (np.arange(n, dtype=np.float64) - c) / sigma
    psi = hermite_functions(nmax, t).T.copy()             # [n, nmax]
    psi /= np.sqrt(np.sum(psi * psi, axis=0, keepdims=True))
    return psi


def hg_basis(ny: int, nx: int, k: int, sigma: float, center: Optional[Tuple[float, float]] = None) -> np.ndarray:
    """Phi in R^{(ny*nx) x k}: Phi[y*nx + x, j] = psi_{n_y(j)}[y] * psi_{n_x(j)}[x].

    Phi^T vec(A) equals the reduction H(A) of Section 5 with its L x L entries
    re-listed in shell order (the transpose in H only relabels entries)."""
    pairs = basis_order(k)
    lsz = basis_size_1d(k)
    cy, cx = default_center(ny, nx) if center is None else center
    py = sampled_hermite(ny, lsz, sigma, cy)
    px = sampled_hermite(nx, lsz, sigma, cx)
    phi = py[:, None, pairs[:, 0]] * px[None, :, pairs[:, 1]]   # [ny, nx, k]
    return phi.reshape(ny * nx, k)


def fourier_basis(ny: int, nx: int) -> np.ndarray:
    """Full-Fourier 'basis': Phi^T vec(A) = ifft2(A) (numpy normalisation).  With it the
    reduced method becomes conventional WDD exactly."""
    qy = np.arange(ny)
    qx = np.arange(nx)
    ey = np.exp(2j * np.pi * np.outer(qy, qy) / ny)          # [q_y, rho_y]
    ex = np.exp(2j * np.pi * np.outer(qx, qx) / nx)
    phi = ey[:, None, :, None] * ex[None, :, None, :] / (ny * nx)
    return phi.reshape(ny * nx, ny * nx)


# ----------------------------------------------------------------------------
# Plan: pre-computed Wiener filter (Algorithm "pre-computed Wiener filter")
# ----------------------------------------------------------------------------


@dataclasses.dataclass
class Plan:
    sy: int
    sx: int
    ny: int
    nx: int
    radius: float
    amplitude: float
    defocus_edge: float
    step: float
    eps_rel: float
    freqs: np.ndarray        # int32 [n_hat, 2], (0, 0) first
    phi: np.ndarray          # [ny*nx, k] real (HG) or complex (Fourier)
    yb: np.ndarray           # complex [n_hat, k]: Phi^T vec(Y_v)
    eps_abs: float
    w: np.ndarray            # complex [n_hat, k]
    center: Optional[Tuple[float, float]] = None   # aperture centre; None: (ny//2, nx//2)

    @property
    def k(self) -> int:
        return self.phi.shape[1]

    @property
    def n_hat(self) -> int:
        return len(self.freqs)


def reduce_hg(a: np.ndarray, psi_y: np.ndarray, psi_x: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    """Phi^T vec(A) for the HG basis through the paper's operator H(A) = psi_x^T A^T psi_y
    (Section 5): entry (n_x, n_y) of H(A) is the coefficient of psi_{n_y}(y) psi_{n_x}(x).
    `a` may hold a stack of matrices [..., ny, nx]."""
    red_t = np.swapaxes(psi_y.T @ (a @ psi_x), -1, -2)   # H(A) = psi_x^T A^T psi_y
    return red_t[..., pairs[:, 1], pairs[:, 0]]


def make_plan(sy: int, sx: int, ny: int, nx: int, radius: float, k: Optional[int] = None,
              amplitude: float = 1.0, defocus_edge: float = 0.0, step: float = 1.0,
              eps_rel: float = 0.01, sigma: Optional[float] = None, phi: Optional[np.ndarray] = None,
              freqs: Optional[np.ndarray] = None, eps_abs: Optional[float] = None, chunk: int = 256,
              center: Optional[Tuple[float, float]] = None) -> Plan:
    """Frequencies with overlap, the reduced probe Wigner functions and the Wiener filter.

    For each kept v: Y_v (probe autocorrelation at q + q_v), its reduction
    Y^B_v = Phi^T vec(Y_v), and W_v = conj(Y^B_v) / (|Y^B_v|^2 + eps)
    (pre-computed Wiener filter algorithm).  `freqs` restricts the plan to a
    subset of the kept frequencies; `eps_abs` then supplies the regularisation
    of the full set (it is a maximum over all kept v).
    """
    hg = phi is None
    if hg:
        if sigma is None:
            sigma = default_sigma(radius, k)
        phi = hg_basis(ny, nx, k, sigma, center)
        lsz = basis_size_1d(k)
        cy, cx = default_center(ny, nx) if center is None else center
        psi_y, psi_x, pairs = sampled_hermite(ny, lsz, sigma, cy), sampled_hermite(nx, lsz, sigma, cx), basis_order(k)
    if freqs is None:
        freqs = nonzero_frequencies(sy, sx, ny, nx, radius, step, center=center)
    yb = np.empty((len(freqs), phi.shape[1]), dtype=np.complex128)
    for c0 in range(0, len(freqs), chunk):
        ys = np.stack([probe_wigner(int(vy), int(vx), sy, sx, ny, nx, radius, amplitude, defocus_edge, step, center)
                       for vy, vx in freqs[c0:c0 + chunk]])
        if hg:
            yb[c0:c0 + chunk] = reduce_hg(ys, psi_y, psi_x, pairs)
        else:
            yb[c0:c0 + chunk] = ys.reshape(len(ys), -1) @ phi
    if eps_abs is None:
        eps_abs = eps_rel * float(np.max(np.abs(yb) ** 2))
    w = np.conj(yb) / (np.abs(yb) ** 2 + eps_abs)
    return Plan(sy, sx, ny, nx, radius, amplitude, defocus_edge, step, eps_rel, freqs, phi, yb, eps_abs, w, center)


# ----------------------------------------------------------------------------
# Per-frame steps of the modified (live) WDD
# ----------------------------------------------------------------------------


def project(frames: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """h_s = Phi^T vec(I_s) for each frame (dimensionality reduction, Section 5)."""
    x = np.asarray(frames, dtype=np.float64).reshape(len(frames), phi.shape[0])  # (0 frames: an empty batch)
    return x @ phi


def scan_phase(freqs: np.ndarray, positions: np.ndarray, sy: int, sx: int) -> np.ndarray:
    """F[v, s] = S^{-1/2} exp(-2 pi i (v_y s_y / S_y + v_x s_x / S_x)): the columns of the
    unitary 2D DFT matrix F_y (x) F_x at the given scan positions (Section 6.1).
    Angles are reduced in integers and looked up in FP64 tables (reading R7)."""
    ty = np.exp(-2j * np.pi * np.arange(sy) / sy)
    tx = np.exp(-2j * np.pi * np.arange(sx) / sx)
    my = (freqs[:, 0:1].astype(np.int64) * positions[None, :, 0].astype(np.int64)) % sy
    mx = (freqs[:, 1:2].astype(np.int64) * positions[None, :, 1].astype(np.int64)) % sx
    return ty[my] * tx[mx] / math.sqrt(sy * sx)


def display(d_grid: np.ndarray) -> np.ndarray:
    """O~ = conj(IDFT2_unitary(D)) / sqrt(|D[0, 0]|) (equation "extract" and the final step
    of the modified-WDD algorithm); all zeros when D[0, 0] = 0."""
    d0 = abs(d_grid[0, 0])
    if d0 == 0.0:
        return np.zeros_like(d_grid)
    return np.conj(np.fft.ifft2(d_grid, norm="ortho")) / math.sqrt(d0)


def scatter(plan: Plan, d: np.ndarray) -> np.ndarray:
    """Place D[v] for kept v into the Sy x Sx grid, zero elsewhere."""
    g = np.zeros((plan.sy, plan.sx), dtype=np.complex128)
    g[plan.freqs[:, 0], plan.freqs[:, 1]] = d
    return g


def extract(plan: Plan, a: np.ndarray) -> np.ndarray:
    """D[v] = sum_k W[v, k] A[v, k]: Hadamard with the Wiener filter, then the sum of all
    entries (modified-WDD algorithm, deconvolution and zero-frequency steps)."""
    return np.sum(plan.w * a, axis=1)


class Live:
    """The modified WDD, one frame batch at a time (Section 6.3).

    order "N": accumulate the spectrum A[v, k] += sum_s F[v, s] h_s[k] and apply the
    Wiener filter when a snapshot is taken.  order "P": apply it per frame,
    O[v] += F[v, s] sum_k W[v, k] h_s[k], as written in the algorithm.
    """

    def __init__(self, plan: Plan, order: str = "N"):
        assert order in ("N", "P")
        self.plan = plan
        self.order = order
        if order == "N":
            self.acc = np.zeros((plan.n_hat, plan.k), dtype=np.complex128)
        else:
            self.acc = np.zeros(plan.n_hat, dtype=np.complex128)
        self.frames_seen = 0

    def push(self, frames: np.ndarray, positions: np.ndarray) -> None:
        positions = np.asarray(positions)
        if len(positions) == 0:
            return
        h = project(frames, self.plan.phi)                                  # [b, k]
        f = scan_phase(self.plan.freqs, positions, self.plan.sy, self.plan.sx)  # [n_hat, b]
        if self.order == "N":
            self.acc += f @ h
        else:
            o = self.plan.w @ h.T                                           # [n_hat, b]
            self.acc += np.sum(f * o, axis=1)
        self.frames_seen += len(positions)

    def spectrum(self) -> np.ndarray:
        """D on the kept frequencies."""
        if self.order == "N":
            return extract(self.plan, self.acc)
        return self.acc.copy()

    def snapshot(self) -> np.ndarray:
        return display(scatter(self.plan, self.spectrum()))


# ----------------------------------------------------------------------------
# Offline forms
# ----------------------------------------------------------------------------


def offline_reduced(plan: Plan, frames: np.ndarray, positions: np.ndarray):
    """Reduced WDD on a complete raster: A = unitary FFT over the scan axes of the
    projected frames, then extraction and display.  Returns (A, D, O~)."""
    h = project(frames, plan.phi)
    cube = np.zeros((plan.sy, plan.sx, plan.k), dtype=h.dtype)
    np.add.at(cube, (positions[:, 0], positions[:, 1]), h)
    a_full = np.fft.fft2(cube, axes=(0, 1), norm="ortho")
    a = a_full[plan.freqs[:, 0], plan.freqs[:, 1]]
    d = extract(plan, a)
    return a, d, display(scatter(plan, d))


def offline_conventional(frames4d: np.ndarray, radius: float, amplitude: float = 1.0,
                         defocus_edge: float = 0.0, step: float = 1.0, eps_rel: float = 0.01):
    """Conventional WDD (equations "deconv_mat" and "extract"; Figure "schematic_WDD").

    frames4d: [Sy, Sx, Ny, Nx].  G = FFT over the scan; H = IFFT over the detector;
    W_P = IFFT over the detector of Y_v; W_O = H conj(W_P) / (|W_P|^2 + eps);
    D[v] = sum over rho of W_O (its Fourier transform at q = 0); then display.
    Returns (D grid, O~).
    """
    sy, sx, ny, nx = frames4d.shape
    g = np.fft.fft2(frames4d.astype(np.float64), axes=(0, 1), norm="ortho")
    hh = np.fft.ifft2(g, axes=(2, 3))
    wp = np.empty((sy, sx, ny, nx), dtype=np.complex128)
    for vy in range(sy):
        for vx in range(sx):
            y = probe_wigner(vy, vx, sy, sx, ny, nx, radius, amplitude, defocus_edge, step)
            wp[vy, vx] = np.fft.ifft2(y)
    eps_abs = eps_rel * float(np.max(np.abs(wp) ** 2))
    wo = hh * np.conj(wp) / (np.abs(wp) ** 2 + eps_abs)
    d = np.sum(wo, axis=(2, 3))
    return d, display(d)


def frequency_fraction(theta: float, step: float, wavelength: float) -> float:
    """The paper's sufficient bound on the fraction of scan frequencies with overlap,
    sqrt(2) * step * sin(theta) / lambda (equation "low_correlation")."""
    return math.sqrt(2.0) * step * math.sin(theta) / wavelength


# ----------------------------------------------------------------------------
# Field-of-view patches (Section 10, Discussion: a large field of view subdivided into
# patches reconstructed independently and merged).  The paper gives no patch geometry or
# merge rule; the reading used here:
#   * a patch is a Py x Px sub-raster; patch origins step by (Py - oy, Px - ox) from 0 and the
#     last one on each axis sits at S - P, so patches stay inside the raster and cover it
#     (oy, ox = overlap in scan positions);
#   * every patch is a live WDD of its own over its Py x Px raster: a frame at scan position
#     s enters every patch p that contains it, at the local position s - o_p;
#   * the merged image is the weighted mean of the patch images over the patches covering a
#     pixel, with the separable trapezoid window w(i) = min(1, (i + 1) / (o + 1),
#     (P - i) / (o + 1)) per axis: the patch's own scan DFT treats it as periodic, so its
#     edges carry wrap-around errors and are de-weighted where another patch covers them.
# One patch covering the whole raster reproduces the full-scan result.
# ----------------------------------------------------------------------------


def patch_origins(s: int, p: int, overlap: int) -> np.ndarray:
    """Origins of the patches of length p along an axis of s positions (0 <= overlap < p <= s)."""
    if not (0 < p <= s and 0 <= overlap < p):
        raise ValueError("need 0 < p <= s and 0 <= overlap < p")
    step = p - overlap
    out = list(range(0, s - p + 1, step))
    if out[-1] != s - p:
        out.append(s - p)
    return np.array(out, dtype=np.int64)


def patch_window(p: int, overlap: int) -> np.ndarray:
    """The 1D merge weight over a patch of length p: 1 inside, linear ramps over the overlap.
    Parity unpinned: the paper gives no window; this shape is the reading's choice."""
    i = np.arange(p, dtype=np.float64)
    return np.minimum(1.0, np.minimum((i + 1) / (overlap + 1), (p - i) / (overlap + 1)))


def merge_patches(images: Sequence[np.ndarray], oy: np.ndarray, ox: np.ndarray, sy: int, sx: int,
                  overlap_y: int, overlap_x: int) -> np.ndarray:
    """Weighted mean of the patch images (listed row-major over the origin grid oy x ox) on
    the sy x sx raster."""
    py, px = images[0].shape
    wy, wx = patch_window(py, overlap_y), patch_window(px, overlap_x)
    num = np.zeros((sy, sx), dtype=np.complex128)
    den = np.zeros((sy, sx), dtype=np.float64)
    for idx, img in enumerate(images):
        y0, x0 = oy[idx // len(ox)], ox[idx % len(ox)]
        w = wy[:, None] * wx[None, :]
        num[y0:y0 + py, x0:x0 + px] += w * img
        den[y0:y0 + py, x0:x0 + px] += w
    return num / den


def patched_reconstruction(frames: np.ndarray, positions: np.ndarray, sy: int, sx: int, py: int, px: int,
                           overlap_y: int, overlap_x: int, plan: Plan):
    """Every patch reconstructed from the frames inside it (offline form of each patch's
    live WDD, `plan` built for the Py x Px patch raster), then merged.  Returns (merged
    image, patch images in origin order)."""
    oy, ox = patch_origins(sy, py, overlap_y), patch_origins(sx, px, overlap_x)
    images = []
    for y0 in oy:
        for x0 in ox:
            inside = ((positions[:, 0] >= y0) & (positions[:, 0] < y0 + py) &
                      (positions[:, 1] >= x0) & (positions[:, 1] < x0 + px))
            local = positions[inside] - np.array([y0, x0])
            _, _, img = offline_reduced(plan, frames[inside], local)
            images.append(img)
    return merge_patches(images, oy, ox, sy, sx, overlap_y, overlap_x), images
