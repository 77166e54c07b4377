"""Pins of the oracle's scan DFT and display against brute-force sums (Section 6.1)."""
import cmath
import math

import numpy as np
import pytest

import oracle.wdd as O


def _all_freqs(sy, sx):
    vy, vx = np.meshgrid(np.arange(sy), np.arange(sx), indexing="ij")
    return np.stack([vy.ravel(), vx.ravel()], axis=1).astype(np.int32)


@pytest.mark.parametrize("sy,sx", [(8, 8), (4, 6), (5, 3)])
def test_scan_phase_matches_bruteforce(sy, sx):
    grid = _all_freqs(sy, sx)
    f = O.scan_phase(grid, grid, sy, sx)
    for i, (vy, vx) in enumerate(grid):
        for j, (py, px) in enumerate(grid):
            ref = cmath.exp(-2j * math.pi * (vy * py / sy + vx * px / sx)) / math.sqrt(sy * sx)
            assert abs(f[i, j] - ref) < 1e-14


def test_scan_phase_is_unitary():
    grid = _all_freqs(8, 6)
    f = O.scan_phase(grid, grid, 8, 6)
    assert np.allclose(f.conj().T @ f, np.eye(48), atol=1e-13)


def test_large_products_reduced_exactly():
    # v*s up to 511*511: the integer reduction must agree with a direct FP64 angle
    fr = np.array([[511, 3], [257, 500]], dtype=np.int32)
    ps = np.array([[509, 511], [1, 2]], dtype=np.int32)
    f = O.scan_phase(fr, ps, 512, 512)
    for i in range(2):
        for j in range(2):
            ang = -2 * math.pi * (((int(fr[i, 0]) * int(ps[j, 0])) % 512) / 512 + ((int(fr[i, 1]) * int(ps[j, 1])) % 512) / 512)
            assert abs(f[i, j] - cmath.exp(1j * ang) / 512) < 1e-15


def test_display_matches_bruteforce():
    rng = np.random.default_rng(5)
    sy, sx = 6, 8
    d = rng.normal(size=(sy, sx)) + 1j * rng.normal(size=(sy, sx))
    out = O.display(d)
    for y in range(sy):
        for x in range(sx):
            acc = 0j
            for vy in range(sy):
                for vx in range(sx):
                    acc += d[vy, vx] * cmath.exp(2j * math.pi * (vy * y / sy + vx * x / sx))
            ref = (acc / math.sqrt(sy * sx)).conjugate() / math.sqrt(abs(d[0, 0]))
            assert abs(out[y, x] - ref) < 1e-13


def test_display_zero_dc_gives_zero():
    d = np.ones((4, 4), dtype=np.complex128)
    d[0, 0] = 0
    assert np.all(O.display(d) == 0)


def test_offline_spectrum_is_outer_product_sum():
    """A from the FFT over the scan equals sum_s f_s h_s^T written out (equation outer_prod)."""
    rng = np.random.default_rng(1)
    sy, sx, ny, nx, k = 4, 4, 8, 8, 4
    phi = rng.normal(size=(ny * nx, k))
    grid = _all_freqs(sy, sx)
    plan = O.Plan(sy, sx, ny, nx, 2.0, 1.0, 0.0, 1.0, 0.01, grid, phi,
                  np.ones((16, k), complex), 1.0, np.ones((16, k), complex))
    frames = rng.normal(size=(16, ny, nx))
    a, _, _ = O.offline_reduced(plan, frames, grid)
    h = frames.reshape(16, -1) @ phi
    for i, (vy, vx) in enumerate(grid):
        for kk in range(k):
            acc = 0j
            for s, (py, px) in enumerate(grid):
                acc += cmath.exp(-2j * math.pi * (vy * py / sy + vx * px / sx)) * h[s, kk]
            assert abs(a[i, kk] - acc / 4.0) < 1e-12
