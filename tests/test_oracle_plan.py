"""Pins of the oracle's frequency set, probe Wigner function and Wiener filter
(pre-computed Wiener filter algorithm; Section 6.2)."""
import json
import math
import os

import numpy as np
import pytest

import oracle.wdd as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _bruteforce_kept(sy, sx, n, radius):
    kept = set()
    c = n // 2
    for vy in range(sy):
        for vx in range(sx):
            svy = vy - sy if 2 * vy >= sy else vy
            svx = vx - sx if 2 * vx >= sx else vx
            dy, dx = svy * n / sy, svx * n / sx
            hit = False
            for qy in range(n):
                for qx in range(n):
                    a = (qy - c) ** 2 + (qx - c) ** 2 <= radius ** 2
                    b = (qy - c + dy) ** 2 + (qx - c + dx) ** 2 <= radius ** 2
                    if a and b:
                        hit = True
                        break
                if hit:
                    break
            if hit:
                kept.add((vy, vx))
    return kept


@pytest.mark.parametrize("sy,sx,n,radius", [(8, 8, 8, 2.0), (16, 16, 8, 2.5), (12, 10, 8, 3.0)])
def test_kept_frequencies_match_bruteforce(sy, sx, n, radius):
    got = O.nonzero_frequencies(sy, sx, n, n, radius)
    assert set(map(tuple, got.tolist())) == _bruteforce_kept(sy, sx, n, radius)
    assert tuple(got[0]) == (0, 0)


def test_kept_frequencies_obey_the_papers_disc_condition():
    """Every kept v has |d_v|^2 <= 4 R^2 (the intersection condition of Section 6.2),
    and every v well inside that disc is kept."""
    sy = sx = 128
    n, radius = 64, 16.0
    got = O.nonzero_frequencies(sy, sx, n, n, radius)
    dy, dx = O.detector_shift(got[:, 0], got[:, 1], sy, sx, n, n)
    assert np.all(dy ** 2 + dx ** 2 <= 4 * radius ** 2)
    vy, vx = np.meshgrid(np.arange(sy), np.arange(sx), indexing="ij")
    ay, ax = O.detector_shift(vy.ravel(), vx.ravel(), sy, sx, n, n)
    inner = np.sqrt(ay ** 2 + ax ** 2) <= 2 * radius - 2
    kept = set(map(tuple, got.tolist()))
    for y, x in zip(vy.ravel()[inner], vx.ravel()[inner]):
        assert (y, x) in kept
    # count approaches the area of the disc of radius 2R (in frequency units)
    area = math.pi * (2 * radius * sy / n) ** 2
    assert abs(len(got) - area) / area < 0.03


def test_kept_frequencies_symmetric():
    sy = sx = 64
    got = set(map(tuple, O.nonzero_frequencies(sy, sx, 32, 32, 8.0).tolist()))
    for vy, vx in got:
        if 2 * vy == sy or 2 * vx == sx:
            continue
        assert ((-vy) % sy, (-vx) % sx) in got


def test_papers_worked_fraction_example():
    g = json.load(open(os.path.join(GOLDEN, "frequency_fraction_example.json")))
    val = O.frequency_fraction(g["theta_rad"], g["step_m"], g["wavelength_m"])
    assert round(val, g["decimals"]) == g["fraction_printed"]


def test_wigner_at_zero_is_aperture_intensity():
    y0 = O.probe_wigner(0, 0, 32, 32, 32, 32, 8.0, amplitude=2.0, defocus_edge=1.3)
    ap = O.aperture(32, 32, 8.0, amplitude=2.0, defocus_edge=1.3)
    assert np.allclose(y0, np.abs(ap) ** 2, atol=1e-15)
    assert np.all(y0.real >= 0) and np.max(np.abs(y0.imag)) < 1e-15


def test_wigner_hermitian_pairing():
    """For integer shifts, Y_{-v}(q) = conj(Y_v(q - d_v))."""
    s = n = 32
    for vy, vx in [(1, 0), (3, 5), (30, 2)]:
        yv = O.probe_wigner(vy, vx, s, s, n, n, 8.0, defocus_edge=0.7)
        ym = O.probe_wigner((-vy) % s, (-vx) % s, s, s, n, n, 8.0, defocus_edge=0.7)
        dy, dx = O.detector_shift(vy, vx, s, s, n, n)
        dy, dx = int(dy), int(dx)
        for qy in range(n):
            for qx in range(n):
                sy_, sx_ = qy - dy, qx - dx
                ref = np.conj(yv[sy_, sx_]) if (0 <= sy_ < n and 0 <= sx_ < n) else 0.0
                assert abs(ym[qy, qx] - ref) < 1e-15


def test_wiener_gain_is_real_and_below_one():
    plan = O.make_plan(32, 32, 32, 32, 8.0, 64)
    gain = plan.w * plan.yb
    assert np.max(np.abs(gain.imag)) < 1e-15
    assert np.all(gain.real >= 0) and np.all(gain.real < 1)
    ref = np.abs(plan.yb) ** 2 / (np.abs(plan.yb) ** 2 + plan.eps_abs)
    assert np.allclose(gain.real, ref, rtol=1e-14, atol=0)
    assert plan.eps_abs == pytest.approx(0.01 * np.max(np.abs(plan.yb) ** 2), rel=1e-15)


def test_eps_is_relative():
    p1 = O.make_plan(32, 32, 32, 32, 8.0, 64, amplitude=1.0)
    p17 = O.make_plan(32, 32, 32, 32, 8.0, 64, amplitude=17.0)
    assert np.linalg.norm(p17.w * 17 ** 2 - p1.w) <= 1e-13 * np.linalg.norm(p1.w)
    assert p17.eps_abs == pytest.approx(p1.eps_abs * 17 ** 4, rel=1e-13)


def test_aperture_value_17_gives_the_same_reconstruction():
    """Simulate and reconstruct with aperture value 17 instead of 1 (Section 3, validation):
    D and the displayed object must not change."""
    wl = synth.periodic_workload(s=16, n=16, radius=4.0, k=16)
    pos = synth.raster_positions(wl.sy, wl.sx)
    obj = wl.object()
    out = []
    for a in (1.0, 17.0):
        probe = synth.real_space_probe(synth.fourier_aperture(wl.n, wl.radius, 0.0, a), unit_intensity=False)
        frames = synth.intensities(obj, probe, pos)
        plan = O.make_plan(wl.sy, wl.sx, wl.n, wl.n, wl.radius, wl.k, amplitude=a)
        _, d, ot = O.offline_reduced(plan, frames, pos)
        out.append((d, ot))
    assert np.linalg.norm(out[0][0] - out[1][0]) <= 1e-12 * np.linalg.norm(out[0][0])
    assert np.linalg.norm(out[0][1] - out[1][1]) <= 1e-12 * np.linalg.norm(out[0][1])


@pytest.mark.parametrize("s,n,radius", [(16, 32, 4.0), (32, 32, 6.0), (16, 16, 3.5)])
def test_scan_step_enters_as_a_finer_frequency_grid(s, n, radius):
    """Section 6.2: a scan frequency is v / (S step) cycles per object pixel.  A raster of S
    positions at step 2 and one of 2S positions at step 1 therefore sample the same
    frequencies wherever both grids have them: the kept signed frequencies of (S, step 2)
    are exactly those of (2S, step 1) with |v| < S/2, and the probe Wigner functions agree."""
    def signed_set(sz, step):
        got = O.nonzero_frequencies(sz, sz, n, n, radius, step)
        vy = O.signed_index(got[:, 0], sz)
        vx = O.signed_index(got[:, 1], sz)
        return set(zip(vy.tolist(), vx.tolist()))
    coarse = signed_set(s, 2.0)
    fine = {(a, b) for a, b in signed_set(2 * s, 1.0) if -s / 2 <= a < s / 2 and -s / 2 <= b < s / 2}
    assert coarse == fine
    for a, b in sorted(coarse)[:: max(1, len(coarse) // 12)]:
        y2 = O.probe_wigner(a % s, b % s, s, s, n, n, radius, defocus_edge=0.9, step=2.0)
        y1 = O.probe_wigner(a % (2 * s), b % (2 * s), 2 * s, 2 * s, n, n, radius, defocus_edge=0.9, step=1.0)
        assert np.max(np.abs(y2 - y1)) < 1e-15


def test_aperture_centre_moves_the_whole_method_with_the_frames():
    """Reading R3 with the aperture centre c as an acquisition setting: frames whose
    diffraction disc sits at c + (dy, dx) on the detector, reconstructed with that centre,
    give exactly the D of the same frames centred at c, because aperture, basis and kept
    set all move with c (the detector is large enough that nothing reaches its edge)."""
    wl = synth.Workload("c", 16, 16, 64, 8.0, 16, 16, 32, 12, 1.5, 0.3, None, seed=5)
    pos = synth.raster_positions(wl.sy, wl.sx)
    frames = wl.frames(pos)
    amp = wl.aperture_amplitude()
    base = O.make_plan(wl.sy, wl.sx, wl.n, wl.n, wl.radius, wl.k, amplitude=amp, defocus_edge=0.8)
    _, d0, _ = O.offline_reduced(base, frames, pos)
    for dy, dx in [(-3, 5), (2, -4)]:
        moved = np.roll(frames, (dy, dx), axis=(1, 2))
        plan = O.make_plan(wl.sy, wl.sx, wl.n, wl.n, wl.radius, wl.k, amplitude=amp, defocus_edge=0.8,
                           center=(wl.n // 2 + dy, wl.n // 2 + dx))
        assert np.array_equal(plan.freqs, base.freqs)
        _, d1, _ = O.offline_reduced(plan, moved, pos)
        assert np.linalg.norm(d1 - d0) <= 1e-12 * np.linalg.norm(d0)
        # the unmoved centre on moved frames is a different reconstruction
        _, dwrong, _ = O.offline_reduced(base, moved, pos)
        assert np.linalg.norm(dwrong - d0) > 1e-3 * np.linalg.norm(d0)


@pytest.mark.parametrize("center", [(15.5, 16.0), (16.5, 14.5), (13.0, 17.5)])
def test_kept_frequencies_match_bruteforce_off_centre(center):
    sy = sx = 16
    n, radius = 32, 5.0
    got = set(map(tuple, O.nonzero_frequencies(sy, sx, n, n, radius, center=center).tolist()))
    kept = set()
    for vy in range(sy):
        for vx in range(sx):
            dy = (vy - sy if 2 * vy >= sy else vy) * n / sy
            dx = (vx - sx if 2 * vx >= sx else vx) * n / sx
            if any((qy - center[0]) ** 2 + (qx - center[1]) ** 2 <= radius ** 2 and
                   (qy - center[0] + dy) ** 2 + (qx - center[1] + dx) ** 2 <= radius ** 2
                   for qy in range(n) for qx in range(n)):
                kept.add((vy, vx))
    assert got == kept
