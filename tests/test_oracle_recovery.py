"""Physics pin: noiseless weak-phase objects are recovered inside the WDD passband
(Section 3, validation): band-limited to twice the aperture, up to a global phase
and a positive scale, in the right orientation."""
import numpy as np
import pytest

import oracle.wdd as O
import synth


def _bandlimit(phi, cutoff):
    m = phi.shape[0]
    f = np.fft.fft2(phi)
    fy = np.fft.fftfreq(m) * m
    r = np.sqrt(fy[:, None] ** 2 + fy[None, :] ** 2)
    f[r > cutoff] = 0
    return np.real(np.fft.ifft2(f))


def _corr(a, b):
    return float(np.corrcoef(a.ravel(), b.ravel())[0, 1])


def _recovered_phase(ot):
    return np.angle(ot * np.exp(-1j * np.angle(np.mean(ot))))


@pytest.mark.parametrize("basis,threshold", [("fourier", 0.95), ("hg", 0.90)])
def test_periodic_recovery(basis, threshold):
    wl = synth.periodic_workload()
    pos = synth.raster_positions(wl.sy, wl.sx)
    obj = wl.object()
    frames = wl.frames(pos, obj)
    amp = wl.aperture_amplitude()
    phi = O.fourier_basis(wl.n, wl.n) if basis == "fourier" else None
    plan = O.make_plan(wl.sy, wl.sx, wl.n, wl.n, wl.radius, wl.k, amplitude=amp, phi=phi)
    _, _, ot = O.offline_reduced(plan, frames, pos)
    truth = _bandlimit(np.angle(obj), 2 * wl.radius * wl.sy / wl.n)
    # recovered pixel s sits at object pixel s + N/2 (probe centred in its window)
    truth = np.roll(truth, (-(wl.n // 2), -(wl.n // 2)), axis=(0, 1))
    rec = _recovered_phase(ot)
    c = _corr(rec, truth)
    assert c >= threshold
    # orientation: negated, flipped and conjugate-transposed truths are far worse
    assert c - _corr(rec, -truth) > 0.5
    assert c - _corr(rec, truth[::-1, ::-1]) > 0.5
    assert c - _corr(rec, truth.T[::-1]) > 0.5


def test_small_workload_recovery_interior():
    wl = synth.WORKLOADS["small"]
    pos = synth.raster_positions(wl.sy, wl.sx)
    obj = wl.object()
    frames = wl.frames(pos, obj)
    plan = O.make_plan(wl.sy, wl.sx, wl.n, wl.n, wl.radius, phi=O.fourier_basis(wl.n, wl.n),
                       amplitude=wl.aperture_amplitude())
    _, _, ot = O.offline_reduced(plan, frames, pos)
    c0 = wl.n // 2
    truth = _bandlimit(np.angle(obj), 2 * wl.radius * wl.m / wl.n)[c0:c0 + wl.sy, c0:c0 + wl.sx]
    rec = _recovered_phase(ot)
    cut = 8
    assert _corr(rec[cut:-cut, cut:-cut], truth[cut:-cut, cut:-cut]) >= 0.90


@pytest.mark.parametrize("basis,threshold", [("fourier", 0.95), ("hg", 0.80)])
def test_defocused_probe_recovery(basis, threshold):
    """A probe with a quadratic phase of pi rad at the rim: the Wigner function is complex,
    so deconvolving by its conjugate (or the wrong factor) would fail here."""
    wl = synth.periodic_workload()
    wl.defocus_edge = np.pi
    pos = synth.raster_positions(wl.sy, wl.sx)
    obj = wl.object()
    frames = wl.frames(pos, obj)
    phi = O.fourier_basis(wl.n, wl.n) if basis == "fourier" else None
    plan = O.make_plan(wl.sy, wl.sx, wl.n, wl.n, wl.radius, wl.k, amplitude=wl.aperture_amplitude(),
                       defocus_edge=np.pi, phi=phi)
    _, _, ot = O.offline_reduced(plan, frames, pos)
    truth = np.roll(_bandlimit(np.angle(obj), 2 * wl.radius * wl.sy / wl.n), (-(wl.n // 2),) * 2, axis=(0, 1))
    assert _corr(_recovered_phase(ot), truth) >= threshold


@pytest.mark.parametrize("basis,threshold", [("fourier", 0.93), ("hg", 0.93)])
def test_recovery_at_scan_step_two(basis, threshold):
    """Scan step 2 object pixels (Section 6.2, physical coordinates: the detector shift of a
    scan frequency is v N / (S step)).  Periodic 64 x 64 object, 32 x 32 positions at step
    2, aperture radius 4 on a 32 x 32 detector, so the passband 2R/N = 1/4 cycle per pixel
    is the step-2 grid's Nyquist limit.  Reconstructed with step 1 instead, the kept set
    and the Wigner shifts are wrong and the recovery drops (about 0.8 here)."""
    wl = synth.Workload("step2", 32, 32, 32, 4.0, 16, 32, 64, 12, 1.5, 0.3, None, step=2, seed=11)
    pos = synth.raster_positions(wl.sy, wl.sx)
    obj = wl.object()
    frames = wl.frames(pos, obj)
    phi = O.fourier_basis(wl.n, wl.n) if basis == "fourier" else None
    truth = np.roll(_bandlimit(np.angle(obj), 2 * wl.radius * wl.m / wl.n), (-(wl.n // 2),) * 2, axis=(0, 1))
    truth = truth[::2, ::2]                       # recovered pixel s <-> object pixel 2 s + N/2
    corr = {}
    for step in (2.0, 1.0):
        plan = O.make_plan(wl.sy, wl.sx, wl.n, wl.n, wl.radius, wl.k, amplitude=wl.aperture_amplitude(), phi=phi,
                           step=step)
        _, _, ot = O.offline_reduced(plan, frames, pos)
        corr[step] = _corr(_recovered_phase(ot), truth)
    assert corr[2.0] >= threshold
    assert corr[2.0] - corr[1.0] > 0.1
