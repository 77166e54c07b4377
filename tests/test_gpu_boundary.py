"""The C ABI's boundary on the GPU: integer counts decode exactly, the plan holds exactly
the tables it exports, and an off-centre probe (aperture centre as an acquisition setting,
reading R3) reconstructs as the oracle does."""
import numpy as np
import pytest

import oracle.wdd as O
import paper_2212_01309_amd as wdd
import synth
from gpu_util import device, rel, rel_d, rel_img, say

pytestmark = pytest.mark.gpu


def test_decode_of_counts_is_bit_exact():
    """K = 1: h = sum_q I[q] psi_0[y] psi_0[x].  For a frame with one non-zero count c at
    (y, x), both stages of the projection have a single non-zero product, so the FP32
    result is exactly fl(psi_y[y] * fl(c * psi_x[x])) with psi rounded to FP32 once.  Any
    mistake in decoding the count (a lost bit, swapped halves of a 32-bit word, a wrong
    lane of the 16-byte load) changes that value.  Counts cover 1 .. 65535, columns every
    residue mod 8 and rows every residue mod 16."""
    ny = nx = 64
    radius = 12.0
    rng = np.random.default_rng(11)
    counts = np.array([65535, 65534, 32768, 32767, 257, 256, 255, 1, 12345, 54321, 4096, 3] * 11, np.uint16)
    nfr = len(counts)
    ys = (np.arange(nfr) * 5 + rng.integers(0, 4, nfr)) % ny
    xs = (np.arange(nfr) * 9 + 3 * rng.integers(0, 8, nfr)) % nx
    frames = np.zeros((nfr, ny, nx), np.uint16)
    frames[np.arange(nfr), ys, xs] = counts
    pos = np.zeros((nfr, 2), np.int32)
    with wdd.Plan(radius, 4, 4, ny, nx, 1, dtype=wdd.WDD_U16, max_batch=nfr) as plan:
        plan.push(device(frames), pos)
        h = plan.projection()[:, 0]
    sigma = O.default_sigma(radius, 1)
    psy = O.sampled_hermite(ny, 1, sigma)[:, 0].astype(np.float32)
    psx = O.sampled_hermite(nx, 1, sigma)[:, 0].astype(np.float32)
    ref = psy[ys] * (counts.astype(np.float32) * psx[xs])       # float32 products, each rounded
    assert ref.dtype == np.float32
    bad = np.nonzero(h.view(np.uint32) != ref.view(np.uint32))[0]
    say(f"[boundary] decode: {nfr} one-hot frames, {len(bad)} differ")
    assert len(bad) == 0, (bad[:5], h[bad[:5]], ref[bad[:5]])


@pytest.mark.parametrize("center", [None, (13.5, 18.0)])
def test_plan_holds_the_tables_it_exports(center):
    """wdd_plan_export returns the plan's own FP64 tables: they equal the oracle's plan
    (<= 1e-12), and the Wiener filter the device holds is exactly their FP32 rounding."""
    sy, sx, n, k, radius = 24, 32, 32, 50, 7.0
    with wdd.Plan(radius, sy, sx, n, n, k, defocus=0.8, center=center, max_batch=16) as plan:
        phi, w, freqs = plan.export()
        w_dev = plan.wiener()
    ref = O.make_plan(sy, sx, n, n, radius, k, defocus_edge=0.8, center=center)
    assert np.array_equal(freqs, ref.freqs)
    assert np.max(np.abs(phi - ref.phi)) <= 1e-12 * np.max(np.abs(ref.phi))
    assert np.linalg.norm(w - ref.w) <= 1e-12 * np.linalg.norm(ref.w)
    assert np.array_equal(w_dev.real, w.real.astype(np.float32)) and np.array_equal(w_dev.imag, w.imag.astype(np.float32))


def test_plan_export_fourier_basis():
    with wdd.Plan(6.0, 16, 16, 16, 16, 256, basis=wdd.WDD_BASIS_FOURIER, dtype=wdd.WDD_F32, max_batch=8) as plan:
        phi, w, freqs = plan.export()
    ref = O.make_plan(16, 16, 16, 16, 6.0, phi=O.fourier_basis(16, 16))
    assert np.array_equal(freqs, ref.freqs)
    assert np.max(np.abs(phi - ref.phi)) <= 1e-15
    assert np.linalg.norm(w - ref.w) <= 1e-12 * np.linalg.norm(ref.w)


@pytest.mark.parametrize("order", [wdd.WDD_ORDER_SPECTRUM, wdd.WDD_ORDER_OBJECT])
def test_off_centre_probe(order):
    """Frames whose diffraction disc sits off the detector's centre, reconstructed with that
    centre: D and the image against the oracle with the same centre, and equal (up to FP32
    rounding) to the centred reconstruction of the same frames moved back."""
    wl = synth.Workload("offc", 32, 32, 64, 10.0, 64, 64, 64, 16, 1.5, 0.3, 2e4, seed=7)
    pos = synth.raster_positions(wl.sy, wl.sx)
    centred = wl.frames(pos)
    dy, dx = -5, 7
    moved = np.roll(centred, (dy, dx), axis=(1, 2))
    center = (wl.n // 2 + dy, wl.n // 2 + dx)
    amp = wl.aperture_amplitude()
    out = {}
    for name, frames, c in (("moved", moved, center), ("centred", centred, None)):
        dev = device(frames)
        with wdd.Plan(wl.radius, wl.sy, wl.sx, wl.n, wl.n, wl.k, amplitude=amp, center=c, max_batch=wl.batch,
                      order=order) as plan:
            for b in range(0, len(pos), wl.batch):
                plan.push(dev[b:b + wl.batch], pos[b:b + wl.batch])
            out[name] = (plan.snapshot(), plan.spectrum())
    live = O.Live(O.make_plan(wl.sy, wl.sx, wl.n, wl.n, wl.radius, wl.k, amplitude=amp, center=center), "N")
    live.push(moved, pos)
    errs = dict(D=rel_d(out["moved"][1], live.spectrum()), O=rel_img(out["moved"][0], live.snapshot()),
                moved_vs_centred=rel_img(out["moved"][0], out["centred"][0]))
    say(f"[boundary] off-centre probe, order {order}: {errs}")
    assert max(errs.values()) <= 1e-5


@pytest.mark.parametrize("sy,sx", [(1, 1), (4, 6), (32, 32), (24, 40), (128, 64), (512, 512), (96, 200)])
def test_display_of_a_spectrum_grid(sy, sx):
    """wdd_display: eq. extract on any spectrum grid (radix-2 passes for power-of-two sides,
    direct sums otherwise) against the oracle's display."""
    import torch
    rng = np.random.default_rng(sy * 1000 + sx)
    d = (rng.normal(size=(sy, sx)) + 1j * rng.normal(size=(sy, sx))) * 0.01
    d[0, 0] = 3.0 + 0.5j
    dev = torch.from_numpy(d.astype(np.complex64)).to("cuda")
    out = wdd.display(dev)
    torch.cuda.synchronize()
    ref = O.display(d.astype(np.complex64).astype(np.complex128))
    err = rel_img(out.cpu().numpy(), ref)
    say(f"[boundary] display {sy}x{sx}: {err:.2e}")
    assert err <= 1e-5
    # D[0, 0] = 0: the normalisation is undefined and the image is zero
    dev[0, 0] = 0
    out2 = wdd.display(dev)
    torch.cuda.synchronize()
    assert not torch.any(out2)


def test_display_of_a_plans_spectrum_is_its_snapshot():
    import torch
    wl = synth.WORKLOADS["small"]
    pos = synth.raster_positions(wl.sy, wl.sx)
    frames = wl.frames(pos)
    with wdd.Plan(wl.radius, wl.sy, wl.sx, wl.n, wl.n, wl.k, dtype=wdd.WDD_F32, amplitude=wl.aperture_amplitude(),
                  max_batch=len(pos)) as plan:
        plan.push(device(frames), pos)
        snap = plan.snapshot()
        d = plan.spectrum()
        _, _, freqs = plan.export()
    grid = np.zeros((wl.sy, wl.sx), np.complex64)
    grid[freqs[:, 0], freqs[:, 1]] = d
    out = wdd.display(torch.from_numpy(grid).to("cuda"))
    torch.cuda.synchronize()
    assert rel_img(out.cpu().numpy(), snap) <= 1e-6
