"""Pins of the field-of-view patch reading (Section 10, Discussion: patches reconstructed
independently and merged).  The geometry and the merge rule are this build's reading; the
pins fix what any such reading must satisfy: a patch covering the raster is the full-scan
result, the merge is a normalised (partition-of-unity), linear and order-independent
average, and a patched weak-phase reconstruction still recovers the object."""
import numpy as np
import pytest

import oracle.wdd as O
import synth


@pytest.mark.parametrize("s,p,o", [(32, 32, 0), (32, 16, 0), (32, 16, 4), (40, 16, 5), (33, 10, 3), (7, 7, 6)])
def test_patch_origins_cover_the_raster(s, p, o):
    org = O.patch_origins(s, p, o)
    assert org[0] == 0 and org[-1] == s - p
    assert np.all(np.diff(org) > 0) and np.all(np.diff(org) <= p - o)
    covered = np.zeros(s, int)
    for a in org:
        covered[a:a + p] += 1
    assert np.all(covered >= 1)


def test_patch_window_is_a_trapezoid():
    w = O.patch_window(10, 3)
    assert np.allclose(w, [0.25, 0.5, 0.75, 1, 1, 1, 1, 0.75, 0.5, 0.25])
    assert np.all(O.patch_window(8, 0) == 1.0)


@pytest.mark.parametrize("s,p,o", [(24, 12, 4), (30, 10, 3), (16, 16, 0), (20, 8, 0)])
def test_merge_is_a_normalised_linear_order_independent_mean(s, p, o):
    rng = np.random.default_rng(s + p + o)
    oy = O.patch_origins(s, p, o)
    ox = O.patch_origins(s + 4, p, o)
    n = len(oy) * len(ox)
    # partition of unity: identical constant patches merge to that constant
    const = [np.full((p, p), 2.5 - 1j) for _ in range(n)]
    assert np.allclose(O.merge_patches(const, oy, ox, s, s + 4, o, o), 2.5 - 1j, atol=1e-14)
    a = [rng.normal(size=(p, p)) + 1j * rng.normal(size=(p, p)) for _ in range(n)]
    b = [rng.normal(size=(p, p)) + 1j * rng.normal(size=(p, p)) for _ in range(n)]
    ma, mb = O.merge_patches(a, oy, ox, s, s + 4, o, o), O.merge_patches(b, oy, ox, s, s + 4, o, o)
    mab = O.merge_patches([2 * x - 3j * y for x, y in zip(a, b)], oy, ox, s, s + 4, o, o)
    assert np.allclose(mab, 2 * ma - 3j * mb, atol=1e-12)
    # a pixel covered by one patch only takes that patch's value
    cover = np.zeros((s, s + 4), int)
    for y0 in oy:
        for x0 in ox:
            cover[y0:y0 + p, x0:x0 + p] += 1
    for idx, img in enumerate(a):
        y0, x0 = oy[idx // len(ox)], ox[idx % len(ox)]
        one = cover[y0:y0 + p, x0:x0 + p] == 1
        assert np.allclose(ma[y0:y0 + p, x0:x0 + p][one], img[one])
    # order independence: the patches listed in another order, with their origins
    perm = rng.permutation(n)
    num = np.zeros((s, s + 4), complex)
    den = np.zeros((s, s + 4))
    w = O.patch_window(p, o)[:, None] * O.patch_window(p, o)[None, :]
    for idx in perm:
        y0, x0 = oy[idx // len(ox)], ox[idx % len(ox)]
        num[y0:y0 + p, x0:x0 + p] += w * a[idx]
        den[y0:y0 + p, x0:x0 + p] += w
    assert np.allclose(num / den, ma, atol=1e-13)


def test_one_patch_covering_the_raster_is_the_full_scan():
    wl = synth.WORKLOADS["small"]
    pos = synth.raster_positions(wl.sy, wl.sx)
    frames = wl.frames(pos)
    plan = O.make_plan(wl.sy, wl.sx, wl.n, wl.n, wl.radius, wl.k, amplitude=wl.aperture_amplitude())
    _, _, full = O.offline_reduced(plan, frames, pos)
    merged, images = O.patched_reconstruction(frames, pos, wl.sy, wl.sx, wl.sy, wl.sx, 0, 0, plan)
    assert len(images) == 1
    assert np.linalg.norm(merged - full) <= 1e-12 * np.linalg.norm(full)


def test_each_patch_is_the_live_wdd_of_its_own_frames():
    """A patch's image equals the live (frame by frame, any order) reconstruction of the
    frames inside it at their local positions."""
    wl = synth.periodic_workload(s=24, n=32, radius=8.0, k=36)
    pos = synth.raster_positions(24, 24)
    frames = wl.frames(pos)
    p, o = 12, 4
    plan = O.make_plan(p, p, wl.n, wl.n, wl.radius, wl.k, amplitude=wl.aperture_amplitude())
    _, images = O.patched_reconstruction(frames, pos, 24, 24, p, p, o, o, plan)
    oy = O.patch_origins(24, p, o)
    rng = np.random.default_rng(1)
    for idx in (0, len(images) - 1, len(images) // 2):
        y0, x0 = oy[idx // len(oy)], oy[idx % len(oy)]
        inside = np.nonzero((pos[:, 0] >= y0) & (pos[:, 0] < y0 + p) & (pos[:, 1] >= x0) & (pos[:, 1] < x0 + p))[0]
        inside = rng.permutation(inside)
        live = O.Live(plan, "P")
        for c in np.array_split(inside, 5):
            live.push(frames[c], pos[c] - np.array([y0, x0]))
        assert np.linalg.norm(live.snapshot() - images[idx]) <= 1e-12 * np.linalg.norm(images[idx])


def test_patched_weak_phase_recovery():
    """Patches of 32 x 32 with 8 positions of overlap on a 64 x 64 raster over a periodic
    128 x 128 object: the merged phase correlates with the band-limited object about as
    well as the full-scan reconstruction (physics pin, stated tolerance)."""
    s, n, radius, k = 64, 32, 8.0, 64
    wl = synth.Workload("fov", s, s, n, radius, k, 64, 2 * s, 48, 1.5, 0.3, None, seed=21)
    pos = synth.raster_positions(s, s)
    obj = wl.object()
    frames = wl.frames(pos, obj)
    amp = wl.aperture_amplitude()
    full_plan = O.make_plan(s, s, n, n, radius, k, amplitude=amp)
    _, _, full = O.offline_reduced(full_plan, frames, pos)
    patch_plan = O.make_plan(32, 32, n, n, radius, k, amplitude=amp)
    merged, _ = O.patched_reconstruction(frames, pos, s, s, 32, 32, 8, 8, patch_plan)
    f = np.fft.fft2(np.angle(obj))
    fy = np.fft.fftfreq(wl.m) * wl.m
    f[np.sqrt(fy[:, None] ** 2 + fy[None, :] ** 2) > 2 * radius * wl.m / n] = 0
    truth = np.real(np.fft.ifft2(f))[n // 2:n // 2 + s, n // 2:n // 2 + s]

    def corr(img):
        ph = np.angle(img * np.exp(-1j * np.angle(np.mean(img))))[4:-4, 4:-4]
        return float(np.corrcoef(ph.ravel(), truth[4:-4, 4:-4].ravel())[0, 1])
    c_full, c_patch = corr(full), corr(merged)
    assert c_full >= 0.85
    assert c_patch >= 0.85 and c_patch >= c_full - 0.05


def test_a_patch_without_frames_has_a_zero_image():
    """Part way through an acquisition some patches have no frames yet: D = 0 there, and
    the display's normalisation then gives a zero image (eq. extract with D[0] = 0)."""
    wl = synth.periodic_workload(s=24, n=32, radius=8.0, k=16)
    pos = synth.raster_positions(24, 24)[:100]
    frames = wl.frames(pos)
    plan = O.make_plan(12, 12, wl.n, wl.n, wl.radius, wl.k, amplitude=wl.aperture_amplitude())
    merged, images = O.patched_reconstruction(frames, pos, 24, 24, 12, 12, 0, 0, plan)
    assert not np.any(images[-1]) and np.any(images[0])
    assert not np.any(merged[12:, 12:])
