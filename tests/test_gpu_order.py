"""Object order (the Wiener filter applied per frame, accumulating D directly, as the
modified-WDD algorithm is written) against the oracle's per-frame order and the
spectrum order, including batches that need several row passes."""
import numpy as np
import pytest

import oracle.wdd as O
import paper_2212_01309_amd as wdd
import synth
from gpu_util import device, rel, rel_d, rel_img, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def medium_raster():
    """The medium workload's full raster and the oracle's object-order result for it."""
    wl = synth.WORKLOADS["medium"]
    pos = synth.raster_positions(wl.sy, wl.sx)
    frames = wl.frames(pos)
    amp = wl.aperture_amplitude()
    live = O.Live(O.make_plan(wl.sy, wl.sx, wl.n, wl.n, wl.radius, wl.k, amplitude=amp), "P")
    live.push(frames, pos)
    return wl, pos, frames, live.spectrum(), live.snapshot()


@pytest.mark.parametrize("mode", ["blocking", "deferred"])
def test_object_order_full_raster(medium_raster, mode):
    """Every batch through push_snapshot: blocking host images, or (as the bench drives it)
    device images each written by the next push's first launch."""
    import torch
    wl, pos, frames, d_ref, o_ref = medium_raster
    dev = device(frames)
    shown = torch.empty((wl.sy, wl.sx), dtype=torch.complex64, device="cuda")
    with wdd.Plan(wl.radius, wl.sy, wl.sx, wl.n, wl.n, wl.k, amplitude=wl.aperture_amplitude(), max_batch=wl.batch,
                  order=wdd.WDD_ORDER_OBJECT) as plan:
        for b in range(0, len(pos), wl.batch):
            if mode == "blocking":
                o = plan.push_snapshot(dev[b:b + wl.batch], pos[b:b + wl.batch])
            else:
                plan.push_snapshot(dev[b:b + wl.batch], pos[b:b + wl.batch], out=shown, wait=False, defer=True)
        plan.sync()
        if mode == "deferred":
            o = shown.cpu().numpy()
        d = plan.spectrum()
        with pytest.raises(wdd.WddError) as ei:
            plan.accumulator()
        assert ei.value.code == wdd.WDD_ESTATE
    errs = (rel_d(d, d_ref), rel_img(o, o_ref))
    say(f"[order] object, medium full raster, {mode} images: D/O {errs}")
    assert max(errs) <= 1e-5


@pytest.mark.parametrize("rows,k", [(3, 100), (40, 100), (5, 20), (7, 64)])
def test_object_order_matches_spectrum_order(rows, k):
    """K = 20, 64, 100 give 8, 16 and 32 lanes per kept frequency in the fused update;
    40 rows take three passes."""
    s, n = 48, 32
    rng = np.random.default_rng(31 + rows)
    ys = rng.choice(s, size=rows, replace=False)
    b = 160
    pos = np.stack([ys[rng.integers(0, rows, size=b)], rng.integers(0, s, size=b)], axis=1).astype(np.int32)
    frames = rng.poisson(20.0, size=(b, n, n)).astype(np.uint16)
    dev = device(frames)
    out = {}
    for order in (wdd.WDD_ORDER_SPECTRUM, wdd.WDD_ORDER_OBJECT):
        with wdd.Plan(8.0, s, s, n, n, k, max_batch=b, order=order) as plan:
            plan.push(dev[:100], pos[:100])
            plan.push(dev[100:], pos[100:])
            out[order] = (plan.snapshot(), plan.spectrum())
            image = plan.checkpoint()
            plan.reset()
            assert not np.any(plan.snapshot())
            plan.restore(image)
            assert np.array_equal(plan.snapshot(), out[order][0])
    e = (rel_d(out[1][1], out[0][1]), rel_img(out[1][0], out[0][0]))
    say(f"[order] rows={rows}: object vs spectrum D/O {e}")
    assert max(e) <= 1e-6
    live = O.Live(O.make_plan(s, s, n, n, 8.0, k), "P")
    live.push(frames, pos)
    assert rel_img(out[1][0], live.snapshot()) <= 1e-5


def test_object_order_long_row():
    """One scan row with more frames than the fused update stages at once (positions repeat)."""
    s, n, k, b = 48, 32, 64, 700
    rng = np.random.default_rng(77)
    pos = np.stack([np.full(b, 17), rng.integers(0, s, size=b)], axis=1).astype(np.int32)
    frames = rng.poisson(12.0, size=(b, n, n)).astype(np.uint16)
    with wdd.Plan(8.0, s, s, n, n, k, max_batch=b, order=wdd.WDD_ORDER_OBJECT) as plan:
        got = plan.push_snapshot(device(frames), pos)
    live = O.Live(O.make_plan(s, s, n, n, 8.0, k), "P")
    live.push(frames, pos)
    err = rel_img(got, live.snapshot())
    say(f"[order] one row of {b} frames: {err:.2e}")
    assert err <= 1e-5


def test_object_order_host_frames_and_float32():
    """Host-memory float32 frames through the staging copy; wdd_update_probe needs A."""
    s, n, k = 16, 32, 36
    rng = np.random.default_rng(5)
    pos = np.stack([np.repeat(np.arange(s), s), np.tile(np.arange(s), s)], axis=1).astype(np.int32)
    frames = rng.random((s * s, n, n)).astype(np.float32)
    with wdd.Plan(8.0, s, s, n, n, k, dtype=wdd.WDD_F32, max_batch=64, order=wdd.WDD_ORDER_OBJECT) as plan:
        for b in range(0, s * s, 64):
            plan.push(frames[b:b + 64], pos[b:b + 64])
        got = plan.snapshot()
        with pytest.raises(wdd.WddError) as ei:
            plan.update_probe(8.0, defocus=0.5)
        assert ei.value.code == wdd.WDD_ESTATE
    live = O.Live(O.make_plan(s, s, n, n, 8.0, k), "P")
    live.push(frames, pos)
    assert rel_img(got, live.snapshot()) <= 1e-5


@pytest.mark.parametrize("radius,sy,sx,n,k,rows", [(8.0, 64, 64, 32, 64, 3), (8.0, 64, 32, 32, 36, 20),
                                                   (8.0, 32, 128, 32, 64, 1), (4.0, 256, 16, 16, 20, 2)])
def test_display_rows_left_by_the_update(radius, sy, sx, n, k, rows):
    """Before a snapshot the object-order update also leaves the display's first pass (the
    DFT along v_y) as one partial row per chunk of frequencies, and the column pass sums
    them.  The image must match the two-pass display of the same D and the oracle, in
    every case: 2 to 4 chunks per v_x, two row passes (20 rows), Sx > Sy, and a tall scan
    whose 16 chunks per v_x exceed what the column pass sums (the two-pass display)."""
    rng = np.random.default_rng(1000 + sy + sx + rows)
    b = 200
    ys = rng.choice(sy, size=rows, replace=False)
    pos = np.stack([ys[rng.integers(0, rows, size=b)], rng.integers(0, sx, size=b)], axis=1).astype(np.int32)
    frames = rng.poisson(15.0, size=(b, n, n)).astype(np.uint16)
    dev = device(frames)
    errs = []
    with wdd.Plan(radius, sy, sx, n, n, k, max_batch=b, order=wdd.WDD_ORDER_OBJECT) as a, \
            wdd.Plan(radius, sy, sx, n, n, k, max_batch=b, order=wdd.WDD_ORDER_OBJECT) as two:
        for part in (slice(0, 120), slice(120, 200)):
            got = a.push_snapshot(dev[part], pos[part])
            two.push(dev[part], pos[part])
            ref = two.snapshot()
            errs.append(rel_img(got, ref))
            assert np.array_equal(a.spectrum(), two.spectrum())
        # a snapshot with no push in between reads the same partial rows
        assert np.array_equal(a.snapshot(), got)
        live = O.Live(O.make_plan(sy, sx, n, n, radius, k), "P")
        live.push(frames, pos)
        errs.append(rel_img(got, live.snapshot()))
        # a plain push leaves them stale: both plans then take the two-pass display
        a.push(dev[:7], pos[:7])
        two.push(dev[:7], pos[:7])
        assert np.array_equal(a.snapshot(), two.snapshot())
    say(f"[order] display rows from the update, {sy}x{sx} scan, {rows} rows: vs two-pass, vs oracle {errs}")
    assert max(errs[:2]) <= 1e-6 and errs[2] <= 1e-5


@pytest.mark.parametrize("sy,sx", [(1, 1), (2, 8), (4, 4), (8, 2), (16, 32)])
def test_display_rows_on_short_scan_columns(sy, sx):
    """Short scan columns (S_y = 1, 2, 4: fewer outputs than the workgroup's waves; 8 and 16:
    several lanes per output) through push_snapshot in object order, whose update transforms
    each chunk's display row itself, against the oracle's per-frame order."""
    n, k, b = 16, 16, 3 * sy * sx
    rng = np.random.default_rng(500 + sy * 64 + sx)
    lin = rng.integers(0, sy * sx, size=b)
    pos = np.stack([lin // sx, lin % sx], axis=1).astype(np.int32)
    order = np.argsort(pos[:, 0], kind="stable")  # whole rows per push, at most 16 rows per pass
    pos = np.ascontiguousarray(pos[order])
    frames = rng.poisson(15.0, size=(b, n, n)).astype(np.uint16)
    dev = device(frames)
    half = b // 2
    with wdd.Plan(4.0, sy, sx, n, n, k, max_batch=b, order=wdd.WDD_ORDER_OBJECT) as plan:
        plan.push_snapshot(dev[:half], pos[:half])
        got = plan.push_snapshot(dev[half:], pos[half:])
    live = O.Live(O.make_plan(sy, sx, n, n, 4.0, k), "P")
    live.push(frames, pos)
    err = rel_img(got, live.snapshot())
    say(f"[order] display rows, {sy}x{sx} scan: {err:.2e}")
    assert err <= 1e-5
