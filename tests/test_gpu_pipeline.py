"""Pipelined pushes (wdd_options.pipeline): each batch's object-order update runs in the next
push's launch beside that push's projection (k_row_fused_obj_next); with two stages the
batch's x-DFT runs one launch ahead of its update, once per kept v_x (k_row_fused_obj_next2).

Detectors of at most 128 rows give every tile a wave of its own in both projections, so the
pipelined plan must reproduce the unpipelined one bit for bit: D, the projections, the
checkpoints, and with one stage every image.  Two-stage plans cut the update into longer
chunks, so the display's partial rows (one per chunk) are summed in another grouping: their
images equal the unpipelined plan's to FP32 rounding.  Larger detectors (two 16-row tiles
per wave in the merged launch) sum the projection in another order and are compared with the
oracle instead."""
import numpy as np
import pytest

import oracle.wdd as O
import paper_2212_01309_amd as wdd
from gpu_util import device, rel_d, rel_img, say

pytestmark = pytest.mark.gpu

TOL = 1e-5
IMG_TOL = 1e-6   # two stages against the unpipelined plan: partial display rows grouped otherwise


def same_image(a, b, stages):
    """Bit for bit with one stage; to FP32 rounding of the display's partial-row sums with two."""
    a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
    b = b.cpu().numpy() if hasattr(b, "cpu") else np.asarray(b)
    if stages == 1:
        return np.array_equal(a, b)
    return np.isfinite(a).all() and rel_img(a, b) <= IMG_TOL


def _case(seed, s, n, count, raster=False):
    rng = np.random.default_rng(seed)
    if raster:   # row-major walk: a batch covers one or two scan rows
        lin = np.arange(count) % (s * s)
    else:        # scattered: a batch of 64 touches most rows (several update passes)
        lin = rng.integers(0, s * s, size=count)
    pos = np.stack([lin // s, lin % s], axis=1).astype(np.int32)
    frames = rng.poisson(20.0, size=(count, n, n)).astype(np.uint16)
    return frames, pos


@pytest.mark.parametrize("stages", [1, 2])
@pytest.mark.parametrize("s,n,raster,precision", [(32, 64, False, "fp32"), (32, 64, True, "fp32"),
                                                  (64, 128, True, "fp32"), (16, 32, False, "fp32"),
                                                  (32, 64, False, "bf16_hilo"), (32, 128, True, "fp16_hilo"),
                                                  (32, 96, True, "bf16")])
def test_pipelined_pushes_equal_unpipelined_ones(s, n, raster, precision, stages):
    """Deferred snapshots after every push, then the calls that must run a held update first
    (inspection of D and of the last projections, a blocking snapshot, a checkpoint, a reset):
    D, the projections and the checkpoints equal the unpipelined plan's bit for bit, in FP32 and
    in the reduced-precision projections (one tile per wave in both launches), with one stage or
    two (scattered batches on more than 16 rows run unpipelined there, after the held ones); the
    images too with one stage, to FP32 rounding with two.  A blocking snapshot right after a
    push equals the unpipelined wdd_push_snapshot."""
    import torch
    b, steps = 64, 9
    say(f"[pipeline] {stages} stage(s), scan {s}^2, detector {n}^2, {precision}, "
        f"{'raster' if raster else 'scattered'} batches of {b}")
    frames, pos = _case(7 + s + n, s, n, b * (steps + 3), raster)
    dev = device(frames)
    blk = lambda i: (dev[i * b:(i + 1) * b], pos[i * b:(i + 1) * b])
    img = lambda: torch.empty((s, s), dtype=torch.complex64, device="cuda")
    outs = {True: [img() for _ in range(steps)], False: [img() for _ in range(steps)]}
    kw = dict(max_batch=b, order=wdd.WDD_ORDER_OBJECT, precision=precision)
    with wdd.Plan(8.0, s, s, n, n, 64, pipeline=stages, **kw) as p, wdd.Plan(8.0, s, s, n, n, 64, **kw) as r:
        assert p.info().pipelined == stages and r.info().pipelined == 0
        for i in range(steps):
            p.push_snapshot(*blk(i), out=outs[True][i], wait=False, defer=True)
            r.push_snapshot(*blk(i), out=outs[False][i], wait=False, defer=True)
        p.sync()
        r.sync()
        for i in range(steps):
            assert same_image(outs[True][i], outs[False][i], stages), i
        # held updates run before every call that reads the state
        for q in (p, r):
            q.push(*blk(steps))
        assert np.array_equal(p.spectrum(), r.spectrum())
        for q in (p, r):
            q.push(*blk(steps + 1))
        assert np.array_equal(p.projection(), r.projection())
        assert same_image(p.snapshot(), r.snapshot(), stages)
        assert p.info().frames_seen == r.info().frames_seen == b * (steps + 2)
        for q in (p, r):
            q.push(*blk(steps + 2))
        assert p.checkpoint() == r.checkpoint()
        p.reset()
        r.reset()
        # a snapshot right after a push: a held update leaves the display's first pass, as
        # wdd_push_snapshot's update does (not the two-pass display of push + snapshot); two
        # stages hold batches of at most 16 scan rows, others run at once
        p.push(*blk(0))
        held = stages == 1 or len(np.unique(blk(0)[1][:, 0])) <= 16
        if held:
            ref = r.push_snapshot(*blk(0))
        else:
            r.push(*blk(0))
            ref = r.snapshot()
        assert same_image(p.snapshot(), ref, stages)


@pytest.mark.parametrize("stages", [1, 2])
def test_deferred_image_lands_stages_plus_one_pushes_later(stages):
    """A deferred snapshot after push i: the held update (in push i + stages' launch) leaves
    its partial rows, push i + stages + 1's launch writes the image; the stream alone then
    completes it."""
    import torch
    s, n, b = 32, 64, 64
    frames, pos = _case(3, s, n, b * 5)
    dev = device(frames)
    blk = lambda i: (dev[i * b:(i + 1) * b], pos[i * b:(i + 1) * b])
    outs = [torch.full((s, s), float("nan"), dtype=torch.complex64, device="cuda") for _ in range(2)]
    kw = dict(max_batch=b, order=wdd.WDD_ORDER_OBJECT)
    with wdd.Plan(8.0, s, s, n, n, 64, pipeline=stages, **kw) as p, wdd.Plan(8.0, s, s, n, n, 64, **kw) as r:
        p.push(*blk(0))
        r.push(*blk(0))
        p.push_snapshot(*blk(1), out=outs[0], wait=False, defer=True)
        ref = r.push_snapshot(*blk(1))
        for i in range(stages + 1):
            p.push(*blk(2 + i))
        torch.cuda.synchronize()     # no plan call in between: the pushes' launches wrote it
        assert same_image(outs[0], ref, stages)


@pytest.mark.parametrize("stages", [1, 2])
@pytest.mark.parametrize("n,raster", [(160, True), (256, False)])
def test_two_tiles_per_wave_against_the_oracle(n, raster, stages):
    """Detectors of more than 128 rows: the merged launch's 8 waves take two 16-row tiles each.
    D and the images against the oracle, and against the unpipelined plan within FP32
    rounding of the projection's summation order."""
    import torch
    s, b, steps, k, radius = 16, 32, 4, 64, 0.3 * n
    say(f"[pipeline] detector {n}^2 (two tiles per wave), scan {s}^2")
    frames, pos = _case(11 + n, s, n, b * steps, raster)
    dev = device(frames)
    kw = dict(max_batch=b, order=wdd.WDD_ORDER_OBJECT)
    outs = [torch.empty((s, s), dtype=torch.complex64, device="cuda") for _ in range(steps)]
    with wdd.Plan(radius, s, s, n, n, k, pipeline=stages, **kw) as p, wdd.Plan(radius, s, s, n, n, k, **kw) as r:
        for i in range(steps):
            p.push_snapshot(dev[i * b:(i + 1) * b], pos[i * b:(i + 1) * b], out=outs[i], wait=False, defer=True)
            r.push(dev[i * b:(i + 1) * b], pos[i * b:(i + 1) * b])
        p.sync()
        got_d, ref_d = p.spectrum(), r.spectrum()
        got_o = outs[-1].cpu().numpy()
    oplan = O.make_plan(s, s, n, n, radius, k)
    live = O.Live(oplan, "N")
    live.push(frames, pos)
    errs = dict(D=rel_d(got_d, live.spectrum()), O=rel_img(got_o, live.snapshot()), D_vs_unpipelined=rel_d(got_d, ref_d))
    say(f"[pipeline] errors {errs}")
    assert errs["D"] <= TOL and errs["O"] <= TOL and errs["D_vs_unpipelined"] <= 1e-6


@pytest.mark.parametrize("stages", [1, 2])
def test_pipelined_host_frames_and_ragged_batches(stages):
    """Frames from host memory (staged through the plan's pinned slots) and batches of changing
    size, some on many scan rows (several update passes): D bit for bit the unpipelined plan's,
    the images as in the first test."""
    import torch
    s, n = 32, 64
    sizes = [64, 7, 33, 1, 64, 50, 2]
    frames, pos = _case(23, s, n, sum(sizes))
    dev = device(frames)
    outs = {True: [], False: []}
    kw = dict(max_batch=64, order=wdd.WDD_ORDER_OBJECT)
    with wdd.Plan(8.0, s, s, n, n, 64, pipeline=stages, **kw) as p, wdd.Plan(8.0, s, s, n, n, 64, **kw) as r:
        b0 = 0
        for i, m in enumerate(sizes):
            fr = frames[b0:b0 + m] if i % 2 == 0 else dev[b0:b0 + m]   # host and device frames in turn
            for q, key in ((p, True), (r, False)):
                out = torch.empty((s, s), dtype=torch.complex64, device="cuda")
                q.push_snapshot(fr, pos[b0:b0 + m], out=out, wait=False, defer=True)
                outs[key].append(out)
            b0 += m
        p.sync()
        r.sync()
        for i in range(len(sizes)):
            assert same_image(outs[True][i], outs[False][i], stages), i
        assert np.array_equal(p.spectrum(), r.spectrum())
        assert p.info().frames_seen == r.info().frames_seen == sum(sizes)


@pytest.mark.parametrize("stages", [1, 2])
@pytest.mark.parametrize("sy,sx", [(1, 1), (1, 8), (2, 4), (4, 16)])
def test_deferred_images_on_short_scan_columns(sy, sx, stages):
    """Deferred images of pipelined plans, whose column pass rides in the update launches with
    two output rows per workgroup: a one-row scan (an odd row count: both halves of the
    workgroup take the row), two and four rows; each image against the oracle."""
    import torch
    n, k = 32, 16
    b = 3 * sy * sx
    rng = np.random.default_rng(700 + 64 * sy + sx + stages)
    lin = rng.integers(0, sy * sx, size=2 * b)
    pos = np.stack([lin // sx, lin % sx], axis=1).astype(np.int32)
    frames = rng.poisson(15.0, size=(2 * b, n, n)).astype(np.uint16)
    dev = device(frames)
    say(f"[pipeline] {stages} stage(s), deferred images on a {sy}x{sx} scan")
    outs = [torch.full((sy, sx), float("nan"), dtype=torch.complex64, device="cuda") for _ in range(2)]
    with wdd.Plan(4.0, sy, sx, n, n, k, max_batch=b, order=wdd.WDD_ORDER_OBJECT, pipeline=stages) as p:
        for i in range(2):
            p.push_snapshot(dev[i * b:(i + 1) * b], pos[i * b:(i + 1) * b], out=outs[i], wait=False, defer=True)
        p.sync()
    oplan = O.make_plan(sy, sx, n, n, 4.0, k)
    for i in range(2):
        live = O.Live(oplan, "P")
        live.push(frames[:(i + 1) * b], pos[:(i + 1) * b])
        got = outs[i].cpu().numpy()
        assert np.isfinite(got).all(), i
        err = rel_img(got, live.snapshot())
        say(f"[pipeline] image {i}: {err:.2e}")
        assert err <= TOL


@pytest.mark.parametrize("stages", [1, 2])
def test_batches_on_few_rows_out_of_row_order(stages):
    """Batches whose frames alternate between a few scan rows (held, but not in row order:
    the update and the x-DFT read the projections through the batch's row grouping): D bit
    for bit the unpipelined plan's, the images as in the first test."""
    import torch
    s, n, b, steps = 32, 64, 48, 6
    rng = np.random.default_rng(31 + stages)
    rows = [rng.choice(s, size=int(rng.integers(2, 5)), replace=False) for _ in range(steps)]
    pos = np.concatenate([np.stack([r[rng.integers(0, len(r), size=b)], rng.integers(0, s, size=b)], axis=1)
                          for r in rows]).astype(np.int32)
    frames = rng.poisson(20.0, size=(b * steps, n, n)).astype(np.uint16)
    dev = device(frames)
    say(f"[pipeline] {stages} stage(s), batches on 2..4 rows out of row order")
    outs = {True: [], False: []}
    kw = dict(max_batch=b, order=wdd.WDD_ORDER_OBJECT)
    with wdd.Plan(8.0, s, s, n, n, 64, pipeline=stages, **kw) as p, wdd.Plan(8.0, s, s, n, n, 64, **kw) as r:
        for i in range(steps):
            for q, key in ((p, True), (r, False)):
                out = torch.empty((s, s), dtype=torch.complex64, device="cuda")
                q.push_snapshot(dev[i * b:(i + 1) * b], pos[i * b:(i + 1) * b], out=out, wait=False, defer=True)
                outs[key].append(out)
        p.sync()
        r.sync()
        for i in range(steps):
            assert same_image(outs[True][i], outs[False][i], stages), i
        assert np.array_equal(p.spectrum(), r.spectrum())


@pytest.mark.parametrize("stages", [1, 2])
def test_restore_while_batches_are_held(stages):
    """A checkpoint restored into a pipelined plan that holds batches: the held updates run
    first and are then replaced by the image, so the plan continues exactly as an
    unpipelined plan given the same calls (D bit for bit, frame count)."""
    s, n, b = 32, 64, 64
    frames, pos = _case(41 + stages, s, n, b * 6, raster=True)
    dev = device(frames)
    blk = lambda i: (dev[i * b:(i + 1) * b], pos[i * b:(i + 1) * b])
    kw = dict(max_batch=b, order=wdd.WDD_ORDER_OBJECT)
    with wdd.Plan(8.0, s, s, n, n, 64, pipeline=stages, **kw) as p, wdd.Plan(8.0, s, s, n, n, 64, **kw) as r:
        for q in (p, r):
            q.push(*blk(0))
        image = r.checkpoint()
        for i in (1, 2):
            for q in (p, r):
                q.push(*blk(i))
        for q in (p, r):           # p still holds batches 1 (and 2) here
            q.restore(image)
        for i in (3, 4, 5):
            for q in (p, r):
                q.push(*blk(i))
        assert np.array_equal(p.spectrum(), r.spectrum())
        assert p.info().frames_seen == r.info().frames_seen == 4 * b
