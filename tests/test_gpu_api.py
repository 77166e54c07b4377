"""GPU edge cases through the C ABI: ragged batches, non-square and non-power-of-two
geometries, degenerate sizes, error paths and state handling."""
import numpy as np
import pytest

import oracle.wdd as O
import paper_2212_01309_amd as wdd
from gpu_util import device, rel, rel_a, rel_d, rel_img, say

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _oracle(radius, sy, sx, ny, nx, k, frames, pos, defocus=0.0, amplitude=1.0, step=1.0):
    plan = O.make_plan(sy, sx, ny, nx, radius, k, amplitude=amplitude, defocus_edge=defocus, step=step)
    live = O.Live(plan, "N")
    live.push(frames, pos)
    return plan, live.acc, live.spectrum(), live.snapshot()


def _random_case(seed, sy, sx, ny, nx, n, dtype):
    rng = np.random.default_rng(seed)
    lin = rng.integers(0, sy * sx, size=n)
    pos = np.stack([lin // sx, lin % sx], axis=1).astype(np.int32)
    if dtype == wdd.WDD_U16:
        frames = rng.poisson(20.0, size=(n, ny, nx)).astype(np.uint16)
    else:
        frames = rng.uniform(0, 1, size=(n, ny, nx)).astype(np.float32)
    return frames, pos


@pytest.mark.parametrize("case", [
    # non-square scan and detector, K not a multiple of 32, odd scan lengths (direct DFT path)
    dict(radius=5.5, sy=24, sx=40, ny=40, nx=48, k=50, defocus=1.1, dtype=wdd.WDD_F32, batches=[7, 33, 1, 64, 0, 95]),
    dict(radius=3.0, sy=30, sx=18, ny=12, nx=16, k=10, step=0.75, dtype=wdd.WDD_U16, batches=[31, 32, 33, 100]),
    # K = 1 and a scan of a single position
    dict(radius=4.0, sy=1, sx=1, ny=16, nx=16, k=1, dtype=wdd.WDD_U16, batches=[3, 1]),
    dict(radius=8.0, sy=32, sx=32, ny=32, nx=32, k=256, dtype=wdd.WDD_U16, batches=[256, 5, 200]),
])
def test_ragged_batches_and_odd_geometries(case):
    batches = case.pop("batches")
    dtype = case.pop("dtype")
    n = sum(batches)
    say(f"[api] geometry {case}, batches {batches}")
    frames, pos = _random_case(1, case["sy"], case["sx"], case["ny"], case["nx"], n, dtype)
    dev = device(frames)
    mb = max(batches)
    with wdd.Plan(case["radius"], case["sy"], case["sx"], case["ny"], case["nx"], case["k"], dtype=dtype,
                  defocus=case.get("defocus", 0.0), step=case.get("step", 1.0), max_batch=mb) as plan:
        b0 = 0
        for nb in batches:
            plan.push(dev[b0:b0 + nb], pos[b0:b0 + nb])
            b0 += nb
        got_o = plan.snapshot()
        got_a, got_d = plan.accumulator(), plan.spectrum()
        assert plan.info().frames_seen == n
    oplan, a, d, o = _oracle(case["radius"], case["sy"], case["sx"], case["ny"], case["nx"], case["k"], frames, pos,
                             defocus=case.get("defocus", 0.0), step=case.get("step", 1.0))
    errs = (rel_a(got_a, a), rel_d(got_d, d), rel_img(got_o, o))
    say(f"[api] errors A/D/O {errs}")
    assert max(errs) <= TOL


def test_decode_of_full_range_counts():
    """Every uint16 value decodes exactly: one-hot frames of 65535 and a full-range random frame."""
    ny = nx = 32
    frames = np.zeros((40, ny, nx), np.uint16)
    rng = np.random.default_rng(3)
    for i in range(32):
        frames[i, rng.integers(0, ny), rng.integers(0, nx)] = 65535 - i
    frames[32:] = rng.integers(0, 65536, size=(8, ny, nx), dtype=np.uint16)
    pos = np.zeros((40, 2), np.int32)
    with wdd.Plan(8.0, 4, 4, ny, nx, 64, dtype=wdd.WDD_U16, max_batch=64) as plan:
        plan.push(device(frames), pos)
        h = plan.projection()
        sig = plan.info().sigma_px
    ref = O.project(frames, O.hg_basis(ny, nx, 64, sig))
    for i in range(40):
        assert rel(h[i], ref[i]) <= 1e-6, i


def test_host_and_device_frames_agree_bitwise():
    frames, pos = _random_case(2, 16, 16, 32, 32, 300, wdd.WDD_U16)
    out = []
    for on_dev in (True, False):
        with wdd.Plan(8.0, 16, 16, 32, 32, 64, max_batch=128) as plan:
            src = device(frames) if on_dev else frames
            for b in range(0, 300, 128):
                plan.push(src[b:b + 128], pos[b:b + 128])
            out.append((plan.accumulator(), plan.snapshot()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_deterministic_and_reset():
    frames, pos = _random_case(4, 16, 16, 32, 32, 200, wdd.WDD_U16)
    dev = device(frames)
    with wdd.Plan(8.0, 16, 16, 32, 32, 64, max_batch=100) as p1, wdd.Plan(8.0, 16, 16, 32, 32, 64, max_batch=100) as p2:
        for b in range(0, 200, 100):
            p1.push(dev[b:b + 100], pos[b:b + 100])
            p2.push(dev[b:b + 100], pos[b:b + 100])
        a1, a2 = p1.accumulator(), p2.accumulator()
        assert np.array_equal(a1, a2)
        p1.reset()
        assert p1.info().frames_seen == 0
        assert not np.any(p1.accumulator())
        for b in range(0, 200, 100):
            p1.push(dev[b:b + 100], pos[b:b + 100])
        assert np.array_equal(p1.accumulator(), a1)


def test_out_of_range_position_rejects_the_whole_batch():
    frames, pos = _random_case(5, 16, 16, 32, 32, 64, wdd.WDD_U16)
    dev = device(frames)
    with wdd.Plan(8.0, 16, 16, 32, 32, 64, max_batch=64) as plan:
        plan.push(dev[:32], pos[:32])
        before = plan.accumulator()
        bad = pos[32:].copy()
        bad[7] = (16, 0)
        with pytest.raises(wdd.WddError) as ei:
            plan.push(dev[32:], bad)
        assert ei.value.code == wdd.WDD_ERANGE
        bad[7] = (0, -1)
        with pytest.raises(wdd.WddError):
            plan.push(dev[32:], bad)
        assert np.array_equal(plan.accumulator(), before)
        assert plan.info().frames_seen == 32
        with pytest.raises(wdd.WddError) as ei:
            plan.push(np.zeros((65, 32, 32), np.uint16), np.zeros((65, 2), np.int32))
        assert ei.value.code == wdd.WDD_EINVAL
        plan.push(dev[32:32], pos[32:32])        # n = 0 is a no-op
        assert np.array_equal(plan.accumulator(), before)


def test_snapshot_before_any_frame_is_zero_and_device_output():
    import torch
    with wdd.Plan(8.0, 16, 16, 32, 32, 64) as plan:
        assert not np.any(plan.snapshot())
        frames, pos = _random_case(6, 16, 16, 32, 32, 50, wdd.WDD_U16)
        plan.push(device(frames), pos)
        host = plan.snapshot()
        out = torch.empty((16, 16), dtype=torch.complex64, device="cuda")
        plan.snapshot(out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), host)


def test_repeated_positions_are_summed():
    frames, pos = _random_case(7, 8, 8, 16, 16, 10, wdd.WDD_F32)
    with wdd.Plan(4.0, 8, 8, 16, 16, 16, dtype=wdd.WDD_F32) as once, wdd.Plan(4.0, 8, 8, 16, 16, 16, dtype=wdd.WDD_F32) as twice:
        once.push(device(frames * 2), pos)
        twice.push(device(frames), pos)
        twice.push(device(frames), pos)
        assert rel_a(twice.accumulator(), once.accumulator()) <= 1e-6


def test_arrival_order_does_not_matter():
    frames, pos = _random_case(8, 32, 32, 32, 32, 1024, wdd.WDD_U16)
    perm = np.random.default_rng(9).permutation(1024)
    res = []
    for order in (np.arange(1024), perm):
        with wdd.Plan(8.0, 32, 32, 32, 32, 64, max_batch=256) as plan:
            fr, ps = device(frames[order]), pos[order]
            for b in range(0, 1024, 256):
                plan.push(fr[b:b + 256], ps[b:b + 256])
            res.append(plan.snapshot())
    assert rel(res[1], res[0]) <= 1e-6


def test_invalid_plans_are_rejected():
    with pytest.raises(wdd.WddError) as ei:
        wdd.Plan(8.0, 16, 16, 32, 30, 64)
    assert ei.value.code == wdd.WDD_EINVAL
    with pytest.raises(wdd.WddError):
        wdd.Plan(8.0, 16, 16, 32, 32, 64, max_batch=0)


def _oracle_all(radius, s, n, k, frames, pos):
    plan = O.make_plan(s, s, n, n, radius, k)
    live = O.Live(plan, "N")
    live.push(frames, pos)
    return live.acc, live.spectrum(), live.snapshot()


@pytest.mark.parametrize("rows", [1, 2, 16, 17, 40])
def test_row_factored_and_direct_updates_agree(rows):
    """Batches on <= 16 scan rows take the row-factored update, others the direct one;
    both must reproduce the oracle, also at the boundary."""
    s, n, k = 48, 32, 64
    rng = np.random.default_rng(100 + rows)
    ys = rng.choice(s, size=rows, replace=False)
    b = 96
    pos = np.stack([ys[rng.integers(0, rows, size=b)], rng.integers(0, s, size=b)], axis=1).astype(np.int32)
    frames = rng.poisson(30.0, size=(b, n, n)).astype(np.uint16)
    with wdd.Plan(8.0, s, s, n, n, k, max_batch=b) as plan:
        plan.profile_enable(wdd.STAGE_ALL)
        plan.push(device(frames), pos)
        o = plan.snapshot()
        prof = plan.profile_read()
        a, d = plan.accumulator(), plan.spectrum()
    assert prof["factored_launches"] == (1 if rows <= 16 else 0)
    ra, rd, ro = _oracle_all(8.0, s, n, k, frames, pos)
    errs = (rel_a(a, ra), rel_d(d, rd), rel_img(o, ro))
    say(f"[api] rows={rows}: A/D/O {errs}")
    assert max(errs) <= TOL


def test_push_snapshot_matches_push_then_snapshot():
    s, n, k = 32, 32, 100          # K not a power of two
    rng = np.random.default_rng(11)
    frames = rng.poisson(10.0, size=(6 * 32, n, n)).astype(np.uint16)
    lin = np.concatenate([np.arange(32) + 32 * r for r in range(3)] + [rng.integers(0, s * s, size=96)])
    pos = np.stack([lin // s, lin % s], axis=1).astype(np.int32)
    dev = device(frames)
    with wdd.Plan(8.0, s, s, n, n, k, max_batch=32) as p1, wdd.Plan(8.0, s, s, n, n, k, max_batch=32) as p2:
        for b in range(0, len(pos), 32):
            p1.push(dev[b:b + 32], pos[b:b + 32])
            o1 = p1.snapshot()
            o2 = p2.push_snapshot(dev[b:b + 32], pos[b:b + 32])
            assert rel_img(o2, o1) <= 1e-6, b
            assert rel_d(p2.spectrum(), p1.spectrum()) <= 1e-6
        assert np.array_equal(p1.accumulator(), p2.accumulator())
        o3 = p2.push_snapshot(dev[:0], pos[:0])     # n = 0: a plain snapshot
        assert rel_img(o3, o1) <= 1e-6


def test_snapshot_into_the_plans_pinned_buffer():
    frames, pos = _random_case(12, 16, 16, 32, 32, 64, wdd.WDD_U16)
    with wdd.Plan(8.0, 16, 16, 32, 32, 64) as plan:
        plan.push(device(frames), pos)
        ref = plan.snapshot()
        buf = plan.snapshot_buffer()
        got = plan.snapshot(out=buf)
        assert got is buf
        assert np.array_equal(buf, ref)
        buf[:] = 0
        again = plan.push_snapshot(device(frames[:0]), pos[:0], out=buf)
        assert np.array_equal(again, ref)


@pytest.mark.parametrize("order", [0, 1])
def test_asynchronous_device_snapshots_match_blocking_ones(order):
    """WDD_OUT_DEVICE_ASYNC: pushes and snapshots pipeline on the plan's stream; after
    sync() each output holds the image of its own point in the sequence."""
    import torch
    frames, pos = _random_case(13, 32, 32, 32, 32, 512, wdd.WDD_U16)
    dev = device(frames)
    outs = [torch.empty((32, 32), dtype=torch.complex64, device="cuda") for _ in range(8)]
    with wdd.Plan(8.0, 32, 32, 32, 32, 64, max_batch=64, order=order) as a, \
            wdd.Plan(8.0, 32, 32, 32, 32, 64, max_batch=64, order=order) as b:
        ref = []
        for i in range(8):
            a.push_snapshot(dev[64 * i:64 * (i + 1)], pos[64 * i:64 * (i + 1)], out=outs[i], wait=False)
            ref.append(b.push_snapshot(dev[64 * i:64 * (i + 1)], pos[64 * i:64 * (i + 1)]).copy())
        a.sync()
        for i in range(8):
            assert np.array_equal(outs[i].cpu().numpy(), ref[i]), i
        assert a.info().frames_seen == 512
        bad = torch.empty((31, 32), dtype=torch.complex64, device="cuda")
        with pytest.raises(ValueError):
            a.snapshot(out=bad, wait=False)
        lib = wdd.load_library()
        assert lib.wdd_snapshot(a._h, outs[0].data_ptr(), 4, None) == wdd.WDD_EINVAL


def test_profile_period_samples_one_push_in_n():
    frames, pos = _random_case(14, 16, 16, 32, 32, 256, wdd.WDD_U16)
    dev = device(frames)
    with wdd.Plan(8.0, 16, 16, 32, 32, 64, max_batch=32, order=wdd.WDD_ORDER_OBJECT) as plan:
        plan.profile_period(4)
        plan.profile_enable(wdd.STAGE_ALL)
        for b in range(0, 256, 32):
            plan.push(dev[b:b + 32], pos[b:b + 32])
        prof = plan.profile_read()
        assert prof["project_launches"] == 2 and prof["accumulate_launches"] >= 2
        assert prof["factored_launches"] == prof["accumulate_launches"]
        assert prof["accumulate_ms"] > 0
        with pytest.raises(wdd.WddError) as ei:
            plan.profile_period(0)
        assert ei.value.code == wdd.WDD_EINVAL


@pytest.mark.parametrize("order", [0, 1])
def test_many_asynchronous_steps_keep_their_own_positions(order):
    """More asynchronous push + snapshot steps than the library keeps in flight (the host
    runs ahead of the GPU and must wait for pinned upload blocks to come free): each step
    must still see its own positions, so the spectrum equals that of the same pushes made
    one at a time, bit for bit."""
    import torch
    s, n, b, steps = 64, 32, 64, 3 * wdd.WDD_MAX_PUSHES_IN_FLIGHT
    rng = np.random.default_rng(21 + order)
    lin = rng.integers(0, s * s, size=b * steps)
    pos = np.stack([lin // s, lin % s], axis=1).astype(np.int32)
    dev = device(rng.poisson(30.0, size=(b * steps, n, n)).astype(np.uint16))
    out = torch.empty((s, s), dtype=torch.complex64, device="cuda")
    with wdd.Plan(8.0, s, s, n, n, 64, max_batch=b, order=order) as a, \
            wdd.Plan(8.0, s, s, n, n, 64, max_batch=b, order=order) as one:
        for i in range(steps):
            a.push_snapshot(dev[i * b:(i + 1) * b], pos[i * b:(i + 1) * b], out=out, wait=False)
        for i in range(steps):
            one.push(dev[i * b:(i + 1) * b], pos[i * b:(i + 1) * b])
            one.sync()
        a.sync()
        if order == 0:  # A itself; D there is formed at a snapshot (in the update for a)
            assert np.array_equal(a.accumulator(), one.accumulator())
            one.snapshot()
            assert rel_d(a.spectrum(), one.spectrum()) <= 1e-6
        else:
            assert np.array_equal(a.spectrum(), one.spectrum())
        assert a.info().frames_seen == one.info().frames_seen == b * steps


def test_temporary_device_frames_outlive_the_call():
    """A device tensor made only for the call (freed when it returns) is held by the binding
    until the plan's stream has read it, even while another plan allocates and pushes."""
    frames, pos = _random_case(17, 8, 8, 16, 16, 10, wdd.WDD_F32)
    for _ in range(3):
        with wdd.Plan(4.0, 8, 8, 16, 16, 16, dtype=wdd.WDD_F32) as a, \
                wdd.Plan(4.0, 8, 8, 16, 16, 16, dtype=wdd.WDD_F32) as b:
            a.push(device(frames * 3), pos)
            for _ in range(3):
                b.push(device(frames), pos)
            assert rel_a(b.accumulator(), a.accumulator()) <= 1e-6


def test_plans_take_device_memory_from_the_callers_allocator():
    """wdd_set_allocator: a plan created under torch's caching allocator takes every device
    buffer from it, gives each back when destroyed, and computes what a plan with its own
    allocations does; an allocator that returns nothing makes creation fail cleanly."""
    import torch
    frames, pos = _random_case(23, 16, 16, 32, 32, 64, wdd.WDD_U16)
    dev = device(frames)
    live = {}

    def alloc(n):
        ptr = torch.cuda.caching_allocator_alloc(n)
        live[ptr] = n
        return ptr

    def release(ptr):
        del live[ptr]
        torch.cuda.caching_allocator_delete(ptr)

    try:
        wdd.set_allocator(alloc, release)
        with wdd.Plan(8.0, 16, 16, 32, 32, 64, order=wdd.WDD_ORDER_OBJECT) as lent:
            assert len(live) > 5 and sum(live.values()) >= lent.info().device_bytes
            got = lent.push_snapshot(dev, pos)
        assert not live
        wdd.set_allocator(lambda n: 0, lambda p: None)
        with pytest.raises(wdd.WddError) as ei:
            wdd.Plan(8.0, 16, 16, 32, 32, 64)
        assert ei.value.code == wdd.WDD_ENOMEM
    finally:
        wdd.set_allocator(None)
    with wdd.Plan(8.0, 16, 16, 32, 32, 64, order=wdd.WDD_ORDER_OBJECT) as own:
        assert np.array_equal(own.push_snapshot(dev, pos), got)


@pytest.mark.parametrize("order,s,precision,n", [(1, 32, "fp32", 32), (0, 32, "fp32", 32), (1, 24, "fp32", 32),
                                                  (0, 24, "fp32", 32), (1, 32, "bf16_hilo", 32),
                                                  (1, 32, "fp32", 160), (0, 32, "fp32", 160),
                                                  (1, 32, "bf16_hilo", 160)])
def test_deferred_device_snapshots_match_asynchronous_ones(order, s, precision, n):
    """WDD_OUT_DEVICE_DEFERRED: the display's last pass is written by the next push's first
    launch (power-of-two Sx: from the partial rows in object order, from the first pass's
    grid in spectrum order; with a 160-row detector in object order, by the first update
    launch, from the previous push's copy of the partial rows and D[0], while a 64-frame
    batch over about 28 scan rows takes two update passes) or queued at once otherwise;
    either way each output holds the image of its own point, bit for bit the asynchronous
    one, and a plain push, or a call that waits for the stream or changes the state
    (inspection, checkpoint, reset, destroy), writes a pending image first."""
    import torch
    b, steps = 64, 8
    frames, pos = _random_case(31 + s + order, s, s, n, n, b * (steps + 5), wdd.WDD_U16)
    dev = device(frames)
    blk = lambda i: (dev[i * b:(i + 1) * b], pos[i * b:(i + 1) * b])
    img = lambda: torch.empty((s, s), dtype=torch.complex64, device="cuda")
    outs = {True: [img() for _ in range(steps + 5)], False: [img() for _ in range(steps + 5)]}
    kw = dict(max_batch=b, order=order, precision=precision)
    with wdd.Plan(8.0, s, s, n, n, 64, **kw) as a, wdd.Plan(8.0, s, s, n, n, 64, **kw) as r:
        for i in range(steps):
            a.push_snapshot(*blk(i), out=outs[True][i], wait=False, defer=True)
            r.push_snapshot(*blk(i), out=outs[False][i], wait=False)
        a.sync()
        r.sync()
        for i in range(steps):
            assert torch.equal(outs[True][i], outs[False][i]), i
        # a pending image is written by a plain push, and before an inspection, a checkpoint
        # and a reset
        for i, settle in zip(range(steps, steps + 4), (lambda p: p.push(*blk(0)), lambda p: p.spectrum(),
                                                        lambda p: p.checkpoint(), lambda p: p.reset())):
            a.push_snapshot(*blk(i), out=outs[True][i], wait=False, defer=True)
            r.push_snapshot(*blk(i), out=outs[False][i], wait=False)
            settle(a)
            settle(r)
            torch.cuda.synchronize()
            assert torch.equal(outs[True][i], outs[False][i]), i
        i = steps + 4
        a.push_snapshot(*blk(i), out=outs[True][i], wait=False, defer=True)
        r.push_snapshot(*blk(i), out=outs[False][i], wait=False)
    torch.cuda.synchronize()  # both plans destroyed: the pending image was written first
    assert torch.equal(outs[True][i], outs[False][i])
