"""Serving runtime: admission by device-memory budget, continuous batching of many
acquisitions of different geometries, and results that are the same alone and in the mix
within the FP32 bar (relative L2 <= 1e-5 on the image and on the image minus its mean;
batch boundaries differ, so the accumulation's rounding differs and results are not
bitwise equal), under each launch mode: per-acquisition streams, grouped rounds (one
projection and one update launch per row pass for all object-order acquisitions) and
grouped rounds replayed from a HIP graph."""
import numpy as np
import pytest

import oracle.wdd as O
import paper_2212_01309_amd as wdd
from gpu_util import device, rel, rel_img, say

pytestmark = pytest.mark.gpu

GEOMS = [  # (radius, scan, detector, K)
    (8.0, 32, 32, 64),
    (6.0, 48, 32, 36),
    (16.0, 64, 64, 128),
    (8.0, 40, 32, 64),
]


def _acquisition(i, radius, s, n, k):
    rng = np.random.default_rng(500 + i)
    count = s * s if s <= 48 else 1500
    lin = rng.permutation(s * s)[:count]
    pos = np.stack([lin // s, lin % s], axis=1).astype(np.int32)
    frames = rng.poisson(15.0 + 5 * i, size=(count, n, n)).astype(np.uint16)
    return frames, pos


def test_admission_by_memory_budget():
    radius, s, n, k = 8.0, 32, 32, 64
    with wdd.Server(hbm_budget_bytes=0) as probe_srv:
        a = probe_srv.open(radius, s, s, n, n, k)
        per_plan = probe_srv.stats()["device_bytes"]
    with wdd.Server(hbm_budget_bytes=int(2.5 * per_plan)) as srv:
        a = srv.open(radius, s, s, n, n, k)
        b = srv.open(radius, s, s, n, n, k)
        assert a is not None and b is not None
        assert srv.open(radius, s, s, n, n, k) is None        # over budget: deferred
        assert srv.stats()["open"] == 2
        srv.close(a)
        c = srv.open(radius, s, s, n, n, k)                   # memory freed: admitted
        assert c is not None and srv.stats()["open"] == 2


# relative L2 bound against the FP64 oracle for each projection arithmetic (as in the
# precision tests: basis rounding ~2^-17 for bf16 hi+lo)
ORACLE_BOUND = {"fp32": 1e-5, "bf16_hilo": 3e-5}


@pytest.mark.parametrize("mode", ["streams", "grouped", "graph"])
@pytest.mark.parametrize("order,precision", [(wdd.WDD_ORDER_SPECTRUM, "fp32"), (wdd.WDD_ORDER_OBJECT, "fp32"),
                                             (wdd.WDD_ORDER_OBJECT, "bf16_hilo"),
                                             (wdd.WDD_ORDER_SPECTRUM, "bf16_hilo")])
def test_each_result_is_the_same_alone_and_in_the_mix(order, precision, mode):
    """The serving mix pushes frames through a per-frame address table (frames from many
    submitted buffers in one batch); with a reduced-precision projection that is the
    bf16 kernel's address-table path, and under the grouped modes the grouped projection
    and the grouped updates of either order over all acquisitions (random submissions over
    up to 48 scan rows give rounds of several row passes).  Alone and in the mix the projections of a frame
    agree; only the accumulation's batch boundaries differ."""
    rng = np.random.default_rng(9)
    data = [_acquisition(i, *g) for i, g in enumerate(GEOMS)]
    devs = [device(f) for f, _ in data]
    with wdd.Server(hbm_budget_bytes=0, snapshot_interval_us=200.0, batch_frames=256, launch_mode=mode) as srv:
        ids = [srv.open(r, s, s, n, n, k, order=order, precision=precision) for (r, s, n, k) in GEOMS]
        cursor = [0] * len(GEOMS)
        while any(c < len(d[1]) for c, d in zip(cursor, data)):
            for _ in range(3):
                i = int(rng.integers(0, len(GEOMS)))
                c = cursor[i]
                if c >= len(data[i][1]):
                    continue
                nb = int(min(rng.integers(1, 65), len(data[i][1]) - c))
                srv.submit(ids[i], devs[i][c:c + nb], data[i][1][c:c + nb])
                cursor[i] += nb
            srv.step()
        mixed = [srv.snapshot(a) for a in ids]
        st = srv.stats()
    total = sum(len(p) for _, p in data)
    assert st["frames"] == total and st["latency_samples"] == total and st["opening"] == 0
    assert 0 < st["latency_p50_us"] <= st["latency_p99_us"] <= st["latency_max_us"]
    assert (st["group_rounds"] > 0) == (mode != "streams")
    say(f"[serving] {mode}: mix of {len(GEOMS)} acquisitions, {total} frames, {st['batches']} batches, "
        f"{st['group_rounds']} grouped rounds ({st['graph_replays']} graph replays), {st['snapshots']} snapshots, "
        f"latency p50 {st['latency_p50_us']:.0f} us p99 {st['latency_p99_us']:.0f} us")
    for i, (r, s, n, k) in enumerate(GEOMS):
        frames, pos = data[i]
        with wdd.Plan(r, s, s, n, n, k, max_batch=256, order=order, precision=precision) as plan:
            for b in range(0, len(pos), 256):
                plan.push(devs[i][b:b + 256], pos[b:b + 256])
            alone = plan.snapshot()
        e = rel_img(mixed[i], alone)
        say(f"[serving] {mode}, order {order}, {precision}, acquisition {i}: mix vs alone {e:.2e}")
        assert e <= 1e-5
    r, s, n, k = GEOMS[0]
    live = O.Live(O.make_plan(s, s, n, n, r, k), "N")
    live.push(*data[0])
    e = rel_img(mixed[0], live.snapshot())
    say(f"[serving] order {order}, {precision}, acquisition 0 vs oracle {e:.2e}")
    assert e <= ORACLE_BOUND[precision]


def test_same_geometry_in_two_bases():
    """A Hermite-Gauss and a Fourier-basis acquisition of one geometry (16 x 16 detector,
    K = 256 = ny nx) open together: each must keep its own tables and match its own plan."""
    r, s, n, k = 5.0, 16, 16, 256
    rng = np.random.default_rng(21)
    pos = synth_raster(s)
    frames = rng.poisson(25.0, size=(len(pos), n, n)).astype(np.uint16)
    dev = device(frames)
    bases = (wdd.WDD_BASIS_HERMITE_GAUSS, wdd.WDD_BASIS_FOURIER)
    with wdd.Server(hbm_budget_bytes=0, snapshot_interval_us=0.0, batch_frames=64) as srv:
        ids = [srv.open(r, s, s, n, n, k, basis=b) for b in bases]
        for b0 in range(0, len(pos), 48):
            for a in ids:
                srv.submit(a, dev[b0:b0 + 48], pos[b0:b0 + 48])
            srv.step()
        mixed = [srv.snapshot(a) for a in ids]
    for basis, got in zip(bases, mixed):
        with wdd.Plan(r, s, s, n, n, k, basis=basis, max_batch=256) as plan:
            plan.push(dev, pos)
            alone = plan.snapshot()
        e = rel_img(got, alone)
        say(f"[serving] basis {basis}: mix vs alone {e:.2e}")
        assert e <= 1e-5
    assert rel_img(mixed[0], mixed[1]) > 1e-3   # the two bases give different reconstructions


def synth_raster(s):
    yy, xx = np.meshgrid(np.arange(s, dtype=np.int32), np.arange(s, dtype=np.int32), indexing="ij")
    return np.stack([yy.ravel(), xx.ravel()], axis=1)


def test_submit_rejects_positions_off_the_raster():
    with wdd.Server(hbm_budget_bytes=0) as srv:
        a = srv.open(8.0, 16, 16, 32, 32, 64)
        fr = device(np.zeros((4, 32, 32), np.uint16))
        with pytest.raises(wdd.WddError) as ei:
            srv.submit(a, fr, np.array([[0, 0], [1, 1], [16, 2], [3, 3]], np.int32))
        assert ei.value.code == wdd.WDD_ERANGE
        assert srv.stats()["pending_frames"] == 0


@pytest.mark.parametrize("mode", ["grouped", "graph"])
def test_grouped_rounds_over_mixed_acquisitions(mode):
    """One server holding acquisitions of two frame types and two arithmetics (several
    grouped projection launches per round), a 160-row detector (one wave per 16 rows in the
    projection), object and spectrum order in the same rounds (grouped object-order updates,
    grouped row DFTs and A updates), and a steady phase of equal rounds (the graph is then
    replayed with updated arguments); each result against its own plan."""
    import torch
    cases = [  # (radius, scan, detector, K, dtype, precision, order)
        (8.0, 32, 32, 64, wdd.WDD_U16, "fp32", wdd.WDD_ORDER_OBJECT),
        (8.0, 32, 32, 64, wdd.WDD_F32, "fp32", wdd.WDD_ORDER_OBJECT),
        (6.0, 32, 32, 36, wdd.WDD_U16, "bf16_hilo", wdd.WDD_ORDER_OBJECT),
        (20.0, 32, 160, 100, wdd.WDD_U16, "fp32", wdd.WDD_ORDER_OBJECT),
        (8.0, 32, 32, 64, wdd.WDD_U16, "fp32", wdd.WDD_ORDER_SPECTRUM),
        (6.0, 32, 64, 36, wdd.WDD_U16, "bf16_hilo", wdd.WDD_ORDER_SPECTRUM),
    ]
    rng = np.random.default_rng(77)
    data = []
    for r, s, n, k, dt, prec, order in cases:
        pos = np.stack([np.repeat(np.arange(s), s), np.tile(np.arange(s), s)], axis=1).astype(np.int32)
        fr = rng.poisson(20.0, size=(s * s, n, n))
        fr = fr.astype(np.uint16) if dt == wdd.WDD_U16 else fr.astype(np.float32)
        data.append((device(fr), pos))
    with wdd.Server(hbm_budget_bytes=0, snapshot_interval_us=0.0, batch_frames=64, launch_mode=mode) as srv:
        ids = [srv.open(r, s, s, n, n, k, dtype=dt, precision=prec, order=order)
               for r, s, n, k, dt, prec, order in cases]
        for a in ids:
            srv.wait_open(a)
        for b in range(0, 32 * 32, 64):   # 16 equal rounds of 64 raster frames (two scan rows) each
            for a, (dev, pos) in zip(ids, data):
                srv.submit(a, dev[b:b + 64], pos[b:b + 64])
            srv.step()
        mixed = [srv.snapshot(a) for a in ids]
        st = srv.stats()
    say(f"[serving] {mode}, mixed classes: {st['group_rounds']} rounds, {st['graph_replays']} graph replays")
    assert st["group_rounds"] == 16
    if mode == "graph":
        assert st["graph_replays"] >= 14
    for (r, s, n, k, dt, prec, order), (dev, pos), got in zip(cases, data, mixed):
        with wdd.Plan(r, s, s, n, n, k, dtype=dt, precision=prec, order=order, max_batch=64) as plan:
            for b in range(0, len(pos), 64):
                plan.push(dev[b:b + 64], pos[b:b + 64])
            alone = plan.snapshot()
        e = rel_img(got, alone)
        say(f"[serving] {mode}, n={n} dtype={dt} {prec} order={order}: mix vs alone {e:.2e}")
        assert e <= 1e-5


def test_open_does_not_wait_for_the_tables():
    """wdd_server_open returns once the acquisition is admitted; the plan is made on a worker
    thread, frames submitted meanwhile wait, and a snapshot waits for the plan."""
    r, s, n, k = 16.0, 64, 64, 128
    rng = np.random.default_rng(3)
    pos = np.stack([np.repeat(np.arange(s), s), np.tile(np.arange(s), s)], axis=1).astype(np.int32)[:512]
    dev = device(rng.poisson(10.0, size=(512, n, n)).astype(np.uint16))
    with wdd.Server(hbm_budget_bytes=0, snapshot_interval_us=1e9, batch_frames=256) as srv:
        a = srv.open(r, s, s, n, n, k, order=wdd.WDD_ORDER_OBJECT)
        st = srv.stats()
        assert st["open"] == 1 and st["opening"] in (0, 1)
        srv.submit(a, dev, pos)
        srv.step()
        got = srv.snapshot(a)
        assert srv.stats()["opening"] == 0 and srv.stats()["frames"] == 512
    with wdd.Plan(r, s, s, n, n, k, order=wdd.WDD_ORDER_OBJECT, max_batch=256) as plan:
        plan.push(dev[:256], pos[:256])
        plan.push(dev[256:], pos[256:])
        alone = plan.snapshot()
    assert rel_img(got, alone) <= 1e-5


def test_graph_rounds_while_acquisitions_close():
    """WDD_SERVE_GRAPH while acquisitions are closed between steps: the plans are freed on
    closer threads while the scheduling thread captures the next rounds.  A closer must not
    wait on the server's stream (a wait on a capturing stream invalidates the capture) nor free
    device memory during a capture; every step succeeds and the survivors' images match the
    same acquisitions served alone."""
    radius, s, n, k = 8.0, 32, 32, 64
    frames, pos = _acquisition(7, radius, s, n, k)
    dev = device(frames)
    with wdd.Server(hbm_budget_bytes=1 << 30, batch_frames=128, launch_mode="graph") as srv:
        keep = srv.open(radius, s, s, n, n, k, order=wdd.WDD_ORDER_OBJECT)
        srv.wait_open(keep)
        for cycle in range(12):
            extra = [srv.open(radius, s, s, n, n, k, order=wdd.WDD_ORDER_OBJECT) for _ in range(3)]
            for e in extra:
                srv.wait_open(e)
            b0 = (cycle * 64) % len(pos)
            for e in extra:
                srv.submit(e, dev[b0:b0 + 64], pos[b0:b0 + 64])
            srv.submit(keep, dev[b0:b0 + 64], pos[b0:b0 + 64])
            srv.step()
            for e in extra:   # closed while the next steps capture their rounds
                srv.close(e)
            srv.step()
        got = srv.snapshot(keep)
        st = srv.stats()
    with wdd.Plan(radius, s, s, n, n, k, order=wdd.WDD_ORDER_OBJECT, max_batch=128) as plan:
        for cycle in range(12):
            b0 = (cycle * 64) % len(pos)
            plan.push(dev[b0:b0 + 64], pos[b0:b0 + 64])
        ref = plan.snapshot()
    say(f"[serving] graph rounds with closes: {st['group_rounds']} rounds, {st['graph_replays']} replays, "
        f"error vs alone {rel_img(got, ref):.2e}")
    assert rel_img(got, ref) <= 1e-5
