"""Reduced-precision projection (BF16 / FP16 MFMA, FP32 accumulation) against the FP64
oracle: the error of every result is stated per mode, and the FP32 path is run on
the same frames beside it."""
import numpy as np
import pytest

import oracle.wdd as O
import paper_2212_01309_amd as wdd
import synth
from gpu_util import device, golden_workload, rel, rel_a, rel_d, rel_img, say

pytestmark = pytest.mark.gpu

# bound on the relative L2 error of h, A and D for each projection arithmetic:
# basis rounding 2^-9 (bf16), 2^-12 (fp16), ~2^-17 (bf16 hi+lo), ~2^-22 (fp16 hi+lo)
BOUNDS = {"fp32": 1e-5, "bf16_hilo": 3e-5, "fp16_hilo": 2e-6, "bf16": 6e-3, "fp16": 8e-4}
# bound on the displayed image, whole and minus its mean (the signal beside the zero
# frequency): the FP32 accumulation and display set a floor of the FP32 bar under every mode
IMAGE_BOUNDS = {m: max(1e-5, b) for m, b in BOUNDS.items()}


@pytest.fixture(scope="module")
def defocus_case():
    wl = synth.WORKLOADS["defocus"]
    g = golden_workload("defocus")
    rng = np.random.default_rng(77)
    lin = np.concatenate([np.arange(256) + 256 * 100, rng.choice(wl.sy * wl.sx, size=512, replace=False)])
    pos = np.stack([lin // wl.sx, lin % wl.sx], axis=1).astype(np.int32)
    frames = wl.frames(pos)
    all_f = O.nonzero_frequencies(wl.sy, wl.sx, wl.n, wl.n, wl.radius, wl.step)
    pick = np.concatenate([[0], np.sort(rng.choice(np.arange(1, len(all_f)), size=200, replace=False))])
    oplan = O.make_plan(wl.sy, wl.sx, wl.n, wl.n, wl.radius, wl.k, amplitude=wl.aperture_amplitude(),
                        defocus_edge=wl.defocus_edge, step=wl.step, freqs=all_f[pick], eps_abs=g["eps_abs"])
    h = O.project(frames, oplan.phi)
    a = O.scan_phase(oplan.freqs, pos, wl.sy, wl.sx) @ h
    d = O.extract(oplan, a)
    return wl, pos, frames, pick, h, a, d


@pytest.mark.parametrize("mode", list(BOUNDS))
def test_projection_precision_against_oracle(defocus_case, mode):
    wl, pos, frames, pick, h, a, d = defocus_case
    dev = device(frames)
    with wdd.Plan(wl.radius, wl.sy, wl.sx, wl.n, wl.n, wl.k, dtype=wdd.WDD_U16, defocus=wl.defocus_edge,
                  amplitude=wl.aperture_amplitude(), max_batch=wl.batch, precision=mode) as plan:
        hs = []
        for b in range(0, len(pos), wl.batch):
            plan.push(dev[b:b + wl.batch], pos[b:b + wl.batch])
            hs.append(plan.projection())
        plan.snapshot()
        got_a, got_d = plan.accumulator()[pick], plan.spectrum()[pick]
    errs = dict(h=rel(np.concatenate(hs), h), A=rel_a(got_a, a), D=rel_d(got_d, d))
    say(f"[precision] {mode}: {errs}")
    assert max(errs.values()) <= BOUNDS[mode]


@pytest.mark.parametrize("mode", ["fp32", "bf16_hilo", "fp16_hilo"])
def test_two_stage_precision_against_oracle(defocus_case, mode):
    """The bench's precision lines run object order with two pipeline stages: D against the
    FP64 oracle within the mode's bound (the first, raster batch held and pipelined, the
    scattered ones, on more than 16 scan rows, unpipelined after it)."""
    wl, pos, frames, pick, h, a, d = defocus_case
    dev = device(frames)
    with wdd.Plan(wl.radius, wl.sy, wl.sx, wl.n, wl.n, wl.k, dtype=wdd.WDD_U16, defocus=wl.defocus_edge,
                  amplitude=wl.aperture_amplitude(), max_batch=wl.batch, precision=mode,
                  order=wdd.WDD_ORDER_OBJECT, pipeline=2) as plan:
        assert plan.info().pipelined == 2
        for b in range(0, len(pos), wl.batch):
            plan.push(dev[b:b + wl.batch], pos[b:b + wl.batch])
        got_d = plan.spectrum()[pick]
    err = rel_d(got_d, d)
    say(f"[precision] {mode}, two pipeline stages: D {err:.2e}")
    assert err <= BOUNDS[mode]


# Full-range counts (up to 65535) through one-hot frames: every coefficient is
# count * psi_y * psi_x at one pixel, including pixels in the basis tails where the
# 16-bit parts of psi_x lose precision (FP16 flushes values below 6e-8).  The error of a
# frame is measured relative to max(||h_ref||, 1e-3 * count).
FULL_RANGE_BOUNDS = {"bf16_hilo": 2e-5, "fp16_hilo": 1e-4, "bf16": 6e-3, "fp16": 2e-3}


@pytest.mark.parametrize("mode", list(FULL_RANGE_BOUNDS))
def test_full_range_counts_split_exactly(mode):
    """Counts above 2^8 / 2^11 take the two-digit split; one-hot frames isolate it."""
    ny = nx = 64
    frames = np.zeros((48, ny, nx), np.uint16)
    rng = np.random.default_rng(5)
    for i in range(32):
        frames[i, rng.integers(0, ny), rng.integers(0, nx)] = 65535 - 997 * i
    frames[32:] = rng.integers(0, 65536, size=(16, ny, nx), dtype=np.uint16)
    with wdd.Plan(16.0, 8, 8, ny, nx, 256, dtype=wdd.WDD_U16, max_batch=64, precision=mode) as plan:
        plan.push(device(frames), np.zeros((48, 2), np.int32))
        got = plan.projection()
        sig = plan.info().sigma_px
    ref = O.project(frames, O.hg_basis(ny, nx, 256, sig))
    errs = [float(np.linalg.norm(got[i] - ref[i]) /
                  max(np.linalg.norm(ref[i]), 1e-3 * float(frames[i].max()))) for i in range(48)]
    bad = [i for i, e in enumerate(errs) if not e <= FULL_RANGE_BOUNDS[mode]]
    if bad:
        i = bad[0]
        say(f"[precision] {mode}: frame {i} max|got| {np.max(np.abs(got[i])):.3e} max|ref| {np.max(np.abs(ref[i])):.3e} "
            f"finite {np.all(np.isfinite(got[i]))}")
    err = float(np.max(errs))
    say(f"[precision] {mode} full-range counts: worst frame {err:.2e}")
    assert err <= FULL_RANGE_BOUNDS[mode]


def test_reduced_precision_needs_uint16_frames():
    with pytest.raises(wdd.WddError) as ei:
        wdd.Plan(8.0, 16, 16, 32, 32, 64, dtype=wdd.WDD_F32, precision="bf16")
    assert ei.value.code == wdd.WDD_EINVAL


@pytest.mark.parametrize("ny,nx,dtype,mode", [(1024, 1024, wdd.WDD_U16, "fp32"), (1000, 1024, wdd.WDD_F32, "fp32"),
                                              (520, 1024, wdd.WDD_U16, "fp16_hilo"), (256, 256, wdd.WDD_U16, "fp32")])
def test_projection_of_large_detectors(ny, nx, dtype, mode):
    """The projection's basis tables at the largest detectors: 1024 x 1024 (the tables take
    most of the LDS), 1000 rows loop the waves over 63 tiles with a partial last one, 520 rows
    with the 16-bit tables, and 256 x 256 (the large workload's detector)."""
    rng = np.random.default_rng(ny + nx)
    n, k, radius = 3, 10, ny / 8.0
    frames = (rng.poisson(30.0, size=(n, ny, nx)).astype(np.uint16) if dtype == wdd.WDD_U16
              else rng.uniform(0.0, 4.0, size=(n, ny, nx)).astype(np.float32))
    pos = np.array([[0, 1], [3, 2], [1, 3]], np.int32)
    with wdd.Plan(radius, 4, 4, ny, nx, k, dtype=dtype, max_batch=n, precision=mode) as plan:
        plan.push(device(frames), pos)
        got = plan.projection()
    oplan = O.make_plan(4, 4, ny, nx, radius, k)
    err = rel(got, O.project(frames, oplan.phi))
    say(f"[precision] projection {ny}x{nx} {mode}: {err:.2e}")
    assert err <= (1e-6 if mode == "fp32" else BOUNDS[mode])


@pytest.mark.parametrize("mode", ["bf16_hilo", "fp16_hilo"])
def test_reduced_precision_with_the_deferred_display(mode):
    """Object order with a reduced-precision projection, each image's column pass left to the
    next push's projection launch (the merged launch) as the bench drives it: every image
    equals the blocking push + snapshot image bit for bit, and the last one is within the
    mode's bound of the FP64 oracle."""
    import torch
    s, n, k, b = 64, 64, 64, 256
    rng = np.random.default_rng(88)
    pos = np.stack([np.repeat(np.arange(s), s), np.tile(np.arange(s), s)], axis=1).astype(np.int32)
    frames = rng.poisson(40.0, size=(s * s, n, n)).astype(np.uint16)
    dev = device(frames)
    shown = [torch.empty((s, s), dtype=torch.complex64, device="cuda") for _ in range(s * s // b)]
    blocking = []
    with wdd.Plan(16.0, s, s, n, n, k, max_batch=b, precision=mode, order=wdd.WDD_ORDER_OBJECT) as pa, \
            wdd.Plan(16.0, s, s, n, n, k, max_batch=b, precision=mode, order=wdd.WDD_ORDER_OBJECT) as pb:
        for i, b0 in enumerate(range(0, s * s, b)):
            pa.push_snapshot(dev[b0:b0 + b], pos[b0:b0 + b], out=shown[i], wait=False, defer=True)
            blocking.append(pb.push_snapshot(dev[b0:b0 + b], pos[b0:b0 + b]))
        pa.sync()
    for i in range(len(blocking)):
        assert np.array_equal(shown[i].cpu().numpy(), blocking[i]), i
    live = O.Live(O.make_plan(s, s, n, n, 16.0, k), "P")
    live.push(frames, pos)
    err = rel_img(blocking[-1], live.snapshot())
    say(f"[precision] {mode} deferred display: vs oracle {err:.2e}")
    assert err <= IMAGE_BOUNDS[mode]
