"""The large workload's whole acquisition on the GPU: 512 x 512 raster positions (262 144
frames of 256 x 256 uint16 counts, K = 128, 115 169 kept frequencies), pushed in raster
batches of 256 as the benchmark drives it, with FP32 accumulation over every frame.

Frame values are cycled from a pool of the workload's first 1024 frames (the work per
frame does not depend on the values; position s carries pool frame s mod 1024).  The
oracle then needs the projections of the pool only; D (and A in the spectrum order) is
compared on a sample of kept frequencies, without the zero frequency as well as with it,
and the 512 x 512 image against the oracle's display of the plan's own D (eq. extract)."""
import numpy as np
import pytest

import oracle.wdd as O
import paper_2212_01309_amd as wdd
import synth
from gpu_util import device, golden_workload, rel_a, rel_d, rel_img, say

pytestmark = pytest.mark.gpu

POOL = 1024
N_SAMPLE = 511


@pytest.fixture(scope="module")
def large_whole_acquisition():
    wl = synth.WORKLOADS["large"]
    g = golden_workload("large")
    pos = synth.raster_positions(wl.sy, wl.sx)
    pool = wl.frames(pos[:POOL])
    rng = np.random.default_rng(2024)
    all_f = O.nonzero_frequencies(wl.sy, wl.sx, wl.n, wl.n, wl.radius, wl.step)
    assert len(all_f) == g["n_freq"]
    pick = np.concatenate([[0], np.sort(rng.choice(np.arange(1, len(all_f)), size=N_SAMPLE, replace=False))])
    oplan = O.make_plan(wl.sy, wl.sx, wl.n, wl.n, wl.radius, wl.k, amplitude=wl.aperture_amplitude(),
                        defocus_edge=wl.defocus_edge, step=wl.step, freqs=all_f[pick], eps_abs=g["eps_abs"])
    h_pool = O.project(pool, oplan.phi)                                    # [POOL, K]
    a = np.zeros((len(pick), wl.k), np.complex128)
    lin = np.arange(wl.sy * wl.sx)
    for c0 in range(0, len(lin), 16384):                                   # A = sum_s F[v, s] h_s
        part = lin[c0:c0 + 16384]
        a += O.scan_phase(oplan.freqs, pos[part], wl.sy, wl.sx) @ h_pool[part % POOL]
    d = O.extract(oplan, a)
    return wl, pos, pool, all_f, pick, a, d


@pytest.mark.parametrize("order,pipeline", [(wdd.WDD_ORDER_OBJECT, 0), (wdd.WDD_ORDER_OBJECT, 1),
                                            (wdd.WDD_ORDER_OBJECT, 2), (wdd.WDD_ORDER_SPECTRUM, 0)])
def test_whole_large_acquisition(large_whole_acquisition, order, pipeline):
    import torch
    wl, pos, pool, all_f, pick, a_ref, d_ref = large_whole_acquisition
    obj = order == wdd.WDD_ORDER_OBJECT
    say(f"[fullsize] large, {'object' if obj else 'spectrum'} order, pipeline {pipeline}: "
        f"{len(pos)} frames in batches of {wl.batch}")
    dev = device(pool)
    shown = torch.empty((wl.sy, wl.sx), dtype=torch.complex64, device="cuda")
    with wdd.Plan(wl.radius, wl.sy, wl.sx, wl.n, wl.n, wl.k, amplitude=wl.aperture_amplitude(), max_batch=wl.batch,
                  order=order, pipeline=pipeline) as plan:
        for i, b in enumerate(range(0, len(pos), wl.batch)):
            fr = dev[b % POOL:b % POOL + wl.batch]
            if obj:   # the bench's step: push, snapshot into HBM, image finished by the next push
                plan.push_snapshot(fr, pos[b:b + wl.batch], out=shown, wait=False, defer=True)
            else:     # the configuration's cadence: a snapshot every 16 384 frames
                plan.push(fr, pos[b:b + wl.batch])
                if (b + wl.batch) % wl.snapshot_every == 0:
                    plan.snapshot(out=shown, wait=False)
        plan.sync()
        assert plan.info().frames_seen == len(pos)
        got_o = shown.cpu().numpy()
        got_d = plan.spectrum()
        got_a = None if obj else plan.accumulator()[pick]
    errs = dict(D=rel_d(got_d[pick], d_ref))
    if got_a is not None:
        errs["A"] = rel_a(got_a, a_ref)
    grid = np.zeros((wl.sy, wl.sx), np.complex128)
    grid[all_f[:, 0], all_f[:, 1]] = got_d
    errs["O vs display of D"] = rel_img(got_o, O.display(grid))
    say(f"[fullsize] errors {errs}")
    assert max(errs.values()) <= 1e-5
