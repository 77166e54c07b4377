"""Field-of-view patches on the GPU (wdd_patches_*) against the oracle's patched
reconstruction (the reading of Section 10's subdivision into independently reconstructed,
merged patches): merged images within the FP32 bar, on raster and scattered pushes, several
patch grids, and a single patch equal to the plain plan."""
import numpy as np
import pytest

import oracle.wdd as O
import paper_2212_01309_amd as wdd
import synth
from gpu_util import device, rel_img, say

pytestmark = pytest.mark.gpu


def _case(s_y, s_x, n, radius, k, seed):
    wl = synth.Workload("fov", s_y, s_x, n, radius, k, 64, 2 * max(s_y, s_x), 40, 1.5, 0.3, 4e4, seed=seed)
    pos = synth.raster_positions(s_y, s_x)
    return wl, pos, wl.frames(pos)


@pytest.mark.parametrize("sy,sx,py,px,oy,ox,batch,scatter", [
    (64, 64, 32, 32, 8, 8, 128, False),     # 3 x 3 patches, raster batches of two scan rows
    (48, 40, 16, 20, 4, 0, 100, True),      # scattered positions, no overlap in x
    (40, 40, 24, 17, 6, 5, 64, False),      # non-power-of-two patch sides (direct DFT display)
    (32, 32, 32, 32, 0, 0, 96, False),      # one patch: the plain plan
    (64, 64, 48, 40, 32, 16, 256, True),    # scattered: up to 48 scan rows of a patch in one push (3 passes)
])
def test_patches_against_the_oracle(sy, sx, py, px, oy, ox, batch, scatter):
    n, radius, k = 32, 8.0, 36
    wl, pos, frames = _case(sy, sx, n, radius, k, seed=sy + sx + py)
    order = np.random.default_rng(5).permutation(len(pos)) if scatter else np.arange(len(pos))
    say(f"[patches] {sy}x{sx} raster, patches {py}x{px} overlap {oy},{ox}, batch {batch}, scatter {scatter}")
    dev = device(frames[order])
    amp = wl.aperture_amplitude()
    with wdd.Patches(radius, sy, sx, n, n, k, py, px, oy, ox, amplitude=amp, max_batch=batch) as ps:
        info = ps.info()
        for b in range(0, len(pos), batch):
            ps.push(dev[b:b + batch], pos[order[b:b + batch]])
        got = ps.snapshot()
    plan = O.make_plan(py, px, n, n, radius, k, amplitude=amp)
    ref, _ = O.patched_reconstruction(frames, pos, sy, sx, py, px, oy, ox, plan)
    assert info["npatch_y"] == len(O.patch_origins(sy, py, oy)) and info["npatch_x"] == len(O.patch_origins(sx, px, ox))
    err = rel_img(got, ref)
    say(f"[patches] {info}: merged vs oracle {err:.2e}")
    assert err <= 1e-5
    if (py, px) == (sy, sx):
        with wdd.Plan(radius, sy, sx, n, n, k, amplitude=amp, max_batch=batch, order=wdd.WDD_ORDER_OBJECT) as plan_:
            for b in range(0, len(pos), batch):
                plan_.push(dev[b:b + batch], pos[order[b:b + batch]])
            single = plan_.snapshot()
        assert rel_img(got, single) <= 1e-6


def test_patches_partial_acquisition_and_errors():
    """Snapshots part way (patches without frames contribute zero images), a position off
    the raster rejects the whole push, and geometries that do not fit are refused."""
    sy = sx = 48
    n, radius, k = 32, 8.0, 25
    wl, pos, frames = _case(sy, sx, n, radius, k, seed=9)
    amp = wl.aperture_amplitude()
    dev = device(frames)
    with wdd.Patches(radius, sy, sx, n, n, k, 24, 24, 6, 6, amplitude=amp, max_batch=96) as ps:
        for b in range(0, 96 * 10, 96):
            ps.push(dev[b:b + 96], pos[b:b + 96])
        got = ps.snapshot()
        bad = pos[:4].copy()
        bad[2] = (48, 0)
        with pytest.raises(wdd.WddError) as ei:
            ps.push(dev[:4], bad)
        assert ei.value.code == wdd.WDD_ERANGE
        again = ps.snapshot()
    assert np.array_equal(got, again)
    plan = O.make_plan(24, 24, n, n, radius, k, amplitude=amp)
    ref, _ = O.patched_reconstruction(frames[:960], pos[:960], sy, sx, 24, 24, 6, 6, plan)
    assert rel_img(got, ref) <= 1e-5
    for geo in [(49, 24, 0, 0), (24, 24, 24, 0), (0, 24, 0, 0)]:
        with pytest.raises(wdd.WddError) as ei:
            wdd.Patches(radius, sy, sx, n, n, k, *geo, amplitude=amp)
        assert ei.value.code == wdd.WDD_EINVAL
