"""Full Fourier basis on the GPU (K = ny nx, complex projections): the live path then computes
conventional WDD.  Compared with the oracle's live path on the same basis and with its
conventional WDD (equations deconv_mat and extract)."""
import numpy as np
import pytest

import oracle.wdd as O
import paper_2212_01309_amd as wdd
import synth
from gpu_util import device, rel, rel_d, rel_img, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("order", [wdd.WDD_ORDER_SPECTRUM, wdd.WDD_ORDER_OBJECT])
def test_small_workload_is_conventional_wdd(order):
    wl = synth.WORKLOADS["small"]
    pos = synth.raster_positions(wl.sy, wl.sx)
    frames = wl.frames(pos)
    n, k = wl.n, wl.n * wl.n
    amp = wl.aperture_amplitude()
    dev = device(frames)
    with wdd.Plan(wl.radius, wl.sy, wl.sx, n, n, k, dtype=wdd.WDD_F32, amplitude=amp, max_batch=wl.batch,
                  order=order, basis=wdd.WDD_BASIS_FOURIER) as plan:
        for b in range(0, len(pos), wl.batch):
            plan.push(dev[b:b + wl.batch], pos[b:b + wl.batch])
        h_last = plan.projection()
        o = plan.snapshot()
        d = plan.spectrum()
    op = O.make_plan(wl.sy, wl.sx, n, n, wl.radius, amplitude=amp, phi=O.fourier_basis(n, n))
    h_ref = O.project(frames[-wl.batch:], op.phi)
    live = O.Live(op, "N")
    live.push(frames, pos)
    frames4d = np.zeros((wl.sy, wl.sx, n, n))
    frames4d[pos[:, 0], pos[:, 1]] = frames
    d_conv, o_conv = O.offline_conventional(frames4d, wl.radius, amplitude=amp)
    errs = dict(h=rel(h_last, h_ref), D=rel_d(d, live.spectrum()), O=rel_img(o, live.snapshot()),
                O_conventional=rel_img(o, o_conv), D_conventional=rel_d(d, d_conv[op.freqs[:, 0], op.freqs[:, 1]]))
    say(f"[fourier] small workload, order {order}: {errs}")
    assert errs["h"] <= 1e-6
    assert max(errs["D"], errs["O"], errs["O_conventional"], errs["D_conventional"]) <= 1e-5


@pytest.mark.parametrize("order", [wdd.WDD_ORDER_SPECTRUM, wdd.WDD_ORDER_OBJECT])
def test_rectangular_detector_scattered_batches(order):
    """16 x 8 detector, scattered uint16 frames on more than 16 rows (several passes),
    push_snapshot equal to push + snapshot."""
    sy, sx, ny, nx, r = 24, 20, 16, 8, 3.5
    rng = np.random.default_rng(21 + order)
    lin = rng.permutation(sy * sx)[:300]
    pos = np.stack([lin // sx, lin % sx], axis=1).astype(np.int32)
    frames = rng.poisson(40.0, size=(300, ny, nx)).astype(np.uint16)
    dev = device(frames)
    kw = dict(max_batch=100, order=order, basis=wdd.WDD_BASIS_FOURIER, defocus=0.8)
    with wdd.Plan(r, sy, sx, ny, nx, ny * nx, **kw) as a, wdd.Plan(r, sy, sx, ny, nx, ny * nx, **kw) as b:
        for i in range(0, 300, 100):
            a.push(dev[i:i + 100], pos[i:i + 100])
            oa = a.snapshot()
            ob = b.push_snapshot(dev[i:i + 100], pos[i:i + 100])
            assert rel_img(ob, oa) <= 1e-6
    op = O.make_plan(sy, sx, ny, nx, r, defocus_edge=0.8, phi=O.fourier_basis(ny, nx))
    live = O.Live(op, "P")
    live.push(frames, pos)
    err = rel_img(oa, live.snapshot())
    say(f"[fourier] 16x8 detector, 300 scattered frames, order {order}: {err:.2e}")
    assert err <= 1e-5
