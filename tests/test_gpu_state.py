"""State handling on the GPU: re-deconvolution of the resident spectrum with a new probe
or regularisation, and checkpoint / restore of the live state."""
import numpy as np
import pytest

import oracle.wdd as O
import paper_2212_01309_amd as wdd
from gpu_util import device, rel, rel_d, rel_img, say

pytestmark = pytest.mark.gpu


def _frames(seed, s, n, count):
    rng = np.random.default_rng(seed)
    lin = rng.permutation(s * s)[:count]
    pos = np.stack([lin // s, lin % s], axis=1).astype(np.int32)
    return rng.poisson(25.0, size=(count, n, n)).astype(np.uint16), pos


def test_update_probe_redeconvolves_all_frames_seen():
    s, n, k, radius = 32, 32, 64, 8.0
    frames, pos = _frames(1, s, n, 600)
    with wdd.Plan(radius, s, s, n, n, k, max_batch=128) as plan:
        dev = device(frames)
        for b in range(0, 600, 128):
            plan.push(dev[b:b + 128], pos[b:b + 128])
        first = plan.snapshot()
        plan.update_probe(radius, defocus=1.3, amplitude=2.0, eps_rel=0.05)
        second = plan.snapshot()
        d2 = plan.spectrum()
        plan.update_probe(radius, eps_rel=0.01)
        third = plan.snapshot()
        with pytest.raises(wdd.WddError) as ei:
            plan.update_probe(radius + 1.0)
        assert ei.value.code == wdd.WDD_EINVAL
    op = O.make_plan(s, s, n, n, radius, k, amplitude=2.0, defocus_edge=1.3, eps_rel=0.05)
    live = O.Live(op, "N")
    live.push(frames, pos)
    errs = (rel_d(d2, live.spectrum()), rel_img(second, live.snapshot()))
    say(f"[state] update_probe D/O {errs}")
    assert max(errs) <= 1e-5
    assert rel_img(third, first) <= 1e-6


def test_checkpoint_restore_continues_bitwise():
    s, n, k, radius = 32, 32, 64, 8.0
    frames, pos = _frames(2, s, n, 512)
    dev = device(frames)
    with wdd.Plan(radius, s, s, n, n, k, max_batch=128) as a, wdd.Plan(radius, s, s, n, n, k, max_batch=128) as b:
        for i in range(0, 256, 128):
            a.push(dev[i:i + 128], pos[i:i + 128])
        image = a.checkpoint()
        b.restore(image)
        assert b.info().frames_seen == 256
        assert np.array_equal(b.accumulator(), a.accumulator())
        for i in range(256, 512, 128):
            a.push(dev[i:i + 128], pos[i:i + 128])
            b.push(dev[i:i + 128], pos[i:i + 128])
        assert np.array_equal(b.accumulator(), a.accumulator())
        assert np.array_equal(b.snapshot(), a.snapshot())
        assert b.info().frames_seen == a.info().frames_seen == 512
    with wdd.Plan(radius, s, s, n, n, 100) as other:
        with pytest.raises(wdd.WddError) as ei:
            other.restore(image)
        assert ei.value.code == wdd.WDD_EINVAL
