"""wdd_display_noalloc (scratch in a fixed device array, no allocation) against wdd_display
(scratch from hipMallocAsync) through the C ABI: two calls in a row, the second on a smaller
grid, each compared with the allocating entry point's output and with the oracle's display
(eq. extract) at the FP32 bar."""
import ctypes

import numpy as np
import pytest

import oracle.wdd as O
import paper_2212_01309_amd as wdd
from gpu_util import rel_img, say

pytestmark = pytest.mark.gpu


def _grid(rng, sy, sx):
    d = (rng.normal(size=(sy, sx)) + 1j * rng.normal(size=(sy, sx))) * 0.01
    d[0, 0] = 2.0 - 0.25j
    return d.astype(np.complex64)


def test_display_without_allocation_matches_the_allocating_call():
    import torch
    lib = wdd.load_library()
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(123)
    for sy, sx in [(512, 512), (96, 200)]:                     # the second call is smaller
        say(f"[noalloc] display {sy}x{sx}")
        d = _grid(rng, sy, sx)
        dev = torch.from_numpy(d).to("cuda")
        a = torch.full((sy, sx), float("nan"), dtype=torch.complex64, device="cuda")
        b = torch.full((sy, sx), float("nan"), dtype=torch.complex64, device="cuda")
        assert lib.wdd_display(dev.data_ptr(), sy, sx, a.data_ptr(), ctypes.c_void_p(stream)) == wdd.WDD_OK
        assert lib.wdd_display_noalloc(dev.data_ptr(), sy, sx, b.data_ptr(), ctypes.c_void_p(stream)) == wdd.WDD_OK
        torch.cuda.synchronize()
        got_a, got_b = a.cpu().numpy(), b.cpu().numpy()
        assert np.all(np.isfinite(got_b))
        ref = O.display(d.astype(np.complex128))
        errs = (rel_img(got_b, got_a), rel_img(got_b, ref))
        say(f"[noalloc] {sy}x{sx}: vs wdd_display {errs[0]:.2e}, vs oracle {errs[1]:.2e}")
        assert np.array_equal(got_b, got_a)
        assert errs[1] <= 1e-5


def test_display_without_allocation_rejects_grids_beyond_its_scratch():
    import torch
    lib = wdd.load_library()
    dev = torch.zeros((4, 4), dtype=torch.complex64, device="cuda")
    # 2048 x 1024 cells exceed the fixed scratch; the pointers are never dereferenced
    assert lib.wdd_display_noalloc(dev.data_ptr(), 2048, 1024, dev.data_ptr(), None) == wdd.WDD_EINVAL
    assert lib.wdd_display_noalloc(dev.data_ptr(), 0, 8, dev.data_ptr(), None) == wdd.WDD_EINVAL
