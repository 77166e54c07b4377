"""Host-side checks of libwdd that need no GPU: the C ABI loads and exports every
declared symbol, the FP64 host tables agree with the oracle, and bad arguments
are rejected."""
import ctypes
import os

import numpy as np
import pytest

import oracle.wdd as O
import paper_2212_01309_amd as wdd
import synth


def test_library_exports_every_declared_symbol():
    lib = wdd.load_library()
    names = wdd.header_symbols()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    # and the binding describes each one
    assert set(names) == set(wdd._SIGNATURES)


def _compare(radius, sy, sx, ny, nx, k, defocus=0.0, amplitude=1.0, step=1.0, sigma=None, eps_rel=0.01,
             center=None):
    t = wdd.Tables(radius, sy, sx, ny, nx, k, defocus=defocus, amplitude=amplitude, step=step,
                   sigma=sigma or 0.0, eps_rel=eps_rel, center=center)
    freqs, psy, psx, pairs, w = t.export()
    p = O.make_plan(sy, sx, ny, nx, radius, k, amplitude=amplitude, defocus_edge=defocus, step=step,
                    sigma=sigma, eps_rel=eps_rel, center=center)
    assert np.array_equal(freqs, p.freqs)
    assert np.array_equal(pairs, O.basis_order(k))
    sig = sigma or O.default_sigma(radius, k)
    assert t.sigma == pytest.approx(sig, rel=1e-15)
    cy, cx = O.default_center(ny, nx) if center is None else center
    assert np.max(np.abs(psy - O.sampled_hermite(ny, t.l, sig, cy))) < 1e-13
    assert np.max(np.abs(psx - O.sampled_hermite(nx, t.l, sig, cx))) < 1e-13
    assert t.eps_abs == pytest.approx(p.eps_abs, rel=1e-12)
    assert np.linalg.norm(w - p.w) <= 1e-12 * np.linalg.norm(p.w)


@pytest.mark.parametrize("args", [
    dict(radius=8.0, sy=32, sx=32, ny=32, nx=32, k=64),
    dict(radius=8.0, sy=32, sx=32, ny=32, nx=32, k=64, defocus=np.pi, amplitude=17.0),
    dict(radius=16.0, sy=64, sx=64, ny=64, nx=64, k=256),
    dict(radius=5.5, sy=24, sx=40, ny=40, nx=48, k=50, defocus=1.1),     # non-square, ragged K
    dict(radius=3.0, sy=30, sx=18, ny=12, nx=16, k=10, step=0.75),        # non-power-of-two shifts
    dict(radius=20.0, sy=16, sx=16, ny=32, nx=32, k=9),                   # aperture clipped by the detector
    dict(radius=8.0, sy=32, sx=32, ny=32, nx=32, k=128, sigma=3.0, eps_rel=0.1),
    dict(radius=8.0, sy=32, sx=32, ny=32, nx=32, k=64, center=(14.5, 17.0), defocus=0.6),   # off-centre probe
    dict(radius=6.0, sy=16, sx=24, ny=24, nx=32, k=30, center=(10.0, 20.5), step=0.75),
    dict(radius=9.0, sy=16, sx=16, ny=32, nx=32, k=16, center=(3.5, 29.0)),                # partly off the detector
])
def test_host_tables_match_oracle(args):
    _compare(**args)


def test_host_tables_medium_workload():
    wl = synth.WORKLOADS["medium"]
    t = wdd.Tables(wl.radius, wl.sy, wl.sx, wl.n, wl.n, wl.k, amplitude=wl.aperture_amplitude())
    freqs, *_ = t.export()
    assert np.array_equal(freqs, O.nonzero_frequencies(wl.sy, wl.sx, wl.n, wl.n, wl.radius))


@pytest.mark.parametrize("bad", [
    dict(k=0), dict(k=257), dict(radius=0.0), dict(radius=-1.0), dict(sy=0), dict(sx=5000),
    dict(nx=12), dict(ny=0), dict(step=0.0), dict(eps_rel=0.0), dict(amplitude=0.0),
])
def test_tables_reject_bad_arguments(bad):
    args = dict(radius=8.0, sy=32, sx=32, ny=32, nx=32, k=64)
    extra = {}
    for key in ("step", "eps_rel", "amplitude"):
        if key in bad:
            extra[key] = bad.pop(key)
    args.update(bad)
    with pytest.raises(wdd.WddError) as ei:
        wdd.Tables(args["radius"], args["sy"], args["sx"], args["ny"], args["nx"], args["k"], **extra)
    assert ei.value.code == wdd.WDD_EINVAL
    assert wdd.load_library().wdd_last_error()


@pytest.mark.parametrize("center", [(-40.0, 16.0), (16.0, 100.0), (float("nan"), 16.0), (16.0, float("inf"))])
def test_tables_reject_an_aperture_off_the_detector(center):
    with pytest.raises(wdd.WddError) as ei:
        wdd.Tables(8.0, 32, 32, 32, 32, 64, center=center)
    assert ei.value.code == wdd.WDD_EINVAL


def test_default_options():
    o = wdd.Options()
    assert wdd.load_library().wdd_default_options(ctypes.byref(o)) == 0
    assert o.eps_rel == 0.01 and o.sigma_px == 0.0 and o.max_batch == 256 and o.precision == wdd.WDD_FP32
    assert o.order == wdd.WDD_ORDER_SPECTRUM and o.basis == wdd.WDD_BASIS_HERMITE_GAUSS
    assert o.pipeline == 0


@pytest.mark.parametrize("radius,s,ny,nx,defocus", [
    (8.0, 32, 32, 32, 0.0), (4.0, 24, 16, 8, 0.7), (2.5, 16, 8, 16, 0.0), (12.0, 20, 32, 64, np.pi),
])
def test_fourier_tables_match_oracle(radius, s, ny, nx, defocus):
    """Full Fourier basis: Y^B = the oracle's reduction with fourier_basis (numpy ifft2)."""
    t = wdd.Tables(radius, s, s, ny, nx, ny * nx, defocus=defocus, basis=wdd.WDD_BASIS_FOURIER)
    freqs, psy, psx, pairs, w = t.export()
    p = O.make_plan(s, s, ny, nx, radius, defocus_edge=defocus, phi=O.fourier_basis(ny, nx))
    assert t.l == 0 and t.k == ny * nx and psy.size == 0
    assert np.array_equal(freqs, p.freqs)
    assert t.eps_abs == pytest.approx(p.eps_abs, rel=1e-12)
    assert np.linalg.norm(w - p.w) <= 1e-12 * np.linalg.norm(p.w)


@pytest.mark.parametrize("ny,nx,k", [(32, 32, 1000), (48, 32, 48 * 32), (128, 128, 128 * 128), (4, 8, 32)])
def test_fourier_tables_reject_bad_shapes(ny, nx, k):
    with pytest.raises(wdd.WddError) as ei:
        wdd.Tables(4.0, 16, 16, ny, nx, k, basis=wdd.WDD_BASIS_FOURIER)
    assert ei.value.code == wdd.WDD_EINVAL


def test_fourier_plan_rejects_reduced_precision_before_touching_a_device():
    with pytest.raises(wdd.WddError) as ei:
        wdd.Plan(8.0, 16, 16, 32, 32, 1024, basis=wdd.WDD_BASIS_FOURIER, precision=wdd.WDD_BF16_HILO)
    assert ei.value.code == wdd.WDD_EINVAL


@pytest.mark.parametrize("kw", [
    dict(order=wdd.WDD_ORDER_SPECTRUM),                       # the update holds A, not D
    dict(dtype=wdd.WDD_F32),                                  # uint16 frames only
    dict(precision=wdd.WDD_BF16_HILO, ny=160),                # reduced precision: at most 128 rows
    dict(nx=48),                                              # columns in multiples of 32
    dict(nx=288),                                             # at most 256 columns
    dict(ny=288),                                             # at most 256 rows
])
def test_pipelined_plan_rejects_unsupported_settings_before_touching_a_device(kw):
    """wdd_options.pipeline: the merged update + projection launch exists for object order and
    uint16 frames of 32..256 columns in multiples of 32 and <= 256 rows (128 with a reduced
    precision)."""
    args = dict(ny=64, nx=64, order=wdd.WDD_ORDER_OBJECT, dtype=wdd.WDD_U16)
    args.update(kw)
    ny, nx = args.pop("ny"), args.pop("nx")
    for stages in (1, 2):
        with pytest.raises(wdd.WddError) as ei:
            wdd.Plan(8.0, 16, 16, ny, nx, 64, pipeline=stages, **args)
        assert ei.value.code == wdd.WDD_EINVAL
        assert "pipelined" in str(ei.value)


@pytest.mark.parametrize("bad", [-1, 3])
def test_pipeline_option_takes_zero_one_or_two(bad):
    o = wdd._options(0.01, 0.0, 256, order=wdd.WDD_ORDER_OBJECT)
    o.pipeline = bad
    h = wdd._P()
    st = wdd.load_library().wdd_plan(ctypes.byref(wdd._probe(8.0, 64, 64, None, 0.0, 1.0)),
                                     ctypes.byref(wdd.Scan(16, 16, 1.0)), ctypes.byref(wdd.Detector(64, 64, 0)),
                                     64, ctypes.byref(o), None, ctypes.byref(h))
    assert st == wdd.WDD_EINVAL and not h.value


def test_binding_constants_match_the_header():
    """The binding's copy of the in-flight bound (it holds that many device tensors) and of
    the enumerations must be the header's."""
    import re
    text = open(os.path.join(os.path.dirname(__file__), "..", "include", "wdd.h")).read()
    assert int(re.search(r"#define WDD_MAX_PUSHES_IN_FLIGHT (\d+)", text).group(1)) == wdd.WDD_MAX_PUSHES_IN_FLIGHT
    for name in ("WDD_OUT_HOST", "WDD_OUT_DEVICE", "WDD_OUT_DEVICE_ASYNC", "WDD_OUT_DEVICE_DEFERRED", "WDD_ORDER_SPECTRUM",
                 "WDD_ORDER_OBJECT",
                 "WDD_BASIS_HERMITE_GAUSS", "WDD_BASIS_FOURIER", "WDD_SERVE_STREAMS", "WDD_SERVE_GROUPED",
                 "WDD_SERVE_GRAPH"):
        assert int(re.search(name + r" = (\d+)", text).group(1)) == getattr(wdd, name), name


def test_allocator_hook_arguments():
    """wdd_set_allocator: an allocator without its release function is refused; setting and
    clearing one needs no device."""
    lib = wdd.load_library()
    alloc = wdd._ALLOC_FN(lambda n, ctx: None)
    assert lib.wdd_set_allocator(alloc, wdd._RELEASE_FN(), None) == wdd.WDD_EINVAL
    assert lib.wdd_set_allocator(alloc, wdd._RELEASE_FN(lambda p, ctx: None), None) == wdd.WDD_OK
    assert lib.wdd_set_allocator(wdd._ALLOC_FN(), wdd._RELEASE_FN(), None) == wdd.WDD_OK
