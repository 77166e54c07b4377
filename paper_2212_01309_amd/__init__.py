"""Python binding of libwdd, the live WDD per-frame update for MI355X.

Argument marshalling only: every step of the reconstruction runs in the HIP
library.  Device buffers are passed as torch tensors on the GPU (their data
pointers), host buffers as numpy arrays.  The library must have been built
(``paper_2212_01309_amd.build.build_library()``); there is no fallback.
"""
from __future__ import annotations

import collections
import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libwdd.so")
_lib: Optional[ctypes.CDLL] = None

WDD_OK, WDD_EINVAL, WDD_ENOMEM, WDD_ERANGE, WDD_EDEVICE, WDD_EBUSY, WDD_ESTATE = 0, -1, -2, -3, -4, -5, -6
WDD_U16, WDD_F32 = 0, 1
WDD_FP32, WDD_BF16_HILO, WDD_FP16_HILO, WDD_BF16, WDD_FP16 = 0, 1, 2, 3, 4
PRECISIONS = {"fp32": WDD_FP32, "bf16_hilo": WDD_BF16_HILO, "fp16_hilo": WDD_FP16_HILO, "bf16": WDD_BF16,
              "fp16": WDD_FP16}
WDD_ORDER_SPECTRUM, WDD_ORDER_OBJECT = 0, 1
WDD_BASIS_HERMITE_GAUSS, WDD_BASIS_FOURIER = 0, 1
WDD_OUT_HOST, WDD_OUT_DEVICE, WDD_OUT_DEVICE_ASYNC, WDD_OUT_DEVICE_DEFERRED = 0, 1, 2, 3
WDD_SERVE_STREAMS, WDD_SERVE_GROUPED, WDD_SERVE_GRAPH = 0, 1, 2
SERVE_MODES = {"streams": WDD_SERVE_STREAMS, "grouped": WDD_SERVE_GROUPED, "graph": WDD_SERVE_GRAPH}
WDD_MAX_PUSHES_IN_FLIGHT = 64
STAGE_PROJECT, STAGE_ACCUMULATE, STAGE_WIENER, STAGE_DISPLAY, STAGE_ROWDFT, STAGE_ALL = 1, 2, 4, 8, 16, 31

_STATUS_NAMES = {0: "WDD_OK", -1: "WDD_EINVAL", -2: "WDD_ENOMEM", -3: "WDD_ERANGE", -4: "WDD_EDEVICE",
                 -5: "WDD_EBUSY", -6: "WDD_ESTATE"}


class WddError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Probe(ctypes.Structure):
    _fields_ = [("radius_px", ctypes.c_double), ("center_y", ctypes.c_double), ("center_x", ctypes.c_double),
                ("defocus_edge_rad", ctypes.c_double), ("amplitude", ctypes.c_double)]


def _probe(radius: float, ny: int, nx: int, center, defocus: float, amplitude: float) -> Probe:
    """The aperture centre defaults to the detector's zero frequency (ny/2, nx/2)."""
    cy, cx = (ny // 2, nx // 2) if center is None else center
    return Probe(radius, float(cy), float(cx), defocus, amplitude)


class Scan(ctypes.Structure):
    _fields_ = [("sy", ctypes.c_int32), ("sx", ctypes.c_int32), ("step_px", ctypes.c_double)]


class Detector(ctypes.Structure):
    _fields_ = [("ny", ctypes.c_int32), ("nx", ctypes.c_int32), ("dtype", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("eps_rel", ctypes.c_double), ("sigma_px", ctypes.c_double), ("precision", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("order", ctypes.c_int32), ("basis", ctypes.c_int32),
                ("pipeline", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_freq", ctypes.c_int64), ("k", ctypes.c_int32), ("l", ctypes.c_int32),
                ("sigma_px", ctypes.c_double), ("eps_abs", ctypes.c_double), ("frames_seen", ctypes.c_uint64),
                ("device_bytes", ctypes.c_int64), ("update_chunks", ctypes.c_int32), ("display_slots", ctypes.c_int32),
                ("pipelined", ctypes.c_int32), ("kept_columns", ctypes.c_int32)]


class Profile(ctypes.Structure):
    _fields_ = [("project_ms", ctypes.c_double), ("accumulate_ms", ctypes.c_double), ("wiener_ms", ctypes.c_double),
                ("display_ms", ctypes.c_double), ("project_launches", ctypes.c_int64),
                ("accumulate_launches", ctypes.c_int64), ("wiener_launches", ctypes.c_int64),
                ("display_launches", ctypes.c_int64), ("factored_launches", ctypes.c_int64),
                ("rowdft_ms", ctypes.c_double), ("rowdft_launches", ctypes.c_int64)]


class PatchGeometry(ctypes.Structure):
    _fields_ = [("py", ctypes.c_int32), ("px", ctypes.c_int32), ("overlap_y", ctypes.c_int32),
                ("overlap_x", ctypes.c_int32)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("snapshot_interval_us", ctypes.c_double),
                ("batch_frames", ctypes.c_int32), ("launch_mode", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("frames", ctypes.c_uint64), ("batches", ctypes.c_uint64), ("snapshots", ctypes.c_uint64),
                ("steps", ctypes.c_uint64), ("open", ctypes.c_int32), ("device_bytes", ctypes.c_int64),
                ("pending_frames", ctypes.c_int64), ("latency_samples", ctypes.c_int64),
                ("latency_p50_us", ctypes.c_double), ("latency_p99_us", ctypes.c_double),
                ("latency_max_us", ctypes.c_double), ("opening", ctypes.c_int32),
                ("group_rounds", ctypes.c_uint64), ("graph_replays", ctypes.c_uint64)]


_P = ctypes.c_void_p
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_SIGNATURES = {
    "wdd_last_error": (ctypes.c_char_p, []),
    "wdd_set_allocator": (ctypes.c_int, [_ALLOC_FN, _RELEASE_FN, ctypes.c_void_p]),
    "wdd_default_options": (ctypes.c_int, [ctypes.POINTER(Options)]),
    "wdd_tables_build": (ctypes.c_int, [ctypes.POINTER(Probe), ctypes.POINTER(Scan), ctypes.POINTER(Detector),
                                        ctypes.c_int32, ctypes.POINTER(Options), ctypes.POINTER(_P)]),
    "wdd_tables_info": (ctypes.c_int, [_P, ctypes.POINTER(PlanInfo)]),
    "wdd_tables_export": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "wdd_tables_free": (ctypes.c_int, [_P]),
    "wdd_plan": (ctypes.c_int, [ctypes.POINTER(Probe), ctypes.POINTER(Scan), ctypes.POINTER(Detector),
                                ctypes.c_int32, ctypes.POINTER(Options), _P, ctypes.POINTER(_P)]),
    "wdd_push": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32]),
    "wdd_snapshot": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]),
    "wdd_push_snapshot": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_uint64)]),
    "wdd_snapshot_buffer": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.POINTER(ctypes.c_float))]),
    "wdd_spectrum": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "wdd_get_wiener": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "wdd_plan_export": (ctypes.c_int, [_P, _P, _P, _P]),
    "wdd_get_accumulator": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "wdd_get_projection": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "wdd_plan_get_info": (ctypes.c_int, [_P, ctypes.POINTER(PlanInfo)]),
    "wdd_profile_enable": (ctypes.c_int, [_P, ctypes.c_int32]),
    "wdd_profile_period": (ctypes.c_int, [_P, ctypes.c_int32]),
    "wdd_profile_read": (ctypes.c_int, [_P, ctypes.POINTER(Profile)]),
    "wdd_update_probe": (ctypes.c_int, [_P, ctypes.POINTER(Probe), ctypes.c_double]),
    "wdd_checkpoint_size": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "wdd_checkpoint_save": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "wdd_checkpoint_load": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "wdd_reset": (ctypes.c_int, [_P]),
    "wdd_sync": (ctypes.c_int, [_P]),
    "wdd_destroy": (ctypes.c_int, [_P]),
    "wdd_display": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P]),
    "wdd_display_noalloc": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P]),
    "wdd_patches_create": (ctypes.c_int, [ctypes.POINTER(Probe), ctypes.POINTER(Scan), ctypes.POINTER(Detector),
                                          ctypes.c_int32, ctypes.POINTER(PatchGeometry), ctypes.POINTER(Options), _P,
                                          ctypes.POINTER(_P)]),
    "wdd_patches_push": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32]),
    "wdd_patches_snapshot": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]),
    "wdd_patches_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "wdd_patches_sync": (ctypes.c_int, [_P]),
    "wdd_patches_destroy": (ctypes.c_int, [_P]),
    "wdd_server_default_options": (ctypes.c_int, [ctypes.POINTER(ServerOptions)]),
    "wdd_server_create": (ctypes.c_int, [ctypes.POINTER(ServerOptions), ctypes.POINTER(_P)]),
    "wdd_server_open": (ctypes.c_int, [_P, ctypes.POINTER(Probe), ctypes.POINTER(Scan), ctypes.POINTER(Detector),
                                       ctypes.c_int32, ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_int32)]),
    "wdd_server_wait_open": (ctypes.c_int, [_P, ctypes.c_int32]),
    "wdd_server_submit": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.c_int32]),
    "wdd_server_step": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "wdd_server_snapshot": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_uint64)]),
    "wdd_server_acq_shape": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32)]),
    "wdd_server_acq_state": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int64)]),
    "wdd_server_close": (ctypes.c_int, [_P, ctypes.c_int32]),
    "wdd_server_get_stats": (ctypes.c_int, [_P, ctypes.POINTER(ServerStats)]),
    "wdd_server_destroy": (ctypes.c_int, [_P]),
}


def library_path() -> str:
    return _LIB_PATH


def load_library() -> ctypes.CDLL:
    """Loads libwdd.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with paper_2212_01309_amd.build.build_library()")
    # PyTorch ships its own HIP runtime and names it without the version suffix.  Loaded after
    # libwdd.so (which binds the system runtime, libamdhip64.so.7), it would come in as a
    # second runtime that sees no device; loaded first, libwdd.so binds to it and the process
    # has one HIP runtime, whose device pointers both sides share.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(_LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


_allocator_refs = None  # the ctypes callbacks in use (kept alive while the library may call them)


def set_allocator(alloc=None, release=None) -> None:
    """Device memory for plans created from now on comes from alloc(nbytes) -> int device
    address (0 if none) and goes back through release(address) (wdd_set_allocator); with
    alloc None the library allocates with hipMalloc again.  Existing plans keep theirs."""
    global _allocator_refs
    if alloc is None:
        _check(load_library().wdd_set_allocator(_ALLOC_FN(), _RELEASE_FN(), None))
        return
    if release is None:
        raise ValueError("an allocator needs a release function")

    def _alloc(nbytes, _ctx):
        try:
            return int(alloc(int(nbytes))) or None
        except Exception:  # the library reports the failure as WDD_ENOMEM
            return None

    def _release(ptr, _ctx):
        release(int(ptr))

    refs = (_ALLOC_FN(_alloc), _RELEASE_FN(_release))
    _check(load_library().wdd_set_allocator(refs[0], refs[1], None))
    # plans created with the previous callbacks release through them: keep every set alive
    _allocator_refs = (refs, _allocator_refs)


def use_torch_allocator() -> None:
    """Plans created from now on take their device memory from torch's caching allocator
    (one pool with the caller's tensors)."""
    import torch
    set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n), torch.cuda.caching_allocator_delete)


def _check(code: int) -> None:
    if code != WDD_OK:
        msg = load_library().wdd_last_error().decode(errors="replace")
        raise WddError(code, msg)


def _options(eps_rel: float, sigma_px: float, max_batch: int, precision: int = WDD_FP32,
             order: int = WDD_ORDER_SPECTRUM, basis: int = WDD_BASIS_HERMITE_GAUSS, pipeline=False) -> Options:
    o = Options()
    _check(load_library().wdd_default_options(ctypes.byref(o)))
    o.eps_rel, o.sigma_px, o.max_batch, o.precision, o.order = eps_rel, sigma_px, max_batch, precision, order
    o.basis = basis
    o.pipeline = int(pipeline)  # False / True / 2 (two-stage)
    return o


_I32 = np.dtype(np.int32)


def _is_device_tensor(x) -> bool:
    return hasattr(x, "data_ptr") and hasattr(x, "is_cuda") and bool(x.is_cuda)


def _host_array(x, dtype) -> np.ndarray:
    if hasattr(x, "numpy"):
        x = x.numpy()
    return np.ascontiguousarray(x, dtype=dtype)


class Tables:
    """FP64 host tables of a geometry (kept frequencies, basis, Wiener filter)."""

    def __init__(self, radius: float, sy: int, sx: int, ny: int, nx: int, k: int, *, defocus: float = 0.0,
                 amplitude: float = 1.0, step: float = 1.0, eps_rel: float = 0.01, sigma: float = 0.0,
                 dtype: int = WDD_U16, basis: int = WDD_BASIS_HERMITE_GAUSS, center=None):
        lib = load_library()
        self._h = _P()
        _check(lib.wdd_tables_build(ctypes.byref(_probe(radius, ny, nx, center, defocus, amplitude)),
                                    ctypes.byref(Scan(sy, sx, step)),
                                    ctypes.byref(Detector(ny, nx, dtype)), k,
                                    ctypes.byref(_options(eps_rel, sigma, 256, basis=basis)), ctypes.byref(self._h)))
        info = PlanInfo()
        _check(lib.wdd_tables_info(self._h, ctypes.byref(info)))
        self.n_freq, self.k, self.l = int(info.n_freq), int(info.k), int(info.l)
        self.sigma, self.eps_abs = float(info.sigma_px), float(info.eps_abs)
        self.ny, self.nx = ny, nx

    def export(self):
        """Returns (freqs [n,2] int32, psi_y [ny,l], psi_x [nx,l], pairs [k,2] int32, w [n,k] complex128)."""
        freqs = np.zeros((self.n_freq, 2), np.int32)
        psi_y = np.zeros((self.ny, self.l))
        psi_x = np.zeros((self.nx, self.l))
        pairs = np.zeros((self.k, 2), np.int32)
        w = np.zeros((self.n_freq, self.k, 2))
        _check(load_library().wdd_tables_export(self._h, freqs.ctypes.data, psi_y.ctypes.data, psi_x.ctypes.data,
                                                pairs.ctypes.data, w.ctypes.data))
        return freqs, psi_y, psi_x, pairs, w[..., 0] + 1j * w[..., 1]

    def close(self):
        if self._h:
            load_library().wdd_tables_free(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """A live reconstruction on the current HIP device (wdd_plan ... wdd_destroy).
    pipeline=True (object order): each push's update runs in the next push's launch, beside
    that push's projection; pipeline=2: two stages, the x-DFT one launch ahead of the update
    (wdd_options.pipeline)."""

    def __init__(self, radius: float, sy: int, sx: int, ny: int, nx: int, k: int, *, dtype: int = WDD_U16,
                 defocus: float = 0.0, amplitude: float = 1.0, step: float = 1.0, eps_rel: float = 0.01,
                 sigma: float = 0.0, max_batch: int = 256, stream: Optional[int] = None, precision: int = WDD_FP32,
                 order: int = WDD_ORDER_SPECTRUM, basis: int = WDD_BASIS_HERMITE_GAUSS, center=None,
                 pipeline=False):
        lib = load_library()
        self._h = _P()
        self.sy, self.sx, self.ny, self.nx, self.dtype = sy, sx, ny, nx, dtype
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        self._np_dtype = np.uint16 if dtype == WDD_U16 else np.float32
        self.basis = basis
        self.center = (ny // 2, nx // 2) if center is None else tuple(center)
        _check(lib.wdd_plan(ctypes.byref(_probe(radius, ny, nx, center, defocus, amplitude)),
                            ctypes.byref(Scan(sy, sx, step)), ctypes.byref(Detector(ny, nx, dtype)), k,
                            ctypes.byref(_options(eps_rel, sigma, max_batch, precision, order, basis, pipeline)),
                            _P(stream) if stream else None, ctypes.byref(self._h)))
        info = self.info()
        self.n_freq, self.k, self.l = int(info.n_freq), int(info.k), int(info.l)
        self._last_batch = 0
        # per-call state of the hot path (a plan is used from one thread at a time)
        self._fn_push, self._fn_push_snapshot = lib.wdd_push, lib.wdd_push_snapshot
        self._seen = ctypes.c_uint64()
        self._seen_ref = ctypes.byref(self._seen)
        self._addr_cache = {}
        self._pinned = None
        # device tensors (frames, asynchronous outputs) of the latest calls: the plan's stream may
        # still use them after the call returns (a temporary would go back to torch's allocator
        # at once).  The library keeps at most WDD_MAX_PUSHES_IN_FLIGHT pushes queued, so holding
        # that many covers every batch still in flight; sync() releases them.
        self._held = collections.deque(maxlen=2 * WDD_MAX_PUSHES_IN_FLIGHT)

    # -- lifecycle ---------------------------------------------------------
    def close(self) -> None:
        if self._h:
            load_library().wdd_destroy(self._h)
            self._h = _P()
            self._pinned = None          # the pinned buffer is freed with the plan
            self._addr_cache = {}

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self) -> int:
        return self._h.value or 0

    def info(self) -> PlanInfo:
        info = PlanInfo()
        _check(load_library().wdd_plan_get_info(self._h, ctypes.byref(info)))
        return info

    # -- hot path ------------------------------------------------------------
    def _host_addr(self, a: np.ndarray) -> int:
        """Data address of a small host array, remembered for the arrays seen recently (they
        are kept alive while remembered, so their ids cannot be taken by other arrays)."""
        e = self._addr_cache.get(id(a))
        if e is not None and e[0] is a:
            return e[1]
        if len(self._addr_cache) >= 256:
            self._addr_cache.clear()
        addr = a.ctypes.data
        self._addr_cache[id(a)] = (a, addr)
        return addr

    def _frames_arg(self, frames, positions):
        if (type(positions) is np.ndarray and positions.dtype == _I32 and positions.ndim == 2
                and positions.shape[1] == 2 and positions.flags.c_contiguous):
            pos = positions
            pos_addr = self._host_addr(pos)
        else:
            pos = _host_array(positions, np.int32).reshape(-1, 2)
            pos_addr = pos.ctypes.data
        n = pos.shape[0]
        if _is_device_tensor(frames):
            if frames.element_size() != np.dtype(self._np_dtype).itemsize:
                raise ValueError("device frames have the wrong element size for the detector dtype")
            if frames.numel() != n * self.ny * self.nx:
                raise ValueError("frames and positions disagree in count or frame shape")
            if not frames.is_contiguous():
                raise ValueError("device frames must be contiguous")
            ptr, on_dev, keep = frames.data_ptr(), 1, frames
        else:
            keep = _host_array(frames, self._np_dtype)
            if keep.size != n * self.ny * self.nx:
                raise ValueError("frames and positions disagree in count or frame shape")
            ptr, on_dev = keep.ctypes.data, 0
        return pos_addr, n, ptr, on_dev, keep

    def push(self, frames, positions) -> None:
        """frames: [n, ny, nx] (torch GPU tensor or host array of the detector dtype);
        positions: host int32 [n, 2] scan indices (y, x)."""
        pos, n, ptr, on_dev, keep = self._frames_arg(frames, positions)
        _check(self._fn_push(self._h, ptr, pos, n, on_dev))
        if n:
            self._last_batch = n
            if on_dev:
                self._held.append(keep)

    def push_snapshot(self, frames, positions, out=None, wait: bool = True, defer: bool = False):
        """push() then snapshot() in one call (one pass over the spectrum when possible).
        With a device `out` and wait=False the call returns once the work is enqueued; `out`
        is complete after sync().  defer=True (with wait=False) lets the image be written by
        the next push's first launch (WDD_OUT_DEVICE_DEFERRED; with pipeline=True, by the push
        after next)."""
        pos, n, ptr, on_dev, keep = self._frames_arg(frames, positions)
        if out is not None and out is self._pinned:
            res = out
            _check(self._fn_push_snapshot(self._h, ptr, pos, n, on_dev, self._pinned_addr, 0, self._seen_ref))
        elif out is not None and _is_device_tensor(out):
            kind = WDD_OUT_DEVICE if wait else (WDD_OUT_DEVICE_DEFERRED if defer else WDD_OUT_DEVICE_ASYNC)
            _check(self._fn_push_snapshot(self._h, ptr, pos, n, on_dev, self._device_out(out), kind, self._seen_ref))
            res = out
            if not wait:
                self._held.append(out)
        else:
            res = self._host_out(out)
            _check(self._fn_push_snapshot(self._h, ptr, pos, n, on_dev, res.ctypes.data, 0, self._seen_ref))
        if n:
            self._last_batch = n
            if on_dev and not wait:
                self._held.append(keep)
        return res

    def _device_out(self, out) -> int:
        if out.numel() * out.element_size() != 8 * self.sy * self.sx or not out.is_contiguous():
            raise ValueError("device output must be a contiguous tensor of sy*sx complex64 values")
        return out.data_ptr()

    def snapshot(self, out=None, wait: bool = True):
        """Displayed estimate [sy, sx] complex64.  With `out` (a torch GPU tensor of
        sy*sx complex64 or 2*sy*sx float32, or a host complex64 array) it is written there
        and returned.  With a device `out` and wait=False the call returns once the work is
        enqueued; `out` is complete after sync()."""
        seen = ctypes.c_uint64()
        if out is not None and _is_device_tensor(out):
            kind = WDD_OUT_DEVICE if wait else WDD_OUT_DEVICE_ASYNC
            _check(load_library().wdd_snapshot(self._h, self._device_out(out), kind, ctypes.byref(seen)))
            if not wait:
                self._held.append(out)
            return out
        host = self._host_out(out)
        _check(load_library().wdd_snapshot(self._h, host.ctypes.data, 0, ctypes.byref(seen)))
        return host

    def _host_out(self, out):
        if out is None:
            return np.empty((self.sy, self.sx), np.complex64)
        if not (isinstance(out, np.ndarray) and out.dtype == np.complex64 and out.size == self.sy * self.sx
                and out.flags.c_contiguous):
            raise ValueError("host output must be a C-contiguous complex64 array of sy*sx elements")
        return out

    def snapshot_buffer(self) -> np.ndarray:
        """The plan's pinned host array [sy, sx] complex64 that host snapshots pass through;
        give it as `out` to avoid the final copy.  Overwritten by every host snapshot."""
        if self._pinned is None:
            ptr = ctypes.POINTER(ctypes.c_float)()
            _check(load_library().wdd_snapshot_buffer(self._h, ctypes.byref(ptr)))
            flat = np.ctypeslib.as_array(ptr, shape=(2 * self.sy * self.sx,))
            self._pinned = flat.view(np.complex64).reshape(self.sy, self.sx)
            self._pinned_addr = self._pinned.ctypes.data
        return self._pinned

    def spectrum(self) -> np.ndarray:
        """D on the kept frequencies from the last snapshot, complex64 [n_freq]."""
        d = np.empty(self.n_freq, np.complex64)
        _check(load_library().wdd_spectrum(self._h, d.ctypes.data, 0))
        return d

    def export(self):
        """The plan's own FP64 tables: (phi [ny*nx, k] float64 (complex128 with the Fourier
        basis), w [n_freq, k] complex128, freqs [n_freq, 2] int32)."""
        fourier = self.basis == WDD_BASIS_FOURIER
        phi = np.zeros((self.ny * self.nx, self.k, 2) if fourier else (self.ny * self.nx, self.k))
        w = np.zeros((self.n_freq, self.k, 2))
        freqs = np.zeros((self.n_freq, 2), np.int32)
        _check(load_library().wdd_plan_export(self._h, phi.ctypes.data, w.ctypes.data, freqs.ctypes.data))
        if fourier:
            phi = phi[..., 0] + 1j * phi[..., 1]
        return phi, w[..., 0] + 1j * w[..., 1], freqs

    def wiener(self) -> np.ndarray:
        """W as the device holds it, complex64 [n_freq, k]."""
        w = np.empty((self.n_freq, self.k), np.complex64)
        _check(load_library().wdd_get_wiener(self._h, w.ctypes.data, 0))
        return w

    def accumulator(self) -> np.ndarray:
        """A, complex64 [n_freq, k]."""
        a = np.empty((self.n_freq, self.k), np.complex64)
        _check(load_library().wdd_get_accumulator(self._h, a.ctypes.data, 0))
        return a

    def projection(self) -> np.ndarray:
        """h of the last pushed batch: float32 [n, k], or complex64 [n, k] with the Fourier basis."""
        h = np.empty((self._last_batch, self.k), np.complex64 if self.basis == WDD_BASIS_FOURIER else np.float32)
        _check(load_library().wdd_get_projection(self._h, h.ctypes.data, 0))
        return h

    def profile_enable(self, stages: int = 31) -> None:
        """Time the stages in the bit mask (STAGE_* constants; 0 turns timing off)."""
        _check(load_library().wdd_profile_enable(self._h, int(stages)))

    def profile_period(self, period: int) -> None:
        """Time one push in every `period` (and the snapshot after it); zeroes the totals."""
        _check(load_library().wdd_profile_period(self._h, int(period)))

    def profile_read(self) -> dict:
        pr = Profile()
        _check(load_library().wdd_profile_read(self._h, ctypes.byref(pr)))
        return {f: getattr(pr, f) for f, _ in Profile._fields_}

    def update_probe(self, radius: float, defocus: float = 0.0, amplitude: float = 1.0, eps_rel: float = 0.01):
        """New Wiener filter for the frames already accumulated (same aperture radius and centre)."""
        _check(load_library().wdd_update_probe(
            self._h, ctypes.byref(_probe(radius, self.ny, self.nx, self.center, defocus, amplitude)), eps_rel))

    def checkpoint(self) -> bytes:
        """Image of the live state (spectrum A and frame count)."""
        size = ctypes.c_size_t()
        _check(load_library().wdd_checkpoint_size(self._h, ctypes.byref(size)))
        buf = ctypes.create_string_buffer(size.value)
        _check(load_library().wdd_checkpoint_save(self._h, ctypes.cast(buf, _P), size.value))
        return buf.raw

    def restore(self, image: bytes) -> None:
        buf = ctypes.create_string_buffer(image, len(image))
        _check(load_library().wdd_checkpoint_load(self._h, ctypes.cast(buf, _P), len(image)))

    def reset(self) -> None:
        _check(load_library().wdd_reset(self._h))
        self._last_batch = 0

    def sync(self) -> None:
        _check(load_library().wdd_sync(self._h))
        self._held.clear()


class Patches:
    """A large field of view as independently reconstructed, merged patches (wdd_patches_*)."""

    def __init__(self, radius: float, sy: int, sx: int, ny: int, nx: int, k: int, py: int, px: int,
                 overlap_y: int = 0, overlap_x: int = 0, *, dtype: int = WDD_U16, defocus: float = 0.0,
                 amplitude: float = 1.0, step: float = 1.0, eps_rel: float = 0.01, sigma: float = 0.0,
                 max_batch: int = 256, stream: Optional[int] = None, precision: int = WDD_FP32, center=None):
        lib = load_library()
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        self.sy, self.sx, self.ny, self.nx, self.dtype = sy, sx, ny, nx, dtype
        self._np_dtype = np.uint16 if dtype == WDD_U16 else np.float32
        self._h = _P()
        _check(lib.wdd_patches_create(ctypes.byref(_probe(radius, ny, nx, center, defocus, amplitude)),
                                      ctypes.byref(Scan(sy, sx, step)), ctypes.byref(Detector(ny, nx, dtype)), k,
                                      ctypes.byref(PatchGeometry(py, px, overlap_y, overlap_x)),
                                      ctypes.byref(_options(eps_rel, sigma, max_batch, precision, WDD_ORDER_OBJECT)),
                                      _P(stream) if stream else None, ctypes.byref(self._h)))
        self._held = collections.deque(maxlen=8)

    def info(self) -> dict:
        a, b, nf, dev = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _check(load_library().wdd_patches_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(nf),
                                               ctypes.byref(dev)))
        return {"npatch_y": a.value, "npatch_x": b.value, "n_freq": nf.value, "device_bytes": dev.value}

    def push(self, frames, positions) -> None:
        """frames: contiguous torch GPU tensor [n, ny, nx]; positions: host int32 [n, 2] on the whole raster."""
        if not _is_device_tensor(frames) or not frames.is_contiguous():
            raise ValueError("patch frames must be a contiguous GPU tensor")
        pos = _host_array(positions, np.int32).reshape(-1, 2)
        if frames.numel() != pos.shape[0] * self.ny * self.nx:
            raise ValueError("frames and positions disagree in count or frame shape")
        _check(load_library().wdd_patches_push(self._h, frames.data_ptr(), pos.ctypes.data, pos.shape[0]))
        self._held.append(frames)

    def snapshot(self, out=None, wait: bool = True):
        """The merged image [sy, sx] complex64 (host array, or into a torch GPU tensor `out`)."""
        seen = ctypes.c_uint64()
        if out is not None and _is_device_tensor(out):
            if out.numel() * out.element_size() != 8 * self.sy * self.sx or not out.is_contiguous():
                raise ValueError("device output must be a contiguous tensor of sy*sx complex64 values")
            kind = WDD_OUT_DEVICE if wait else WDD_OUT_DEVICE_ASYNC
            _check(load_library().wdd_patches_snapshot(self._h, out.data_ptr(), kind, ctypes.byref(seen)))
            return out
        host = np.empty((self.sy, self.sx), np.complex64) if out is None else out
        _check(load_library().wdd_patches_snapshot(self._h, host.ctypes.data, WDD_OUT_HOST, ctypes.byref(seen)))
        return host

    def sync(self) -> None:
        _check(load_library().wdd_patches_sync(self._h))
        self._held.clear()

    def close(self) -> None:
        if self._h:
            load_library().wdd_patches_destroy(self._h)
            self._h = _P()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Many concurrent acquisitions with continuous batching (wdd_server_*)."""

    def __init__(self, hbm_budget_bytes: int = 1 << 30, snapshot_interval_us: float = 1000.0, batch_frames: int = 256,
                 launch_mode=None):
        """launch_mode: a WDD_SERVE_* value or "streams" / "grouped" / "graph" (None: the
        library's default)."""
        lib = load_library()
        o = ServerOptions()
        _check(lib.wdd_server_default_options(ctypes.byref(o)))
        o.hbm_budget_bytes, o.snapshot_interval_us, o.batch_frames = hbm_budget_bytes, snapshot_interval_us, batch_frames
        if launch_mode is not None:
            o.launch_mode = SERVE_MODES[launch_mode] if isinstance(launch_mode, str) else launch_mode
        self._h = _P()
        _check(lib.wdd_server_create(ctypes.byref(o), ctypes.byref(self._h)))
        self._keep = {}

    def open(self, radius: float, sy: int, sx: int, ny: int, nx: int, k: int, *, dtype: int = WDD_U16,
             defocus: float = 0.0, amplitude: float = 1.0, step: float = 1.0, eps_rel: float = 0.01,
             sigma: float = 0.0, precision=WDD_FP32, order: int = WDD_ORDER_SPECTRUM,
             basis: int = WDD_BASIS_HERMITE_GAUSS, center=None) -> Optional[int]:
        """Acquisition id, or None when it does not fit the memory budget now."""
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        aid = ctypes.c_int32()
        code = load_library().wdd_server_open(self._h, ctypes.byref(_probe(radius, ny, nx, center, defocus, amplitude)),
                                              ctypes.byref(Scan(sy, sx, step)), ctypes.byref(Detector(ny, nx, dtype)),
                                              k, ctypes.byref(_options(eps_rel, sigma, 256, precision, order, basis)),
                                              ctypes.byref(aid))
        if code == WDD_EBUSY:
            return None
        _check(code)
        self._keep[aid.value] = []
        return aid.value

    def state(self, acq: int) -> Tuple[bool, int]:
        """(plan ready, submitted frames not yet pushed)."""
        r, n = ctypes.c_int32(), ctypes.c_int64()
        _check(load_library().wdd_server_acq_state(self._h, acq, ctypes.byref(r), ctypes.byref(n)))
        return bool(r.value), n.value

    def wait_open(self, acq: int) -> None:
        """Waits until the acquisition's plan (made on a worker thread) is ready."""
        _check(load_library().wdd_server_wait_open(self._h, acq))

    def submit(self, acq: int, frames, positions) -> None:
        """frames: contiguous torch GPU tensor [n, ny, nx]; kept referenced until pushed."""
        if not _is_device_tensor(frames) or not frames.is_contiguous():
            raise ValueError("server frames must be a contiguous GPU tensor")
        pos = _host_array(positions, np.int32).reshape(-1, 2)
        _check(load_library().wdd_server_submit(self._h, acq, frames.data_ptr(), pos.ctypes.data, pos.shape[0]))
        self._keep[acq].append(frames)

    def step(self) -> int:
        """One scheduling round; returns the number of frames pushed.  Submitted tensors stay
        referenced until the acquisition's next snapshot() or close()."""
        n = ctypes.c_int32()
        _check(load_library().wdd_server_step(self._h, ctypes.byref(n)))
        return n.value

    def snapshot(self, acq: int) -> np.ndarray:
        sy, sx = ctypes.c_int32(), ctypes.c_int32()
        _check(load_library().wdd_server_acq_shape(self._h, acq, ctypes.byref(sy), ctypes.byref(sx)))
        out = np.empty((sy.value, sx.value), np.complex64)
        seen = ctypes.c_uint64()
        _check(load_library().wdd_server_snapshot(self._h, acq, out.ctypes.data, ctypes.byref(seen)))
        self._keep[acq].clear()
        return out

    def close(self, acq: int) -> None:
        _check(load_library().wdd_server_close(self._h, acq))
        self._keep.pop(acq, None)

    def stats(self) -> dict:
        st = ServerStats()
        _check(load_library().wdd_server_get_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def destroy(self) -> None:
        if self._h:
            load_library().wdd_server_destroy(self._h)
            self._h = _P()
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def display(spectrum, out=None, stream: Optional[int] = None):
    """O~ = conj(IDFT2_unitary(D)) / sqrt(|D[0, 0]|) of a spectrum grid D [sy, sx] (complex64
    torch GPU tensor) into `out` (a new complex64 GPU tensor if None), queued on `stream`
    (a hipStream_t; None: torch's current stream) (wdd_display)."""
    import torch
    if not (_is_device_tensor(spectrum) and spectrum.dtype == torch.complex64 and spectrum.dim() == 2
            and spectrum.is_contiguous()):
        raise ValueError("spectrum must be a contiguous 2-D complex64 GPU tensor")
    sy, sx = spectrum.shape
    if out is None:
        out = torch.empty_like(spectrum)
    elif not (_is_device_tensor(out) and out.dtype == torch.complex64 and tuple(out.shape) == (sy, sx)
              and out.is_contiguous()):
        raise ValueError("out must be a contiguous complex64 GPU tensor of the spectrum's shape")
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    _check(load_library().wdd_display(spectrum.data_ptr(), sy, sx, out.data_ptr(), _P(stream) if stream else None))
    return out


def header_symbols(header: Optional[str] = None) -> Tuple[str, ...]:
    """Names of the functions declared in include/wdd.h."""
    import re
    if header is None:
        header = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "wdd.h")
    text = open(header).read()
    return tuple(sorted(set(re.findall(r"^\s*(?:wdd_status|const char\*)\s+(wdd_\w+)\s*\(", text, re.M))))
