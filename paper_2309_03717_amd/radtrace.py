"""Python binding of libradtrace (include/radtrace.h): argument marshalling
only. Every step of the computation runs in the library's HIP kernels; torch
provides device memory and streams.

The low-level functions carry the C names (``rt_plan_create``,
``rt_accumulate``, ...). ``Plan`` bundles a detector, a plan handle and a
workspace for convenience. Importing this module loads the compiled library
and raises ImportError if it is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import torch  # loads the HIP runtime the library must share

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libradtrace.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(or python paper_2309_03717_amd/build_lib.py)")

_lib = C.CDLL(LIB_PATH)

RT_OK, RT_E_INVALID, RT_E_UNSUPPORTED, RT_E_NO_DEVICE, RT_E_HIP, RT_E_WORKSPACE = range(6)
RT_ENDPOINT, RT_ZHS = 0, 1
RT_FP64, RT_MIXED = 0, 1
RT_UNIFORM, RT_EXPONENTIAL, RT_TABULATED, RT_SPHERICAL = 0, 1, 2, 3
MEDIUM_KIND = {"uniform": RT_UNIFORM, "exponential": RT_EXPONENTIAL, "tabulated": RT_TABULATED,
               "spherical": RT_SPHERICAL}
FORMALISM = {"endpoint": RT_ENDPOINT, "zhs": RT_ZHS}
PRECISION = {"fp64": RT_FP64, "mixed": RT_MIXED}
K_SI = 4.80320471518522e-18


class rt_medium(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n0_minus_1", C.c_double), ("scale_height", C.c_double),
                ("table", C.c_void_p), ("n_table", C.c_int32), ("table_z0", C.c_double),
                ("table_dz", C.c_double), ("earth_radius", C.c_double)]


class rt_detector(C.Structure):
    _fields_ = [("n_antennas", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p),
                ("z", C.c_void_p), ("t_start", C.c_void_p), ("dt", C.c_double),
                ("n_bins", C.c_int32)]


_TRACK_FIELDS = ("x0", "y0", "z0", "t0", "x1", "y1", "z1", "t1", "bx", "by", "bz", "qw")


class rt_tracks(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(f, C.c_void_p) for f in _TRACK_FIELDS]


class rt_tiling(C.Structure):
    _fields_ = [("antennas_per_block", C.c_int32), ("track_splits", C.c_int32),
                ("block_threads", C.c_int32), ("bins_per_segment", C.c_int32),
                ("tracks_per_pass", C.c_int64)]

    def as_tuple(self):
        return (self.antennas_per_block, self.track_splits, self.block_threads,
                self.bins_per_segment, self.tracks_per_pass)


class rt_shower(C.Structure):
    _fields_ = [("det", rt_detector), ("med", rt_medium), ("formalism", C.c_int32),
                ("tracks", rt_tracks), ("traces", C.c_void_p)]


class rt_batch_options(C.Structure):
    _fields_ = [("block_threads", C.c_int32), ("items_per_cu", C.c_int32),
                ("max_antennas_per_tile", C.c_int32), ("direct_launch", C.c_int32),
                ("per_shower", C.POINTER(rt_tiling))]


_P = C.c_void_p
_lib.rt_abi_version.restype = C.c_int
ABI_VERSION = 2   # the structure layouts below
if _lib.rt_abi_version() != ABI_VERSION:
    raise ImportError(f"{LIB_PATH} has ABI version {_lib.rt_abi_version()}, the binding expects "
                      f"{ABI_VERSION}: rebuild the library")
_lib.rt_status_string.restype = C.c_char_p
_lib.rt_status_string.argtypes = [C.c_int]
_lib.rt_last_error.restype = C.c_char_p
_lib.rt_plan_create.argtypes = [C.POINTER(_P), C.POINTER(rt_detector), C.POINTER(rt_medium),
                                C.c_int, C.c_int, C.c_double]
_lib.rt_plan_destroy.argtypes = [_P]
_lib.rt_plan_set_tiling.argtypes = [_P, C.POINTER(rt_tiling)]
_lib.rt_plan_get_tiling.argtypes = [_P, C.c_int64, C.POINTER(rt_tiling)]
_lib.rt_plan_workspace_bytes.argtypes = [_P, C.c_int64, C.POINTER(C.c_size_t)]
_lib.rt_accumulate.argtypes = [_P, C.POINTER(rt_tracks), _P, _P, C.c_size_t, _P]
_lib.rt_accumulate_static.argtypes = [_P, C.POINTER(rt_tracks), _P, _P]
RT_STATIC_WORKSPACE_BYTES = 64 << 20   # include/radtrace.h
_lib.rt_propagate.argtypes = [_P, C.POINTER(rt_tracks), _P, _P, _P]
_lib.rt_plan_set_timing_events.argtypes = [_P, _P, _P]
_lib.rt_plan_set_n0m1_device.argtypes = [_P, _P]
_lib.rt_plan_vjp_workspace_bytes.argtypes = [_P, C.c_int64, C.POINTER(C.c_size_t)]
_lib.rt_zhs_vjp.argtypes = [_P, C.POINTER(rt_tracks), _P, _P, _P, _P, _P, _P, C.c_size_t, _P]
_lib.rt_endpoint_vjp.argtypes = _lib.rt_zhs_vjp.argtypes
_lib.rt_batch_create.argtypes = [C.POINTER(_P), C.POINTER(rt_shower), C.c_int32, C.c_int,
                                 C.c_double, C.POINTER(rt_batch_options)]
_lib.rt_batch_destroy.argtypes = [_P]
_lib.rt_batch_workspace_bytes.argtypes = [_P, C.POINTER(C.c_size_t)]
_lib.rt_batch_get_info.argtypes = [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
_lib.rt_batch_launch.argtypes = [_P, _P, C.c_size_t, _P]
_lib.rt_batch_set_timing_events.argtypes = [_P, _P, _P]
_lib.rt_filter_tracks.argtypes = [C.POINTER(rt_tracks), C.c_int, C.c_double,
                                  C.POINTER(rt_tracks), _P, _P, C.c_size_t, _P]
_lib.rt_filter_workspace_bytes.argtypes = [C.c_int64, C.POINTER(C.c_size_t)]
_lib.rt_plan_autotune.argtypes = [_P, C.POINTER(rt_tracks), _P, _P, C.c_size_t,
                                  C.POINTER(rt_tiling), C.c_int32, C.c_int32, _P,
                                  C.POINTER(C.c_float), C.POINTER(C.c_int32)]
_lib.rt_batch_autotune.argtypes = [C.POINTER(rt_shower), C.c_int32, C.c_int, C.c_double,
                                   C.POINTER(rt_batch_options), C.c_int32, _P, C.c_size_t,
                                   C.c_int32, _P, C.POINTER(C.c_float), C.POINTER(C.c_int32)]


class RadtraceError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.rt_last_error().decode()
        super().__init__(f"{where}: {_lib.rt_status_string(status).decode()} ({status}): {msg}")


def _check(status: int, where: str):
    if status != RT_OK:
        raise RadtraceError(status, where)


def _stream(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _on_stream(stream):
    """Context for a call on an explicit torch.cuda.Stream other than the
    current one: that stream first waits for the current stream's work (the
    call's inputs), and the tensors allocated for the call are taken from
    that stream's memory pool, so the caching allocator reuses them only
    after the stream's work on them is done. A no-op for the current stream
    (or a raw handle)."""
    import contextlib
    if not isinstance(stream, torch.cuda.Stream):
        return contextlib.nullcontext()
    cur = torch.cuda.current_stream(stream.device)
    if stream == cur:
        return contextlib.nullcontext()
    stream.wait_stream(cur)
    return torch.cuda.stream(stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


# ------------------------------------------------------------------ device data
@dataclass
class DeviceDetector:
    """Antenna arrays on the device (float64 tensors) plus the time binning."""
    x: torch.Tensor
    y: torch.Tensor
    z: torch.Tensor
    t_start: torch.Tensor
    dt: float
    n_bins: int

    @property
    def m(self) -> int:
        return int(self.x.numel())

    @staticmethod
    def from_array(array, device="cuda") -> "DeviceDetector":
        f = lambda a: torch.as_tensor(a, dtype=torch.float64).contiguous().to(device)
        return DeviceDetector(f(array.x), f(array.y), f(array.z), f(array.t_start),
                              float(array.dt), int(array.n_bins))

    def struct(self) -> rt_detector:
        for t in (self.x, self.y, self.z, self.t_start):
            if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != self.m:
                raise ValueError("antenna arrays must be contiguous float64 of equal length")
        return rt_detector(self.m, _ptr(self.x), _ptr(self.y), _ptr(self.z), _ptr(self.t_start),
                           self.dt, self.n_bins)


@dataclass
class DeviceTracks:
    """Structure-of-arrays tracks on the device: geometry float64; beta and
    qw float64 (FP64 plans) or float32 (mixed plans)."""
    x0: torch.Tensor
    y0: torch.Tensor
    z0: torch.Tensor
    t0: torch.Tensor
    x1: torch.Tensor
    y1: torch.Tensor
    z1: torch.Tensor
    t1: torch.Tensor
    bx: torch.Tensor
    by: torch.Tensor
    bz: torch.Tensor
    qw: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.x0.numel())

    @staticmethod
    def from_tracks(tracks, device="cuda") -> "DeviceTracks":
        return DeviceTracks(**{f: torch.from_numpy(getattr(tracks, f).copy()).to(device)
                               for f in _TRACK_FIELDS})

    def struct(self, precision: int) -> rt_tracks:
        want = torch.float64 if precision == RT_FP64 else torch.float32
        n = self.n
        for f in _TRACK_FIELDS:
            t = getattr(self, f)
            dt = torch.float64 if f in _TRACK_FIELDS[:8] else want
            if t.dtype != dt or not t.is_contiguous() or t.numel() != n:
                raise ValueError(f"track field {f} must be contiguous {dt} of length {n}")
        return rt_tracks(n, *[_ptr(getattr(self, f)) for f in _TRACK_FIELDS])

    def slice(self, lo: int, hi: int) -> "DeviceTracks":
        return DeviceTracks(**{f: getattr(self, f)[lo:hi] for f in _TRACK_FIELDS})


# ------------------------------------------------------------------ C names
def rt_abi_version() -> int:
    return _lib.rt_abi_version()


def rt_status_string(status: int) -> str:
    return _lib.rt_status_string(status).decode()


def rt_last_error() -> str:
    return _lib.rt_last_error().decode()


def rt_plan_create(det: DeviceDetector, medium_kind: int, n0_minus_1: float, scale_height: float,
                   formalism: int, precision: int, k: float, table: Optional[torch.Tensor] = None,
                   table_z0: float = 0.0, table_dz: float = 1.0, earth_radius: float = 0.0) -> int:
    """table: device float64 tensor of the tabulated profile (kept alive by
    the caller for the plan's lifetime); earth_radius: spherical medium only."""
    handle = _P()
    d = det.struct()
    m = rt_medium(medium_kind, n0_minus_1, scale_height, _ptr(table),
                  0 if table is None else table.numel(), table_z0, table_dz, earth_radius)
    _check(_lib.rt_plan_create(C.byref(handle), C.byref(d), C.byref(m), formalism, precision,
                               float(k)), "rt_plan_create")
    return handle.value


def rt_plan_destroy(plan: int) -> None:
    _check(_lib.rt_plan_destroy(plan), "rt_plan_destroy")


def rt_plan_set_tiling(plan: int, antennas_per_block=0, track_splits=0, block_threads=0,
                       bins_per_segment=0, tracks_per_pass=0) -> None:
    tl = rt_tiling(antennas_per_block, track_splits, block_threads, bins_per_segment,
                   tracks_per_pass)
    _check(_lib.rt_plan_set_tiling(plan, C.byref(tl)), "rt_plan_set_tiling")


def rt_plan_get_tiling(plan: int, n_tracks: int):
    """(antennas_per_block, track_splits, block_threads, bins_per_segment,
    tracks_per_pass) the plan uses for n_tracks tracks."""
    tl = rt_tiling()
    _check(_lib.rt_plan_get_tiling(plan, n_tracks, C.byref(tl)), "rt_plan_get_tiling")
    return tl.as_tuple()


def rt_plan_workspace_bytes(plan: int, n_tracks: int) -> int:
    b = C.c_size_t()
    _check(_lib.rt_plan_workspace_bytes(plan, n_tracks, C.byref(b)), "rt_plan_workspace_bytes")
    return b.value


def rt_accumulate(plan: int, tracks: rt_tracks, traces: torch.Tensor, workspace: torch.Tensor,
                  stream=None) -> None:
    _check(_lib.rt_accumulate(plan, C.byref(tracks), _ptr(traces), _ptr(workspace),
                              workspace.numel() * workspace.element_size(), _stream(stream)),
           "rt_accumulate")


def rt_accumulate_static(plan: int, tracks: rt_tracks, traces: torch.Tensor, stream=None) -> None:
    """rt_accumulate with the library's static device workspace (no
    allocation; calls overlapping in time on one device race)."""
    _check(_lib.rt_accumulate_static(plan, C.byref(tracks), _ptr(traces), _stream(stream)),
           "rt_accumulate_static")


def _event_handle(ev):
    if ev is None or isinstance(ev, int):
        return ev
    if not ev.cuda_event:   # torch creates events lazily: force creation
        ev.record()
    return ev.cuda_event


def rt_plan_set_timing_events(plan: int, start_event, stop_event) -> None:
    """start_event / stop_event: torch.cuda.Event (timing enabled) or raw
    hipEvent_t handles; None clears."""
    _check(_lib.rt_plan_set_timing_events(plan, _event_handle(start_event),
                                          _event_handle(stop_event)),
           "rt_plan_set_timing_events")


def rt_plan_set_n0m1_device(plan: int, n0m1: Optional[torch.Tensor]) -> None:
    """n0m1: a device float64 tensor of one element (kept alive by the
    caller while work reading it can run), or None for the plan's medium
    value."""
    if n0m1 is not None and (n0m1.dtype != torch.float64 or n0m1.numel() != 1
                             or not n0m1.is_cuda):
        raise ValueError("n0m1 must be a one-element float64 device tensor")
    _check(_lib.rt_plan_set_n0m1_device(plan, _ptr(n0m1)), "rt_plan_set_n0m1_device")


def rt_propagate(plan: int, tracks: rt_tracks, t_arrival: Optional[torch.Tensor],
                 bins: Optional[torch.Tensor], stream=None) -> None:
    _check(_lib.rt_propagate(plan, C.byref(tracks), _ptr(t_arrival), _ptr(bins), _stream(stream)),
           "rt_propagate")


def rt_plan_vjp_workspace_bytes(plan: int, n_tracks: int) -> int:
    b = C.c_size_t()
    _check(_lib.rt_plan_vjp_workspace_bytes(plan, n_tracks, C.byref(b)),
           "rt_plan_vjp_workspace_bytes")
    return b.value


def rt_zhs_vjp(plan: int, tracks: rt_tracks, grad_traces: torch.Tensor, grad_qw: torch.Tensor,
               grad_p0: torch.Tensor, grad_p1: torch.Tensor, grad_n0m1: torch.Tensor,
               workspace: torch.Tensor, stream=None) -> None:
    _check(_lib.rt_zhs_vjp(plan, C.byref(tracks), _ptr(grad_traces), _ptr(grad_qw), _ptr(grad_p0),
                           _ptr(grad_p1), _ptr(grad_n0m1), _ptr(workspace),
                           workspace.numel() * workspace.element_size(), _stream(stream)),
           "rt_zhs_vjp")


def rt_endpoint_vjp(plan: int, tracks: rt_tracks, grad_traces: torch.Tensor,
                    grad_qw: torch.Tensor, grad_p0: torch.Tensor, grad_p1: torch.Tensor,
                    grad_n0m1: torch.Tensor, workspace: torch.Tensor, stream=None) -> None:
    _check(_lib.rt_endpoint_vjp(plan, C.byref(tracks), _ptr(grad_traces), _ptr(grad_qw),
                                _ptr(grad_p0), _ptr(grad_p1), _ptr(grad_n0m1), _ptr(workspace),
                                workspace.numel() * workspace.element_size(), _stream(stream)),
           "rt_endpoint_vjp")


def rt_filter_workspace_bytes(n_tracks: int) -> int:
    b = C.c_size_t()
    _check(_lib.rt_filter_workspace_bytes(n_tracks, C.byref(b)), "rt_filter_workspace_bytes")
    return b.value


def rt_filter_tracks(tracks: rt_tracks, precision: int, qw_min: float, out: rt_tracks,
                     n_kept: torch.Tensor, workspace: torch.Tensor, stream=None) -> None:
    _check(_lib.rt_filter_tracks(C.byref(tracks), precision, qw_min, C.byref(out), _ptr(n_kept),
                                 _ptr(workspace), workspace.numel() * workspace.element_size(),
                                 _stream(stream)), "rt_filter_tracks")


def filter_tracks(tracks: "DeviceTracks", precision: str = "mixed", qw_min: float = 0.0,
                  stream=None) -> "DeviceTracks":
    """The tracks that can radiate (rt_filter_tracks), compacted in input
    order into new device tensors, on the current stream or on `stream` (a
    torch.cuda.Stream). Waits for that stream to read the count."""
    prec = PRECISION[precision]
    src = tracks.struct(prec)
    dev = tracks.x0.device
    out = DeviceTracks(**{f: torch.empty_like(getattr(tracks, f)) for f in _TRACK_FIELDS})
    n_kept = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(max(rt_filter_workspace_bytes(tracks.n), 256), dtype=torch.uint8, device=dev)
    if stream is not None:
        stream.wait_stream(torch.cuda.current_stream(dev))   # the new tensors are ready
        for t in [getattr(out, f) for f in _TRACK_FIELDS] + [n_kept, ws]:
            t.record_stream(stream)
    rt_filter_tracks(src, prec, float(qw_min), out.struct(prec), n_kept, ws, stream)
    if stream is not None:
        stream.synchronize()
    k = int(n_kept.item())
    return out.slice(0, k)


def rt_batch_create(showers, precision: int, k: float, options: Optional[rt_batch_options] = None
                    ) -> int:
    """showers: a sequence of rt_shower structs."""
    arr = (rt_shower * len(showers))(*showers)
    handle = _P()
    _check(_lib.rt_batch_create(C.byref(handle), arr, len(showers), precision, float(k),
                                C.byref(options) if options is not None else None),
           "rt_batch_create")
    return handle.value


def rt_batch_destroy(batch: int) -> None:
    _check(_lib.rt_batch_destroy(batch), "rt_batch_destroy")


def rt_batch_workspace_bytes(batch: int) -> int:
    b = C.c_size_t()
    _check(_lib.rt_batch_workspace_bytes(batch, C.byref(b)), "rt_batch_workspace_bytes")
    return b.value


def rt_batch_get_info(batch: int) -> dict:
    items, lds, pairs = C.c_int64(), C.c_int64(), C.c_int64()
    wgs = C.c_int32()
    _check(_lib.rt_batch_get_info(batch, C.byref(items), C.byref(wgs), C.byref(lds),
                                  C.byref(pairs)), "rt_batch_get_info")
    return {"items": items.value, "workgroups": wgs.value, "lds_bytes": lds.value,
            "pairs": pairs.value}


def rt_batch_launch(batch: int, workspace: Optional[torch.Tensor], stream=None) -> None:
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check(_lib.rt_batch_launch(batch, _ptr(workspace), nbytes, _stream(stream)),
           "rt_batch_launch")


def rt_batch_set_timing_events(batch: int, start_event, stop_event) -> None:
    _check(_lib.rt_batch_set_timing_events(batch, _event_handle(start_event),
                                           _event_handle(stop_event)),
           "rt_batch_set_timing_events")


# ------------------------------------------------------------------ convenience
class Plan:
    """A radio process for one detector, medium, formalism and precision
    (§4, Listing 2), with its own workspace per stream (calls on one stream
    run in order and share it; calls on different streams get their own)."""

    def __init__(self, det: DeviceDetector, medium, formalism: str = "endpoint",
                 precision: str = "fp64", k: float = 1.0):
        self.det = det
        self.medium = medium
        self.formalism = FORMALISM[formalism]
        self.precision = PRECISION[precision]
        self._table = _device_table(medium, det.x.device)
        self.handle = rt_plan_create(det, MEDIUM_KIND[medium.kind], float(medium.n0m1),
                                     float(medium.h), self.formalism, self.precision, k,
                                     self._table, float(getattr(medium, "z0", 0.0)),
                                     float(getattr(medium, "dz", 1.0)),
                                     float(getattr(medium, "earth_radius", 0.0)))
        self._ws = {}   # stream handle -> workspace
        self.dtype = torch.float64 if self.precision == RT_FP64 else torch.float32

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:   # module globals are cleared at interpreter exit
            _lib.rt_plan_destroy(h)
            self.handle = None

    def set_tiling(self, antennas_per_block=0, track_splits=0, block_threads=0,
                   bins_per_segment=0, tracks_per_pass=0):
        rt_plan_set_tiling(self.handle, antennas_per_block, track_splits, block_threads,
                           bins_per_segment, tracks_per_pass)

    def tiling(self, n_tracks: int):
        return rt_plan_get_tiling(self.handle, n_tracks)

    def workspace(self, n_tracks: int, stream=None) -> torch.Tensor:
        """The workspace of calls on ``stream`` (default: the current one),
        grown to what n_tracks tracks need (allocated from that stream's
        memory pool, so that a replaced workspace is reused only after the
        stream's work on it)."""
        need = rt_plan_workspace_bytes(self.handle, n_tracks)
        key = _stream(stream)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < need:
            with _on_stream(stream):
                ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.det.x.device)
            self._ws[key] = ws
        return ws

    def set_n0m1_device(self, n0m1: Optional[torch.Tensor]) -> None:
        """Read n0 - 1 from a one-element float64 device tensor in every
        later call (rt_plan_set_n0m1_device); None returns to the medium's
        value. The plan keeps a reference to the tensor."""
        rt_plan_set_n0m1_device(self.handle, n0m1)
        self._n0m1_dev = n0m1

    def new_traces(self) -> torch.Tensor:
        return torch.zeros((self.det.m, self.det.n_bins, 3), dtype=self.dtype,
                           device=self.det.x.device)

    def accumulate(self, tracks: DeviceTracks, traces: torch.Tensor, stream=None) -> torch.Tensor:
        """traces += this plan's contribution of the tracks, on ``stream``
        (default: the current one). With another torch.cuda.Stream, that
        stream first waits for the current one."""
        if traces.dtype != self.dtype or not traces.is_contiguous() or \
                tuple(traces.shape) != (self.det.m, self.det.n_bins, 3):
            raise ValueError("traces must be a contiguous [M, n_bins, 3] tensor of the plan dtype")
        ws = self.workspace(tracks.n, stream)
        with _on_stream(stream):
            rt_accumulate(self.handle, tracks.struct(self.precision), traces, ws, stream)
        return traces

    def traces(self, tracks: DeviceTracks, stream=None) -> torch.Tensor:
        """New traces of the tracks, allocated and zeroed on ``stream``."""
        with _on_stream(stream):
            out = self.new_traces()
        return self.accumulate(tracks, out, stream)

    def zhs_vjp(self, tracks: DeviceTracks, grad_traces: torch.Tensor, stream=None):
        """Gradients (qw [n], p0 [3, n], p1 [3, n], n0m1 [1]) of sum(grad * A),
        all float64, for a ZHS plan."""
        if self.formalism != RT_ZHS:
            raise ValueError("zhs_vjp needs a ZHS plan")
        return self.vjp(tracks, grad_traces, stream)

    def endpoint_vjp(self, tracks: DeviceTracks, grad_traces: torch.Tensor, stream=None):
        """Gradients (qw [n], p0 [3, n], p1 [3, n], n0m1 [1]) of sum(grad * E),
        all float64, for an Endpoint plan (landing bins held fixed)."""
        if self.formalism != RT_ENDPOINT:
            raise ValueError("endpoint_vjp needs an Endpoint plan")
        return self.vjp(tracks, grad_traces, stream)

    def vjp(self, tracks: DeviceTracks, grad_traces: torch.Tensor, stream=None):
        """The vector-Jacobian product of the plan's formalism, on ``stream``
        (default: the current one; with another torch.cuda.Stream the
        outputs belong to that stream, which first waits for the current
        one)."""
        dev = self.det.x.device
        n = tracks.n
        with _on_stream(stream):
            g = grad_traces.to(self.dtype).contiguous()
            if tuple(g.shape) != (self.det.m, self.det.n_bins, 3):
                raise ValueError("grad_traces must be [M, n_bins, 3]")
            gq = torch.empty(n, dtype=torch.float64, device=dev)
            gp0 = torch.empty((3, n), dtype=torch.float64, device=dev)
            gp1 = torch.empty((3, n), dtype=torch.float64, device=dev)
            gn = torch.empty(1, dtype=torch.float64, device=dev)
            ws = torch.empty(max(rt_plan_vjp_workspace_bytes(self.handle, n), 256),
                             dtype=torch.uint8, device=dev)
            fn = rt_zhs_vjp if self.formalism == RT_ZHS else rt_endpoint_vjp
            fn(self.handle, tracks.struct(self.precision), g, gq, gp0, gp1, gn, ws, stream)
        return gq, gp0, gp1, gn

    def propagate(self, tracks: DeviceTracks, stream=None):
        shape = (2, tracks.n, self.det.m)
        with _on_stream(stream):
            t = torch.empty(shape, dtype=torch.float64, device=self.det.x.device)
            b = torch.empty(shape, dtype=torch.int32, device=self.det.x.device)
            rt_propagate(self.handle, tracks.struct(self.precision), t, b, stream)
        return t, b


def _device_table(medium, device) -> Optional[torch.Tensor]:
    if medium.kind != "tabulated":
        return None
    return torch.tensor(medium.table, dtype=torch.float64, device=device)


def _medium_struct(medium, table: Optional[torch.Tensor] = None) -> rt_medium:
    return rt_medium(MEDIUM_KIND[medium.kind], float(medium.n0m1), float(medium.h), _ptr(table),
                     0 if table is None else table.numel(), float(getattr(medium, "z0", 0.0)),
                     float(getattr(medium, "dz", 1.0)), float(getattr(medium, "earth_radius", 0.0)))


@dataclass
class BatchOptions:
    """Launch shape of a batch (rt_batch_options); 0 keeps the automatic
    choice. block_threads 1024 (with max_antennas_per_tile 1) runs one-antenna
    tiles in one kernel per formalism. per_shower: None or a list of
    (antennas_per_block, track_splits, bins_per_segment) per shower."""
    block_threads: int = 0
    items_per_cu: int = 0
    max_antennas_per_tile: int = 0
    direct_launch: int = 0
    per_shower: Optional[list] = None

    def struct(self):
        o = rt_batch_options(self.block_threads, self.items_per_cu, self.max_antennas_per_tile,
                             self.direct_launch, None)
        keep = None
        if self.per_shower is not None:
            keep = (rt_tiling * len(self.per_shower))(
                *[rt_tiling(a, s, 0, b, 0) for a, s, b in self.per_shower])
            o.per_shower = C.cast(keep, C.POINTER(rt_tiling))
        return o, keep


def rt_plan_autotune(plan: "Plan", tracks: "DeviceTracks", tilings, reps: int = 2,
                  stream=None):
    """rt_plan_autotune: times each tiling (tuples of the five rt_tiling
    fields) on the tracks; returns the median seconds per candidate (None for
    a skipped one) and leaves the fastest tiling set on the plan. Allocates
    one workspace for the largest candidate and a scratch trace tensor."""
    cands = (rt_tiling * len(tilings))(*[rt_tiling(*map(int, t)) for t in tilings])
    need = 0
    for t in cands:   # the workspace of the largest candidate
        if _lib.rt_plan_set_tiling(plan.handle, C.byref(t)) == RT_OK:
            need = max(need, rt_plan_workspace_bytes(plan.handle, tracks.n))
    dev = plan.det.x.device
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    scratch = plan.new_traces()
    ms = (C.c_float * len(tilings))()
    best = C.c_int32(-1)
    _check(_lib.rt_plan_autotune(plan.handle, C.byref(tracks.struct(plan.precision)),
                                 _ptr(scratch), _ptr(ws), ws.numel(), cands, len(tilings),
                                 int(reps), _stream(stream), ms, C.byref(best)),
           "rt_plan_autotune")
    return [m * 1e-3 if m >= 0 else None for m in ms]


def _shower_structs(showers, precision: int, traces=None):
    """rt_shower structures for (DeviceDetector, medium, formalism name,
    DeviceTracks) tuples, with new zeroed traces unless given; returns the
    structures and the tensors they point into (keep them alive)."""
    dtype = torch.float64 if precision == RT_FP64 else torch.float32
    structs, keep, out = [], [], []
    for i, (det, medium, formalism, tracks) in enumerate(showers):
        tr = traces[i] if traces is not None else torch.zeros(
            (det.m, det.n_bins, 3), dtype=dtype, device=det.x.device)
        table = _device_table(medium, det.x.device)
        out.append(tr)
        keep.append(table)
        structs.append(rt_shower(det.struct(), _medium_struct(medium, table),
                                 FORMALISM[formalism], tracks.struct(precision), _ptr(tr)))
    return structs, keep, out


def rt_batch_autotune(showers, precision: str, k: float, options, reps: int = 2, stream=None):
    """rt_batch_autotune: times a whole launch of the showers with each
    BatchOptions; returns the median seconds per candidate (None for a
    skipped one). The traces are scratch tensors of this call."""
    prec = PRECISION[precision]
    structs, keep, traces = _shower_structs(showers, prec)
    arr = (rt_shower * len(structs))(*structs)
    opts, keeps = zip(*[o.struct() for o in options])
    oarr = (rt_batch_options * len(opts))(*opts)
    need = 0
    for o in opts:   # the workspace of the largest candidate (host planning only)
        h = _P()
        if _lib.rt_batch_create(C.byref(h), arr, len(structs), prec, float(k), C.byref(o)) == RT_OK:
            n = C.c_size_t(0)
            _lib.rt_batch_workspace_bytes(h, C.byref(n))
            need = max(need, n.value)
            _lib.rt_batch_destroy(h)
    dev = traces[0].device if traces else "cuda"
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    ms = (C.c_float * len(opts))()
    best = C.c_int32(-1)
    _check(_lib.rt_batch_autotune(arr, len(structs), prec, float(k), oarr, len(opts), _ptr(ws),
                                  ws.numel(), int(reps), _stream(stream), ms, C.byref(best)),
           "rt_batch_autotune")
    del keeps, keep
    return [m * 1e-3 if m >= 0 else None for m in ms]


class Batch:
    """Many showers in one persistent launch (rt_batch_*). showers: a list of
    (DeviceDetector, medium, formalism name, DeviceTracks). The batch owns one
    trace tensor per shower (zeroed at construction; launches add to them) and
    its workspace; it keeps references to every input tensor."""

    def __init__(self, showers, precision: str = "mixed", k: float = 1.0,
                 options: Optional[BatchOptions] = None):
        self.precision = PRECISION[precision]
        self.dtype = torch.float64 if self.precision == RT_FP64 else torch.float32
        self.inputs = list(showers)
        self.options = options or BatchOptions()
        structs, self._tables, self.traces = _shower_structs(self.inputs, self.precision)
        opt, keep = self.options.struct()
        self.handle = rt_batch_create(structs, self.precision, k, opt)
        self.info = rt_batch_get_info(self.handle)
        need = rt_batch_workspace_bytes(self.handle)
        device = self.traces[0].device if self.traces else "cuda"
        self.workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=device)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:   # module globals are cleared at interpreter exit
            _lib.rt_batch_destroy(h)
            self.handle = None

    @property
    def pairs(self) -> int:
        return self.info["pairs"]

    def zero_traces(self):
        for t in self.traces:
            t.zero_()

    def launch(self, stream=None):
        rt_batch_launch(self.handle, self.workspace, stream)
        return self.traces

    def set_timing_events(self, start_event, stop_event):
        rt_batch_set_timing_events(self.handle, start_event, stop_event)
