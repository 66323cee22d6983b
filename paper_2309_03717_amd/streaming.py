"""Host-resident track streams.

In the radio module every track the cascade produces on the CPU goes to the
radio process, which loops over the antennas (Section 2, Fig. 1). Here the
tracks arrive in chunks instead of one at a time: ``HostTrackStream`` takes
chunks that live in pinned host memory, copies each one to the device on a
copy stream of its own while the previous chunk deposits, two device buffers
alternating, and runs every given plan on each chunk (Endpoint and ZHS can
share the copy). The deposits are the
library's (``Plan.accumulate``); the copies are plain DMA transfers.

With a threshold ``qw_min`` the stream also runs the track filter (the check
a track passes before the antenna loop, Section 2) on each copied chunk and
deposits only the kept tracks. The kept count lives in device memory; rather
than wait for it right after each filter, a chunk's deposits are enqueued at
the next push (or at ``flush``), by which time its filter has long finished:
the host waits only for that filter, while the deposits enqueued before it
keep the GPU busy.
"""
from __future__ import annotations

import math
from typing import Dict, Optional, Sequence

import torch

from . import radtrace as rt
from .workloads import TRACK_FIELDS


class HostTrackStream:
    """Double-buffered host-to-device track stream for one or more plans on
    the same device and precision.

    push(chunk, traces): ``chunk`` maps every track field name (x0, y0, z0, t0,
    x1, y1, z1, t1, bx, by, bz, qw) to a pinned host tensor of n <= max_chunk
    elements (positions and times float64; velocities and weights float64 for
    FP64 plans, float32 for mixed ones); ``traces`` holds one trace tensor per
    plan, to which the chunk's traces are added. The deposits are enqueued on
    the current stream (the caller orders that stream after any other stream
    that uses the same trace tensors), the copy on the object's copy stream,
    and push returns at once: the caller leaves each pushed host chunk unchanged until
    ``synchronize`` returns (dropping the tensors early is safe: torch's pinned
    allocator reuses a block only after the copies that read it).

    qw_min (None: no filter): filter each chunk with rt_filter_tracks at this
    threshold and deposit only the kept tracks. A chunk's deposits still go on
    the stream current at its push, but they are enqueued one push later, or
    by ``flush``/``synchronize``: call ``flush`` before another stream waits
    for the traces. ``kept`` counts the tracks deposited so far.

    The device buffers are read on streams the allocator does not track, so
    call ``synchronize`` before dropping the object, or use it as a context
    manager, whose exit does.
    """

    def __init__(self, plans: Sequence["rt.Plan"], max_chunk: int,
                 qw_min: Optional[float] = None):
        if not plans:
            raise ValueError("need at least one plan")
        if max_chunk < 1:
            raise ValueError("max_chunk must be >= 1")
        if qw_min is not None and not (math.isfinite(qw_min) and qw_min >= 0):
            raise ValueError("qw_min must be finite and >= 0")
        precisions = {p.precision for p in plans}
        if len(precisions) != 1:
            raise ValueError("the plans of one stream share one precision")
        self.plans = list(plans)
        self.max_chunk = int(max_chunk)
        self.device = plans[0].det.x.device
        low = torch.float64 if plans[0].precision == rt.RT_FP64 else torch.float32
        self.dtypes = {f: (low if f in ("bx", "by", "bz", "qw") else torch.float64)
                       for f in TRACK_FIELDS}
        self.buffers = [{f: torch.empty(self.max_chunk, dtype=self.dtypes[f], device=self.device)
                         for f in TRACK_FIELDS} for _ in range(2)]
        self.copy_stream = torch.cuda.Stream(self.device)
        for buf in self.buffers:
            for t in buf.values():
                t.record_stream(self.copy_stream)
        self.copied = [torch.cuda.Event() for _ in range(2)]
        self.done = [torch.cuda.Event() for _ in range(2)]
        self.pushed = 0
        self.qw_min = None if qw_min is None else float(qw_min)
        self.kept = 0
        self.pending = None   # (slot, traces, stream) of a filtered chunk not yet deposited
        if self.qw_min is not None:
            self.prec = plans[0].precision
            # per slot: the compacted tracks, the kept count (device and pinned
            # host copies) and the filter's workspace
            self.compact = [{f: torch.empty(self.max_chunk, dtype=self.dtypes[f],
                                            device=self.device) for f in TRACK_FIELDS}
                            for _ in range(2)]
            self.count_dev = [torch.zeros(1, dtype=torch.int64, device=self.device)
                              for _ in range(2)]
            self.count_host = [torch.zeros(1, dtype=torch.int64).pin_memory() for _ in range(2)]
            wsb = max(rt.rt_filter_workspace_bytes(self.max_chunk), 256)
            self.filter_ws = [torch.empty(wsb, dtype=torch.uint8, device=self.device)
                              for _ in range(2)]
            self.filtered = [torch.cuda.Event() for _ in range(2)]
            self.deposited = [torch.cuda.Event() for _ in range(2)]

    def push(self, chunk: Dict[str, torch.Tensor], traces: Sequence[torch.Tensor]) -> None:
        if len(traces) != len(self.plans):
            raise ValueError("one trace tensor per plan")
        n = None
        for f in TRACK_FIELDS:
            t = chunk.get(f)
            if t is None:
                raise ValueError(f"chunk lacks the field {f}")
            if t.device.type != "cpu" or not t.is_pinned():
                raise ValueError(f"field {f} must be a pinned host tensor")
            if t.dtype != self.dtypes[f] or t.dim() != 1 or not t.is_contiguous():
                raise ValueError(f"field {f} must be a contiguous 1-d {self.dtypes[f]} tensor")
            if n is None:
                n = t.numel()
            elif t.numel() != n:
                raise ValueError("every field of a chunk has the same length")
        if n > self.max_chunk:
            raise ValueError(f"chunk of {n} tracks exceeds max_chunk {self.max_chunk}")
        if n == 0:
            return
        b = self.pushed % 2
        self.pushed += 1
        compute = torch.cuda.current_stream(self.device)
        # the buffer is free once the chunk before last has been read from it
        # (by its deposits, or by its filter)
        self.copy_stream.wait_event(self.done[b])
        with torch.cuda.stream(self.copy_stream):
            for f in TRACK_FIELDS:
                self.buffers[b][f][:n].copy_(chunk[f], non_blocking=True)
        self.copied[b].record(self.copy_stream)
        compute.wait_event(self.copied[b])
        dev = rt.DeviceTracks(**{f: self.buffers[b][f][:n] for f in TRACK_FIELDS})
        if self.qw_min is None:
            for plan, tr in zip(self.plans, traces):
                plan.accumulate(dev, tr)
            self.done[b].record(compute)
            self.kept += n
            return
        # the compacted slot is free once the deposits of the chunk before
        # last are done (they may have run on another stream)
        compute.wait_event(self.deposited[b])
        out = rt.DeviceTracks(**{f: self.compact[b][f][:n] for f in TRACK_FIELDS})
        rt.rt_filter_tracks(dev.struct(self.prec), self.prec, self.qw_min, out.struct(self.prec),
                            self.count_dev[b], self.filter_ws[b], compute)
        self.done[b].record(compute)
        self.count_host[b].copy_(self.count_dev[b], non_blocking=True)
        self.filtered[b].record(compute)
        self.flush()
        self.pending = (b, list(traces), compute)

    def flush(self) -> None:
        """Enqueues the deposits of a filtered chunk still waiting for them,
        on the stream of its push (no-op without a filter). Waits on the host
        for that chunk's filter only."""
        if self.pending is None:
            return
        b, traces, stream = self.pending
        self.pending = None
        self.filtered[b].synchronize()   # the kept count is in host memory
        k = int(self.count_host[b][0])
        self.kept += k
        if k > 0:
            kept = rt.DeviceTracks(**{f: self.compact[b][f][:k] for f in TRACK_FIELDS})
            with torch.cuda.stream(stream):
                for plan, tr in zip(self.plans, traces):
                    plan.accumulate(kept, tr)
        self.deposited[b].record(stream)

    def __enter__(self) -> "HostTrackStream":
        return self

    def __exit__(self, *exc) -> None:
        self.synchronize()

    def synchronize(self) -> None:
        """Flushes, then waits for every push so far; the host chunks are free
        again and the traces complete."""
        self.flush()
        for ev in self.done:
            ev.synchronize()
        if self.qw_min is not None:
            for ev in self.deposited:
                ev.synchronize()
        self.copy_stream.synchronize()


def pinned_chunk(tracks) -> Dict[str, torch.Tensor]:
    """The fields of a host Tracks container as pinned tensors (new pinned
    allocations holding a copy)."""
    return {f: torch.from_numpy(getattr(tracks, f)).pin_memory() for f in TRACK_FIELDS}
