"""Host-resident track streams.

In the radio module every track the cascade produces on the CPU goes to the
radio process, which loops over the antennas (Section 2, Fig. 1). Here the
tracks arrive in chunks instead of one at a time: ``HostTrackStream`` takes
chunks that live in pinned host memory, copies each one to the device on a
copy stream of its own while the previous chunk deposits, two device buffers
alternating, and runs every given plan on each chunk (Endpoint and ZHS can
share the copy). The deposits are the
library's (``Plan.accumulate``); the copies are plain DMA transfers.
"""
from __future__ import annotations

from typing import Dict, Sequence

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
    """

    def __init__(self, plans: Sequence["rt.Plan"], max_chunk: int):
        if not plans:
            raise ValueError("need at least one plan")
        if max_chunk < 1:
            raise ValueError("max_chunk must be >= 1")
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
        # the buffer is free once the deposits of the chunk before last are done
        self.copy_stream.wait_event(self.done[b])
        with torch.cuda.stream(self.copy_stream):
            for f in TRACK_FIELDS:
                self.buffers[b][f][:n].copy_(chunk[f], non_blocking=True)
        self.copied[b].record(self.copy_stream)
        compute.wait_event(self.copied[b])
        dev = rt.DeviceTracks(**{f: self.buffers[b][f][:n] for f in TRACK_FIELDS})
        for plan, tr in zip(self.plans, traces):
            plan.accumulate(dev, tr)
        self.done[b].record(compute)

    def synchronize(self) -> None:
        """Waits for every push so far; the host chunks are free again."""
        for ev in self.done:
            ev.synchronize()
        self.copy_stream.synchronize()


def pinned_chunk(tracks) -> Dict[str, torch.Tensor]:
    """The fields of a host Tracks container as pinned tensors (new pinned
    allocations holding a copy)."""
    return {f: torch.from_numpy(getattr(tracks, f)).pin_memory() for f in TRACK_FIELDS}
