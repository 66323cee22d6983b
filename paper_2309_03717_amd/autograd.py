"""Differentiable traces: a torch.autograd.Function whose forward is the
library's deposit (ZHS or Endpoint) and whose backward is the matching
hand-written adjoint (rt_zhs_vjp, rt_endpoint_vjp). Differentiable inputs:
per-track weights qw [n], start points p0 [3, n], end points p1 [3, n] and
the refractivity n0 - 1 (0-d tensor); the emission times, the velocities, the
antenna array and the shape of the medium (scale height, table, Earth radius)
are held fixed (and, for the Endpoint formalism, the bins the impulses land
in). Every medium is differentiable.
"""
from __future__ import annotations

import dataclasses

import torch

from . import radtrace as rt
from .workloads import Medium


# One plan per (detector, medium shape, formalism, precision, k), kept on the
# detector object (so it lives as long as the detector): n0 - 1 reaches the
# kernels from device memory (rt_plan_set_n0m1_device), so neither a host copy
# of it nor a new plan is needed per call.
def _plan(det, medium, formalism, precision, k):
    shape = dataclasses.replace(medium, n0m1=0.0)
    key = (repr(shape), formalism, precision, float(k))
    plans = det.__dict__.setdefault("_autograd_plans", {})
    plan = plans.get(key)
    if plan is None:
        plan = plans[key] = rt.Plan(det, shape, formalism, precision, k)
    return plan


class RadioTraces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, qw, p0, p1, n0m1, t0, t1, beta, det, formalism, medium, precision, k):
        plan = _plan(det, medium, formalism, precision, k)
        n0 = n0m1.detach().to(device=det.x.device, dtype=torch.float64).reshape(1).contiguous()
        plan.set_n0m1_device(n0)
        in_dtype = torch.float64 if precision == "fp64" else torch.float32
        tracks = rt.DeviceTracks(
            x0=p0[0].detach().double().contiguous(), y0=p0[1].detach().double().contiguous(),
            z0=p0[2].detach().double().contiguous(), t0=t0.double().contiguous(),
            x1=p1[0].detach().double().contiguous(), y1=p1[1].detach().double().contiguous(),
            z1=p1[2].detach().double().contiguous(), t1=t1.double().contiguous(),
            bx=beta[0].to(in_dtype).contiguous(), by=beta[1].to(in_dtype).contiguous(),
            bz=beta[2].to(in_dtype).contiguous(), qw=qw.detach().to(in_dtype).contiguous())
        traces = plan.traces(tracks)
        ctx.plan, ctx.tracks, ctx.n0 = plan, tracks, n0
        ctx.dtypes = (qw.dtype, p0.dtype, p1.dtype, n0m1.dtype)
        return traces

    @staticmethod
    def backward(ctx, grad):
        # the plan is shared: point it at this forward's n0 - 1 again
        ctx.plan.set_n0m1_device(ctx.n0)
        gq, gp0, gp1, gn = ctx.plan.vjp(ctx.tracks, grad)
        dq, d0, d1, dn = ctx.dtypes
        return (gq.to(dq), gp0.to(d0), gp1.to(d1), gn.reshape(()).to(dn),
                None, None, None, None, None, None, None, None)


# kept for callers of the ZHS-only name
ZHSTraces = RadioTraces


def radio_traces(formalism: str, qw, p0, p1, n0m1, *, t0, t1, beta, det: rt.DeviceDetector,
                 medium_kind: str = "exponential", scale_height: float = 8000.0,
                 medium: Medium | None = None, precision: str = "mixed", k: float = 1.0):
    """Traces [M, n_bins, 3] of the given tracks in the given formalism
    ("zhs" or "endpoint"), differentiable in qw, p0, p1 and n0m1. The medium is
    ``medium`` (any kind; its own n0m1 is replaced by the n0m1 tensor, which
    the kernels read from device memory: no host synchronisation) or, if that
    is None, the uniform or exponential profile named by medium_kind."""
    if medium is None:
        medium = Medium(medium_kind, 0.0, float(scale_height))
    return RadioTraces.apply(qw, p0, p1, n0m1, t0, t1, beta, det, formalism, medium, precision, k)


def zhs_traces(qw, p0, p1, n0m1, **kw):
    """ZHS traces, differentiable in qw, p0, p1 and n0m1."""
    return radio_traces("zhs", qw, p0, p1, n0m1, **kw)


def endpoint_traces(qw, p0, p1, n0m1, **kw):
    """Endpoint traces, differentiable in qw, p0, p1 and n0m1 (bins fixed)."""
    return radio_traces("endpoint", qw, p0, p1, n0m1, **kw)
