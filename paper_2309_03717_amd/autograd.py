"""Differentiable ZHS traces: a torch.autograd.Function whose forward is the
library's ZHS deposit and whose backward is its hand-written adjoint
(rt_zhs_vjp). Differentiable inputs: per-track weights qw [n], start points
p0 [3, n], end points p1 [3, n] and the refractivity n0 - 1 (0-d tensor);
the emission times, the velocities and the antenna array are held fixed.
"""
from __future__ import annotations

import torch

from . import radtrace as rt
from .workloads import Medium


class ZHSTraces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, qw, p0, p1, n0m1, t0, t1, beta, det, medium_kind, scale_height, precision, k):
        medium = Medium(medium_kind, float(n0m1.detach().cpu()), float(scale_height))
        plan = rt.Plan(det, medium, "zhs", precision, k)
        in_dtype = torch.float64 if precision == "fp64" else torch.float32
        tracks = rt.DeviceTracks(
            x0=p0[0].detach().double().contiguous(), y0=p0[1].detach().double().contiguous(),
            z0=p0[2].detach().double().contiguous(), t0=t0.double().contiguous(),
            x1=p1[0].detach().double().contiguous(), y1=p1[1].detach().double().contiguous(),
            z1=p1[2].detach().double().contiguous(), t1=t1.double().contiguous(),
            bx=beta[0].to(in_dtype).contiguous(), by=beta[1].to(in_dtype).contiguous(),
            bz=beta[2].to(in_dtype).contiguous(), qw=qw.detach().to(in_dtype).contiguous())
        traces = plan.traces(tracks)
        ctx.plan, ctx.tracks = plan, tracks
        ctx.dtypes = (qw.dtype, p0.dtype, p1.dtype, n0m1.dtype)
        return traces

    @staticmethod
    def backward(ctx, grad):
        gq, gp0, gp1, gn = ctx.plan.zhs_vjp(ctx.tracks, grad)
        dq, d0, d1, dn = ctx.dtypes
        return (gq.to(dq), gp0.to(d0), gp1.to(d1), gn.reshape(()).to(dn),
                None, None, None, None, None, None, None, None)


def zhs_traces(qw, p0, p1, n0m1, *, t0, t1, beta, det: rt.DeviceDetector, medium_kind: str,
               scale_height: float = 8000.0, precision: str = "mixed", k: float = 1.0):
    """ZHS traces [M, n_bins, 3] of the given tracks, differentiable in qw,
    p0, p1 and n0m1."""
    return ZHSTraces.apply(qw, p0, p1, n0m1, t0, t1, beta, det, medium_kind, scale_height,
                           precision, k)
