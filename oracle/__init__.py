"""FP64 CPU oracle of the radio-emission loop (ctypes wrapper of radio_oracle.c).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline may import this package. The product (``paper_2309_03717_amd``)
never imports it, and the two share no code.

Inputs are the numpy containers of ``paper_2309_03717_amd.workloads`` (which
hold no emission arithmetic); float32 fields are widened to float64 here.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "radio_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-pthread",
          "-std=c11", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile radio_oracle.c with gcc into oracle/liborc.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Tracks(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(f, C.POINTER(C.c_double)) for f in
                                     ("x0", "y0", "z0", "t0", "x1", "y1", "z1", "t1",
                                      "bx", "by", "bz", "qw")]


class _Antennas(C.Structure):
    _fields_ = [("m", C.c_int64), ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)),
                ("z", C.POINTER(C.c_double)), ("t_start", C.POINTER(C.c_double)),
                ("dt", C.c_double), ("n_bins", C.c_int32)]


class _Medium(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n0m1", C.c_double), ("h", C.c_double),
                ("f", C.POINTER(C.c_double)), ("n_f", C.c_int32), ("z0", C.c_double),
                ("dz", C.c_double), ("re", C.c_double)]


_lib = None
ORC_VERSION = 2   # the structure layouts above


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        lib.orc_traces.argtypes = [C.c_int, C.POINTER(_Tracks), C.POINTER(_Antennas),
                                   C.POINTER(_Medium), C.c_double, dp, C.c_int, C.c_int64]
        lib.orc_propagate.argtypes = [C.POINTER(_Tracks), C.POINTER(_Antennas), C.POINTER(_Medium),
                                      dp, dp, C.POINTER(C.c_int32)]
        lib.orc_zhs_vjp.argtypes = [C.POINTER(_Tracks), C.POINTER(_Antennas), C.POINTER(_Medium),
                                    C.c_double, dp, dp, dp, dp, dp, C.c_int]
        lib.orc_endpoint_vjp.argtypes = lib.orc_zhs_vjp.argtypes
        lib.orc_version.restype = C.c_int
        lib.orc_gl_rule.argtypes = [dp, dp]
        if lib.orc_version() != ORC_VERSION:
            raise ImportError(f"{_LIB} is stale (version {lib.orc_version()}); rebuild the oracle")
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class _Args:
    """Keeps the float64 copies alive while the C call runs."""

    def __init__(self, tracks, array, medium):
        self.keep = []
        t = {f: _f64(getattr(tracks, f)) for f in _Tracks._fields_names()}
        self.keep += list(t.values())
        self.tr = _Tracks(tracks.n, *[_dp(t[f]) for f in _Tracks._fields_names()])
        a = [_f64(array.x), _f64(array.y), _f64(array.z), _f64(array.t_start)]
        self.keep += a
        self.ar = _Antennas(array.m, *[_dp(v) for v in a], float(array.dt), int(array.n_bins))
        if medium.kind == "tabulated":
            f = _f64(np.asarray(medium.table, dtype=np.float64))
            self.keep.append(f)
            self.md = _Medium(medium.code, float(medium.n0m1), float(medium.h), _dp(f), f.size,
                              float(medium.z0), float(medium.dz), 0.0)
        else:
            self.md = _Medium(medium.code, float(medium.n0m1), float(medium.h), None, 0, 0.0, 1.0,
                              float(getattr(medium, "earth_radius", 0.0)))


_Tracks._fields_names = staticmethod(lambda: [f for f, _ in _Tracks._fields_[1:]])

FORMALISMS = {"endpoint": 0, "zhs": 1}


def traces(formalism: str, tracks, array, medium, k: float = 1.0, n_threads: int = 1,
           bunch: int = 0, out: Optional[np.ndarray] = None) -> np.ndarray:
    """Traces [m, n_bins, 3] float64 of every (track, antenna) pair, added to
    ``out`` if given (else to zeros)."""
    lib = _load()
    args = _Args(tracks, array, medium)
    if out is None:
        out = np.zeros((array.m, array.n_bins, 3), dtype=np.float64)
    assert out.dtype == np.float64 and out.flags.c_contiguous
    assert out.shape == (array.m, array.n_bins, 3)
    rc = lib.orc_traces(FORMALISMS[formalism], C.byref(args.tr), C.byref(args.ar),
                        C.byref(args.md), float(k), _dp(out), int(n_threads), int(bunch))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return out


def gl_rule():
    """Nodes (ascending, on [0, 1]) and weights of the quadrature rule the
    spherical-Earth path mean uses."""
    lib = _load()
    s, w = np.zeros(16), np.zeros(16)
    n = lib.orc_gl_rule(_dp(s), _dp(w))
    return s[:n].copy(), w[:n].copy()


def propagate(tracks, array, medium):
    """Arrival time t, window coordinate u and bin (-1 outside) for every
    (end, track, antenna): arrays of shape [2, n, m]."""
    lib = _load()
    args = _Args(tracks, array, medium)
    shape = (2, tracks.n, array.m)
    t = np.empty(shape, np.float64)
    u = np.empty(shape, np.float64)
    b = np.empty(shape, np.int32)
    rc = lib.orc_propagate(C.byref(args.tr), C.byref(args.ar), C.byref(args.md), _dp(t), _dp(u),
                           b.ctypes.data_as(C.POINTER(C.c_int32)))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return t, u, b


def zhs_vjp(tracks, array, medium, grad: np.ndarray, k: float = 1.0, n_threads: int = 1):
    """Gradients of sum(grad * A_zhs) with respect to qw [n], p0 [3, n],
    p1 [3, n] and n0m1 (scalar), with beta and the emission times fixed."""
    return _vjp("orc_zhs_vjp", tracks, array, medium, grad, k, n_threads)


def endpoint_vjp(tracks, array, medium, grad: np.ndarray, k: float = 1.0, n_threads: int = 1):
    """Gradients of sum(grad * E_endpoint) with respect to qw [n], p0 [3, n],
    p1 [3, n] and n0m1 (scalar), with beta, the emission times and the bins the
    impulses land in held fixed."""
    return _vjp("orc_endpoint_vjp", tracks, array, medium, grad, k, n_threads)


def _vjp(name, tracks, array, medium, grad, k, n_threads):
    lib = _load()
    args = _Args(tracks, array, medium)
    g = _f64(grad)
    assert g.shape == (array.m, array.n_bins, 3)
    n = tracks.n
    gq = np.zeros(n)
    gp0 = np.zeros((3, n))
    gp1 = np.zeros((3, n))
    gn = np.zeros(1)
    rc = getattr(lib, name)(C.byref(args.tr), C.byref(args.ar), C.byref(args.md), float(k),
                            _dp(g), _dp(gq), _dp(gp0), _dp(gp1), _dp(gn), int(n_threads))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return {"qw": gq, "p0": gp0, "p1": gp1, "n0m1": float(gn[0])}
