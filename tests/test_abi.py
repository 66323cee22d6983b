"""The C ABI without a GPU: the library loads, exports every function that
include/radtrace.h declares, and rejects invalid arguments before touching a
device (or reports that there is none)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "radtrace.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(rt_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def rt():
    from paper_2309_03717_amd import radtrace
    return radtrace


def test_header_lists_the_entry_points():
    names = declared_functions()
    for n in ("rt_plan_create", "rt_accumulate", "rt_propagate", "rt_plan_workspace_bytes"):
        assert n in names


def test_library_exports_every_declared_symbol(rt):
    lib = C.CDLL(rt.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_python_binding_has_the_same_names(rt):
    for n in declared_functions():
        assert callable(getattr(rt, n, None)), n


def test_version_and_status_strings(rt):
    assert rt.rt_abi_version() == 1
    assert rt.rt_status_string(rt.RT_OK) == "ok"
    assert "workspace" in rt.rt_status_string(rt.RT_E_WORKSPACE)
    assert rt.rt_status_string(99) == "unknown status"


def _detector(rt, n=4, dt=1e-10, n_bins=64, null=False):
    import numpy as np
    buf = (C.c_double * n)()
    p = None if null else C.addressof(buf)
    return rt.rt_detector(n, p, p, p, p, dt, n_bins), buf


@pytest.mark.parametrize("case", ["no_antennas", "bad_dt", "bad_bins", "null_ptr", "bad_formalism",
                                  "bad_precision", "bad_medium", "negative_refractivity",
                                  "bad_height", "nan_k"])
def test_plan_create_rejects_invalid_arguments(rt, case):
    det, keep = _detector(rt)
    med = rt.rt_medium(rt.RT_EXPONENTIAL, 2.92e-4, 8000.0)
    formalism, precision, k = rt.RT_ENDPOINT, rt.RT_FP64, 1.0
    if case == "no_antennas":
        det.n_antennas = 0
    elif case == "bad_dt":
        det.dt = 0.0
    elif case == "bad_bins":
        det.n_bins = 0
    elif case == "null_ptr":
        det.t_start = None
    elif case == "bad_formalism":
        formalism = 7
    elif case == "bad_precision":
        precision = 3
    elif case == "bad_medium":
        med.kind = 5
    elif case == "negative_refractivity":
        med.n0_minus_1 = -1e-4
    elif case == "bad_height":
        med.scale_height = 0.0
    elif case == "nan_k":
        k = float("nan")
    handle = C.c_void_p()
    st = rt._lib.rt_plan_create(C.byref(handle), C.byref(det), C.byref(med), formalism, precision, k)
    assert st == rt.RT_E_INVALID
    assert handle.value is None
    assert rt.rt_last_error()


def test_plan_create_without_gpu_reports_no_device(rt):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    det, keep = _detector(rt)
    med = rt.rt_medium(rt.RT_UNIFORM, 2.92e-4, 8000.0)
    handle = C.c_void_p()
    st = rt._lib.rt_plan_create(C.byref(handle), C.byref(det), C.byref(med), rt.RT_ENDPOINT,
                                rt.RT_FP64, 1.0)
    assert st == rt.RT_E_NO_DEVICE


def test_null_plan_arguments(rt):
    assert rt._lib.rt_plan_destroy(None) == rt.RT_OK
    assert rt._lib.rt_plan_set_tiling(None, C.byref(rt.rt_tiling())) == rt.RT_E_INVALID
    tr = rt.rt_tracks()
    assert rt._lib.rt_accumulate(None, C.byref(tr), None, None, 0, None) == rt.RT_E_INVALID
    assert rt._lib.rt_propagate(None, C.byref(tr), None, None, None) == rt.RT_E_INVALID
