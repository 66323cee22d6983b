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
    assert rt.rt_abi_version() == rt.ABI_VERSION == 2
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
    assert rt._lib.rt_accumulate_static(None, C.byref(tr), None, None) == rt.RT_E_INVALID
    assert rt._lib.rt_propagate(None, C.byref(tr), None, None, None) == rt.RT_E_INVALID
    assert rt._lib.rt_plan_set_n0m1_device(None, None) == rt.RT_E_INVALID


def test_autotuners_reject_invalid_arguments(rt):
    """Both autotuners check their arguments before touching a device."""
    tr = rt.rt_tracks()
    cands = (rt.rt_tiling * 1)()
    ms = (C.c_float * 1)()
    best = C.c_int32(7)
    assert rt._lib.rt_plan_autotune(None, C.byref(tr), None, None, 0, cands, 1, 1, None, ms,
                                    C.byref(best)) == rt.RT_E_INVALID
    assert "required" in rt.rt_last_error()
    sh, keep = _shower(rt)
    opts = (rt.rt_batch_options * 1)()
    assert rt._lib.rt_batch_autotune(None, 1, rt.RT_FP64, 1.0, opts, 1, None, 0, 1, None, ms,
                                     C.byref(best)) == rt.RT_E_INVALID
    assert rt._lib.rt_batch_autotune(C.byref(sh), 1, rt.RT_FP64, 1.0, opts, 0, None, 0, 1, None,
                                     ms, C.byref(best)) == rt.RT_E_INVALID
    assert rt._lib.rt_batch_autotune(C.byref(sh), 1, rt.RT_FP64, 1.0, opts, 1, None, 0, 0, None,
                                     ms, C.byref(best)) == rt.RT_E_INVALID
    assert "reps" in rt.rt_last_error()


def _shower(rt):
    det, keep = _detector(rt)
    med = rt.rt_medium(rt.RT_UNIFORM, 2.92e-4, 8000.0)
    return rt.rt_shower(det, med, rt.RT_ENDPOINT, rt.rt_tracks(), None), keep


@pytest.mark.parametrize("case", ["null_showers", "zero_showers", "bad_block", "bad_block_768",
                                  "bad_at", "bad_items", "bad_detector", "bad_formalism",
                                  "null_traces", "bad_per_shower", "one_antenna_wide_tile",
                                  "bad_precision"])
def test_batch_create_rejects_invalid_arguments(rt, case):
    sh, keep = _shower(rt)
    arr = (rt.rt_shower * 2)(sh, sh)
    n, precision = 2, rt.RT_MIXED
    opt = rt.rt_batch_options()
    tl = (rt.rt_tiling * 2)()
    if case == "null_showers":
        arr = None
    elif case == "zero_showers":
        n = 0
    elif case == "bad_block":   # 1024 threads take one-antenna tiles only
        opt.block_threads = 1024
    elif case == "bad_block_768":
        opt.block_threads = 768
        opt.max_antennas_per_tile = 1
    elif case == "bad_at":
        opt.max_antennas_per_tile = 4
    elif case == "bad_items":
        opt.items_per_cu = -1
    elif case == "bad_detector":
        arr[1].det.dt = -1.0
    elif case == "bad_formalism":
        arr[0].formalism = 3
    elif case == "null_traces":
        buf = (C.c_double * 1)()
        arr[1].tracks = rt.rt_tracks(1, *([C.addressof(buf)] * 12))
    elif case == "bad_per_shower":
        tl[1].bins_per_segment = 100
        opt.per_shower = C.cast(tl, C.POINTER(rt.rt_tiling))
    elif case == "one_antenna_wide_tile":
        opt.block_threads = 1024
        opt.max_antennas_per_tile = 1
        tl[1].antennas_per_block = 2
        opt.per_shower = C.cast(tl, C.POINTER(rt.rt_tiling))
    elif case == "bad_precision":
        precision = 2
    handle = C.c_void_p()
    st = rt._lib.rt_batch_create(C.byref(handle), arr, n, precision, 1.0, C.byref(opt))
    assert st == rt.RT_E_INVALID, rt.rt_last_error()
    assert handle.value is None
    if case in ("bad_detector", "null_traces", "bad_per_shower", "one_antenna_wide_tile"):
        assert rt.rt_last_error().startswith("shower 1:")


def test_batch_create_without_gpu_reports_no_device(rt):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    sh, keep = _shower(rt)
    handle = C.c_void_p()
    st = rt._lib.rt_batch_create(C.byref(handle), C.byref(sh), 1, rt.RT_FP64, 1.0, None)
    assert st == rt.RT_E_NO_DEVICE


def test_null_batch_arguments(rt):
    assert rt._lib.rt_batch_destroy(None) == rt.RT_OK
    assert rt._lib.rt_batch_launch(None, None, 0, None) == rt.RT_E_INVALID
    b = C.c_size_t()
    assert rt._lib.rt_batch_workspace_bytes(None, C.byref(b)) == rt.RT_E_INVALID
    assert rt._lib.rt_batch_get_info(None, None, None, None, None) == rt.RT_E_INVALID
    assert rt._lib.rt_batch_set_timing_events(None, None, None) == rt.RT_E_INVALID


@pytest.mark.parametrize("case", ["no_table", "one_node", "zero_dz", "nan_z0"])
def test_plan_create_rejects_invalid_tables(rt, case):
    det, keep = _detector(rt)
    buf = (C.c_double * 4)(1.0, 0.9, 0.8, 0.7)
    med = rt.rt_medium(rt.RT_TABULATED, 2.92e-4, 8000.0, C.addressof(buf), 4, 0.0, 100.0)
    if case == "no_table":
        med.table = None
    elif case == "one_node":
        med.n_table = 1
    elif case == "zero_dz":
        med.table_dz = 0.0
    elif case == "nan_z0":
        med.table_z0 = float("nan")
    handle = C.c_void_p()
    st = rt._lib.rt_plan_create(C.byref(handle), C.byref(det), C.byref(med), rt.RT_ENDPOINT,
                                rt.RT_FP64, 1.0)
    assert st == rt.RT_E_INVALID, rt.rt_last_error()


@pytest.mark.parametrize("case", ["zero_radius", "small_radius", "nan_radius", "inf_radius",
                                  "zero_scale_height"])
def test_plan_create_rejects_invalid_spheres(rt, case):
    det, keep = _detector(rt)
    med = rt.rt_medium(rt.RT_SPHERICAL, 2.92e-4, 8000.0, None, 0, 0.0, 1.0, 6.371e6)
    if case == "zero_radius":
        med.earth_radius = 0.0
    elif case == "small_radius":
        med.earth_radius = 999.0
    elif case == "nan_radius":
        med.earth_radius = float("nan")
    elif case == "inf_radius":
        med.earth_radius = float("inf")
    elif case == "zero_scale_height":
        med.scale_height = 0.0
    handle = C.c_void_p()
    st = rt._lib.rt_plan_create(C.byref(handle), C.byref(det), C.byref(med), rt.RT_ZHS,
                                rt.RT_MIXED, 1.0)
    assert st == rt.RT_E_INVALID, rt.rt_last_error()
    assert "earth_radius" in rt.rt_last_error() or "scale_height" in rt.rt_last_error()


def test_medium_struct_carries_the_earth_radius(rt):
    from paper_2309_03717_amd.workloads import SPHERICAL_AIR, EXPONENTIAL_AIR
    m = rt._medium_struct(SPHERICAL_AIR)
    assert m.kind == rt.RT_SPHERICAL and m.earth_radius == 6.371e6 and m.scale_height == 8000.0
    assert rt._medium_struct(EXPONENTIAL_AIR).earth_radius == 0.0
    assert C.sizeof(rt.rt_medium) == 64


@pytest.mark.parametrize("medium", ["uniform", "exponential", "layered", "spherical"])
def test_plan_binding_passes_every_medium_field(rt, medium):
    """The Python Plan marshals each medium completely: on a host without a
    GPU the library validates the medium first and then reports the missing
    device (an incomplete medium would be rejected as invalid)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2309_03717_amd import workloads as W
    md = {"uniform": W.UNIFORM_AIR, "exponential": W.EXPONENTIAL_AIR,
          "layered": W.layered_air(), "spherical": W.SPHERICAL_AIR}[medium]
    arr = W.config(0).array
    det = rt.DeviceDetector.from_array(arr, device="cpu")
    with pytest.raises(rt.RadtraceError) as e:
        rt.Plan(det, md, "zhs", "mixed")
    assert e.value.status == rt.RT_E_NO_DEVICE, rt.rt_last_error()
    # a radius the Python check would refuse, set past it to reach the library's
    bad = W.Medium("spherical", W.N0_AIR, W.H_AIR, earth_radius=6.371e6)
    object.__setattr__(bad, "earth_radius", 10.0)
    with pytest.raises(rt.RadtraceError) as e:
        rt.Plan(det, bad, "zhs", "mixed")
    assert e.value.status == rt.RT_E_INVALID


def test_plan_create_rejects_more_than_int32_antennas(rt):
    det, keep = _detector(rt)
    det.n_antennas = 2 ** 31
    med = rt.rt_medium(rt.RT_UNIFORM, 2.92e-4, 8000.0)
    handle = C.c_void_p()
    st = rt._lib.rt_plan_create(C.byref(handle), C.byref(det), C.byref(med), rt.RT_ZHS,
                                rt.RT_MIXED, 1.0)
    assert st == rt.RT_E_UNSUPPORTED and "antennas" in rt.rt_last_error()


def test_filter_workspace_bytes(rt):
    """Two 256-byte-aligned arrays of one int64 per 256-track workgroup."""
    b = C.c_size_t()
    for n, want in [(0, 512), (1, 512), (256 * 32, 512), (256 * 33, 1024), (10 ** 6, 2 * 31488)]:
        assert rt._lib.rt_filter_workspace_bytes(n, C.byref(b)) == rt.RT_OK
        assert b.value == want, (n, b.value)
        assert rt.rt_filter_workspace_bytes(n) == want
    assert rt._lib.rt_filter_workspace_bytes(-1, C.byref(b)) == rt.RT_E_INVALID
    assert rt._lib.rt_filter_workspace_bytes(5, None) == rt.RT_E_INVALID


@pytest.mark.parametrize("case", ["null_in", "null_out", "null_count", "bad_precision",
                                  "negative_qw_min", "nan_qw_min", "inf_qw_min", "null_field",
                                  "small_capacity", "null_out_field", "small_workspace"])
def test_filter_rejects_invalid_arguments(rt, case):
    """Every invalid argument is refused before the device is touched."""
    buf = (C.c_double * 16)()
    p = C.addressof(buf)
    tin = rt.rt_tracks(10, *([p] * 12))
    tout = rt.rt_tracks(10, *([p + 64] * 12))
    count = p + 8
    ws, ws_bytes = p, 1 << 20
    precision, qw_min = rt.RT_MIXED, 0.0
    args = None
    if case == "null_in":
        args = (None, precision, qw_min, C.byref(tout), count, ws, ws_bytes, None)
    elif case == "null_out":
        args = (C.byref(tin), precision, qw_min, None, count, ws, ws_bytes, None)
    elif case == "null_count":
        args = (C.byref(tin), precision, qw_min, C.byref(tout), None, ws, ws_bytes, None)
    elif case == "bad_precision":
        precision = 5
    elif case == "negative_qw_min":
        qw_min = -1e-3
    elif case == "nan_qw_min":
        qw_min = float("nan")
    elif case == "inf_qw_min":
        qw_min = float("inf")
    elif case == "null_field":
        tin.qw = None
    elif case == "small_capacity":
        tout.n = 9
    elif case == "null_out_field":
        tout.x1 = None
    elif case == "small_workspace":
        ws_bytes = 100
    if args is None:
        args = (C.byref(tin), precision, qw_min, C.byref(tout), count, ws, ws_bytes, None)
    st = rt._lib.rt_filter_tracks(*args)
    want = rt.RT_E_WORKSPACE if case == "small_workspace" else rt.RT_E_INVALID
    assert st == want, (case, st, rt.rt_last_error())


def test_library_sources_allocate_no_device_memory():
    """The caller owns every device buffer (workspaces included): no source
    of the library calls a device allocator or free (the static workspace
    of rt_accumulate_static is a device array of the code object)."""
    import glob
    import os
    import re
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    call = re.compile(r"\bhip(Malloc\w*|ExtMalloc\w*|Free\w*|HostMalloc|HostAlloc|MemPool\w*)\s*\(")
    sources = glob.glob(os.path.join(root, "paper_2309_03717_amd", "csrc", "*"))
    assert sources
    for f in sources:
        with open(f) as fh:
            for i, line in enumerate(fh, 1):
                assert not call.search(line.split("//")[0]), f"{f}:{i}: {line.strip()}"
