"""C ABI contract checks that need no GPU: the library loads, exports every
symbol include/mf.h declares, and rejects bad arguments on the host before
touching the device."""
import ctypes
import os
import re

import pytest

import paper_2003_02978_amd as mf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mf.h")).read()
    return sorted(set(re.findall(r"MF_API\s+[\w\s\*]+?\b(mf_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = mf.load_library()
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(mf.EXPORTS)
    assert lib.mf_abi_version() == mf.ABI_VERSION == 4


def test_options_default_and_struct_layout():
    o = mf.default_options()
    assert o.struct_size == ctypes.sizeof(mf.Options)
    assert (o.n_bands, o.n_iter, o.albedo, o.cov, o.refine_steps) == (74, 30, 1, 0, -1)
    assert (o.chunk_lines, o.group, o.save_for_backward, o.track_energy) == (0, 1, 0, 0)
    assert o.lambda_ == 1.0 and o.epsilon == 1e-9


def _create(**kw):
    lib = mf.load_library()
    o = mf.default_options()
    for k, v in kw.items():
        setattr(o, k, v)
    fl = (mf.Flightline * 1)(mf.Flightline(0, 4, 1000))
    h = ctypes.c_void_p()
    rc = lib.mf_plan_create(ctypes.byref(o), fl, 1, ctypes.byref(h))
    return rc, h, lib.mf_last_error().decode()


@pytest.mark.parametrize("field,value,code", [
    ("struct_size", 8, mf.MF_E_ARG),
    ("n_bands", 1, mf.MF_E_UNSUPPORTED),
    ("n_bands", 79, mf.MF_E_UNSUPPORTED),
    ("n_iter", -1, mf.MF_E_ARG),
    ("lambda_", -1.0, mf.MF_E_ARG),
    ("lambda_", float("nan"), mf.MF_E_ARG),
    ("epsilon", 0.0, mf.MF_E_ARG),
    ("albedo", 2, mf.MF_E_ARG),
    ("cov", 7, mf.MF_E_ARG),
    ("cov", -1, mf.MF_E_ARG),
    ("refine_steps", 9, mf.MF_E_ARG),
    ("refine_steps", -2, mf.MF_E_ARG),
    ("chunk_lines", 100, mf.MF_E_ARG),
    ("save_for_backward", 2, mf.MF_E_ARG),
    ("group", 0, mf.MF_E_ARG),
    ("group", -3, mf.MF_E_ARG),
    ("track_energy", 2, mf.MF_E_ARG),
])
def test_bad_options_rejected_on_host(field, value, code):
    rc, h, msg = _create(**{field: value})
    assert rc == code and not h.value and msg


def test_header_limits_match_the_binding():
    src = open(os.path.join(ROOT, "include", "mf.h")).read()

    def define(name):
        return re.search(r"#define\s+" + name + r"\s+(.+?)\s*(/\*|$)", src, re.M).group(1)

    assert int(define("MF_MAX_BANDS")) == 78
    assert int(define("MF_MAX_STREAMS")) == mf.MAX_STREAMS
    assert int(define("MF_MAX_BACKWARD_ITER")) == mf.MAX_BACKWARD_ITER
    assert define("MF_NOALLOC_SCRATCH_BYTES") == "((size_t)64 << 20)" == "((size_t)%d << 20)" % (
        mf.NOALLOC_SCRATCH_BYTES >> 20)


def test_backward_needs_low_rank_form_and_bounded_k():
    rc, h, msg = _create(save_for_backward=1, cov=1)
    assert rc == mf.MF_E_UNSUPPORTED and "low-rank" in msg
    rc, h, msg = _create(save_for_backward=1, n_iter=mf.MAX_BACKWARD_ITER + 1)
    assert rc == mf.MF_E_UNSUPPORTED and str(mf.MAX_BACKWARD_ITER) in msg
    lib = mf.load_library()
    assert lib.mf_backward(None, None, None, None, None, None, None, None, None) == mf.MF_E_ARG


def test_energy_needs_low_rank_form():
    rc, h, msg = _create(track_energy=1, cov=1)
    assert rc == mf.MF_E_UNSUPPORTED and "low-rank" in msg
    lib = mf.load_library()
    assert lib.mf_plan_energy(None, None, None, None) == mf.MF_E_ARG


def test_bad_geometry_rejected_on_host():
    lib = mf.load_library()
    o = mf.default_options()
    h = ctypes.c_void_p()
    fl = (mf.Flightline * 2)(mf.Flightline(0, 4, 1000), mf.Flightline(3000, 2, 1000))
    assert lib.mf_plan_create(ctypes.byref(o), fl, 2, ctypes.byref(h)) == mf.MF_E_SHAPE
    assert b"overlap" in lib.mf_last_error()
    fl = (mf.Flightline * 1)(mf.Flightline(0, 0, 1000))
    assert lib.mf_plan_create(ctypes.byref(o), fl, 1, ctypes.byref(h)) == mf.MF_E_SHAPE
    assert lib.mf_plan_create(ctypes.byref(o), fl, 0, ctypes.byref(h)) == mf.MF_E_SHAPE
    assert lib.mf_plan_create(None, fl, 1, ctypes.byref(h)) == mf.MF_E_ARG
    assert lib.mf_plan_create(ctypes.byref(o), fl, 1, None) == mf.MF_E_ARG


def test_null_arguments_of_retrieve():
    lib = mf.load_library()
    assert lib.mf_retrieve(None, None, None, None, None, None, None, None) == mf.MF_E_ARG
    assert lib.mf_workspace_bytes(None) == 0
    lib.mf_plan_destroy(None)
    assert lib.mf_status_str(3) == b"unsupported configuration"


def test_stream_read_rejects_bad_arguments_on_host():
    lib = mf.load_library()
    # pointers are only checked, never dereferenced, before these errors
    assert lib.mf_stream_read(None, 1024, None, 16, None, None) == mf.MF_E_ARG
    assert lib.mf_stream_read(16, 1022, 32, 16, None, None) == mf.MF_E_ARG      # n not a multiple of 4
    assert lib.mf_stream_read(20, 1024, 32, 16, None, None) == mf.MF_E_ARG      # src not 16-byte aligned
    assert lib.mf_stream_read(16, 1024, 32, 0, None, None) == mf.MF_E_ARG       # no workgroups
    assert lib.mf_stream_read(16, 1 << 31, 32, 1, None, None) == mf.MF_E_ARG    # span over 2^29 floats
    assert b"2^29" in lib.mf_last_error()
