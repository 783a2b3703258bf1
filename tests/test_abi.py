"""CPU checks of the C ABI: the library loads, exports every entry point that
include/vp.h declares, and the binding covers exactly that set.  No compute
call is made here."""
import ctypes
import os
import re

import pytest

from paper_2005_09316_amd import vp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vp_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_binding_set():
    assert _declared() == sorted(vp.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(vp.LIB_PATH):
        pytest.fail("libvp.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(vp.LIB_PATH)
    missing = [s for s in _declared() if not hasattr(lib, s)]
    assert not missing, missing


def test_version_and_last_error_without_gpu():
    assert "libvp" in vp.vp_version()
    assert isinstance(vp.vp_last_error(), str)


def test_header_constants_match_binding():
    src = open(os.path.join(ROOT, "include", "vp.h")).read()
    consts = dict((m.group(1), int(m.group(2))) for m in re.finditer(r"#define (VP_[A-Z0-9_]+) \(?(-?\d+)\)?", src))
    for name, val in consts.items():
        assert getattr(vp, name) == val, name


def test_null_arguments_are_rejected_before_any_device_work():
    lib = vp.load()
    assert lib.vp_create_ctx(0, 0, None) == vp.VP_EINVAL
    assert lib.vp_destroy_ctx(None) == vp.VP_EINVAL
    assert lib.vp_create_obs(None, None, None) == vp.VP_EINVAL
    assert lib.vp_create_sky(None, None, None) == vp.VP_EINVAL
    assert lib.vp_predict(None, None, None, 1, 1, None, None) == vp.VP_EINVAL
    assert lib.vp_predict_noalloc(None, None, None, 1, 1, None, None) == vp.VP_EINVAL
    assert "NULL" in vp.vp_last_error()


def test_other_entry_points_reject_null_arguments_before_any_device_work():
    """Every remaining entry point checks its handles and out-parameters
    first: the serving calls, subtract, destroy and the profiling calls."""
    import ctypes
    lib = vp.load()
    ticket = ctypes.c_uint64(0)
    assert lib.vp_submit(None, None, None) == vp.VP_EINVAL  # NULL ticket
    assert lib.vp_submit(None, None, ctypes.byref(ticket)) == vp.VP_EINVAL  # NULL context and job
    assert lib.vp_poll(None, 1, None) == vp.VP_EINVAL
    assert lib.vp_serve_stats(None, None, None) == vp.VP_EINVAL
    assert lib.vp_job_footprint(None, None, None) == vp.VP_EINVAL
    assert lib.vp_subtract(None, None, None, 1, 1, None, None) == vp.VP_EINVAL
    assert lib.vp_destroy_obs(None) == vp.VP_EINVAL
    assert lib.vp_destroy_sky(None) == vp.VP_EINVAL
    assert lib.vp_profile(None, 1) == vp.VP_EINVAL
    assert lib.vp_profile_read(None, None, None) == vp.VP_EINVAL


def test_peel_null_arguments_are_rejected_before_any_device_work():
    lib = vp.load()
    assert lib.vp_peel(None, None, None, None, None, 4, 1, 0, 0, None, None, None) == vp.VP_EINVAL
