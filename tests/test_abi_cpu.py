"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and host-detectable argument errors return their documented codes without
touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_2104_14547_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nurbsdiff.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nurbs_\w+)\s*\(", text)))


def test_header_declarations_match_binding():
    assert declared_functions() == sorted(N.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = N.lib()
    missing = [s for s in declared_functions() if not hasattr(L, s)]
    assert not missing, missing


def test_status_strings():
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert N.status_string(code)
    assert N.status_string(0) == "ok"
    assert "unknown" in N.status_string(-99)


def test_null_context_is_rejected_before_any_launch():
    L = N.lib()
    rc = L.nurbs_surface_fwd(None, 1, 3, 3, 4, 4, None, None, None, None, 8, 8, None, None, 1, None,
                             None, 0, None)
    assert rc == N.NURBS_EINVAL
    assert L.nurbs_last_error(None).decode() == "ctx is NULL"
    out = ctypes.c_size_t()
    assert L.nurbs_surface_ws_bytes(None, 1, 3, 3, 4, 4, 8, 8, 15, ctypes.byref(out)) == N.NURBS_EINVAL
    h = ctypes.c_void_p()
    assert L.nurbs_plan_create(None, None, 0, 0, ctypes.byref(h), None) == N.NURBS_EINVAL
    assert L.nurbs_ctx_set_flags(None, 0) == N.NURBS_EINVAL
    assert L.nurbs_ctx_set_knot_sigma(None, 0.0) == N.NURBS_EINVAL
    assert L.nurbs_ctx_create(0, None) == N.NURBS_EINVAL
    assert L.nurbs_plan_destroy(None) == N.NURBS_OK
    assert L.nurbs_ctx_destroy(None) == N.NURBS_OK


@pytest.mark.parametrize("p", [0, -1, N.NURBS_MAX_DEGREE + 1])
def test_span_export_rejects_bad_degree(p):
    L = N.lib()
    assert L.nurbs_find_spans(None, 12, p, None, 4, None, None) == N.NURBS_EDEGREE
    assert L.nurbs_basis(None, 12, p, None, 4, None, None) == N.NURBS_EDEGREE


def test_span_export_rejects_short_knot_vector():
    L = N.lib()
    # p = 3 needs at least 2p + 2 = 8 knots; pointers are never dereferenced
    assert L.nurbs_find_spans(ctypes.c_void_p(16), 7, 3, ctypes.c_void_p(16), 4, ctypes.c_void_p(16),
                              None) == N.NURBS_EINVAL
    assert L.nurbs_find_spans(ctypes.c_void_p(16), 8, 3, ctypes.c_void_p(16), 0, ctypes.c_void_p(16),
                              None) == N.NURBS_OK  # nothing to do


def test_plan_calls_reject_null_plan():
    L = N.lib()
    assert L.nurbs_plan_fwd(None, *([None] * 8), 0, None) == N.NURBS_EINVAL
    assert L.nurbs_plan_bwd(None, *([None] * 11), 15, None, 0, None) == N.NURBS_EINVAL
    assert L.nurbs_plan_info(None, None, None, None) == N.NURBS_EINVAL


def test_device_error_read_rejects_null():
    code = ctypes.c_int()
    assert N.lib().nurbs_read_device_error(None, None, ctypes.byref(code)) == N.NURBS_EINVAL
