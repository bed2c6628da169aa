"""ctypes binding of libnurbsdiff (include/nurbsdiff.h): argument marshalling only.

Every entry point keeps the C name.  Pointers are raw device addresses
(``tensor.data_ptr()``) and streams raw ``hipStream_t`` handles.  The library
is loaded from this package directory; if it is missing the import fails
loudly -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnurbsdiff.so")

NURBS_OK = 0
NURBS_EINVAL = -1
NURBS_EDEGREE = -2
NURBS_EKNOTS = -3
NURBS_EDOMAIN = -4
NURBS_EWEIGHTS = -5
NURBS_EWORKSPACE = -6
NURBS_EDEVICE = -7
NURBS_EUNSUPPORTED = -8

NURBS_GRAD_CTRL = 1
NURBS_GRAD_W = 2
NURBS_GRAD_KU = 4
NURBS_GRAD_KV = 8
NURBS_GRAD_ALL = 15
NURBS_VALIDATE = 1
NURBS_PLAN_WS_HEADER = 4352
NURBS_SCHED_STATIC = 0
NURBS_SCHED_DYNAMIC = 1
NURBS_MAX_DEGREE = 7
NURBS_MAX_KNOTS = 256

# every symbol include/nurbsdiff.h declares
EXPORTS = (
    "nurbs_ctx_create", "nurbs_ctx_destroy", "nurbs_ctx_set_flags", "nurbs_ctx_set_knot_sigma",
    "nurbs_ctx_set_tiling",
    "nurbs_status_string", "nurbs_last_error", "nurbs_ctx_device_info",
    "nurbs_surface_ws_bytes", "nurbs_surface_fwd", "nurbs_surface_derivs", "nurbs_surface_bwd",
    "nurbs_plan_create", "nurbs_plan_create_in", "nurbs_plan_destroy", "nurbs_plan_info", "nurbs_plan_fwd", "nurbs_plan_bwd",
    "nurbs_plan_set_timing", "nurbs_plan_read_timing",
    "nurbs_find_spans", "nurbs_basis", "nurbs_read_device_error",
    "nurbs_curve_ws_bytes", "nurbs_curve_fwd", "nurbs_curve_bwd",
    "nurbs_surface_bwd_noalloc",
    "nurbs_chamfer_ws_bytes", "nurbs_nearest", "nurbs_chamfer",
    "nurbs_surface_uv_ws_bytes", "nurbs_surface_uv_fwd", "nurbs_surface_uv_bwd",
    "nurbs_basis_table_bytes", "nurbs_basis_table_build", "nurbs_surface_fwd_tab", "nurbs_surface_bwd_tab",
    "nurbs_ctx_set_schedule",
    "nurbs_server_create", "nurbs_server_submit", "nurbs_server_wait", "nurbs_server_stats",
    "nurbs_server_last_error", "nurbs_server_destroy", "nurbs_server_admit", "nurbs_server_busy",
)


class nurbs_desc(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("p", "q", "nu_c", "nv_c", "nu_s", "nv_s")] + \
               [(n, ctypes.c_int64) for n in ("ctrl_off", "w_off", "ku_off", "kv_off", "us_off",
                                              "vs_off", "pts_off")]


_vp = ctypes.c_void_p
_i = ctypes.c_int
_u = ctypes.c_uint
_sz = ctypes.c_size_t
_szp = ctypes.POINTER(ctypes.c_size_t)
_ip = ctypes.POINTER(ctypes.c_int)
_fp = ctypes.POINTER(ctypes.c_float)
_i64p = ctypes.POINTER(ctypes.c_int64)

_SIGS = {
    "nurbs_ctx_create": (_i, [_i, ctypes.POINTER(_vp)]),
    "nurbs_ctx_destroy": (_i, [_vp]),
    "nurbs_ctx_set_flags": (_i, [_vp, _u]),
    "nurbs_ctx_set_knot_sigma": (_i, [_vp, ctypes.c_float]),
    "nurbs_ctx_set_tiling": (_i, [_vp, _i, _i]),
    "nurbs_ctx_set_schedule": (_i, [_vp, _i]),
    "nurbs_status_string": (ctypes.c_char_p, [_i]),
    "nurbs_last_error": (ctypes.c_char_p, [_vp]),
    "nurbs_ctx_device_info": (_i, [_vp, _ip, _ip]),
    "nurbs_surface_ws_bytes": (_i, [_vp, _i, _i, _i, _i, _i, _i, _i, _u, _szp]),
    "nurbs_surface_fwd": (_i, [_vp, _i, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _i, _i, _vp, _vp, _i, _vp,
                               _vp, _sz, _vp]),
    "nurbs_surface_derivs": (_i, [_vp, _i, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _i, _i, _vp, _vp, _i, _vp, _vp,
                                  _vp, _vp, _vp, _sz, _vp]),
    "nurbs_surface_bwd": (_i, [_vp, _i, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _i, _i, _vp, _vp, _i, _vp,
                               _vp, _vp, _vp, _vp, _u, _vp, _sz, _vp]),
    "nurbs_plan_create": (_i, [_vp, ctypes.POINTER(nurbs_desc), _i, _u, ctypes.POINTER(_vp), _szp]),
    "nurbs_plan_create_in": (_i, [_vp, ctypes.POINTER(nurbs_desc), _i, _u, _vp, _sz, _vp, ctypes.POINTER(_vp),
                                  _szp, _szp]),
    "nurbs_plan_destroy": (_i, [_vp]),
    "nurbs_plan_info": (_i, [_vp, _ip, _ip, _ip]),
    "nurbs_plan_fwd": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "nurbs_plan_bwd": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _u, _vp, _sz,
                            _vp]),
    "nurbs_plan_set_timing": (_i, [_vp, _i]),
    "nurbs_plan_read_timing": (_i, [_vp, _fp, _ip, _fp, _fp, _fp, _ip]),
    "nurbs_find_spans": (_i, [_vp, _i, _i, _vp, _i, _vp, _vp]),
    "nurbs_basis": (_i, [_vp, _i, _i, _vp, _i, _vp, _vp]),
    "nurbs_read_device_error": (_i, [_vp, _vp, _ip]),
    "nurbs_surface_bwd_noalloc": (_i, [_vp, _i, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _i, _i, _vp, _vp, _i, _vp,
                                       _vp, _vp, _vp, _vp, _u, _vp]),
    "nurbs_basis_table_bytes": (_i, [_i, _i, _szp]),
    "nurbs_basis_table_build": (_i, [_vp, _i, _i, _vp, _i, _vp, _sz, _vp]),
    "nurbs_surface_fwd_tab": (_i, [_vp, _i, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _i, _i, _vp, _vp, _i, _vp, _vp, _i,
                                   _vp, _vp, _sz, _vp]),
    "nurbs_surface_bwd_tab": (_i, [_vp, _i, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _i, _i, _vp, _vp, _i, _vp, _vp, _i,
                                   _vp, _vp, _vp, _u, _vp, _sz, _vp]),
    "nurbs_surface_uv_ws_bytes": (_i, [_vp, _i, _i, _i, _i, _i, _i, _u, _szp]),
    "nurbs_surface_uv_fwd": (_i, [_vp, _i, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _i, _vp, _i, _vp, _vp, _vp, _vp, _sz,
                                  _vp]),
    "nurbs_surface_uv_bwd": (_i, [_vp, _i, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _i, _vp, _i, _vp, _vp, _vp, _vp, _vp,
                                  _u, _vp, _sz, _vp]),
    "nurbs_chamfer_ws_bytes": (_i, [_vp, _i, _i, _i, _szp]),
    "nurbs_nearest": (_i, [_vp, _i, _i, _vp, _i, _vp, _i, _vp, _vp, _vp, _sz, _vp]),
    "nurbs_chamfer": (_i, [_vp, _i, _i, _vp, _i, _vp, _i, _vp, _vp, _vp, _vp, _sz, _vp]),
    "nurbs_curve_ws_bytes": (_i, [_vp, _i, _i, _i, _i, _i, _u, _szp]),
    "nurbs_curve_fwd": (_i, [_vp, _i, _i, _i, _i, _vp, _vp, _vp, _i, _vp, _i, _vp, _vp, _vp, _sz, _vp]),
    "nurbs_curve_bwd": (_i, [_vp, _i, _i, _i, _i, _vp, _vp, _vp, _i, _vp, _i, _vp, _vp, _vp, _vp, _u, _vp, _sz,
                             _vp]),
    "nurbs_server_create": (_i, [_i, ctypes.POINTER(nurbs_desc), _i, _vp, _vp, _vp, _vp, _i, _sz, _i,
                                 ctypes.POINTER(_vp)]),
    "nurbs_server_submit": (_i, [_vp, _i, _vp, _i, _vp, _i, _vp, _vp, ctypes.c_double, _i64p]),
    "nurbs_server_wait": (_i, [_vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]),
    "nurbs_server_stats": (_i, [_vp, _i64p, _i64p, _i64p]),
    "nurbs_server_last_error": (ctypes.c_char_p, [_vp]),
    "nurbs_server_busy": (_i, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "nurbs_server_destroy": (_i, [_vp]),
    "nurbs_server_admit": (_i, [ctypes.POINTER(ctypes.c_int32), _szp, _i, _sz, _sz, _i,
                                ctypes.POINTER(ctypes.c_int32), _ip]),
}

_lib = None


class NativeLibraryMissing(ImportError):
    pass


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise NativeLibraryMissing(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


_serve_py = None


def serve_py():
    """The CPython binding of the per-request serving calls, bound to the
    loaded library (raises if it has not been built)."""
    global _serve_py
    if _serve_py is None:
        L = lib()
        try:
            from . import _serve_py as m
        except ImportError as e:
            raise NativeLibraryMissing(
                f"the serving binding _serve_py is missing ({e}): build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'`") from e
        addr = lambda f: ctypes.cast(f, ctypes.c_void_p).value
        m.bind(addr(L.nurbs_server_submit), addr(L.nurbs_server_wait))
        _serve_py = m
    return _serve_py


def status_string(code: int) -> str:
    return lib().nurbs_status_string(int(code)).decode()
