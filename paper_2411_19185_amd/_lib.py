"""ctypes binding of libhope.so (the C ABI in include/hope.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Device buffers are torch CUDA (HIP) FP64 tensors; the stream is
torch's current stream.  The library is loaded from this package directory
and its absence is an error: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
# HOPE_LIB selects another build of the same library (used to compare build variants)
LIB_PATH = os.environ.get("HOPE_LIB") or os.path.join(HERE, "libhope.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "hope.h")

HOPE_OK = 0
HOPE_ERR_NUMERIC = -5
HOPE_PROFILE_SELECT = 0x40000000
HOPE_SCHEME_TPP, HOPE_SCHEME_WENO = 0, 1
HOPE_RK_SSP3, HOPE_RK_WS3 = 0, 1


class HopeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hope error {code}: {msg}")
        self.code = code


# surface_geopotential(count, xyz, phis, user) of hope_grid_desc
SURFACE_FN = ctypes.CFUNCTYPE(None, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                              ctypes.c_void_p)


class GridDesc(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_int32),
        ("n", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
        ("n_gauss", ctypes.c_int32),
        ("ghost_iters", ctypes.c_int32),
        ("radius", ctypes.c_double),
        ("gravity", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("axis_tilt", ctypes.c_double),
        ("weno_eps", ctypes.c_double),
        ("split_theta", ctypes.c_double),
        ("cache_dir", ctypes.c_char_p),
        ("surface_geopotential", SURFACE_FN),
        ("surface_user", ctypes.c_void_p),
    ]


class Layout(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("r", ctypes.c_int32),
        ("padded", ctypes.c_int32),
        ("n_gauss", ctypes.c_int32),
        ("state_elems", ctypes.c_int64),
        ("interior_elems", ctypes.c_int64),
        ("rk_workspace_bytes", ctypes.c_int64),
        ("vjp_workspace_bytes", ctypes.c_int64),
        ("rk_vjp_workspace_bytes", ctypes.c_int64),
        ("ghost_cells", ctypes.c_int64),
        ("ghost_nnz", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64),
        ("ghost_sweeps", ctypes.c_int32),
        ("tables_cached", ctypes.c_int32),
        ("tendency_workspace_bytes", ctypes.c_int64),
        ("fill_blocks", ctypes.c_int64),
    ]


class BatchInfo(ctypes.Structure):
    _fields_ = [
        ("n_members", ctypes.c_int32),
        ("n_grids", ctypes.c_int32),
        ("state_elems", ctypes.c_int64),
        ("field_elems", ctypes.c_int64),
        ("rk_workspace_bytes", ctypes.c_int64),
        ("items", ctypes.c_int64),
        ("blocks", ctypes.c_int64),
        ("ghost_rows", ctypes.c_int64),
        ("fill_blocks", ctypes.c_int64),
    ]


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_SIGS = {
    "hope_grid_create": (_I32, [ctypes.POINTER(GridDesc), ctypes.POINTER(_P)]),
    "hope_grid_destroy": (None, [_P]),
    "hope_grid_derive": (_I32, [_P, ctypes.c_double, ctypes.POINTER(_P)]),
    "hope_grid_layout": (_I32, [_P, ctypes.POINTER(Layout)]),
    "hope_fill_halo": (_I32, [_P, _P, _P]),
    "hope_check_state": (_I32, [_P, _P, ctypes.POINTER(ctypes.c_int64), _P]),
    "hope_tendency": (_I32, [_P, _P, _P, _P, ctypes.c_size_t, _P]),
    "hope_tendency_vjp": (_I32, [_P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "hope_rk_step": (_I32, [_P, _P, ctypes.c_double, _I32, _P, ctypes.c_size_t, _P]),
    "hope_rk_step_vjp": (_I32, [_P, _P, ctypes.c_double, _I32, _P, _P, _P, ctypes.c_size_t, _P]),
    "hope_rk_step_static": (_I32, [_P, _P, ctypes.c_double, _I32, _P]),
    "hope_last_error": (ctypes.c_char_p, []),
    "hope_grid_set_launch": (_I32, [_P, _I32, _I32]),
    "hope_grid_get_launch": (_I32, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "hope_grid_profile": (_I32, [_P, _I32]),
    "hope_grid_profile_read": (_I32, [_P, _I32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "hope_batch_create": (_I32, [ctypes.POINTER(_P), _I32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_P)]),
    "hope_batch_destroy": (None, [_P]),
    "hope_batch_layout": (_I32, [_P, ctypes.POINTER(BatchInfo), ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_int64)]),
    "hope_batch_set_launch": (_I32, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), _I32]),
    "hope_batch_get_launch": (_I32, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "hope_batch_tendency": (_I32, [_P, _P, _P, _P]),
    "hope_batch_rk_stage": (_I32, [_P, _I32, _I32, _P, _P, _P, ctypes.c_size_t, _P]),
    "hope_batch_rk_step": (_I32, [_P, _I32, _P, _P, _P, ctypes.c_size_t, _P]),
    "hope_inspect_ghost_map": (_I32, [ctypes.POINTER(GridDesc), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_I32),
                                      _P, _P, _P, _P]),
}


def header_functions() -> list[str]:
    """Names of the functions include/hope.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hope_[a-z_]+)\s*\(", txt)))


def lib():
    """The loaded library (raises if libhope.so has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2411_19185_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code: int):
    if code != HOPE_OK:
        raise HopeError(code, lib().hope_last_error().decode())


def surface_callback(surface):
    """A SURFACE_FN that evaluates the Python callable surface(p) -> phi_s at
    the unit vectors p (count, 3) the library asks for (marshalling only)."""
    import numpy as np

    def cb(count, xyz, out, user):
        p = np.ctypeslib.as_array(xyz, shape=(count, 3))
        np.ctypeslib.as_array(out, shape=(count,))[:] = np.asarray(surface(p), dtype=np.float64)
    return SURFACE_FN(cb)


def make_desc(n, order, scheme="tpp", radius=6.371e6, omega=7.292e-5, axis_tilt=0.0, weno_eps=1e-12,
              split_theta=3.0, gravity=9.80616, ghost_iters=0, cache_dir=None, surface_fn=None) -> GridDesc:
    d = GridDesc()
    d.struct_size = ctypes.sizeof(GridDesc)
    d.n = n
    d.order = order
    d.scheme = {"tpp": HOPE_SCHEME_TPP, "weno": HOPE_SCHEME_WENO}[scheme]
    d.n_gauss = 0
    d.radius = radius
    d.gravity = gravity
    d.omega = omega
    d.axis_tilt = axis_tilt
    d.weno_eps = weno_eps
    d.split_theta = split_theta
    d.ghost_iters = ghost_iters
    d.cache_dir = None if cache_dir is None else os.fsencode(cache_dir)
    if surface_fn is not None:
        d.surface_geopotential = surface_fn
    return d


def inspect_ghost_map(n, order, scheme="tpp", radius=6.371e6, ghost_iters=0):
    """The ghost map the library builds, as numpy arrays (host only);
    ghost_iters = 0 gives the fixed point, N > 0 the map of N Jacobi sweeps."""
    import numpy as np
    d = make_desc(n, order, scheme, radius, ghost_iters=ghost_iters)
    rows, nnz, sweeps = ctypes.c_int64(), ctypes.c_int64(), _I32()
    check(lib().hope_inspect_ghost_map(ctypes.byref(d), ctypes.byref(rows), ctypes.byref(nnz),
                                       ctypes.byref(sweeps), None, None, None, None))
    dst = np.zeros(rows.value, np.int32)
    ptr = np.zeros(rows.value + 1, np.int32)
    col = np.zeros(nnz.value, np.int32)
    val = np.zeros(5 * nnz.value, np.float64)
    check(lib().hope_inspect_ghost_map(ctypes.byref(d), ctypes.byref(rows), ctypes.byref(nnz),
                                       ctypes.byref(sweeps), dst.ctypes.data, ptr.ctypes.data,
                                       col.ctypes.data, val.ctypes.data))
    return dst, ptr, col, val.reshape(5, -1), sweeps.value
