"""ctypes loader for libmatgraph.so (the C ABI of include/matgraph.h).

Only argument marshalling lives here: every call goes straight to the
library. Loading fails loudly when the library is missing; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MG_LIB_PATH", os.path.join(PKG, "libmatgraph.so"))

MG_OK = 0
MG_ERR_INVALID_ARG = 1
MG_ERR_WORKSPACE = 2
MG_ERR_HIP = 3
MG_ERR_UNSUPPORTED = 4

MG_FLAG_CAPACITY = 1
MG_FLAG_SINGULAR = 2
MG_FLAG_NONFINITE = 4
MG_FLAG_IMAGES = 8
MG_FLAG_RANGE = 16
MG_FLAG_KNN_EXTENDED = 32
MG_FLAG_TIES = 64

MG_OPT_DEFAULT = 0
MG_OPT_CELL_LIST_OFF = 2
MG_OPT_CELL_LIST_FORCE = 4

ABI_VERSION = 1
REPORT_BYTES = 64


class MgTuning(ctypes.Structure):
    _fields_ = [("cutoff_wgs_per_cu", ctypes.c_int32), ("cutoff_slots", ctypes.c_int32),
                ("knn_wgs_per_cu", ctypes.c_int32), ("knn_lambda_x4", ctypes.c_int32),
                ("knn_tau_x8", ctypes.c_int32), ("cutoff_img_group", ctypes.c_int32),
                ("cutoff_cl_span", ctypes.c_int32), ("knn_cl_span", ctypes.c_int32)]


class MatgraphError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"matgraph status {status}: {message}")
        self.status = status


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_F = ctypes.c_float

# name -> (restype, argtypes); the single source of the Python-side signatures
SIGNATURES = {
    "mg_abi_version": (_I32, []),
    "mg_last_error": (ctypes.c_char_p, []),
    "mg_cutoff_workspace_bytes": (_SZ, [_I32, _I64, _I64]),
    "mg_knn_workspace_bytes": (_SZ, [_I32, _I64, _I32, _I64]),
    "mg_geometry_workspace_bytes": (_SZ, [_I32, _I64]),
    "mg_geometry_backward_workspace_bytes": (_SZ, [_I32, _I64, _I64]),
    "mg_cutoff_graph": (_I32, [_P, _P, _P, _I32, _I64, _F, _I64, _P, _P, _P, _P, _P, _P, _P, _SZ,
                               _I32, _P]),
    "mg_cutoff_graph_radii": (_I32, [_P, _P, _P, _I32, _I64, _P, _I64, _P, _P, _P, _P, _P, _P, _P,
                                     _SZ, _I32, _P]),
    "mg_cutoff_graph_vec": (_I32, [_P, _P, _P, _I32, _I64, _F, _P, _I64, _P, _P, _P, _P, _P, _P, _P, _P,
                                   _SZ, _I32, _P]),
    "mg_images_needed": (_I32, [_P, _P, _P, _I32, _I64, _F, _P, _I32, _P, _P, _SZ, _I32, _P]),
    "mg_knn_graph": (_I32, [_P, _P, _P, _I32, _I64, _I32, _P, _P, _P, _P, _P, _P, _SZ, _I32, _P]),
    "mg_edge_geometry": (_I32, [_P, _P, _P, _I32, _I64, _P, _P, _P, _I64, _P, _P, _P, _P, _SZ, _P]),
    "mg_edge_geometry_backward": (_I32, [_P, _P, _P, _I32, _I64, _P, _P, _P, _I64, _P, _P, _P, _P,
                                         _P, _P, _SZ, _P]),
    "mg_edge_geometry_backward_static": (_I32, [_P, _P, _P, _I32, _I64, _P, _P, _P, _I64, _P, _P, _P, _P,
                                                _P, _P]),
    "mg_triplets_workspace_bytes": (_SZ, [_I64]),
    "mg_symmetrize_workspace_bytes": (_SZ, [_I64, _I64]),
    "mg_knn_ties_workspace_bytes": (_SZ, [_I32, _I64, _I32, _I64]),
    "mg_knn_graph_ties": (_I32, [_P, _P, _P, _I32, _I64, _I32, _I64, _P, _P, _P, _P, _P, _P, _P, _SZ, _I32,
                                 _P]),
    "mg_symmetrize": (_I32, [_P, _I64, _P, _P, _P, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "mg_triplets": (_I32, [_P, _I64, _I64, _P, _I64, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "mg_get_tuning": (_I32, [ctypes.POINTER(MgTuning)]),
    "mg_set_tuning": (_I32, [ctypes.POINTER(MgTuning)]),
    "mg_profile_enable": (_I32, [_I32]),
    "mg_profile_read": (_I32, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_int64), _I32]),
}

_lib = None
_lock = threading.Lock()


def load(path: str | None = None):
    """Load libmatgraph.so once (raises if it is missing or has the wrong ABI)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise RuntimeError(
                f"libmatgraph.so not found at {p}: build it with "
                "`python -m paper_2307_05380_amd.build` (there is no CPU fallback)")
        lib = ctypes.CDLL(p)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        v = lib.mg_abi_version()
        if v != ABI_VERSION:
            raise RuntimeError(f"libmatgraph ABI {v}, binding expects {ABI_VERSION}")
        _lib = lib
        return lib


def check(status: int, lib=None):
    if status != MG_OK:
        lib = lib or load()
        raise MatgraphError(status, lib.mg_last_error().decode(errors="replace"))


def get_tuning() -> dict:
    lib = load()
    t = MgTuning()
    check(lib.mg_get_tuning(ctypes.byref(t)), lib)
    return {f: getattr(t, f) for f, _ in MgTuning._fields_}


def set_tuning(**kw):
    lib = load()
    t = MgTuning()
    for k, v in kw.items():
        setattr(t, k, int(v))
    check(lib.mg_set_tuning(ctypes.byref(t)), lib)


def profile_enable(on: bool):
    load().mg_profile_enable(1 if on else 0)


def profile_read(max_phases: int = 64) -> dict:
    """{phase name: (milliseconds summed, launches)} since the last read."""
    lib = load()
    names = ctypes.create_string_buffer(32 * max_phases)
    ms = (ctypes.c_double * max_phases)()
    cnt = (ctypes.c_int64 * max_phases)()
    m = lib.mg_profile_read(names, ms, cnt, max_phases)
    out = {}
    for q in range(min(m, max_phases)):
        nm = names.raw[32 * q:32 * q + 32].split(b"\0", 1)[0].decode()
        out[nm] = (ms[q], cnt[q])
    return out
