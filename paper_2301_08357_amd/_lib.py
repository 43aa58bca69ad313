"""ctypes declarations of the C ABI in include/pressure_cg.h.

Loading fails loudly when the built library is missing: there is no
fallback implementation of any step."""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libpressure.so")

PM_OK, PM_NOT_CONVERGED, PM_EINVAL, PM_EDEGENERATE, PM_ENOMEM, PM_EBREAKDOWN, PM_EHIP = 0, 1, -1, -2, -3, -4, -5
PM_PENDING = 2
PM_ETOOLARGE = -6
PM_ETIMEOUT = -7
PM_NOALLOC_MAX_NODES, PM_NOALLOC_MAX_ITER = 524288, 65535
PM_FP64, PM_FP32_INNER = 1, 2
PM_TILE_256, PM_TILE_512, PM_TILE_128 = 0x10, 0x20, 0x30
PM_MASS_LUMPED = 0x100
PM_VARIANT_AUTO, PM_VARIANT_NODE, PM_VARIANT_TILED = 0, 1, 2
PM_MIXED_KEEP_DIRECTION, PM_MIXED_RESTART = 0, 1

# every symbol the header declares, with (restype, argtypes)
_P = ctypes.c_void_p
_i32, _i64, _dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double


class PmMesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("n_nodes", ctypes.c_int64), ("n_elems", ctypes.c_int64),
                ("coords", _P), ("elems", _P), ("dirichlet", _P), ("lattice", _P), ("period", _P)]


_PMESH = ctypes.POINTER(PmMesh)

SIGNATURES = {
    "pressure_setup": (ctypes.c_int, [_PMESH, _P, _dbl, _dbl, _i32, ctypes.POINTER(_P)]),
    "pressure_update_coef": (ctypes.c_int, [_P, _P, _dbl, _dbl]),
    "pressure_apply": (ctypes.c_int, [_P, _P, _P, _P]),
    "pressure_solve": (ctypes.c_int, [_P, _P, _P, _dbl, _i32, _P, ctypes.POINTER(_i32), _P,
                                      ctypes.POINTER(_dbl), _P]),
    "pressure_solve_noalloc": (ctypes.c_int, [_P, _P, _P, _dbl, _i32, _P, ctypes.POINTER(_i32), _P,
                                              ctypes.POINTER(_dbl), _P]),
    "pressure_solve_mixed": (ctypes.c_int, [_P, _P, _P, _dbl, _dbl, _i32, _P, ctypes.POINTER(_i32),
                                            ctypes.POINTER(_i32), _P, ctypes.POINTER(_dbl), _P]),
    "pressure_footprint": (ctypes.c_int, [_PMESH, _i32, ctypes.POINTER(ctypes.c_uint64)]),
    "pressure_destroy": (None, [_P]),
    "pressure_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "pressure_layout": (ctypes.c_int, [_PMESH, _P, _P, _P, _P, _P]),
    "pressure_set_variant": (ctypes.c_int, [_P, _i32]),
    "pressure_set_mixed_mode": (ctypes.c_int, [_P, _i32]),
    "pressure_timing_enable": (ctypes.c_int, [_P, _i32]),
    "pressure_timing_read": (ctypes.c_int, [_P, ctypes.POINTER(_i64), ctypes.POINTER(_dbl)]),
    "pressure_info": (ctypes.c_int, [_P, ctypes.POINTER(_i64), _i32]),
    "pressure_batch_create": (ctypes.c_int, [_P, _i32, _P, ctypes.POINTER(_P)]),
    "pressure_batch_create_mixed": (ctypes.c_int, [_P, _i32, _P, _dbl, ctypes.POINTER(_P)]),
    "pressure_batch_solve": (ctypes.c_int, [_P, _P, _P, _dbl, _i32, _P, _P, _P, _P, _P]),
    "pressure_batch_set_graph": (ctypes.c_int, [_P, _i32]),
    "pressure_batch_set_persistent": (ctypes.c_int, [_P, _i32]),
    "pressure_batch_set_barrier_limit": (ctypes.c_int, [_P, ctypes.c_int64]),
    "pressure_batch_step_launch": (ctypes.c_int, [_P, _P]),
    "pressure_batch_step_wait": (ctypes.c_int, [_P, _P]),
    "pressure_batch_step_poll": (ctypes.c_int, [_P, _P]),
    "pressure_batch_next_index": (ctypes.c_int, [_P, ctypes.POINTER(_i32)]),
    "pressure_batch_begin": (ctypes.c_int, [_P, _i32, _P, _P, _dbl, _i32, _P]),
    "pressure_batch_step": (ctypes.c_int, [_P, _P, _P]),
    "pressure_batch_finish": (ctypes.c_int, [_P, _i32, _P, _dbl, _P, ctypes.POINTER(_i32), ctypes.POINTER(_dbl), _P]),
    "pressure_batch_destroy": (None, [_P]),
    "pressure_batch_tune": (ctypes.c_int, [_P, _i32, _i32, ctypes.c_char_p, _P, ctypes.POINTER(_dbl)]),
    "pressure_tune_tile": (ctypes.c_int, [_PMESH, _P, _dbl, _dbl, _i32, _i32, ctypes.c_char_p,
                                          ctypes.POINTER(_i32), ctypes.POINTER(_dbl)]),
    "pressure_dual_count": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "pressure_dual_faces": (ctypes.c_int, [_P, _P, _P]),
    "pressure_projection": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _dbl, _dbl, _i32, _dbl, _i32,
                                           _P, _P, _P, _P, _P]),
    "pressure_transport": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _dbl, _dbl, _dbl, _dbl, _dbl, _P, _P, _P, _P]),
    "pressure_transport_lader": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _dbl, _dbl, _dbl, _dbl, _dbl, _P, _P, _P,
                                                _P]),
    "pressure_post_projection": (ctypes.c_int, [_P, _P, _P, _P, _P, _dbl, _dbl, _P, _P]),
}

_lib = None


def load():
    """Load libpressure.so (built by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libpressure.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class PressureError(RuntimeError):
    def __init__(self, status, what):
        msg = load().pressure_strerror(status).decode()
        super().__init__("%s failed: %s (%d)" % (what, msg, status))
        self.status = status


def check(status, what):
    if status < 0:
        raise PressureError(status, what)
    return status
