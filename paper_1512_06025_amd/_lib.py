"""ctypes binding of libbbdg.so (argument marshalling only).

Every entry point of include/bbdg.h is exposed under the same name.  The
library is loaded from this package directory; a missing library is an
error (there is no fallback implementation).
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# BBDG_LIBRARY may name another build of the same library (the host-sanitized
# one of sanitize_build.py); by default the in-tree libbbdg.so is loaded.
LIB_PATH = os.environ.get("BBDG_LIBRARY") or os.path.join(HERE, "libbbdg.so")

BBDG_F64, BBDG_F32 = 0, 1
BBDG_BC_RIGID, BBDG_BC_PRESSURE_RELEASE = 0, 1
BBDG_RHS_FULL, BBDG_RHS_VOLUME, BBDG_RHS_SURFACE = 0, 1, 2
BBDG_STORES_AUTO, BBDG_STORES_PLAIN, BBDG_STORES_NONTEMPORAL = 0, 1, 2

ERRORS = {
    0: "BBDG_OK", -1: "BBDG_E_ARG", -2: "BBDG_E_ORDER", -3: "BBDG_E_MESH",
    -4: "BBDG_E_NONFINITE", -5: "BBDG_E_DTYPE", -6: "BBDG_E_BC", -7: "BBDG_E_DEVICE",
    -8: "BBDG_E_LAUNCH", -9: "BBDG_E_MODE", -10: "BBDG_E_OUTSIDE", -11: "BBDG_E_RESIDENT",
    -12: "BBDG_E_TIMEOUT", -13: "BBDG_E_TOOBIG",
}
BBDG_NOALLOC_WORK_BYTES = 64 << 20

# name -> (restype, argtypes)
_c = ctypes
SIGNATURES = {
    "bbdg_np": (_c.c_int, [_c.c_int]),
    "bbdg_alpha_table": (_c.c_int, [_c.c_int, _c.c_void_p]),
    "bbdg_mesh_geometry": (_c.c_int, [_c.c_int64, _c.c_int64, _c.c_void_p, _c.c_void_p,
                                      _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "bbdg_create": (_c.c_int, [_c.POINTER(_c.c_void_p), _c.c_int, _c.c_int, _c.c_int64,
                               _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                               _c.c_int, _c.c_int]),
    "bbdg_nodal_create": (_c.c_int, [_c.POINTER(_c.c_void_p), _c.c_int, _c.c_int, _c.c_int64,
                                     _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                     _c.c_int, _c.c_int]),
    "bbdg_nodal_ept_create": (_c.c_int, [_c.POINTER(_c.c_void_p), _c.c_int, _c.c_int, _c.c_int64,
                                         _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                         _c.c_int, _c.c_int]),
    "bbdg_nodal_operators": (_c.c_int, [_c.c_int, _c.c_void_p, _c.c_void_p]),
    "bbdg_basis": (_c.c_int, [_c.c_void_p]),
    "bbdg_info": (_c.c_int, [_c.c_void_p, _c.POINTER(_c.c_int), _c.POINTER(_c.c_int),
                             _c.POINTER(_c.c_int64), _c.POINTER(_c.c_int)]),
    "bbdg_rhs": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int, _c.c_void_p]),
    "bbdg_work_bytes": (_c.c_size_t, [_c.c_void_p]),
    "bbdg_run": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_double, _c.c_double,
                            _c.c_int64, _c.c_void_p]),
    "bbdg_run_noalloc": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_double, _c.c_double, _c.c_int64,
                                    _c.c_void_p]),
    "bbdg_set_store_policy": (_c.c_int, [_c.c_void_p, _c.c_int]),
    "bbdg_nontemporal_stores": (_c.c_int, [_c.c_void_p]),
    "bbdg_locate_points": (_c.c_int, [_c.c_int64, _c.c_int64, _c.c_void_p, _c.c_void_p, _c.c_int64,
                                      _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "bbdg_bernstein_eval": (_c.c_int, [_c.c_int, _c.c_int64, _c.c_void_p, _c.c_void_p]),
    "bbdg_source_coeffs": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "bbdg_batched_work_bytes": (_c.c_size_t, [_c.c_void_p, _c.c_int64]),
    "bbdg_run_batched": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_int64, _c.c_void_p, _c.c_void_p,
                                    _c.c_double, _c.c_double, _c.c_int, _c.c_void_p, _c.c_void_p,
                                    _c.c_void_p, _c.c_void_p, _c.c_double, _c.c_double, _c.c_int64,
                                    _c.c_int, _c.c_void_p]),
    "bbdg_status": (_c.c_int, [_c.c_void_p]),
    "bbdg_batched_occupancy": (_c.c_int, [_c.c_void_p, _c.c_int, _c.c_int, _c.c_void_p]),
    "bbdg_set_barrier_timeout": (_c.c_int, [_c.c_void_p, _c.c_double]),
    "bbdg_tune_batched": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_void_p, _c.POINTER(_c.c_int),
                                     _c.c_void_p]),
    "bbdg_set_wavespeed": (_c.c_int, [_c.c_void_p, _c.c_void_p]),
    "bbdg_misfit_work_bytes": (_c.c_size_t, [_c.c_void_p, _c.c_int64, _c.c_int, _c.c_int64, _c.c_int64,
                                             _c.c_int64]),
    "bbdg_misfit": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_double,
                               _c.c_double, _c.c_int, _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_double,
                               _c.c_double, _c.c_int64, _c.c_int64, _c.c_int64, _c.c_void_p, _c.c_void_p,
                               _c.c_void_p]),
    "bbdg_misfit_gradient": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                        _c.c_double, _c.c_double, _c.c_int, _c.c_void_p, _c.c_void_p,
                                        _c.c_void_p, _c.c_double, _c.c_double, _c.c_int64, _c.c_int64,
                                        _c.c_int64, _c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "bbdg_last_hip_error": (_c.c_int, []),
    "bbdg_copy_probe": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "bbdg_destroy": (_c.c_int, [_c.c_void_p]),
    "bbdg_strerror": (_c.c_char_p, [_c.c_int]),
}

_lib = None


class BBDGError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        detail = ""
        if code in (-8, -11) and _lib is not None:
            detail = " [hipError %d]" % _lib.bbdg_last_hip_error()
        super().__init__("%s failed: %s (%d)%s" % (where, ERRORS.get(code, "?"), code, detail))


def load():
    """Load libbbdg.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libbbdg.so is not built (run python paper_1512_06025_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code, where):
    if code != 0:
        raise BBDGError(code, where)
    return code
