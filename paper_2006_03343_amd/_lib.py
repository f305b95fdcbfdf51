"""ctypes declarations of ``libibm.so`` (the C ABI in ``include/ibm.h``).

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""
import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_int64, c_uint8, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libibm.so")

IBM_OK, IBM_E_ARG, IBM_E_STATE, IBM_E_HIP, IBM_E_NOMEM, IBM_E_RANGE, IBM_E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
IBM_F32, IBM_F64 = 0, 1
IBM_PREC_PLAIN, IBM_PREC_MIXED = 0, 1
IBM_GRID_UV, IBM_GRID_W = 0, 1

EXPORTS = ["ibm_create", "ibm_destroy", "ibm_levelset_prepare", "ibm_counts", "ibm_band_size",
           "ibm_band_export", "ibm_mask_export", "ibm_wall_stress", "ibm_apply", "ibm_apply_spectral", "ibm_ab2_predict", "ibm_pressure_project",
           "ibm_sgs_stress", "ibm_apply_sgs", "ibm_stage_vjp", "ibm_chester_prepare",
           "ibm_chester_counts", "ibm_chester_wall_stress", "ibm_apply_noalloc",
           "ibm_stage",
           "ibm_set_tile", "ibm_get_tile", "ibm_last_error", "ibm_autotune", "ibm_batch_create",
           "ibm_batch_destroy", "ibm_batch_prepare", "ibm_batch_bind", "ibm_batch_tune",
           "ibm_batch_run", "ibm_batch_capture", "ibm_batch_launch", "ibm_batch_case"]
IBM_TUNE_FORCE, IBM_TUNE_BATCH = 1, 2


class IbmGrid(ctypes.Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("nz", c_int),
                ("dx", c_double), ("dy", c_double), ("dz", c_double)]


class IbmParams(ctypes.Structure):
    _fields_ = [("band_width", c_double), ("phi_c", c_double), ("kappa", c_double)]


class IbmCaseIO(ctypes.Structure):
    _fields_ = [("u", c_void_p), ("v", c_void_p), ("w", c_void_p), ("log_z0", c_void_p),
                ("tau", c_void_p * 6), ("ustar", c_void_p * 3), ("gradp", c_void_p * 3),
                ("div", c_void_p * 3), ("dt", c_double), ("drag_dev", c_void_p),
                ("stats_dev", c_void_p)]


class IbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          f"(or python paper_2006_03343_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    vp = c_void_p
    L.ibm_create.argtypes = [POINTER(vp), POINTER(IbmGrid), c_int, c_int]
    L.ibm_destroy.argtypes = [vp]
    L.ibm_levelset_prepare.argtypes = [vp, vp, vp, POINTER(IbmParams), vp]
    L.ibm_counts.argtypes = [vp, POINTER(c_int64)]
    L.ibm_band_size.argtypes = [vp, c_int, POINTER(c_int64)]
    L.ibm_band_export.argtypes = [vp, c_int, vp, vp]
    L.ibm_mask_export.argtypes = [vp, vp]
    L.ibm_wall_stress.argtypes = [vp, vp, vp, vp, c_double, vp, vp, vp, vp]
    L.ibm_apply.argtypes = [vp, vp, vp, vp, c_double, vp, vp, vp]
    L.ibm_apply_spectral.argtypes = [vp, vp, vp, vp, c_double, vp, vp, vp]
    L.ibm_apply_noalloc.argtypes = [vp, vp, vp, vp, c_double, vp, vp, vp]
    L.ibm_stage.argtypes = [vp, vp, vp, vp, c_double, vp, vp, vp, vp, c_double, vp, vp, vp, vp]
    L.ibm_ab2_predict.argtypes = [vp, vp, vp, vp, c_double, vp, vp]
    L.ibm_pressure_project.argtypes = [vp, vp, c_double, vp, vp, vp]
    L.ibm_sgs_stress.argtypes = [vp, vp, vp, vp, vp, vp, c_double, vp, c_double, c_double, vp, vp]
    L.ibm_apply_sgs.argtypes = [vp, vp, vp, vp, vp, vp, c_double, vp, c_double, c_double, vp, vp,
                                vp, c_double, vp, vp, vp]
    L.ibm_stage_vjp.argtypes = [vp, vp, vp, vp, c_double, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.ibm_chester_prepare.argtypes = [vp, vp, vp, vp]
    L.ibm_chester_counts.argtypes = [vp, POINTER(c_int64)]
    L.ibm_chester_wall_stress.argtypes = [vp, vp, vp, vp, c_double, vp, vp, c_double, c_int, vp,
                                          vp]
    L.ibm_set_tile.argtypes = [vp, c_int, c_int, c_int, c_int]
    L.ibm_get_tile.argtypes = [vp, vp]
    L.ibm_autotune.argtypes = [vp, c_char_p, c_int, vp]
    L.ibm_batch_create.argtypes = [POINTER(vp), c_int, vp, c_int, c_int]
    L.ibm_batch_destroy.argtypes = [vp]
    L.ibm_batch_prepare.argtypes = [vp, vp, vp, POINTER(IbmParams), vp, vp]
    L.ibm_batch_bind.argtypes = [vp, c_int, POINTER(IbmCaseIO)]
    L.ibm_batch_tune.argtypes = [vp, c_char_p, vp]
    L.ibm_batch_run.argtypes = [vp, vp]
    L.ibm_batch_capture.argtypes = [vp, vp]
    L.ibm_batch_launch.argtypes = [vp, vp]
    L.ibm_batch_case.argtypes = [vp, c_int, POINTER(vp)]
    L.ibm_last_error.restype = c_char_p
    for name in EXPORTS:
        if name not in ("ibm_last_error", "ibm_destroy", "ibm_batch_destroy"):
            getattr(L, name).restype = c_int
    _lib = L
    return L


def check(rc):
    if rc != IBM_OK:
        msg = load().ibm_last_error().decode(errors="replace")
        raise IbmError(rc, msg)
    return rc


def ptr_array(ptrs):
    """A C array of void* (None -> NULL)."""
    return (c_void_p * len(ptrs))(*[p if p else None for p in ptrs])
