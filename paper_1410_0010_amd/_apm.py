"""ctypes binding of libapm.so: the C ABI of include/apm.h under the same names.

Argument marshalling only -- every step of the solve runs in the HIP library.
If the library is missing or fails to load this module raises ImportError; there
is no fallback path.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libapm.so")

APM_OK = 0
APM_ERR_INVALID = 1
APM_ERR_OOM = 2
APM_ERR_DEVICE = 3
APM_ERR_RANGE = 4
APM_ERR_UNSUPPORTED = 5
APM_ERR_STATE = 6
APM_F32 = 1
APM_F64 = 2
APM_GRAD_SPECTRAL = 0
APM_GRAD_FD2 = 1
APM_ACC_F64 = 0
APM_ACC_F32_COMP = 1
APM_BC_ISOLATED = 0
APM_BC_PERIODIC = 1

STATUS_NAMES = {0: "APM_OK", 1: "APM_ERR_INVALID", 2: "APM_ERR_OOM", 3: "APM_ERR_DEVICE",
                4: "APM_ERR_RANGE", 5: "APM_ERR_UNSUPPORTED", 6: "APM_ERR_STATE"}


class apm_config(ctypes.Structure):
    _fields_ = [("G", ctypes.c_double), ("root_n", ctypes.c_int32),
                ("a_cells", ctypes.c_double), ("pad_factor", ctypes.c_double),
                ("ghost", ctypes.c_int32), ("brillouin", ctypes.c_int32),
                ("gradient", ctypes.c_int32), ("workspace_limit", ctypes.c_int64),
                ("boundary", ctypes.c_int32), ("strict", ctypes.c_int32),
                ("deposit_accum", ctypes.c_int32)]


class apm_grid(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("parent", ctypes.c_int32),
                ("lo", ctypes.c_int32 * 3), ("n", ctypes.c_int32 * 3)]


class apm_grid_layout(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("parent", ctypes.c_int32),
                ("lo", ctypes.c_int32 * 3), ("n", ctypes.c_int32 * 3),
                ("gmf_lo", ctypes.c_int32 * 3), ("gmf_n", ctypes.c_int32 * 3),
                ("fld_lo", ctypes.c_int32 * 3), ("fld_n", ctypes.c_int32 * 3),
                ("fft_n", ctypes.c_int32 * 3),
                ("gmf_offset", ctypes.c_int64), ("fld_offset", ctypes.c_int64),
                ("gas_offset", ctypes.c_int64), ("dx", ctypes.c_double)]


class apm_level_layout(ctypes.Structure):
    _fields_ = [("ngrids", ctypes.c_int32), ("first_grid", ctypes.c_int32),
                ("gmf_elems", ctypes.c_int64), ("fld_cells", ctypes.c_int64),
                ("gas_elems", ctypes.c_int64), ("dx", ctypes.c_double)]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_st = ctypes.c_int

# name -> (restype, argtypes); the exported symbols of include/apm.h
SIGNATURES = {
    "apm_config_default": (None, [ctypes.POINTER(apm_config)]),
    "apm_plan_create": (_st, [ctypes.POINTER(apm_config), ctypes.POINTER(apm_grid), _i32,
                              ctypes.POINTER(_vp)]),
    "apm_plan_destroy": (_st, [_vp]),
    "apm_plan_nlevels": (_i32, [_vp]),
    "apm_plan_ngrids": (_i32, [_vp]),
    "apm_plan_grid": (_st, [_vp, _i32, ctypes.POINTER(apm_grid_layout)]),
    "apm_plan_level": (_st, [_vp, _i32, ctypes.POINTER(apm_level_layout)]),
    "apm_last_error": (ctypes.c_char_p, []),
    "apm_create": (_st, [_vp, _i32, _vp, ctypes.POINTER(_vp)]),
    "apm_destroy": (_st, [_vp]),
    "apm_set_stream": (_st, [_vp, _vp]),
    "apm_owner": (_st, [_vp, _st, _vp, _vp, _vp, _i64, _vp]),
    "apm_deposit": (_st, [_vp, _st, _i32, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "apm_solve_level": (_st, [_vp, _st, _i32, _vp, _vp]),
    "apm_accel": (_st, [_vp, _st, _i32, _vp, _vp, _vp]),
    "apm_interp": (_st, [_vp, _st, _i32, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp]),
    "apm_totals": (_st, [_vp, _st, ctypes.POINTER(_vp), _vp, _vp, _i64, _vp, _vp, _vp, _vp,
                         ctypes.POINTER(ctypes.c_double)]),
    "apm_dropped": (_st, [_vp, _st, _vp, _vp, _vp, _vp, _i64, ctypes.POINTER(_i64),
                          ctypes.POINTER(ctypes.c_double)]),
    "apm_totals_noalloc": (_st, [_vp, _st, ctypes.POINTER(_vp), _vp, _vp, _i64, _vp, _vp, _vp,
                                 _vp, _vp]),
    "apm_solve": (_st, [_vp, _st, _vp, _vp, _vp, _vp, _i64, ctypes.POINTER(_vp), _vp, _vp, _vp,
                        _vp]),
    "apm_solve_totals": (_st, [_vp, _st, _vp, _i64, ctypes.POINTER(_vp), _vp, _vp, _vp, _vp,
                               ctypes.POINTER(ctypes.c_double)]),
    "apm_solve_totals_async": (_st, [_vp, _st, _vp, _i64, ctypes.POINTER(_vp), _vp, _vp, _vp, _vp,
                                     _vp]),
    "apm_gas_energy": (_st, [_vp, _st, _i32, _vp, _vp, ctypes.POINTER(ctypes.c_double)]),
    "apm_solve_adjoint": (_st, [_vp, _st, _vp, _vp, _vp, _vp, _i64, ctypes.POINTER(_vp), _vp,
                                _vp, _vp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp, _vp,
                                ctypes.POINTER(_vp)]),
    "apm_kick": (_st, [_vp, _st, _i64, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_double]),
    "apm_drift": (_st, [_vp, _st, _i64, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_double]),
    "apm_kinetic_energy": (_st, [_vp, _st, _vp, _vp, _vp, _vp, _i64,
                                 ctypes.POINTER(ctypes.c_double)]),
    "apm_leapfrog": (_st, [_vp, _st, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, ctypes.POINTER(_vp),
                           ctypes.c_double, _i32, _vp, _vp, _vp, _vp,
                           ctypes.POINTER(ctypes.c_double)]),
    "apm_evolve_subcycled": (_st, [_vp, _st, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64,
                                   ctypes.POINTER(_vp), ctypes.c_double, _i32,
                                   ctypes.POINTER(ctypes.c_double)]),
    "apm_field_ptr": (_vp, [_vp, _st, _i32]),
    "apm_gmf_ptr": (_vp, [_vp, _st, _i32]),
    "apm_set_graph": (_st, [_vp, _i32]),
    "apm_autotune": (_st, [_vp, _st, _i32, ctypes.c_char_p, _i32]),
    "apm_profile": (_st, [_vp, _i32]),
    "apm_profile_count": (_i32, [_vp]),
    "apm_profile_entry": (_st, [_vp, _i32, ctypes.c_char_p, _i32, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(_i64)]),
}


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libapm.so not built ({path}); run __graft_entry__.build() "
                          "or python -m paper_1410_0010_amd.build")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


class APMError(RuntimeError):
    def __init__(self, status, where):
        msg = lib().apm_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status, where):
    if status != APM_OK:
        raise APMError(status, where)
