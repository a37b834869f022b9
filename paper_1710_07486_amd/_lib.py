"""ctypes declarations of the C ABI in include/telbm.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtelbm.so")

OK, ERR_INVAL, ERR_UNSTABLE, ERR_DEVICE, ERR_NOMEM = 0, 1, 2, 3, 4
D2Q9, D3Q27 = 0, 1
FP64, FP32_MIXED = 0, 1
FIELDS = {"rho": 0, "phi": 1, "ux": 2, "uy": 3, "uz": 4, "c1": 5, "c2": 6, "mu_rho": 7, "mu_phi": 8,
          "fx": 9, "fy": 10, "fz": 11}


class TelbmParams(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("eos", ctypes.c_int32),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double), ("T", ctypes.c_double),
        ("rho_g", ctypes.c_double), ("rho_l", ctypes.c_double),
        ("lambda1", ctypes.c_double), ("lambda2", ctypes.c_double), ("lambda3", ctypes.c_double),
        ("kappa1", ctypes.c_double), ("kappa2", ctypes.c_double), ("kappa3", ctypes.c_double),
        ("chi", ctypes.c_double), ("nu", ctypes.c_double), ("mobility", ctypes.c_double),
        ("tau_phi", ctypes.c_double), ("rho_ref", ctypes.c_double),
        ("diag_every", ctypes.c_uint32), ("reserved1", ctypes.c_uint32),
        ("omega", ctypes.c_double),
        ("walls", ctypes.c_int32), ("reserved2", ctypes.c_uint32),
        ("theta_rho_lo", ctypes.c_double), ("theta_rho_hi", ctypes.c_double),
        ("theta_phi_lo", ctypes.c_double), ("theta_phi_hi", ctypes.c_double),
        ("glattice", ctypes.c_int32), ("reserved3", ctypes.c_uint32),
    ]


class TelbmNlParams(ctypes.Structure):
    _fields_ = [("lambda4", ctypes.c_double), ("kappa4", ctypes.c_double)]


NL_FIELDS = {"rho": 0, "phi": 1, "psi": 2, "ux": 3, "uy": 4, "uz": 5, "c1": 6, "c2": 7, "c3": 8, "mu_rho": 9,
             "mu_phi": 10, "mu_psi": 11, "fx": 12, "fy": 13, "fz": 14}


class TelbmDiag(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("mass", ctypes.c_double), ("phi_total", ctypes.c_double),
        ("mom", ctypes.c_double * 3), ("max_u", ctypes.c_double), ("min_rho", ctypes.c_double),
        ("gamma_min", ctypes.c_double), ("gamma_max", ctypes.c_double), ("nonfinite", ctypes.c_int64),
    ]


class TelbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"telbm error {code}: {msg}")
        self.code = code


# name -> (restype, argtypes); mirrors include/telbm.h
_c, _vp, _d, _pd, _i, _i64, _sz = (ctypes.c_char_p, ctypes.c_void_p, ctypes.c_double,
                                   ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int64,
                                   ctypes.c_size_t)
PROTOTYPES = {
    "telbm_version": (_c, []),
    "telbm_critical_temperature": (_i, [_d, _d, _d, _pd]),
    "telbm_coexistence": (_i, [_d, _d, _d, _d, _pd, _pd, _pd, _pd]),
    "telbm_temperature_for_ratio": (_i, [_d, _d, _d, _d, _pd]),
    "telbm_eos_critical_temperature": (_i, [_i, _d, _d, _d, _d, _pd]),
    "telbm_eos_coexistence": (_i, [_i, _d, _d, _d, _d, _d, _pd, _pd, _pd, _pd]),
    "telbm_eos_temperature_for_ratio": (_i, [_i, _d, _d, _d, _d, _d, _pd]),
    "telbm_required_bytes": (_i, [ctypes.POINTER(TelbmParams), ctypes.POINTER(_sz)]),
    "telbm_create": (_i, [ctypes.POINTER(TelbmParams), _vp, _sz, ctypes.POINTER(_vp)]),
    "telbm_set_stream": (_i, [_vp, _vp]),
    "telbm_init_fields": (_i, [_vp, _vp, _vp, _vp, _i]),
    "telbm_step": (_i, [_vp, _i64]),
    "telbm_read": (_i, [_vp, _i, _vp, _i]),
    "telbm_diagnostics": (_i, [_vp, ctypes.POINTER(TelbmDiag)]),
    "telbm_last_diagnostics": (_i, [_vp, ctypes.POINTER(TelbmDiag)]),
    "telbm_sync": (_i, [_vp]),
    "telbm_step_count": (_i, [_vp, ctypes.POINTER(_i64)]),
    "telbm_time_kernels": (_i, [_vp, _i64, _pd, ctypes.POINTER(_i)]),
    "telbm_kernel_name": (_c, [_vp, _i]),
    "telbm_algorithmic_bytes_per_update": (_d, [_vp]),
    "telbm_destroy": (_i, [_vp]),
    "telbm_last_error": (_c, [_vp]),
    "telbm_nl_mobility": (_i, [ctypes.POINTER(TelbmParams), ctypes.POINTER(TelbmNlParams), _pd]),
    "telbm_nl_required_bytes": (_i, [ctypes.POINTER(TelbmParams), ctypes.POINTER(TelbmNlParams),
                                     ctypes.POINTER(_sz)]),
    "telbm_nl_create": (_i, [ctypes.POINTER(TelbmParams), ctypes.POINTER(TelbmNlParams), _vp, _sz,
                             ctypes.POINTER(_vp)]),
    "telbm_nl_set_stream": (_i, [_vp, _vp]),
    "telbm_nl_init_fields": (_i, [_vp, _vp, _vp, _vp, _vp, _i]),
    "telbm_nl_step": (_i, [_vp, _i64]),
    "telbm_nl_read": (_i, [_vp, _i, _vp, _i]),
    "telbm_nl_step_count": (_i, [_vp, ctypes.POINTER(_i64)]),
    "telbm_nl_destroy": (_i, [_vp]),
    "telbm_nl_last_error": (_c, [_vp]),
}

_lib = None


def load():
    """Load the in-tree HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch brings its own HIP runtime (same soname as /opt/rocm's); load it
        # first so that libtelbm binds to that one and the process holds a
        # single HIP runtime
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1710_07486_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
