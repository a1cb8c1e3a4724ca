"""ctypes loader of the in-tree HIP library (liblbm_hip.so).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/lbm.h.  There is no CPU
fallback; a missing or unloadable library raises."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "liblbm_hip.so")

_lib = None


class LbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("lbm status %d: %s" % (status, msg))
        self.status = status


class LbmParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dt", ctypes.c_double),
                ("lam", ctypes.c_double), ("mu", ctypes.c_double), ("rho", ctypes.c_double),
                ("bc", ctypes.c_int32), ("model", ctypes.c_int32), ("flags", ctypes.c_uint32)]


# (name, restype, argtypes) of every exported entry point of include/lbm.h
_VP, _I32, _I64, _D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)
SIGNATURES = [
    ("lbm_workspace_bytes", ctypes.c_size_t, [ctypes.POINTER(LbmParams)]),
    ("lbm_create", ctypes.c_int, [ctypes.POINTER(LbmParams), _VP, ctypes.c_size_t, _VP,
                                  ctypes.POINTER(_VP)]),
    ("lbm_init", ctypes.c_int, [_VP, _VP, _VP, _VP]),
    ("lbm_init_from_gradient", ctypes.c_int, [_VP, _VP, _VP, _VP]),
    ("lbm_set_populations", ctypes.c_int, [_VP, _VP]),
    ("lbm_set_wall_velocity", ctypes.c_int, [_VP, _I32, _VP, _VP, _I64]),
    ("lbm_set_body_force", ctypes.c_int, [_VP, _I32, _VP, _VP, _VP, _I64]),
    ("lbm_init_displacement", ctypes.c_int, [_VP, _VP]),
    ("lbm_displacement", ctypes.c_int, [_VP, _VP]),
    ("lbm_set_reference", ctypes.c_int, [_VP, _I32, _VP, _VP, _VP, _I64]),
    ("lbm_error_track", ctypes.c_int, [_VP, _I32]),
    ("lbm_error_sums", ctypes.c_int, [_VP, _PD]),
    ("lbm_step", ctypes.c_int, [_VP, _I64]),
    ("lbm_step_count", _I64, [_VP]),
    ("lbm_moments", ctypes.c_int, [_VP, _VP]),
    ("lbm_moments_U", ctypes.c_int, [_VP, _VP]),
    ("lbm_populations", ctypes.c_int, [_VP, _VP]),
    ("lbm_energy", ctypes.c_int, [_VP, _PD]),
    ("lbm_rel_l2", ctypes.c_int, [_VP, _VP, _PD]),
    ("lbm_lattice_constants", ctypes.c_int, [_VP, _PD, _PD, _PD]),
    ("lbm_step_config_count", _I32, []),
    ("lbm_step_config_info", ctypes.c_int, [_I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                            ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    ("lbm_get_step_config", ctypes.c_int, [_VP, ctypes.POINTER(_I32)]),
    ("lbm_set_step_config", ctypes.c_int, [_VP, _I32]),
    ("lbm_autotune", ctypes.c_int, [_VP, _I32, _I32, ctypes.POINTER(_I32), _PD]),
    ("lbm_time_step_config", ctypes.c_int, [_VP, _I32, _I32, _PD]),
    ("lbm_copy_f32", ctypes.c_int, [_VP, _VP, _I64, _VP]),
    ("lbm_tblock_config_count", _I32, []),
    ("lbm_tblock_config_info", ctypes.c_int,
     [_I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32),
      ctypes.POINTER(_I32)]),
    ("lbm_steps_per_launch", _I32, [_VP]),
    ("lbm_get_tblock_config", ctypes.c_int, [_VP, ctypes.POINTER(_I32)]),
    ("lbm_set_tblock_config", ctypes.c_int, [_VP, _I32]),
    ("lbm_set_tblock_split", ctypes.c_int, [_VP, _I32]),
    ("lbm_tblock_split_active", _I32, [_VP, _I32]),
    ("lbm_get_tblock_remainder", ctypes.c_int, [_VP, _I32, ctypes.POINTER(_I32)]),
    ("lbm_select_for_steps", ctypes.c_int, [_VP, _I64, ctypes.POINTER(_I32)]),
    ("lbm_time_tblock_config", ctypes.c_int, [_VP, _I32, _I32, _PD]),
    ("lbm_wop_scratch_bytes", ctypes.c_size_t, [ctypes.POINTER(LbmParams)]),
    ("lbm_wop_operand_bytes", ctypes.c_size_t, []),
    ("lbm_wop_build", ctypes.c_int, [ctypes.POINTER(LbmParams), _VP, _VP, _VP, ctypes.c_size_t,
                                     _VP]),
    ("lbm_wop_apply", ctypes.c_int, [ctypes.POINTER(LbmParams), _VP, _VP, _VP, _I32, _VP]),
    ("lbm_batch_workspace_bytes", ctypes.c_size_t, [_I32, _VP]),
    ("lbm_batch_create", ctypes.c_int, [_I32, _VP, _VP, ctypes.c_size_t, _VP,
                                        ctypes.POINTER(_VP)]),
    ("lbm_batch_node_offset", _I64, [_VP, _I32]),
    ("lbm_batch_step_count", _I64, [_VP]),
    ("lbm_batch_init", ctypes.c_int, [_VP, _VP, _VP]),
    ("lbm_batch_init_fields_f32", ctypes.c_int, [_VP, _VP]),
    ("lbm_batch_set_wall_velocity", ctypes.c_int, [_VP, _I32, _I32, _VP, _VP, _I64]),
    ("lbm_batch_step", ctypes.c_int, [_VP, _I64]),
    ("lbm_batch_step_eager", ctypes.c_int, [_VP, _I64]),
    ("lbm_batch_tblock_config_count", _I32, []),
    ("lbm_batch_tblock_config_info", ctypes.c_int,
     [_I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32),
      ctypes.POINTER(_I32)]),
    ("lbm_batch_get_tblock_config", ctypes.c_int, [_VP, ctypes.POINTER(_I32)]),
    ("lbm_batch_set_tblock_config", ctypes.c_int, [_VP, _I32]),
    ("lbm_batch_autotune", ctypes.c_int, [_VP, _I32, ctypes.POINTER(_I32), _PD]),
    ("lbm_batch_moments", ctypes.c_int, [_VP, _VP]),
    ("lbm_batch_moments_U", ctypes.c_int, [_VP, _VP]),
    ("lbm_batch_energy", ctypes.c_int, [_VP, _PD]),
    ("lbm_batch_rel_l2_fields", ctypes.c_int, [_VP, _VP, _PD]),
    ("lbm_batch_rel_l2_pair", ctypes.c_int, [_VP, _VP, _VP, _PD]),
    ("lbm_rel_l2_pair_static", ctypes.c_int, [_I32, _VP, _VP, _VP, _PD, _VP]),
    ("lbm_batch_destroy", ctypes.c_int, [_VP]),
    ("sg_workspace_bytes", ctypes.c_size_t, [_VP]),
    ("sg_param_count", _I64, []),
    ("sg_create", ctypes.c_int, [_VP, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    ("sg_destroy", ctypes.c_int, [_VP]),
    ("sg_set_conv_mode", ctypes.c_int, [_VP, _I32]),
    ("sg_set_params", ctypes.c_int, [_VP, _VP]),
    ("sg_get_params", ctypes.c_int, [_VP, _VP]),
    ("sg_get_grads", ctypes.c_int, [_VP, _VP]),
    ("sg_forward", ctypes.c_int, [_VP, _VP, _I32, _I32, _VP]),
    ("sg_train_step", ctypes.c_int, [_VP, _VP, _VP, _I32, _I32, ctypes.c_float, _PD]),
    ("lbm_destroy", ctypes.c_int, [_VP]),
    ("lbm_last_error", ctypes.c_char_p, []),
]


def load(path: str = LIBPATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("HIP library %s is missing: build it with "
                           "paper_2408_01081_amd/build.py (or __graft_entry__.build())" % path)
    L = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(status: int):
    if status != 0:
        raise LbmError(status, load().lbm_last_error().decode())
