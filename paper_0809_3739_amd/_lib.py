"""ctypes binding of libmpe.so (argument marshalling only).

Every entry point of ``include/mpe.h`` is declared here with the same name.
The library is loaded from this package directory; if it is missing the
import fails loudly -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpe.so")

MPE_OK = 0
STATUS = {
    0: "MPE_OK", 1: "MPE_ERR_INVALID_ARGUMENT", 2: "MPE_ERR_UNSUPPORTED", 3: "MPE_ERR_OUT_OF_MEMORY",
    4: "MPE_ERR_NOT_POSITIVE_DEFINITE", 5: "MPE_ERR_EIG_NO_CONVERGENCE", 6: "MPE_ERR_NONFINITE",
    7: "MPE_ERR_DEVICE", 8: "MPE_ERR_STATE",
}
MPE_FP64, MPE_FP32 = 0, 1
KERNEL_CLASSES = ["plane_fwd", "pencil", "plane_link", "plane_tail", "h_apply", "gram", "small_dense",
                  "rotate", "other"]

_dp = C.POINTER(C.c_double)
_vp = C.c_void_p
_i32 = C.c_int32

class SystemDesc(C.Structure):
    """mpe_system_desc of include/mpe.h."""
    _fields_ = [("grid", C.c_int32 * 3), ("box", C.c_double * 3), ("n_states", C.c_int32),
                ("n_guard", C.c_int32), ("V", C.c_void_p)]


# name -> (restype, argtypes)
SIGNATURES = {
    "mpe_abi_version": (C.c_int, []),
    "mpe_status_string": (C.c_char_p, [C.c_int]),
    "mpe_coefficients": (C.c_int, [_i32, _dp]),
    "mpe_plan_create": (C.c_int, [C.POINTER(_vp), C.POINTER(_i32), _dp, _i32, _i32, C.c_int, _i32, _vp]),
    "mpe_plan_destroy": (C.c_int, [_vp]),
    "mpe_last_error": (C.c_char_p, [_vp]),
    "mpe_workspace_bytes": (C.c_int64, [_vp]),
    "mpe_set_potential": (C.c_int, [_vp, _vp, C.c_double]),
    "mpe_step": (C.c_int, [_vp, _vp, C.c_double]),
    "mpe_apply_h": (C.c_int, [_vp, _vp, _vp]),
    "mpe_orthonormalize": (C.c_int, [_vp, _vp]),
    "mpe_rayleigh_ritz": (C.c_int, [_vp, _vp, _dp]),
    "mpe_residuals": (C.c_int, [_vp, _vp, _dp, _dp, _dp]),
    "mpe_iterate": (C.c_int, [_vp, _vp, C.c_double, _dp, _dp, _dp, _dp]),
    "mpe_forget_cached_h": (C.c_int, [_vp]),
    "mpe_set_states_per_launch": (C.c_int, [_vp, _i32]),
    "mpe_set_locked": (C.c_int, [_vp, _i32]),
    "mpe_set_locked_states": (C.c_int, [_vp, _vp]),
    "mpe_set_variances": (C.c_int, [_vp, _i32]),
    "mpe_get_locked": (_i32, [_vp]),
    "mpe_set_propagator": (C.c_int, [_vp, _i32]),
    "mpe_set_three_pass": (C.c_int, [_vp, _i32]),
    "mpe_get_three_pass": (_i32, [_vp]),
    "mpe_get_propagator": (_i32, [_vp]),
    "mpe_set_plane_shape": (C.c_int, [_vp, _i32, _i32, _i32]),
    "mpe_get_plane_shape": (C.c_int, [_vp, C.POINTER(_i32)]),
    "mpe_set_pencil_shape": (C.c_int, [_vp, _i32]),
    "mpe_get_pencil_shape": (_i32, [_vp]),
    "mpe_set_gemm_precision": (C.c_int, [_vp, _i32]),
    "mpe_autotune": (C.c_int, [_vp, _vp, C.c_double, _i32, C.c_char_p, _dp]),
    "mpe_set_graph": (C.c_int, [_vp, _i32]),
    "mpe_last_jacobi_sweeps": (C.c_int32, [_vp]),
    "mpe_small_dense_phases": (C.c_int, [_vp, _dp]),
    "mpe_profile_enable": (C.c_int, [_vp, _i32]),
    "mpe_get_kernel_times": (C.c_int, [_vp, _dp, C.POINTER(C.c_int64)]),
    "mpe_orthonormalize_noalloc": (C.c_int, [_vp, _i32, C.c_int64, C.c_int, _vp]),
    "mpe_noalloc_last_error": (C.c_char_p, []),
    "mpe_noalloc_prepare": (C.c_int, []),
    "mpe_batch_create": (C.c_int, [C.POINTER(_vp), _i32, C.POINTER(SystemDesc), _i32, C.c_int, C.c_double, _vp]),
    "mpe_batch_destroy": (C.c_int, [_vp]),
    "mpe_batch_last_error": (C.c_char_p, [_vp]),
    "mpe_batch_step": (C.c_int, [_vp, C.POINTER(_vp), C.c_double]),
    "mpe_batch_iterate": (C.c_int, [_vp, C.POINTER(_vp), C.c_double, _dp, _dp, _dp, _dp]),
    "mpe_batch_launches_per_step": (C.c_int32, [_vp]),
    "mpe_batch_set_batched_la": (C.c_int, [_vp, _i32]),
    "wsn_create": (C.c_int, [C.POINTER(_vp), _i32, _i32, _i32, C.c_uint64, _vp]),
    "wsn_destroy": (C.c_int, [_vp]),
    "wsn_last_error": (C.c_char_p, [_vp]),
    "wsn_num_params": (C.c_int64, [_vp]),
    "wsn_get_params": (C.c_int, [_vp, _vp, _i32]),
    "wsn_set_params": (C.c_int, [_vp, _vp]),
    "wsn_zero_grads": (C.c_int, [_vp]),
    "wsn_forward": (C.c_int, [_vp, _vp, C.c_float, C.c_float, _i32, _vp]),
    "wsn_backward": (C.c_int, [_vp, _vp]),
    "wsn_layer_info": (C.c_int, [_vp, _i32, C.POINTER(_i32)]),
    "wsn_layer": (C.c_int, [_vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp]),
    "wsn_adam_step": (C.c_int, [_vp, C.c_float, C.c_float, C.c_float, C.c_float, _i32]),
    "wsn_subspace_loss": (C.c_int, [_vp, _vp, _vp, _i32, C.c_int64, _dp, _vp]),
    "wsn_procrustes_loss": (C.c_int, [_vp, _vp, _vp, _i32, C.c_int64, _dp, _vp]),
    "wsn_upsample_periodic": (C.c_int, [_vp, _i32, _i32, _i32, _vp, _vp]),
}


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libmpe.so not found at {path}; build it with `python -m paper_0809_3739_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


class MpeError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        self.code = code
        self.name = STATUS.get(code, f"status {code}")
        super().__init__(f"{self.name}: {msg}" if msg else self.name)


def check(code: int, plan=None) -> None:
    if code != MPE_OK:
        msg = lib().mpe_last_error(plan).decode() if plan else ""
        raise MpeError(code, msg)


def coefficients(order: int):
    """c_1..c_K of the order-2K expansion, computed by the library."""
    K = order // 2
    buf = (C.c_double * max(K, 1))()
    check(lib().mpe_coefficients(order, buf))
    return [buf[i] for i in range(K)]
