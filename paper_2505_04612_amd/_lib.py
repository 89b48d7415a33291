"""ctypes binding of libfastmap_hip.so (the C ABI in include/fastmap_hip.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  There is no fallback: if the library is missing or no GPU is
present, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfastmap_hip.so")

FM_OK, FM_EINVAL, FM_ESHAPE, FM_EDTYPE, FM_EHIP, FM_ENOMEM, FM_EDEVICE_CHECK, FM_ECOOP = 0, -1, -2, -3, -4, -5, -6, -7
FM_F64, FM_F32, FM_BF16 = 0, 1, 2
STATUS_NAMES = {0: "FM_OK", -1: "FM_EINVAL", -2: "FM_ESHAPE", -3: "FM_EDTYPE", -4: "FM_EHIP",
                -5: "FM_ENOMEM", -6: "FM_EDEVICE_CHECK", -7: "FM_ECOOP"}
# fm_check_bits
FM_CHECK_COORDS, FM_CHECK_PARAMS, FM_CHECK_DEGENERATE, FM_CHECK_LOSS = 1, 2, 4, 8

# Every symbol include/fastmap_hip.h declares.
EXPORTS = [
    "fm_create", "fm_destroy", "fm_last_error", "fm_version", "fm_set_check", "fm_check",
    "fm_scene_create", "fm_scene_destroy", "fm_scene_work_items",
    "fm_build_pair_grams", "fm_reweight", "fm_reweight_build",
    "fm_epipolar_loss_grad", "fm_adam_step", "fm_epipolar_solve", "fm_solve_barrier_failures",
    "fm_profile_enable", "fm_profile_read",
    "fm_match_features", "fm_mlp_forward", "fm_mlp_backward", "fm_mlp_backward_noalloc",
    "fm_translation_directions", "fm_translation_loss_grad", "fm_translation_solve", "fm_translation_merge",
    "fm_rotation_loss_grad", "fm_rotation_solve", "fm_rotation_init", "fm_translation_search",
    "fm_epipolar_focal_loss_grad", "fm_epipolar_focal_solve", "fm_poses_from_centres", "fm_pose_change",
]
(K_GRAM, K_SOLVE, K_ESSENTIALS, K_FINALIZE, K_PAIR, K_CAMERA, K_TA_SOLVE, K_TA_PAIR, K_TA_CAMERA,
 K_RA_SOLVE, K_RA_PAIR, K_RA_CAMERA, K_RA_INIT, K_TS_SEARCH, K_FO_PAIR, K_FO_CAMERA, K_FO_SOLVE, K_GRAM_CALL) = range(18)


class FastMapError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class AdamCfg(ctypes.Structure):
    _fields_ = [
        ("lr_rot", ctypes.c_float), ("lr_t", ctypes.c_float), ("lr_final_frac", ctypes.c_float),
        ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
        ("lr_step0", ctypes.c_int64), ("lr_total_steps", ctypes.c_int64), ("adam_step0", ctypes.c_int64),
        ("blocks", ctypes.c_int32),
    ]


class Mlp(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("W1", "b1", "W2", "b2", "W3", "b3", "feat_mean", "feat_std")]


class MlpGrad(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("W1", "b1", "W2", "b2", "W3", "b3")]


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_F = ctypes.c_float
_D = ctypes.c_double
_S = ctypes.c_int

_SIGNATURES = {
    "fm_create": (_S, [ctypes.POINTER(_P), _S]),
    "fm_destroy": (None, [_P]),
    "fm_last_error": (ctypes.c_char_p, [_P]),
    "fm_version": (ctypes.c_char_p, []),
    "fm_set_check": (_S, [_P, _S]),
    "fm_check": (_S, [_P, _P, ctypes.POINTER(ctypes.c_uint32)]),
    "fm_scene_create": (_S, [_P, _I64, _I64, _I32, _P, _P, _P, _S, _P, ctypes.POINTER(_P)]),
    "fm_scene_destroy": (None, [_P]),
    "fm_scene_work_items": (_I64, [_P]),
    "fm_build_pair_grams": (_S, [_P, _P, _P, _P, _P, _P]),
    "fm_reweight": (_S, [_P, _P, _P, _F, _F, _P, _P, _P, _P]),
    "fm_reweight_build": (_S, [_P, _P, _P, _F, _F, _P, _P, _P, _P]),
    "fm_epipolar_loss_grad": (_S, [_P, _P, _P, _S, _P, _D, _P, _P, _P, _P]),
    "fm_adam_step": (_S, [_P, _I64, _P, _P, _P, _P, _I64, _P, _S, _F, _F, _F, _P]),
    "fm_epipolar_solve": (_S, [_P, _P, _P, _S, _P, _P, _P, _I32, ctypes.POINTER(AdamCfg), _D, _P, _P, _P]),
    "fm_solve_barrier_failures": (_S, [_P, _P, ctypes.POINTER(_I64)]),
    "fm_profile_enable": (_S, [_P, _S]),
    "fm_match_features": (_S, [_P, _P, _P, _F, _P, _P]),
    "fm_mlp_forward": (_S, [_P, _I64, _P, ctypes.POINTER(Mlp), _F, _P, _P, _P]),
    "fm_mlp_backward": (_S, [_P, _I64, _P, ctypes.POINTER(Mlp), _P, _P, ctypes.POINTER(MlpGrad), _P]),
    "fm_mlp_backward_noalloc": (_S, [_P, _I64, _P, ctypes.POINTER(Mlp), _P, _P, ctypes.POINTER(MlpGrad), _P]),
    "fm_profile_read": (_S, [_P, _S, ctypes.POINTER(_D), ctypes.POINTER(_I64)]),
    "fm_translation_directions": (_S, [_P, _P, _P, _P, _P, _P]),
    "fm_translation_loss_grad": (_S, [_P, _P, _P, _I32, _P, _P, _P, _P]),
    "fm_translation_solve": (_S, [_P, _P, _P, _I32, _P, _P, _P, _I32, ctypes.POINTER(AdamCfg), _P, _P]),
    "fm_translation_merge": (_S, [_P, _P, _P, _I32, _P, _P, _P, _P, _P]),
    "fm_rotation_loss_grad": (_S, [_P, _P, _P, _P, _P, _P, _P]),
    "fm_rotation_solve": (_S, [_P, _P, _P, _P, _P, _P, _I32, ctypes.POINTER(AdamCfg), _P, _P]),
    "fm_rotation_init": (_S, [_P, _P, _P, _P, _I32, _I32, _P, _P, _P]),
    "fm_translation_search": (_S, [_P, _P, _P, _P, _P, _I32, _P, _P, _P, _P, _P]),
    "fm_epipolar_focal_loss_grad": (_S, [_P, _P, _P, _S, _P, _P, _D, _P, _P, _P, _P, _P]),
    "fm_epipolar_focal_solve": (_S, [_P, _P, _P, _S, _P, _P, _P, _P, _P, _P, _I32, ctypes.POINTER(AdamCfg), _F, _D,
                                     _P, _P, _P]),
    "fm_poses_from_centres": (_S, [_P, _I32, _P, _P, _P, _P]),
    "fm_pose_change": (_S, [_P, _P, _P, _P, _F, _F, _P, _P, _P, _P]),
}

_lib = None


def load(path: str | None = None) -> ctypes.CDLL:
    """Load the library (once) and declare every exported function."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise FastMapError(FM_EHIP, f"{p} is missing: build it with paper_2505_04612_amd.build.build()")
    lib = ctypes.CDLL(p)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def check(ctx, status: int) -> None:
    if status != FM_OK:
        msg = load().fm_last_error(ctx).decode() if ctx else "no context"
        raise FastMapError(status, msg)
