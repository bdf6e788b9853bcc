"""ctypes loader for libfmap.so (the C ABI in include/fmap.h).

The library is loaded lazily on first use and never replaced by anything else:
if it is missing, every call raises, there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmap.so")

FMAP_OK = 0
STATUS_NAMES = {0: "FMAP_OK", 1: "FMAP_ERR_NULL", 2: "FMAP_ERR_SHAPE", 3: "FMAP_ERR_VALUE", 4: "FMAP_ERR_DTYPE",
                5: "FMAP_ERR_WORKSPACE", 6: "FMAP_ERR_UNSUPPORTED", 7: "FMAP_ERR_HIP"}
FMAP_MASK_LAPLACIAN, FMAP_MASK_RESOLVENT = 0, 1
FMAP_F32, FMAP_BF16 = 0, 1
FMAP_NOALLOC_SCRATCH_BYTES = 32 << 20  # include/fmap.h

# Every symbol include/fmap.h declares, with (restype, argtypes).
_vp, _i32, _i64, _f32, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_size_t
SIGNATURES = {
    "fmap_abi_version": (_i32, []),
    "fmap_max_k": (_i32, []),
    "fmap_status_str": (ctypes.c_char_p, [_i32]),
    "fmap_project_workspace_bytes": (_sz, [_i64, _i64, _i64, _i64, _i32]),
    "fmap_project": (_i32, [_vp, _vp, _vp, _i32, _i64, _i64, _i64, _i64, _vp, _vp, _sz, _vp]),
    "fmap_project_noalloc": (_i32, [_vp, _vp, _vp, _i32, _i64, _i64, _i64, _i64, _vp, _vp]),
    "fmap_project_backward": (_i32, [_vp, _vp, _i32, _vp, _i64, _i64, _i64, _i64, _vp, _vp]),
    "fmap_solve_workspace_bytes": (_sz, [_i64, _i64, _i64, _i64]),
    "fmap_factor_floats": (_sz, [_i64, _i64]),
    "fmap_solve": (_i32, [_vp, _vp, _vp, _vp, _vp, _i32, _f32, _i64, _i64, _i64, _i64, _i32, _f32, _vp, _vp, _vp,
                          _vp, _vp, _sz, _vp]),
    "fmap_solve_backward": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _f32, _i64, _i64, _i64, _i64, _vp, _vp,
                                   _vp, _vp, _vp, _vp, _sz, _vp]),
    "fmap_project_pinv_workspace_bytes": (_sz, [_i64, _i64, _i64, _i64, _i32]),
    "fmap_project_pinv": (_i32, [_vp, _vp, _i32, _i64, _i64, _i64, _i64, _vp, _vp, _sz, _vp]),
    "fmap_project_pinv_backward": (_i32, [_vp, _i32, _vp, _i64, _i64, _i64, _i64, _vp, _vp, _sz, _vp]),
    "fmap_solve_resolutions_workspace_bytes": (_sz, [_i64, _i64, _i64, _i64, _i32, _vp, _vp]),
    "fmap_solve_vectorized_workspace_bytes": (_sz, [_i64, _i64, _i64, _i64]),
    "fmap_solve_vectorized": (_i32, [_vp, _vp, _vp, _vp, _vp, _i64, _i64, _i64, _i64, _vp, _vp, _vp, _sz, _vp]),
    "fmap_solve_resolutions": (_i32, [_vp, _vp, _vp, _vp, _vp, _i32, _f32, _i64, _i64, _i64, _i64, _i32, _vp, _vp,
                                      _vp, _vp, _vp, _sz, _vp]),
    "fmap_gradient_features": (_i32, [_vp, _vp, _vp, _i32, _i64, _i64, _vp, _vp]),
    "fmap_overlap_metrics": (_i32, [_vp, _vp, _vp, _i64, _i64, _f32, _vp, _vp, _vp]),
    "fmap_plan_create": (_i32, [_vp, _i32, _i64, _i32, _f32, _i32, ctypes.c_char_p, _vp, _vp]),
    "fmap_plan_forward": (_i32, [_vp, _vp]),
    "fmap_plan_backward": (_i32, [_vp, _vp]),
    "fmap_plan_tuning": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "fmap_plan_groups": (_i32, [_vp, _vp]),
    "fmap_plan_group": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "fmap_plan_destroy": (_i32, [_vp]),
}


class FmapPair(ctypes.Structure):
    """struct fmap_pair: one shape pair of a plan (device pointers and sizes)."""
    _fields_ = [(name, _vp) for name in ("phi_x", "phi_y", "mass_x", "mass_y", "feat_x", "feat_y", "evals_x",
                                         "evals_y", "lambda_", "C", "info", "A", "B", "dC", "dF_x", "dF_y")] + \
               [("n_x", _i64), ("n_y", _i64), ("k", _i64)]

_lib = None


class FmapError(RuntimeError):
    def __init__(self, fn: str, status: int):
        self.status = status
        super().__init__(f"{fn}: {STATUS_NAMES.get(status, status)} ({status_str(status)})")


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2604_10377_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_str(status: int) -> str:
    return lib().fmap_status_str(int(status)).decode()


def check(fn: str, status: int) -> None:
    if status != FMAP_OK:
        raise FmapError(fn, status)
