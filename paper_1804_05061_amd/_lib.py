"""ctypes declarations of the C ABI in include/srwcr.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# SRWCR_LIB names another build of the same library (the host-sanitizer
# build of the tests); by default the in-tree one.
LIB_PATH = os.environ.get("SRWCR_LIB") or os.path.join(_HERE, "libsrwcr.so")

SRWCR_OK = 0
STATUS_NAMES = {0: "SRWCR_OK", -1: "SRWCR_E_INVALID_ARG", -2: "SRWCR_E_DEGENERATE", -3: "SRWCR_E_WORKSPACE",
                -4: "SRWCR_E_HIP", -5: "SRWCR_E_UNSUPPORTED", -6: "SRWCR_E_NONFINITE", -7: "SRWCR_E_LINESEARCH"}

# symbols the header declares (the ABI test checks every one is exported)
EXPORTED = ["srwcr_ctrl_dims", "srwcr_plan_create", "srwcr_plan_destroy", "srwcr_workspace_bytes",
            "srwcr_normalize", "srwcr_minmax", "srwcr_eval", "srwcr_grad", "ffd_warp",
            "srwcr_grad_noalloc", "srwcr_lbfgs_default_opts", "register_lbfgs", "srwcr_debug_moments", "srwcr_debug_samples",
            "srwcr_plan_info", "srwcr_debug_check_flags",
            "srwcr_profile", "srwcr_profile_read", "srwcr_refine_ffd", "srwcr_bending_energy", "srwcr_lbfgs_minimize",
            "srwcr_eval_dense", "srwcr_grad_dense", "srwcr_batch_create", "srwcr_batch_destroy", "srwcr_batch_workspace_bytes", "srwcr_grad_batched",
            "raptor_patches_create", "raptor_patches_destroy", "raptor_workspace_bytes", "raptor_eval",
            "raptor_grad", "srwcr_grad_fixed", "srwcr_plan_create_tuned", "srwcr_last_error"]

MAX_BATCH = 32
NOALLOC_SCRATCH_BYTES = 64 << 20   # SRWCR_NOALLOC_SCRATCH_BYTES


class SrwcrProblem(ctypes.Structure):
    _fields_ = [("fixed_dims", ctypes.c_int32 * 3), ("moving_dims", ctypes.c_int32 * 3), ("n_bins", ctypes.c_int32),
                ("spatial_bins", ctypes.c_int32 * 3), ("ctrl_spacing", ctypes.c_int32 * 3), ("role", ctypes.c_int32),
                ("fixed_dtype", ctypes.c_int32), ("moving_dtype", ctypes.c_int32)]


class SrwcrLbfgsOpts(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("max_iter", ctypes.c_int32 * 3), ("history", ctypes.c_int32),
                ("stall_window", ctypes.c_int32), ("stall_tol", ctypes.c_double),
                ("bending_weight", ctypes.c_double)]


class SrwcrLbfgsReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32 * 3), ("evaluations", ctypes.c_int32 * 3),
                ("initial_value", ctypes.c_double * 3), ("final_value", ctypes.c_double * 3),
                ("status", ctypes.c_int32 * 3), ("seconds", ctypes.c_double * 3)]


class SrwcrBatchItem(ctypes.Structure):
    _fields_ = [("fixed", ctypes.c_void_p), ("moving", ctypes.c_void_p), ("ffd", ctypes.c_void_p),
                ("d_value", ctypes.c_void_p), ("d_grad", ctypes.c_void_p)]


class SrwcrTuning(ctypes.Structure):
    _fields_ = [("grad_item_voxels", ctypes.c_int32), ("value_workgroups", ctypes.c_int32)]


class SrwcrPatch(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_int32), ("y0", ctypes.c_int32), ("z0", ctypes.c_int32),
                ("x1", ctypes.c_int32), ("y1", ctypes.c_int32), ("z1", ctypes.c_int32)]


# int fg(void *user, const double *x, double *f, double *g)
FG_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double))


class SrwcrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load the in-tree HIP library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first (__graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
    pp = ctypes.POINTER(SrwcrProblem)
    sig = {
        "srwcr_ctrl_dims": (ctypes.c_int, [pp, ctypes.POINTER(i32)]),
        "srwcr_plan_create": (ctypes.c_int, [pp, ctypes.POINTER(vp)]),
        "srwcr_plan_destroy": (None, [vp]),
        "srwcr_workspace_bytes": (sz, [vp]),
        "srwcr_normalize": (ctypes.c_int, [vp, i64, dp, dp, i32, vp, i32, vp]),
        "srwcr_minmax": (ctypes.c_int, [vp, i64, ctypes.POINTER(dp), ctypes.POINTER(dp), vp]),
        "srwcr_eval": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, sz, vp]),
        "srwcr_grad": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp, sz, vp]),
        "srwcr_grad_noalloc": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp]),
        "srwcr_debug_check_flags": (ctypes.c_int, [ctypes.POINTER(i32), i32]),
        "ffd_warp": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "srwcr_lbfgs_default_opts": (None, [ctypes.POINTER(SrwcrLbfgsOpts)]),
        "register_lbfgs": (ctypes.c_int, [pp, vp, vp, vp, ctypes.POINTER(SrwcrLbfgsOpts),
                                          ctypes.POINTER(SrwcrLbfgsReport), vp]),
        "srwcr_debug_moments": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, sz, vp]),
        "srwcr_debug_samples": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, sz, vp]),
        "srwcr_plan_info": (ctypes.c_int, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "srwcr_profile": (ctypes.c_int, [vp, i32]),
        "srwcr_profile_read": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)]),
        "srwcr_refine_ffd": (ctypes.c_int, [ctypes.POINTER(i32), vp, ctypes.POINTER(i32), vp]),
        "srwcr_bending_energy": (ctypes.c_double, [pp, vp, vp]),
        "srwcr_lbfgs_minimize": (ctypes.c_int, [i64, ctypes.POINTER(dp), FG_FN, vp, i32, i32, i32, dp,
                                                ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(dp)]),
        "srwcr_eval_dense": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, sz, vp]),
        "srwcr_grad_dense": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp, sz, vp]),
        "srwcr_batch_create": (ctypes.c_int, [i32, ctypes.POINTER(vp), ctypes.POINTER(vp)]),
        "srwcr_batch_destroy": (None, [vp]),
        "srwcr_batch_workspace_bytes": (sz, [vp]),
        "srwcr_grad_batched": (ctypes.c_int, [vp, ctypes.POINTER(SrwcrBatchItem), vp, sz, vp]),
        "raptor_patches_create": (ctypes.c_int, [vp, ctypes.POINTER(SrwcrPatch), i32, ctypes.POINTER(vp)]),
        "raptor_patches_destroy": (None, [vp]),
        "raptor_workspace_bytes": (sz, [vp, vp]),
        "raptor_eval": (ctypes.c_int, [vp, vp, vp, vp, vp, i32, vp, vp, sz, vp]),
        "raptor_grad": (ctypes.c_int, [vp, vp, vp, vp, vp, i32, vp, vp, vp, sz, vp]),
        "srwcr_grad_fixed": (ctypes.c_int, [vp, vp, vp, vp, i32, vp, vp, vp, sz, vp]),
        "srwcr_plan_create_tuned": (ctypes.c_int, [pp, ctypes.POINTER(SrwcrTuning), ctypes.POINTER(vp)]),
        "srwcr_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(code: int) -> None:
    if code != SRWCR_OK:
        raise SrwcrError(code, load().srwcr_last_error().decode())
