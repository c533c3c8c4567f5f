"""ctypes declarations for libbxmg.so (the C ABI of include/bxmg.h).

The library must have been built in-tree (``__graft_entry__.build()`` or
``python paper_2403_12179_amd/build.py``); importing fails loudly otherwise --
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbxmg.so")

BXMG_OK = 0
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENOCONV", -5: "ENONFINITE", -6: "EBUSY"}
F64, F32 = 0, 1
PERIODIC, DIRICHLET0 = 0, 1


class BxmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(status, "?"), status, msg))
        self.status = status


class SolveParams(C.Structure):
    _fields_ = [("nu1", C.c_int32), ("nu2", C.c_int32), ("max_cycles", C.c_int32), ("precision", C.c_int32),
                ("prolong", C.c_int32), ("fixed_cycles", C.c_int32), ("rel_tol", C.c_double),
                ("abs_tol", C.c_double), ("dx", C.c_double), ("bottom_rtol", C.c_double),
                ("krylov", C.c_int32), ("reserved", C.c_int32), ("alpha", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("cycles", C.c_int32), ("levels", C.c_int32), ("nhist", C.c_int32),
                ("rel_resid_inf", C.c_double), ("resid_l2", C.c_double), ("f_inf", C.c_double),
                ("seconds", C.c_double), ("hist", C.c_double * 256), ("hist_l2", C.c_double * 256)]


_lib = None

I32P = C.POINTER(C.c_int32)
I64P = C.POINTER(C.c_int64)
DP = C.POINTER(C.c_double)
VP = C.c_void_p
H = C.c_void_p  # opaque handles


def _declare(lib):
    sig = {
        "bxmg_version": (C.c_int, []),
        "bxmg_last_error": (C.c_char_p, []),
        "bxmg_ctx_create": (C.c_int, [C.c_int, VP, C.POINTER(H)]),
        "bxmg_ctx_destroy": (None, [H]),
        "bxmg_define_boxarray": (C.c_int, [I32P, I32P, I32P, C.c_int32, C.POINTER(H)]),
        "bxmg_define_boxarray_list": (C.c_int, [I32P, I32P, I32P, C.c_int32, I32P, C.POINTER(H)]),
        "bxmg_boxarray_get": (C.c_int, [H, I32P, I32P]),
        "bxmg_boxarray_hierarchy": (C.c_int, [H, C.c_int32, I32P, I32P, I32P, C.c_int32, I32P]),
        "bxmg_boxarray_release": (None, [H]),
        "bxmg_multifab_bytes": (C.c_size_t, [H, C.c_int32, C.c_int32, C.c_int]),
        "bxmg_alloc_multifab": (C.c_int, [H, H, C.c_int32, C.c_int32, C.c_int, VP, C.POINTER(H)]),
        "bxmg_multifab_box_view": (C.c_int, [H, C.c_int32, C.POINTER(VP), I32P, I32P, I64P]),
        "bxmg_multifab_info": (C.c_int, [H, C.POINTER(VP), C.POINTER(C.c_size_t), I32P, I32P, I32P]),
        "bxmg_multifab_copy_host": (C.c_int, [H, C.c_int32, VP, C.c_int32, VP]),
        "bxmg_multifab_release": (None, [H]),
        "bxmg_fill_boundary": (C.c_int, [H, C.c_int32, C.c_int32, C.c_int32, VP]),
        "bxmg_apply_domain_bc": (C.c_int, [H, C.c_int32, C.c_int32, C.c_int32, VP]),
        "bxmg_fill_boundary_noalloc": (C.c_int, [H, C.c_int32, C.c_int32, C.c_int32, VP]),
        "bxmg_parallel_copy": (C.c_int, [H, C.c_int32, H, C.c_int32, C.c_int32, C.c_int32, VP]),
        "bxmg_solve_params_default": (None, [C.POINTER(SolveParams)]),
        "bxmg_mlmg_solve": (C.c_int, [H, C.POINTER(SolveParams), H, H, H, C.POINTER(SolveInfo)]),
        "bxmg_heat_step": (C.c_int, [H, C.POINTER(SolveParams), H, H, H, C.c_double, C.POINTER(SolveInfo)]),
        "bxmg_nodal_solve": (C.c_int, [H, C.POINTER(SolveParams), H, VP, VP, C.POINTER(SolveInfo)]),
        "bxmg_composite_solve": (C.c_int, [H, C.POINTER(SolveParams), H, H, H, H, C.POINTER(SolveInfo)]),
        "bxmg_ctx_tune": (C.c_int, [H, C.c_int32, C.c_int32]),
        "bxmg_autotune": (C.c_int, [H, C.POINTER(SolveParams), H, H, H, C.c_int32, I32P, DP, I32P]),
        "bxmg_profile_stage": (C.c_int, [H, C.c_int32]),
        "bxmg_profile_read": (C.c_int, [H, I64P, DP, C.c_int32]),
        "bxmg_gs_colour": (C.c_int, [H, H, H, H, C.c_double, C.c_int32]),
        "bxmg_residual": (C.c_int, [H, H, H, H, C.c_double, H, DP]),
        "bxmg_restrict": (C.c_int, [H, H, H]),
        "bxmg_prolong_add": (C.c_int, [H, H, H, C.c_int32]),
        "bxmg_bottom_solve": (C.c_int, [H, H, H, H, C.c_double, C.c_double, I32P]),
        "bxmg_batch_create": (C.c_int, [H, C.c_size_t, C.c_int32, C.c_int32, C.POINTER(SolveParams), C.POINTER(H)]),
        "bxmg_batch_destroy": (None, [H]),
        "bxmg_batch_footprint": (C.c_size_t, [H, H]),
        "bxmg_batch_add": (C.c_int, [H, H, H, H, C.c_double, I64P]),
        "bxmg_batch_step": (C.c_int, [H, C.c_int32, I32P]),
        "bxmg_batch_launch": (C.c_int, [H, C.c_int32]),
        "bxmg_batch_collect": (C.c_int, [H, I32P]),
        "bxmg_batch_poll": (C.c_int, [H, C.c_int32, I64P, C.POINTER(SolveInfo), I32P]),
        "bxmg_batch_remove": (C.c_int, [H, C.c_int64]),
        "bxmg_batch_stats": (C.c_int, [H, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t), I32P, I32P]),
        "bxmg_batch_set": (C.c_int, [H, C.c_int32, C.c_int32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def lib():
    """The loaded library; raises ImportError if it has not been built."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime (same sonames as ROCm's).  Loading it
        # first makes libbxmg.so bind to that copy, so the process holds one
        # HIP runtime that both torch and the library use.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError("libbxmg.so is not built (run __graft_entry__.build() or "
                              "python paper_2403_12179_amd/build.py)")
        _lib = _declare(C.CDLL(LIB_PATH))
    return _lib


def check(status):
    if status != BXMG_OK:
        raise BxmgError(status, lib().bxmg_last_error().decode())
    return status


def i32(seq):
    arr = (C.c_int32 * len(seq))(*[int(x) for x in seq])
    return arr
