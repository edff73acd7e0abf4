"""ctypes binding of libppsolve.so (the C ABI of include/ppsolve.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  There is no fallback: if the library has not been built the import of
the solver fails with an error that says so.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libppsolve.so")

PP_F64, PP_F32, PP_F32_REFINED = 0, 1, 2
PP_GAUGE_MEAN, PP_GAUGE_PIN, PP_GAUGE_PIN_RAW = 0, 1, 2

STATUS = {
    0: "PP_OK", -1: "PP_ERR_ARG", -2: "PP_ERR_BC", -3: "PP_ERR_SIZE", -4: "PP_ERR_ALIAS",
    -5: "PP_ERR_WORKSPACE", -6: "PP_ERR_HIP", -7: "PP_ERR_NOT_CONVERGED", -8: "PP_ERR_NONFINITE",
    -9: "PP_ERR_SCRATCH",
}

# size of the fixed workspace behind pp_solve_noalloc (PP_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 128 * 1024 * 1024

EXPORTED = [
    "pp_plan_create", "pp_plan_set_gauge", "pp_plan_set_zsolver", "pp_plan_set_zsplit", "pp_plan_set_refinement",
    "pp_plan_workspace_bytes",
    "pp_solve", "pp_solve_bc", "pp_solve_adjoint", "pp_plan_last_info", "pp_plan_set_timing", "pp_plan_kernel_times",
    "pp_plan_destroy", "pp_status_string", "pp_solve_noalloc", "pp_stream_copy",
]

_lib = None


class PPError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)} ({status_string(status)})")


def load():
    """Load libppsolve.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_1909_05423_amd.build or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.pp_plan_create.argtypes = [i, i, i, ctypes.c_char_p, ctypes.POINTER(d), i, i, ctypes.POINTER(vp)]
    lib.pp_plan_create.restype = i
    lib.pp_plan_set_gauge.argtypes = [vp, i]
    lib.pp_plan_set_gauge.restype = i
    lib.pp_plan_set_zsolver.argtypes = [vp, i]
    lib.pp_plan_set_zsolver.restype = i
    lib.pp_plan_set_zsplit.argtypes = [vp, i]
    lib.pp_plan_set_zsplit.restype = i
    lib.pp_plan_set_refinement.argtypes = [vp, d, i]
    lib.pp_plan_set_refinement.restype = i
    lib.pp_plan_workspace_bytes.argtypes = [vp]
    lib.pp_plan_workspace_bytes.restype = ctypes.c_size_t
    lib.pp_solve.argtypes = [vp, vp, vp, vp, vp]
    lib.pp_solve.restype = i
    lib.pp_solve_bc.argtypes = [vp, vp, ctypes.POINTER(vp), vp, vp, vp]
    lib.pp_solve_bc.restype = i
    lib.pp_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
    lib.pp_stream_copy.restype = i
    lib.pp_solve_noalloc.argtypes = [vp, vp, vp, vp]
    lib.pp_solve_noalloc.restype = i
    lib.pp_solve_adjoint.argtypes = [vp, vp, vp, vp, vp]
    lib.pp_solve_adjoint.restype = i
    lib.pp_plan_last_info.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(d), ctypes.POINTER(d)]
    lib.pp_plan_last_info.restype = i
    lib.pp_plan_set_timing.argtypes = [vp, i]
    lib.pp_plan_set_timing.restype = i
    lib.pp_plan_kernel_times.argtypes = [vp, ctypes.POINTER(d), ctypes.POINTER(i), i]
    lib.pp_plan_kernel_times.restype = i
    lib.pp_plan_destroy.argtypes = [vp]
    lib.pp_plan_destroy.restype = None
    lib.pp_status_string.argtypes = [i]
    lib.pp_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def status_string(status):
    try:
        return load().pp_status_string(status).decode()
    except Exception:
        return STATUS.get(status, "unknown")


def check(status, what):
    if status != 0:
        raise PPError(status, what)
