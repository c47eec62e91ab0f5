"""ctypes binding of libpwdft.so (declared in include/pw.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
the library.  There is no fallback: if the shared library is missing or
fails to load, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpwdft.so")

c_int64 = ctypes.c_int64
c_int32 = ctypes.c_int32
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p
c_int = ctypes.c_int

PW_OK = 0
PW_FP64, PW_FP32, PW_BF16 = 0, 1, 2
STAGES = ["fft_col_inv", "fft_plane", "fft_col_fwd", "proj", "nonlocal", "gram", "chol",
          "rotate", "eigh", "misc", "fft_col_inv_lp", "fft_plane_lp", "fft_col_fwd_lp", "proj_lp",
          "nonlocal_lp", "density"]


class PwHamDesc(ctypes.Structure):
    _fields_ = [
        ("n", c_int32 * 3),
        ("npw", c_int64),
        ("miller", ctypes.POINTER(c_int32)),
        ("recip", c_double * 9),
        ("kpt", c_double * 3),
        ("vloc_dev", c_void_p),
        ("nproj", c_int64),
        ("proj_dev", c_void_p),
        ("ekb", ctypes.POINTER(c_double)),
        ("nb_max", c_int64),
        ("low_prec", c_int32),
    ]


# name -> (restype, argtypes)
class PwTuning(ctypes.Structure):
    """pw_tuning (include/pw.h)."""
    _fields_ = [("reg_col", c_int32), ("reg_plane", c_int32), ("plane_variant", c_int32),
                ("plane_variant32", c_int32), ("chunk", c_int32), ("gemm_blocks", c_int32),
                ("nn_tile", c_int32), ("nn_tile32", c_int32), ("ms", c_double)]


SIGNATURES = {
    "pw_status_string": (ctypes.c_char_p, [c_int]),
    "pw_version": (ctypes.c_char_p, []),
    "pw_last_error": (ctypes.c_char_p, [c_void_p]),
    "pw_ctx_create": (c_int, [c_int, c_void_p, ctypes.POINTER(c_void_p)]),
    "pw_ctx_destroy": (c_int, [c_void_p]),
    "pw_ham_create": (c_int, [c_void_p, ctypes.POINTER(PwHamDesc), ctypes.POINTER(c_void_p)]),
    "pw_ham_destroy": (c_int, [c_void_p]),
    "pw_ham_info": (c_int, [c_void_p] + [ctypes.POINTER(c_int64)] * 5),
    "pw_apply_h": (c_int, [c_void_p, c_int, c_int64, c_void_p, c_int64, c_void_p, c_int64]),
    "pw_density": (c_int, [c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_int32]),
    "pw_cheb_filter": (c_int, [c_void_p, c_int, c_int32, c_double, c_double, c_double, c_int64,
                               c_void_p, c_int64, c_void_p, c_int64]),
    "pw_orthonormalize": (c_int, [c_void_p, c_int, c_int64, c_void_p, c_int64, c_void_p, c_int64]),
    "pw_rayleigh_ritz": (c_int, [c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_int64, c_void_p,
                                 c_void_p]),
    "pw_upper_bound": (c_int, [c_void_p, ctypes.POINTER(c_double)]),
    "pw_ham_cprj": (c_int, [c_void_p, c_int64, c_void_p, c_int64]),
    "pw_lobpcg": (c_int, [c_void_p, c_int64, c_int32, c_int32, c_void_p, c_int64, c_void_p, c_int64,
                          c_void_p, c_void_p, c_void_p]),
    "pw_rmm_diis": (c_int, [c_void_p, c_int64, c_int32, c_void_p, c_int64, c_void_p, c_int64,
                            c_int32, c_void_p, c_void_p, c_void_p]),
    "pw_gemm_cn": (c_int, [c_void_p, c_int64, c_int64, c_int64, c_double, c_void_p, c_int64,
                           c_void_p, c_int64, c_void_p, c_int64]),
    "pw_gemm_nn": (c_int, [c_void_p, c_int64, c_int64, c_int64, c_double, c_void_p, c_int64,
                           c_void_p, c_int64, c_double, c_void_p, c_int64]),
    "pw_heev": (c_int, [c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_int64]),
    "pw_potrf_inv": (c_int, [c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_int64]),
    "pw_heev_noalloc": (c_int, [c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_int64]),
    "pw_ctx_set_timing": (c_int, [c_void_p, c_int]),
    "pw_ctx_stage_time": (c_int, [c_void_p, c_int, ctypes.POINTER(c_double),
                                  ctypes.POINTER(c_int64)]),
    "pw_ctx_reset_timing": (c_int, [c_void_p]),
    "pw_ctx_last_sweeps": (c_int, [c_void_p, ctypes.POINTER(c_int)]),
    "pw_ctx_check": (c_int, [c_void_p]),
    "pw_ctx_set_sweep_limit": (c_int, [c_void_p, c_int32]),
    "pw_ctx_set_overlap": (c_int, [c_void_p, c_int32]),
    "pw_ham_get_tuning": (c_int, [c_void_p, ctypes.POINTER(PwTuning)]),
    "pw_ham_set_tuning": (c_int, [c_void_p, ctypes.POINTER(PwTuning)]),
    "pw_ham_autotune": (c_int, [c_void_p, c_int, c_int64, c_int32, ctypes.POINTER(PwTuning),
                                ctypes.POINTER(PwTuning)]),
    "pw_batch_create": (c_int, [c_void_p, c_int32, ctypes.POINTER(c_void_p),
                                ctypes.POINTER(c_int64), ctypes.POINTER(c_void_p),
                                ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p),
                                ctypes.POINTER(c_void_p), c_int32, c_int, c_int32,
                                ctypes.POINTER(c_void_p)]),
    "pw_batch_destroy": (c_int, [c_void_p]),
    "pw_batch_start": (c_int, [c_void_p]),
    "pw_batch_iterate": (c_int, [c_void_p, c_int32, c_int32]),
    "pw_batch_max_sweeps": (c_int, [c_void_p, ctypes.POINTER(c_int32)]),
    "pw_batch_chfsi": (c_int, [c_void_p, c_int32, c_int32]),
    "pw_autotune": (c_int, [c_void_p, c_int, c_int64, c_int32, ctypes.c_char_p,
                            ctypes.POINTER(PwTuning), ctypes.POINTER(PwTuning),
                            ctypes.POINTER(c_int32)]),
}


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libpwdft.so not built at {path}; run __graft_entry__.build() "
                          "or python paper_2507_08578_amd/build.py")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


class PWError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(message)
