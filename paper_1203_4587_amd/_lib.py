"""ctypes declarations of the C ABI in include/csmri.h.

Loading is lazy and strict: if libcsmri.so is missing or does not load, the
first use raises.  Nothing here computes anything.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcsmri.so")

CS_OK = 0
CS_EINVAL = 1
CS_EUNSUPPORTED = 2
CS_ENOMEM = 3
CS_EDEVICE = 4
CS_EMU_MISMATCH = 5

CS_PRIOR_TEMPORAL_TV = 0
CS_PRIOR_TEMPORAL_DFT = 1
CS_PRIOR_TEMPORAL_FRAME = 2

CS_FLAG_NO_REFACTOR = 1 << 0
CS_FLAG_GRAPH = 1 << 1
CS_FLAG_COLUMN_RESIDENT = 1 << 2
CS_FLAG_XU_WAVE = 1 << 3
CS_FLAG_XU_GROUP = 1 << 4
CS_FLAG_EIGEN = 1 << 5
CS_FLAG_CHECK_FINITE = 1 << 6

# every function declared in include/csmri.h
EXPORTED = (
    "cs_plan_create",
    "cs_plan_destroy",
    "cs_plan_bytes",
    "cs_apply_A",
    "cs_apply_AH",
    "cs_apply_block_inverse",
    "cs_admm_solve",
    "cs_admm_solve_until",
    "cs_status_string",
    "cs_last_error",
    "cs_version",
    "cs_kernel_timing",
    "cs_kernel_times",
    "cs_plan_flags",
    "cs_plan_set_flags",
    "cs_plan_tune",
    "cs_plan_fft_tiles",
    "cs_plan_set_fft_tiles",
    "cs_batch_create",
    "cs_batch_destroy",
    "cs_batch_size",
    "cs_batch_plan",
    "cs_batch_solve",
    "cs_grad_create",
    "cs_grad_destroy",
    "cs_admm_forward_ckpt",
    "cs_admm_backward",
    "cs_apply_AH_noalloc",
    "cs_read_stream",
)

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class CsPlanDesc(ctypes.Structure):
    _fields_ = [
        ("nv", ctypes.c_int32),
        ("nh", ctypes.c_int32),
        ("nt", ctypes.c_int32),
        ("nc", ctypes.c_int32),
        ("prior", ctypes.c_int32),
        ("mu_ratio", ctypes.c_float),
        ("flags", ctypes.c_uint32),
    ]


class CsAllocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


class CsState(ctypes.Structure):
    _fields_ = [
        ("s0", ctypes.c_void_p),
        ("s1", ctypes.c_void_p),
        ("s2", ctypes.c_void_p),
        ("s3", ctypes.c_void_p),
        ("iter", ctypes.c_int32),
    ]


class CsKernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_int32), ("ms", ctypes.c_double)]


class CsTuneEntry(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("ms_per_iter", ctypes.c_float)]


class CsSliceDesc(ctypes.Structure):
    _fields_ = [("desc", CsPlanDesc), ("coil", ctypes.c_void_p), ("mask", ctypes.c_void_p),
                ("mu", ctypes.c_float)]


class CsmriError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({detail})")


_lib = None


def load() -> ctypes.CDLL:
    """Load libcsmri.so once; raises if it is absent (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run `python -m paper_1203_4587_amd.build` "
            "(the HIP library is the only compute path)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, f32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float, ctypes.c_size_t
    lib.cs_plan_create.argtypes = [ctypes.POINTER(CsPlanDesc), vp, vp, f32, ctypes.POINTER(CsAllocator), vp,
                                   ctypes.POINTER(vp)]
    lib.cs_plan_destroy.argtypes = [vp]
    lib.cs_plan_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    lib.cs_apply_A.argtypes = [vp, vp, vp, vp]
    lib.cs_apply_AH.argtypes = [vp, vp, vp, vp]
    lib.cs_apply_block_inverse.argtypes = [vp, vp, vp, vp]
    lib.cs_admm_solve.argtypes = [vp, vp, f32, f32, i32, vp, ctypes.POINTER(CsState), vp, vp]
    lib.cs_admm_solve_until.argtypes = [vp, vp, f32, f32, i32, f32, i32, vp, ctypes.POINTER(CsState),
                                         ctypes.POINTER(i32), ctypes.POINTER(f32), vp]
    lib.cs_kernel_timing.argtypes = [vp, ctypes.c_int]
    lib.cs_kernel_times.argtypes = [vp, ctypes.POINTER(CsKernelTime), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.cs_plan_flags.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32)]
    lib.cs_plan_set_flags.argtypes = [vp, ctypes.c_uint32]
    lib.cs_plan_tune.argtypes = [vp, vp, f32, i32, ctypes.POINTER(CsTuneEntry), i32, ctypes.POINTER(i32), vp]
    lib.cs_plan_fft_tiles.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.cs_plan_set_fft_tiles.argtypes = [vp, i32, i32]
    lib.cs_batch_create.argtypes = [ctypes.POINTER(CsSliceDesc), i32, ctypes.POINTER(CsAllocator), vp,
                                    ctypes.POINTER(vp)]
    lib.cs_batch_destroy.argtypes = [vp]
    lib.cs_batch_size.argtypes = [vp, ctypes.POINTER(i32)]
    lib.cs_batch_plan.argtypes = [vp, i32, ctypes.POINTER(vp)]
    lib.cs_batch_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(f32), i32, ctypes.POINTER(vp), vp]
    lib.cs_grad_create.argtypes = [vp, i32, i32, ctypes.POINTER(vp)]
    lib.cs_grad_destroy.argtypes = [vp]
    lib.cs_admm_forward_ckpt.argtypes = [vp, vp, f32, f32, vp, vp]
    lib.cs_admm_backward.argtypes = [vp, vp, vp, vp, vp]
    lib.cs_apply_AH_noalloc.argtypes = [ctypes.POINTER(CsPlanDesc), vp, vp, vp, vp, vp]
    lib.cs_read_stream.argtypes = [vp, ctypes.c_size_t, i32, vp, vp]
    for name in EXPORTED:
        if name not in ("cs_status_string", "cs_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    lib.cs_version.argtypes = []
    lib.cs_status_string.argtypes = [ctypes.c_int]
    lib.cs_status_string.restype = ctypes.c_char_p
    lib.cs_last_error.argtypes = []
    lib.cs_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().cs_status_string(status).decode()


def check(status: int, where: str) -> None:
    if status != CS_OK:
        raise CsmriError(status, where, load().cs_last_error().decode())
