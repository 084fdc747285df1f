"""ctypes binding of ``libtdt.so`` (argument marshalling only).

Every step of a solve runs in the HIP kernels behind the C ABI of
``include/tdt.h``; this module only passes device pointers, sizes and the
current HIP stream.  There is no fallback: if the library is not built, every
entry point raises.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
LIB_PATH = os.path.join(_HERE, "libtdt.so")
SOURCES = [os.path.join(_HERE, "csrc", "tdt_kernels.hip"), os.path.join(_HERE, "csrc", "tdt_api.cpp"),
           os.path.join(_HERE, "csrc", "tdt_poisson.hip"), os.path.join(_HERE, "csrc", "tdt_strided.hip")]
HEADER = os.path.join(_ROOT, "include", "tdt.h")

# status codes (include/tdt.h)
TDT_OK = 0
TDT_WARN_NOT_DOMINANT = 1
TDT_ERR_INVALID_ARG = -1
TDT_ERR_SINGULAR = -2
TDT_ERR_HIP = -3
TDT_ERR_OOM = -4
TDT_ERR_NOT_CONVERGED = -5
TDT_ERR_CAPTURE = -6

DTYPES = {"f64": 0, "f32": 1, "f32_refine": 2}

# Every symbol the header declares (checked by the CPU tests).
EXPORTS = [
    "tdt_plan_create", "tdt_plan_varlen_create", "tdt_plan_reserve", "tdt_solve",
    "tdt_solve_varlen", "tdt_solve_backward", "tdt_plan_destroy", "tdt_status_string",
    "tdt_last_info", "tdt_block_constants", "tdt_green_rows", "tdt_segment_merge", "tdt_plan_profile",
    "tdt_plan_profile_read", "tdt_build_info", "tdt_plan_set_option", "tdt_plan_get_option",
    "tdt_plan_autotune", "tdt_plan_quasi_create", "tdt_plan_varlen_quasi_create",
    "tdt_plan_general_create", "tdt_poisson2d_create", "tdt_poisson2d_solve",
    "tdt_poisson2d_line_plan", "tdt_poisson2d_destroy", "tdt_poisson2d_profile",
    "tdt_poisson2d_profile_read", "tdt_plan_strided_create",
    "tdt_solve_strided", "tdt_poisson3d_create", "tdt_poisson3d_solve", "tdt_poisson3d_schedule",
    "tdt_poisson3d_profile", "tdt_poisson3d_profile_read", "tdt_poisson3d_destroy",
    "tdt_adi_parameters", "tdt_green_support", "tdt_plan_green_support", "tdt_solve_noalloc",
]

# tdt_option_t
OPTIONS = {"whole_max_tiles": 0, "wg_per_cu": 1, "max_refine": 2, "shape": 3}
# work shapes of TDT_OPT_SHAPE: (rows per lane, lanes per workgroup)
SHAPES = [(16, 512), (8, 512), (16, 256)]
TUNE_NO_CACHE = 1
TUNE_FORCE = 2
TUNE_ADJOINT = 4


def _flags() -> list:
    return ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(_ROOT, "include"), "-I", os.path.join(_HERE, "csrc")]


def build() -> str:
    """Compile libtdt.so for gfx950 in-tree (always recompiles): each source
    to an object file in parallel, then one link."""
    import tempfile
    with tempfile.TemporaryDirectory(prefix="tdt_build_") as tmpd:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmpd, os.path.basename(src) + ".o")
            objs.append(obj)
            procs.append(subprocess.Popen(["hipcc", *_flags(), "-c", src, "-o", obj]))
        rcs = [q.wait() for q in procs]
        if any(rcs):
            raise subprocess.CalledProcessError(max(rcs, key=abs), "hipcc -c")
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs,
                               "-o", tmp, "-L/opt/rocm/lib", "-lhipfft"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class TDTError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    d, i64, i32, p = ctypes.c_double, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "tdt_plan_create": [d, d, d, i64, i32, pp],
        "tdt_plan_varlen_create": [i64, p, p, p, p, i32, pp],
        "tdt_plan_quasi_create": [d, d, d, d, d, i64, i32, pp],
        "tdt_plan_varlen_quasi_create": [i64, p, p, p, p, p, p, i32, pp],
        "tdt_plan_general_create": [i64, p, p, p, i32, pp],
        "tdt_poisson2d_create": [i64, i64, d, d, i32, pp],
        "tdt_poisson2d_solve": [p, p, p, p],
        "tdt_poisson2d_line_plan": [p, pp],
        "tdt_poisson2d_destroy": [p],
        "tdt_poisson2d_profile": [p, i32],
        "tdt_poisson2d_profile_read": [p, p, ctypes.POINTER(i64)],
        "tdt_plan_strided_create": [i64, i64, p, p, p, i32, pp],
        "tdt_solve_strided": [p, p, p, i64, i64, i64, i64, p],
        "tdt_poisson3d_create": [i64, i64, i64, d, d, d, d, pp],
        "tdt_poisson3d_solve": [p, p, p, p],
        "tdt_poisson3d_schedule": [p, p, p, i64, ctypes.POINTER(i32)],
        "tdt_poisson3d_profile": [p, i32],
        "tdt_poisson3d_profile_read": [p, p, ctypes.POINTER(i64)],
        "tdt_poisson3d_destroy": [p],
        "tdt_adi_parameters": [d, d, i32, p, p],
        "tdt_plan_reserve": [p, i64],
        "tdt_solve": [p, p, p, i64, p],
        "tdt_solve_noalloc": [p, p, p, i64, p],
        "tdt_solve_varlen": [p, p, p, p],
        "tdt_solve_backward": [p, p, p, p, p, i64, p],
        "tdt_plan_destroy": [p],
        "tdt_last_info": [p, ctypes.POINTER(i32), ctypes.POINTER(d), ctypes.POINTER(d),
                          ctypes.POINTER(d)],
        "tdt_block_constants": [d, d, d, i32, p],
        "tdt_segment_merge": [p, p, p],
        "tdt_green_rows": [d, d, d, i64, p, p],
        "tdt_green_support": [d, d, d, i64, ctypes.POINTER(i64), ctypes.POINTER(i64), p],
        "tdt_plan_green_support": [p, p],
        "tdt_plan_profile": [p, i32],
        "tdt_plan_profile_read": [p, p, ctypes.POINTER(i64)],
        "tdt_build_info": [ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                           ctypes.POINTER(i64)],
        "tdt_plan_set_option": [p, i32, i64],
        "tdt_plan_get_option": [p, i32, ctypes.POINTER(i64)],
        "tdt_plan_autotune": [p, p, p, i64, p, i32, ctypes.POINTER(d)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = i32
    L.tdt_status_string.argtypes = [i32]
    L.tdt_status_string.restype = ctypes.c_char_p
    _lib = L
    return L


def status_string(status: int) -> str:
    try:
        return lib().tdt_status_string(int(status)).decode()
    except Exception:
        return "unknown"


def check(status: int, what: str, allow_warn: bool = True) -> int:
    if status == TDT_OK or (allow_warn and status == TDT_WARN_NOT_DOMINANT):
        return status
    raise TDTError(status, what)
