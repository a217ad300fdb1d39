"""ctypes loader for libwilson_mi355x.so and the C structs of include/wilson.h.

Argument marshalling only: no arithmetic of the method happens in Python.
Loading needs the HIP runtime library (present in a ROCm install) but no GPU;
calls that launch kernels need a GPU. If the shared library has not been
built, loading fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwilson_mi355x.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "wilson.h")

WD_F64, WD_F32, WD_BF16, WD_F16, WD_I8 = 0, 1, 2, 3, 4
WD_RHS_SOURCE, WD_RHS_NORMAL = 0, 1
WD_C128, WD_C64 = 0, 1
WD_TWO_ROW_LINKS = 0x100
WD_RELIABLE_UPDATE, WD_ITERATIVE_REFINEMENT = 0, 1
WD_BATCH_AUTO, WD_BATCH_PERSISTENT, WD_BATCH_LOCKSTEP = 0, 1, 2
WD_OK, WD_NOT_CONVERGED = 0, 1
WD_ERR_INVALID, WD_ERR_HIP, WD_ERR_BREAKDOWN, WD_ERR_NAN, WD_ERR_WORKSPACE = -1, -2, -3, -4, -5

PREC_NAMES = {"f64": WD_F64, "f32": WD_F32, "bf16": WD_BF16, "f16": WD_F16, "i8": WD_I8,
              "bf16_rows2": WD_BF16 | WD_TWO_ROW_LINKS, "f16_rows2": WD_F16 | WD_TWO_ROW_LINKS,
              "i8_rows2": WD_I8 | WD_TWO_ROW_LINKS}


class WdLattice(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4)]


class WdCgParams(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("inner_prec", ctypes.c_int32),
        ("reliable_interval", ctypes.c_int32),
        ("rhs_mode", ctypes.c_int32),
        ("io_dtype", ctypes.c_int32),
        ("zero_guess", ctypes.c_int32),
        ("history", ctypes.POINTER(ctypes.c_double)),
        ("history_len", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
        ("ring_len", ctypes.c_int32),
        ("inner_tol", ctypes.c_double),
        ("batch_schedule", ctypes.c_int32),
    ]


class WdCgResult(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32),
        ("reliable_updates", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("two_row_links", ctypes.c_int32),
        ("true_rel_res", ctypes.c_double),
        ("iter_rel_res", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("kernel_seconds", ctypes.c_double * 3),
        ("ooc_slab_planes", ctypes.c_int32),
        ("ooc_slabs", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "kernel_seconds"}
        d["kernel_seconds"] = list(self.kernel_seconds)
        return d


_P = ctypes.c_void_p
_LAT = ctypes.POINTER(WdLattice)
_PAR = ctypes.POINTER(WdCgParams)
_RES = ctypes.POINTER(WdCgResult)

# name -> (restype, argtypes); every function declared in include/wilson.h
SIGNATURES = {
    "wd_last_error": (ctypes.c_char_p, []),
    "wd_device_count": (ctypes.c_int, []),
    "wilson_apply": (ctypes.c_int, [_LAT, ctypes.c_double, _P, _P, _P, _P]),
    "wilson_apply_dagger": (ctypes.c_int, [_LAT, ctypes.c_double, _P, _P, _P, _P]),
    "wd_workspace_bytes": (ctypes.c_size_t, [_LAT, _PAR, ctypes.c_int32]),
    "cg_solve": (ctypes.c_int, [_LAT, ctypes.c_double, _P, _P, _P, _PAR, _RES, _P, ctypes.c_size_t, _P]),
    "cg_solve_noalloc": (ctypes.c_int, [_LAT, ctypes.c_double, _P, _P, _P, _PAR, _RES, _P]),
    "wd_ooc_workspace_bytes": (ctypes.c_int, [_LAT, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t),
                                              ctypes.POINTER(ctypes.c_size_t)]),
    "cg_solve_ooc": (ctypes.c_int, [_LAT, ctypes.c_double, _P, _P, _P, _PAR, _RES, _P, ctypes.c_size_t, _P,
                                    ctypes.c_size_t, _P]),
    "wd_stream": (ctypes.c_int, [ctypes.c_int32, _P, _P, ctypes.c_size_t, _P]),
    "wd_stream_partials": (ctypes.c_size_t, [ctypes.c_size_t]),
    "cg_solve_batched": (ctypes.c_int, [_LAT, ctypes.c_double, _P, ctypes.c_int32, _P, _P, _PAR, _RES, _P,
                                        ctypes.c_size_t, _P]),
    "wilson_force": (ctypes.c_int, [_LAT, _P, _P, ctypes.c_double, ctypes.c_int32, _P, _P]),
    "wd_gauge_bytes": (ctypes.c_size_t, [_LAT, ctypes.c_int32]),
    "wd_spinor_bytes": (ctypes.c_size_t, [_LAT, ctypes.c_int32]),
    "wd_pack_gauge": (ctypes.c_int, [_LAT, _P, ctypes.c_int32, _P, _P]),
    "wd_pack_spinor": (ctypes.c_int, [_LAT, _P, ctypes.c_int32, ctypes.c_int32, _P, _P]),
    "wd_unpack_spinor": (ctypes.c_int, [_LAT, _P, ctypes.c_int32, _P, ctypes.c_int32, _P]),
    "wilson_apply_packed": (ctypes.c_int, [_LAT, ctypes.c_double, ctypes.c_int32, _P, _P, _P, ctypes.c_int32, _P]),
    "laplace_apply": (ctypes.c_int, [_LAT, ctypes.c_double, _P, _P, _P, _P]),
    "laplace_workspace_bytes": (ctypes.c_size_t, [_LAT, _PAR]),
    "laplace_cg_solve": (ctypes.c_int, [_LAT, ctypes.c_double, _P, _P, _P, _PAR, _RES, _P, ctypes.c_size_t, _P]),
}

_lib = None


class WilsonError(RuntimeError):
    def __init__(self, code: int, func: str, msg: str):
        super().__init__(f"{func} returned {code}: {msg}")
        self.code = code


def header_functions() -> list:
    """Names of the functions declared in include/wilson.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b([A-Za-z_][A-Za-z0-9_]*)\s*\([^;{]*\)\s*;", text)
    return sorted(set(n for n in names if n not in ("sizeof",)))


def load(path: str | None = None) -> ctypes.CDLL:
    """Load the shared library (once). Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    # WILSON_MI355X_LIB selects another build of this library (the host
    # sanitizer build); there is no other implementation to fall back to
    p = path or os.environ.get("WILSON_MI355X_LIB") or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(
            f"{p} not found: build the HIP library first (python -m paper_2001_05218_amd.build); "
            "there is no CPU fallback")
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().wd_last_error().decode()


def check(code: int, func: str, ok=(WD_OK,)) -> int:
    if code not in ok:
        raise WilsonError(code, func, last_error())
    return code


def lattice(dims) -> WdLattice:
    lat = WdLattice()
    for i in range(4):
        lat.L[i] = int(dims[i])
    return lat
