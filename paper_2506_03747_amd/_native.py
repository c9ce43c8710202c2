"""ctypes view of the C ABI in include/nlos.h (libnlos.so, built in-tree).

Argument marshalling only: the structs below mirror nlos_grid / nlos_params
field by field, and every entry point is bound with its exact signature.
Loading fails loudly when the library has not been built; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnlos.so")

NLOS_OK = 0
NLOS_EINVAL = -1
NLOS_ENOSPC = -2
NLOS_EHIP = -3
NLOS_ENODEV = -4
NLOS_F_COSINES = 1
NLOS_MAX_BINS = 1 << 22
NLOS_MAX_RADIUS = 127
NLOS_MAX_PATCHES = 1 << 24
NLOS_RECORD_FLOATS = 8


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("half_x", C.c_double),
                ("half_y", C.c_double), ("cx", C.c_double), ("cy", C.c_double)]


class Params(C.Structure):
    _fields_ = [("relay", Grid), ("laser", Grid), ("standoff_m", C.c_double),
                ("bin_ps", C.c_double), ("n_bins", C.c_int32), ("flags", C.c_uint32),
                ("fwhm_ps", C.c_double)]


class DepthRequest(C.Structure):
    _fields_ = [("grid", Grid), ("depth", C.c_void_p), ("albedo", C.c_void_p), ("mask", C.c_void_p),
                ("flags", C.c_uint32), ("patches", C.c_void_p), ("n_active", C.c_void_p)]


class Request(C.Structure):
    _fields_ = [("params", Params), ("patches", C.c_void_p), ("n_patches", C.c_int32),
                ("n_active", C.c_void_p), ("out", C.c_void_p)]


class NlosError(RuntimeError):
    def __init__(self, code: int, where: str, hip: int = 0):
        self.code = code
        msg = f"{where}: {strerror(code)} ({code})"
        if code == NLOS_EHIP:
            msg += f", hipError {hip}"
        super().__init__(msg)


_lib = None

# (name, restype, argtypes) for every entry point of include/nlos.h
SIGNATURES = [
    ("nlos_abi_version", C.c_int, []),
    ("nlos_strerror", C.c_char_p, [C.c_int]),
    ("nlos_last_hip_error", C.c_int, []),
    ("nlos_patches_workspace_bytes", C.c_int, [C.POINTER(Grid), C.POINTER(C.c_size_t)]),
    ("nlos_patches_from_depth", C.c_int,
     [C.POINTER(Grid), C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p,
      C.c_void_p, C.c_size_t, C.c_void_p]),
    ("nlos_forward_workspace_bytes", C.c_int, [C.POINTER(Params), C.c_int32, C.POINTER(C.c_size_t)]),
    ("nlos_forward", C.c_int,
     [C.POINTER(Params), C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
      C.c_void_p]),
    ("nlos_simulate_workspace_bytes", C.c_int, [C.POINTER(Params), C.POINTER(Grid), C.POINTER(C.c_size_t)]),
    ("nlos_simulate", C.c_int,
     [C.POINTER(Params), C.POINTER(Grid), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
      C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    ("nlos_patches_batched_sizes", C.c_int,
     [C.POINTER(DepthRequest), C.c_int32, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    ("nlos_patches_batched", C.c_int,
     [C.POINTER(DepthRequest), C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("nlos_forward_batched_sizes", C.c_int,
     [C.POINTER(Request), C.c_int32, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    ("nlos_forward_batched", C.c_int,
     [C.POINTER(Request), C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("nlos_forward_smooth_workspace_bytes", C.c_int, [C.POINTER(Params), C.c_int32, C.POINTER(C.c_size_t)]),
    ("nlos_forward_smooth", C.c_int,
     [C.POINTER(Params), C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("nlos_adjoint_workspace_bytes", C.c_int, [C.POINTER(Params), C.c_int32, C.POINTER(C.c_size_t)]),
    ("nlos_adjoint", C.c_int,
     [C.POINTER(Params), C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
      C.c_void_p]),
    ("nlos_patches_adjoint_workspace_bytes", C.c_int, [C.POINTER(Grid), C.POINTER(C.c_size_t)]),
    ("nlos_patches_adjoint", C.c_int,
     [C.POINTER(Grid), C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
      C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("nlos_noise_scale_workspace_bytes", C.c_int, [C.c_int64, C.POINTER(C.c_size_t)]),
    ("nlos_noise_scale", C.c_int,
     [C.c_void_p, C.c_int64, C.c_double, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("nlos_poisson_noise", C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p]),
    ("nlos_lct_workspace_bytes", C.c_int, [C.POINTER(Params), C.POINTER(C.c_size_t)]),
    ("nlos_lct_forward", C.c_int,
     [C.POINTER(Params), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("nlos_debug_bins", C.c_int,
     [C.POINTER(Params), C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
      C.c_void_p]),
]


def lib():
    """The loaded library; raises if libnlos.so is missing (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2506_03747_amd.build` "
                              "(or __graft_entry__.build()) first")
        h = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def strerror(code: int) -> str:
    return lib().nlos_strerror(int(code)).decode()


def check(code: int, where: str) -> None:
    if code != NLOS_OK:
        raise NlosError(code, where, lib().nlos_last_hip_error())
