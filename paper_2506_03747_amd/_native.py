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
NLOS_NOALLOC_MAX_PATCHES = 1 << 22


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


class SimRequest(C.Structure):
    _fields_ = [("params", Params), ("grid", Grid), ("depth", C.c_void_p), ("albedo", C.c_void_p),
                ("mask", C.c_void_p), ("patches", C.c_void_p), ("n_active", C.c_void_p), ("out", C.c_void_p)]


class TickCaps(C.Structure):
    _fields_ = [("max_requests", C.c_int32), ("max_pixels", C.c_int64)]


class TuningEntry(C.Structure):
    _fields_ = [("confocal", C.c_int32), ("t_min", C.c_int32), ("t_max", C.c_int32), ("h_min", C.c_int64),
                ("h_max", C.c_int64), ("tl", C.c_int32), ("tx", C.c_int32), ("ty", C.c_int32)]


class PlanInfo(C.Structure):
    _fields_ = [("tl", C.c_int32), ("tx", C.c_int32), ("ty", C.c_int32), ("pair", C.c_int32),
                ("n_split", C.c_int32), ("n_windows", C.c_int32), ("workgroups", C.c_int64),
                ("lds_bytes", C.c_int64)]


class Probe(C.Structure):
    _fields_ = [("forward_mark", C.c_void_p), ("evaluated_pairs", C.c_void_p)]


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
    ("nlos_forward_noalloc", C.c_int,
     [C.POINTER(Params), C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("nlos_simulate_workspace_bytes", C.c_int, [C.POINTER(Params), C.POINTER(Grid), C.POINTER(C.c_size_t)]),
    ("nlos_simulate", C.c_int,
     [C.POINTER(Params), C.POINTER(Grid), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
      C.c_void_p, C.c_size_t, C.POINTER(Probe), C.c_void_p]),
    ("nlos_patches_batched_sizes", C.c_int,
     [C.POINTER(DepthRequest), C.c_int32, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    ("nlos_patches_batched", C.c_int,
     [C.POINTER(DepthRequest), C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("nlos_forward_batched_sizes", C.c_int,
     [C.POINTER(Request), C.c_int32, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    ("nlos_forward_batched", C.c_int,
     [C.POINTER(Request), C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("nlos_tick_sizes", C.c_int, [C.POINTER(TickCaps), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    ("nlos_tick_plan", C.c_int,
     [C.POINTER(TickCaps), C.POINTER(SimRequest), C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t]),
    ("nlos_tick_launch", C.c_int, [C.POINTER(TickCaps), C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("nlos_tick_graph_create", C.c_int,
     [C.POINTER(TickCaps), C.c_void_p, C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p)]),
    ("nlos_tick_graph_launch", C.c_int, [C.c_void_p, C.c_void_p]),
    ("nlos_tick_graph_destroy", C.c_int, [C.c_void_p]),
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
    ("nlos_set_tuning", C.c_int, [C.POINTER(TuningEntry), C.c_int32]),
    ("nlos_get_plan", C.c_int, [C.POINTER(Params), C.c_int32, C.POINTER(PlanInfo)]),
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
        _install_tuning(h)
        _lib = h
    return _lib


TUNING_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def _install_tuning(h) -> None:
    """Install the autotuner's table (tuning.json beside the library) unless
    NLOS_NO_TUNING is set; without a table the library's built-in rule plans."""
    if os.environ.get("NLOS_NO_TUNING") or not os.path.exists(TUNING_PATH):
        return
    import json
    with open(TUNING_PATH) as f:
        ents = json.load(f)["entries"]
    arr = (TuningEntry * max(len(ents), 1))()
    for i, e in enumerate(ents):
        arr[i] = TuningEntry(int(e["confocal"]), int(e["t_min"]), int(e["t_max"]), int(e["h_min"]),
                             int(e["h_max"]), int(e["tl"]), int(e["tx"]), int(e["ty"]))
    rc = h.nlos_set_tuning(arr, len(ents))
    if rc != NLOS_OK:
        raise RuntimeError(f"{TUNING_PATH}: rejected by nlos_set_tuning ({h.nlos_strerror(rc).decode()})")


def strerror(code: int) -> str:
    return lib().nlos_strerror(int(code)).decode()


def check(code: int, where: str) -> None:
    if code != NLOS_OK:
        raise NlosError(code, where, lib().nlos_last_hip_error())
