"""FP64 brute-force oracle of the transient NLOS forward operator.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline use it; the product path never imports it.  It shares no code with
the HIP library.  The arithmetic lives in ``nlos_oracle.c`` (plain C, fp64,
no FMA contraction); this module only compiles it and marshals arrays.

Functions follow arXiv 2506.03747: Section 2 Eq. (1) (forward model),
Section 2 depth-to-volume mapping / Algorithm 1 step 2.1 (patches from a
depth map), Section 2 temporal jitter / Algorithm 1 step 2.3 (Gaussian taps).
The smooth forward and its gradient (a continuous Gaussian time response so
that the depth has a gradient) are a reading: the paper bins hard.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nlos_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11"]


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("half_x", C.c_double),
                ("half_y", C.c_double), ("cx", C.c_double), ("cy", C.c_double)]


class Params(C.Structure):
    _fields_ = [("relay", Grid), ("laser", Grid), ("standoff_m", C.c_double),
                ("bin_ps", C.c_double), ("n_bins", C.c_int32), ("fwhm_ps", C.c_double),
                ("cosines", C.c_int32)]


def compile_library(src: str = _SRC, out: str = _LIB, extra=()) -> str:
    """Compile the oracle with gcc (plain C, OpenMP, no FMA contraction)."""
    cmd = ["gcc", *CFLAGS, *extra, src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def load(path: str | None = None, rebuild: bool = False):
    """Load (compiling first if needed) the oracle library."""
    global _lib
    with _lock:
        if path is not None:
            return _bind(C.CDLL(path))
        if _lib is None or rebuild:
            stale = (not os.path.exists(_LIB)) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
            if stale or rebuild:
                compile_library()
            _lib = _bind(C.CDLL(_LIB))
        return _lib


def _bind(lib):
    dp = C.POINTER(C.c_double)
    lib.oracle_grid_coords.argtypes = [C.POINTER(Grid), dp, dp]
    lib.oracle_inv_bin.argtypes = [C.c_double]
    lib.oracle_inv_bin.restype = C.c_double
    lib.oracle_patches.argtypes = [C.POINTER(Grid), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, dp]
    lib.oracle_patches.restype = C.c_int32
    lib.oracle_taps.argtypes = [C.c_double, C.c_double, dp, C.c_int32]
    lib.oracle_taps.restype = C.c_int32
    lib.oracle_forward.argtypes = [C.POINTER(Params), dp, C.c_int32, C.c_void_p, C.c_int32,
                                   C.c_void_p, C.c_void_p, C.c_void_p]
    lib.oracle_forward.restype = C.c_int32
    lib.oracle_num_threads.restype = C.c_int
    lib.oracle_patches_f64.argtypes = [C.POINTER(Grid), dp, C.c_void_p, C.c_void_p, C.c_int32, dp]
    lib.oracle_patches_f64.restype = C.c_int32
    lib.oracle_smooth_radius.argtypes = [C.c_double, C.c_double]
    lib.oracle_smooth_radius.restype = C.c_int32
    lib.oracle_forward_smooth.argtypes = [C.POINTER(Params), dp, C.c_int32, C.c_void_p, C.c_int32, dp]
    lib.oracle_forward_smooth.restype = C.c_int32
    lib.oracle_smooth_grad.argtypes = [C.POINTER(Params), C.POINTER(Grid), dp, C.c_void_p, C.c_void_p, dp,
                                       dp, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.oracle_smooth_grad.restype = C.c_int32
    lib.oracle_adjoint_records.argtypes = [C.POINTER(Params), dp, C.c_int32, dp, C.c_void_p, C.c_int32, dp]
    lib.oracle_adjoint_records.restype = C.c_int32
    lib.oracle_forward_error_model.argtypes = [C.POINTER(Params), dp, C.c_int32, C.c_void_p, C.c_int32, C.c_double,
                                               C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.oracle_forward_error_model.restype = C.c_int32
    u64p = C.POINTER(C.c_uint64)
    lib.oracle_philox4x64.argtypes = [u64p, u64p, u64p]
    lib.oracle_nx_exp.argtypes = [C.c_double]
    lib.oracle_nx_exp.restype = C.c_double
    lib.oracle_nx_log.argtypes = [C.c_double]
    lib.oracle_nx_log.restype = C.c_double
    lib.oracle_nx_logfact.argtypes = [C.c_double]
    lib.oracle_nx_logfact.restype = C.c_double
    lib.oracle_poisson_count.argtypes = [C.c_double, C.c_uint64, C.c_int64]
    lib.oracle_poisson_count.restype = C.c_int64
    lib.oracle_poisson_counts.argtypes = [dp, C.c_int64, C.c_uint64, C.c_void_p]
    lib.oracle_noise_scale.argtypes = [C.c_void_p, C.c_int64, C.c_double, dp]
    lib.oracle_poisson_noise.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.c_uint64, C.c_void_p]
    return lib


def num_threads(lib=None) -> int:
    return int((lib or load()).oracle_num_threads())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_grid(g: dict) -> Grid:
    return Grid(int(g["nx"]), int(g["ny"]), float(g["half_x"]), float(g["half_y"]),
                float(g["cx"]), float(g["cy"]))


def make_params(scene) -> Params:
    laser = make_grid(scene.laser) if scene.laser is not None else Grid(0, 0, 0.0, 0.0, 0.0, 0.0)
    return Params(make_grid(scene.relay), laser, float(scene.standoff_m), float(scene.bin_ps),
                  int(scene.n_bins), float(scene.fwhm_ps), 1 if scene.cosines else 0)


def grid_coords(g: dict, lib=None):
    lib = lib or load()
    xs = np.zeros(int(g["nx"]), np.float64)
    ys = np.zeros(int(g["ny"]), np.float64)
    lib.oracle_grid_coords(C.byref(make_grid(g)), _dptr(xs), _dptr(ys))
    return xs, ys


def inv_bin(bin_ps: float, lib=None) -> float:
    lib = lib or load()
    return lib.oracle_inv_bin(float(bin_ps))


def patches(scene, lib=None) -> np.ndarray:
    """[nx*ny, 8] fp64 records (px, py, pz, a, n_x, n_y, n_z, present), x major."""
    lib = lib or load()
    g = scene.patch_grid
    depth = np.ascontiguousarray(scene.depth, np.float32)
    albedo = None if scene.albedo is None else np.ascontiguousarray(scene.albedo, np.float32)
    mask = None if scene.mask is None else np.ascontiguousarray(scene.mask, np.uint8)
    assert depth.shape == (g["nx"], g["ny"])
    rec = np.zeros((g["nx"] * g["ny"], 8), np.float64)
    lib.oracle_patches(C.byref(make_grid(g)), depth.ctypes.data,
                       None if albedo is None else albedo.ctypes.data,
                       None if mask is None else mask.ctypes.data,
                       1 if scene.cosines else 0, _dptr(rec))
    return rec


def taps(fwhm_ps: float, bin_ps: float, lib=None) -> np.ndarray:
    lib = lib or load()
    buf = np.zeros(1024, np.float64)
    R = lib.oracle_taps(float(fwhm_ps), float(bin_ps), _dptr(buf), 1024)
    if R < 0:
        raise ValueError("jitter kernel too long")
    return buf[: 2 * R + 1].copy()


def forward(scene, rec: np.ndarray | None = None, subset=None, want_hist=False,
            want_tau=True, want_bins=False, lib=None):
    """Run the brute-force operator.  Returns a dict with any of
    ``hist`` / ``tau`` ([n_out, T] fp64) and ``bins`` ([n_out, P] int32),
    where n_out = L*S (or len(subset)) in [laser][x'][y'] order."""
    lib = lib or load()
    if rec is None:
        rec = patches(scene, lib)
    rec = np.ascontiguousarray(rec, np.float64)
    P = rec.shape[0]
    prm = make_params(scene)
    n_total = scene.n_laser * scene.n_scan
    sub = None
    if subset is not None:
        sub = np.ascontiguousarray(subset, np.int32)
        n_out = sub.shape[0]
    else:
        n_out = n_total
    T = int(scene.n_bins)
    hist = np.zeros((n_out, T), np.float64) if want_hist else None
    tau = np.zeros((n_out, T), np.float64) if want_tau else None
    bins = np.zeros((n_out, P), np.int32) if want_bins else None
    rc = lib.oracle_forward(C.byref(prm), _dptr(rec), P,
                            None if sub is None else sub.ctypes.data,
                            0 if sub is None else n_out,
                            None if hist is None else hist.ctypes.data,
                            None if tau is None else tau.ctypes.data,
                            None if bins is None else bins.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_forward rejected its arguments")
    out = {}
    if want_hist:
        out["hist"] = hist
    if want_tau:
        out["tau"] = tau
    if want_bins:
        out["bins"] = bins
    return out


# Error model of an fp32 evaluation (the parity tests' per-histogram
# tolerance): e0 relative error of every weight; e1 of each patch-cosine
# numerator relative to the sum of its terms' magnitudes (fp32 normals differ
# from these fp64 ones by a few ulp per component, and fp32 arithmetic adds a
# few more: 16 ulp of 2^-24 bounds both).
ERR_E0 = 2e-6
ERR_E1 = 16 * 2.0 ** -24


def error_model(scene, rec: np.ndarray | None = None, subset=None, e0: float = ERR_E0, e1: float = ERR_E1,
                lib=None):
    """Per bin of each histogram: a bound on the error of an fp32 evaluation
    of the in-window pair weights (``err``) and the in-window pair count
    (``count``), both [n_out, T] fp64, before the jitter; and each
    histogram's stand-off weight g_l g_d (``gain``, [n_out])."""
    lib = lib or load()
    if rec is None:
        rec = patches(scene, lib)
    rec = np.ascontiguousarray(rec, np.float64)
    n_total = scene.n_laser * scene.n_scan
    sub = None if subset is None else np.ascontiguousarray(subset, np.int32)
    n_out = n_total if sub is None else sub.shape[0]
    T = int(scene.n_bins)
    err = np.zeros((n_out, T), np.float64)
    cnt = np.zeros((n_out, T), np.float64)
    gain = np.zeros(n_out, np.float64)
    rc = lib.oracle_forward_error_model(C.byref(make_params(scene)), _dptr(rec), rec.shape[0],
                                        None if sub is None else sub.ctypes.data, 0 if sub is None else n_out,
                                        float(e0), float(e1), err.ctypes.data, cnt.ctypes.data, gain.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_forward_error_model rejected its arguments")
    return {"err": err, "count": cnt, "gain": gain}


def _maps64(scene, depth64=None, albedo64=None):
    d = np.ascontiguousarray(scene.depth if depth64 is None else depth64, np.float64)
    a = None
    if albedo64 is not None:
        a = np.ascontiguousarray(albedo64, np.float64)
    elif scene.albedo is not None:
        a = np.ascontiguousarray(scene.albedo, np.float64)
    m = None if scene.mask is None else np.ascontiguousarray(scene.mask, np.uint8)
    return d, a, m


def patches_f64(scene, depth64=None, albedo64=None, lib=None) -> np.ndarray:
    """Records from fp64 maps (defaults: the scene's fp32 maps, promoted)."""
    lib = lib or load()
    g = scene.patch_grid
    d, a, m = _maps64(scene, depth64, albedo64)
    rec = np.zeros((g["nx"] * g["ny"], 8), np.float64)
    lib.oracle_patches_f64(C.byref(make_grid(g)), _dptr(d), None if a is None else a.ctypes.data,
                           None if m is None else m.ctypes.data, 1 if scene.cosines else 0, _dptr(rec))
    return rec


def smooth_radius(fwhm_ps: float, bin_ps: float, lib=None) -> int:
    return int((lib or load()).oracle_smooth_radius(float(fwhm_ps), float(bin_ps)))


def forward_smooth(scene, rec: np.ndarray | None = None, subset=None, lib=None) -> np.ndarray:
    """Smooth-response histograms [n_out, T] (fp64)."""
    lib = lib or load()
    if rec is None:
        rec = patches(scene, lib)
    rec = np.ascontiguousarray(rec, np.float64)
    n_total = scene.n_laser * scene.n_scan
    sub = None if subset is None else np.ascontiguousarray(subset, np.int32)
    n_out = n_total if sub is None else sub.shape[0]
    tau = np.zeros((n_out, int(scene.n_bins)), np.float64)
    rc = lib.oracle_forward_smooth(C.byref(make_params(scene)), _dptr(rec), rec.shape[0],
                                   None if sub is None else sub.ctypes.data, 0 if sub is None else n_out,
                                   _dptr(tau))
    if rc != 0:
        raise ValueError("oracle_forward_smooth rejected its arguments")
    return tau


def smooth_grad(scene, y: np.ndarray, depth64=None, albedo64=None, lib=None) -> dict:
    """Loss 1/2 ||tau_s - y||^2 and its gradient with respect to the depth and
    albedo maps (and each record), all fp64."""
    lib = lib or load()
    g = scene.patch_grid
    d, a, m = _maps64(scene, depth64, albedo64)
    npx = g["nx"] * g["ny"]
    yy = np.ascontiguousarray(y, np.float64).reshape(-1)
    if yy.size != scene.n_laser * scene.n_scan * int(scene.n_bins):
        raise ValueError("target has the wrong size")
    loss = C.c_double(0.0)
    gd = np.zeros(npx, np.float64)
    ga = np.zeros(npx, np.float64)
    gr = np.zeros((npx, 8), np.float64)
    rc = lib.oracle_smooth_grad(C.byref(make_params(scene)), C.byref(make_grid(g)), _dptr(d),
                                None if a is None else a.ctypes.data, None if m is None else m.ctypes.data,
                                _dptr(yy), C.byref(loss), gd.ctypes.data, ga.ctypes.data, gr.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_smooth_grad rejected its arguments")
    return {"loss": loss.value, "grad_depth": gd.reshape(g["nx"], g["ny"]),
            "grad_albedo": ga.reshape(g["nx"], g["ny"]), "grad_rec": gr}


def adjoint_records(scene, G: np.ndarray, rec: np.ndarray | None = None, subset=None, lib=None) -> np.ndarray:
    """Record gradients [n, 8] (d/d(pz, a, n_x, n_y, n_z) at 2..6) of the
    smooth forward for upstream gradient G [L*S, T], for the records in
    ``subset`` (default all)."""
    lib = lib or load()
    if rec is None:
        rec = patches(scene, lib)
    rec = np.ascontiguousarray(rec, np.float64)
    GG = np.ascontiguousarray(G, np.float64).reshape(-1)
    if GG.size != scene.n_laser * scene.n_scan * int(scene.n_bins):
        raise ValueError("upstream gradient has the wrong size")
    sub = None if subset is None else np.ascontiguousarray(subset, np.int32)
    n = rec.shape[0] if sub is None else sub.shape[0]
    out = np.zeros((n, 8), np.float64)
    rc = lib.oracle_adjoint_records(C.byref(make_params(scene)), _dptr(rec), rec.shape[0], _dptr(GG),
                                    None if sub is None else sub.ctypes.data, 0 if sub is None else n, _dptr(out))
    if rc != 0:
        raise ValueError("oracle_adjoint_records rejected its arguments")
    return out


NOISE_KEY1 = 0x4E4C4F53   # second key word of the noise generator


def philox4x64(ctr, key, lib=None) -> np.ndarray:
    """One Philox4x64-10 block (4 uint64) for counter ctr[4] and key key[2]."""
    lib = lib or load()
    c = np.ascontiguousarray(ctr, np.uint64)
    k = np.ascontiguousarray(key, np.uint64)
    o = np.zeros(4, np.uint64)
    u64p = C.POINTER(C.c_uint64)
    lib.oracle_philox4x64(c.ctypes.data_as(u64p), k.ctypes.data_as(u64p), o.ctypes.data_as(u64p))
    return o


def poisson_counts(lam, seed: int, lib=None) -> np.ndarray:
    """Counts of the noise sampler for means lam (element i uses stream i)."""
    lib = lib or load()
    lm = np.ascontiguousarray(lam, np.float64).ravel()
    k = np.zeros(lm.size, np.int64)
    lib.oracle_poisson_counts(_dptr(lm), lm.size, C.c_uint64(seed), k.ctypes.data)
    return k


def noise_scale(tau: np.ndarray, nr_db: float, lib=None):
    """(mean, population variance, sigma_n = Var / 10^(nr/10)) of an fp32 frame."""
    lib = lib or load()
    t = np.ascontiguousarray(tau, np.float32).ravel()
    o = np.zeros(3, np.float64)
    lib.oracle_noise_scale(t.ctypes.data, t.size, float(nr_db), _dptr(o))
    return float(o[0]), float(o[1]), float(o[2])


def poisson_noise(tau: np.ndarray, sigma_n: float, seed: int, lib=None) -> np.ndarray:
    """Poisson(tau * sigma_n) / sigma_n elementwise, fp32, same shape."""
    lib = lib or load()
    t = np.ascontiguousarray(tau, np.float32)
    out = np.zeros_like(t)
    lib.oracle_poisson_noise(t.ctypes.data, t.size, float(sigma_n), C.c_uint64(seed), out.ctypes.data)
    return out
