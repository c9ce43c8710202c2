"""Shared plumbing of the GPU parity tests: move a seeded scene to the GPU,
run the HIP path through the C ABI, and compare with the FP64 oracle."""
from __future__ import annotations

import math
import sys

import numpy as np

import oracle

REL_L2_TOL = 1e-5   # per histogram, against the fp64 oracle


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_gpu(scene):
    import torch
    dev = "cuda"
    depth = torch.from_numpy(np.ascontiguousarray(scene.depth, np.float32)).to(dev)
    albedo = None if scene.albedo is None else torch.from_numpy(
        np.ascontiguousarray(scene.albedo, np.float32)).to(dev)
    mask = None if scene.mask is None else torch.from_numpy(
        np.ascontiguousarray(scene.mask, np.uint8)).to(dev)
    return depth, albedo, mask


def gpu_patches(scene, stream=None):
    import paper_2506_03747_amd as nl
    depth, albedo, mask = to_gpu(scene)
    return nl.patches_from_depth(depth, scene.patch_grid, albedo, mask, cosines=scene.cosines,
                                 stream=stream)


def gpu_forward(scene, stream=None, use_n_active=True):
    import torch
    import paper_2506_03747_amd as nl
    patches, n_act = gpu_patches(scene, stream)
    prm = nl.params_of(scene)
    if use_n_active:
        tau = nl.forward(prm, patches, n_act, stream=stream)
    else:
        torch.cuda.synchronize()
        n = int(n_act.item())
        tau = nl.forward(prm, patches[:max(n, 0)].contiguous(), None, stream=stream)
    torch.cuda.synchronize()
    return tau, patches, n_act


def rel_l2_rows(got: np.ndarray, ref: np.ndarray) -> np.ndarray:
    got = got.reshape(-1, got.shape[-1]).astype(np.float64)
    ref = ref.reshape(-1, ref.shape[-1])
    num = np.linalg.norm(got - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    out = np.zeros_like(num)
    nz = den > 0
    out[nz] = num[nz] / den[nz]
    out[~nz] = np.where(num[~nz] == 0, 0.0, np.inf)
    return out


def assert_parity(got, ref, tol=REL_L2_TOL, what=""):
    e = rel_l2_rows(got, ref)
    worst = int(np.argmax(e))
    assert e.max() <= tol, f"{what}: rel-L2 {e.max():.3e} at histogram {worst} (tol {tol})"
    return float(e.max())


def guard_delta(T: int) -> float:
    """The guard half-width the kernels use: 16 ulp(1) of T + 2 bins."""
    return float(np.float32(16.0 * (T + 2.0) * math.ldexp(1.0, -24)))


def oracle_bins_for_records(scene, gpu_patches_np, n_act, subset=None):
    """Oracle bins reordered to the GPU record order ([H, n_act])."""
    o = oracle.forward(scene, subset=subset, want_tau=False, want_bins=True)
    idx = gpu_patches_np[:n_act, 7].view(np.int32)
    return o["bins"][:, idx]


# --------------------------------------------------------------------------
# Per-histogram tolerance.  A histogram's GPU result differs from the fp64
# oracle through (i) the fp32 weight of each in-window pair, bounded by the
# oracle's error model (a few ulp per weight, and the cancellation of a
# grazing patch cosine against fp32 record normals), and (ii) the 64-bit
# fixed-point accumulation, which rounds each pair's increment by at most
# g_l g_d W_u / 2^32, W_u the weight bound of the histogram's unit under the
# scale rule nlos.h states (summaries of 256 consecutive records in record
# order).  Both are jittered like the histogram (the taps are positive, so
# the bound carries through), and the tolerance is
#     tol_h = max(1e-5, (||jit(err_h)|| + g_h W_h 2^-32 ||jit(count_h)||) / ||tau_h||).
# For a histogram of well-conditioned pairs the bracket is ~1e-6, so the
# 1e-5 bar holds; it exceeds 1e-5 only for histograms made of a few pairs
# seen edge-on or far weaker than their unit's bound.

def record_order(patch_grid, present):
    """Pixel indices (ix * ny + iy) of the present pixels in the record order
    nlos.h documents: 16x16-pixel blocks, x major over blocks, each as 4
    stride-2 phases (ix mod 2, iy mod 2) of 8x8 pixels."""
    nx, ny = int(patch_grid["nx"]), int(patch_grid["ny"])
    bx, by = -(-nx // 16), -(-ny // 16)
    e = np.arange(256 * bx * by, dtype=np.int64)
    chunk, w = e >> 6, e & 63
    phase, blk = chunk & 3, chunk >> 2
    ix = (blk // by) * 16 + (w >> 3) * 2 + (phase >> 1)
    iy = (blk % by) * 16 + (w & 7) * 2 + (phase & 1)
    ok = (ix < nx) & (iy < ny)
    idx = (ix * ny + iy)[ok]
    return idx[np.asarray(present).reshape(-1)[idx]]


def _approx_coords(g, axis):
    n, half, c = int(g["n" + axis]), float(g["half_" + axis]), float(g["c" + axis])
    a0, step = np.float32(c - half), np.float32((2.0 * half) / n)
    return (a0 + (np.arange(n, dtype=np.float32) + np.float32(0.5)) * step).astype(np.float64)


def unit_weight_bounds(scene, rec):
    """W_u of every histogram ([L*S], output order) under the stated scale
    rule -- the bound of the aligned block of 4 x 4 scan points (confocal) or
    2 lasers x 2 x 2 detectors that holds it -- from fp64 records ``rec``
    (oracle layout)."""
    order = record_order(scene.patch_grid, rec[:, 7] != 0)
    R = rec[order]
    n = len(order)
    S = scene.n_scan
    L = scene.n_laser
    if n == 0:
        return np.zeros(L * S)
    st = np.arange(0, n, 256)
    x0, x1 = np.minimum.reduceat(R[:, 0], st), np.maximum.reduceat(R[:, 0], st)
    y0, y1 = np.minimum.reduceat(R[:, 1], st), np.maximum.reduceat(R[:, 1], st)
    z0, am = np.minimum.reduceat(R[:, 2], st), np.maximum.reduceat(R[:, 3], st)
    tl, tx, ty = (1, 4, 4) if scene.laser is None else (2, 2, 2)
    rx, ry = _approx_coords(scene.relay, "x"), _approx_coords(scene.relay, "y")
    nrx, nry = len(rx), len(ry)
    lpts = None
    if scene.laser is not None:
        lxs, lys = _approx_coords(scene.laser, "x"), _approx_coords(scene.laser, "y")
        lpts = np.stack([np.repeat(lxs, len(lys)), np.tile(lys, len(lxs))], axis=1)

    def axis_d(a0, a1, b0, b1):
        # lateral gap between intervals [a0, a1] (per unit) and [b0, b1] (per summary)
        return np.maximum(np.maximum(a0[:, None] - b1[None, :], b0[None, :] - a1[:, None]), 0.0)

    ix0 = np.arange(0, nrx, tx)
    iy0 = np.arange(0, nry, ty)
    dx = axis_d(rx[ix0], rx[np.minimum(ix0 + tx, nrx) - 1], x0, x1)      # [utx, ns]
    dy = axis_d(ry[iy0], ry[np.minimum(iy0 + ty, nry) - 1], y0, y1)      # [uty, ns]
    z2 = z0 * z0
    rd2 = dx[:, None, :] ** 2 + dy[None, :, :] ** 2 + z2                  # [utx, uty, ns]
    if lpts is None:
        Wu = np.max(am / (rd2 * rd2), axis=2)[None]                       # [1, utx, uty]
        lunit = np.zeros(1, np.int64)
    else:
        l0 = np.arange(0, L, tl)
        lrx0 = np.array([lpts[a:a + tl, 0].min() for a in l0])
        lrx1 = np.array([lpts[a:a + tl, 0].max() for a in l0])
        lry0 = np.array([lpts[a:a + tl, 1].min() for a in l0])
        lry1 = np.array([lpts[a:a + tl, 1].max() for a in l0])
        rl2 = axis_d(lrx0, lrx1, x0, x1) ** 2 + axis_d(lry0, lry1, y0, y1) ** 2 + z2     # [utl, ns]
        Wu = np.stack([np.max(am / (rl2[u][None, None, :] * rd2), axis=2) for u in range(len(l0))])
        lunit = np.arange(L) // tl
    ux = np.arange(nrx) // tx
    uy = np.arange(nry) // ty
    W = Wu[lunit[:, None, None], ux[None, :, None], uy[None, None, :]]  # [L, nrx, nry]
    return W.reshape(-1)


def parity_tolerance(scene, ref_tau, subset=None, rec=None, floor=REL_L2_TOL):
    """Per-histogram tolerance (see above) for the histograms ``subset`` (all
    when None) whose oracle output is ``ref_tau`` [n, T]."""
    from scipy import ndimage
    if rec is None:
        rec = oracle.patches(scene)
    m = oracle.error_model(scene, rec, subset=subset)
    taps = oracle.taps(scene.fwhm_ps, scene.bin_ps)
    jerr = ndimage.convolve1d(m["err"], taps, axis=1, mode="constant")
    jcnt = ndimage.convolve1d(m["count"], taps, axis=1, mode="constant")
    W = unit_weight_bounds(scene, rec)
    if subset is not None:
        W = W[np.asarray(subset)]
    # the kernel's bound is taken in fp32 from fp32 records: 1% margin
    q = 1.01 * m["gain"] * W * 2.0 ** -32
    nrm = np.linalg.norm(ref_tau.reshape(len(W), -1), axis=1)
    bound = np.where(nrm > 0, (np.linalg.norm(jerr, axis=1) + q * np.linalg.norm(jcnt, axis=1)) /
                     np.where(nrm > 0, nrm, 1.0), 0.0)
    return np.maximum(floor, bound)


def assert_parity_model(got, ref, tol, what=""):
    """Every histogram within its own tolerance (exact zeros where the
    oracle's histogram is zero); returns (worst rel-L2, worst ratio to the
    tolerance, histograms whose tolerance exceeds 1e-5)."""
    e = rel_l2_rows(got, ref)
    tol = np.asarray(tol, np.float64).reshape(-1)
    r = e / tol
    worst = int(np.argmax(r))
    loose = int(np.sum(tol > REL_L2_TOL))
    assert r.max() <= 1.0, (f"{what}: rel-L2 {e[worst]:.3e} at histogram {worst} over its tolerance "
                            f"{tol[worst]:.3e}")
    log(f"{what}: worst rel-L2 {e.max():.3e}, worst ratio to tolerance {r.max():.3f}, "
        f"{loose} of {len(tol)} histograms with tolerance above 1e-5 (largest {tol.max():.3e})")
    return float(e.max()), float(r.max()), loose
