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
