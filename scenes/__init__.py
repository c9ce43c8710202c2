"""Seeded synthetic scene generators for the transient NLOS forward operator.

This module only draws inputs: depth fields, albedo maps, masks and the
parameter values of each workload.  It holds none of the operator's
arithmetic (no geometry, no binning, no jitter), so that both the FP64
oracle and the HIP path can be fed from it without sharing any code.

The paper's own workload is ShapeNet-derived 128x128 depth maps over a
2 m x 2 m scan area with 1024 bins (Simulation section).  That dataset is not
available here; smooth, masked random depth fields of the same shapes stand
in for its object silhouettes.  No dataset item is reproduced.

Conventions shared by every scene (they describe inputs, not the method):
  * a grid is ``dict(nx, ny, half_x, half_y, cx, cy)``: ``nx*ny`` cells over
    ``[cx-half_x, cx+half_x] x [cy-half_y, cy+half_y]`` on the wall plane z=0;
  * maps are float32 / uint8 arrays of shape ``[nx, ny]`` indexed ``[x][y]``
    (the paper writes D_{x,y}, A_{x,y});
  * depth is in metres, albedo in [0, 1], ``mask`` nonzero = patch present.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
from scipy import ndimage

__all__ = [
    "Scene",
    "grid",
    "cfg1",
    "cfg2",
    "cfg3",
    "cfg4_request",
    "cfg4_requests",
    "cfg5",
    "pshape",
    "tiny",
    "by_name",
]


@dataclasses.dataclass
class Scene:
    """One simulation request: hidden surface maps plus system parameters."""

    name: str
    relay: dict                 # scan grid (confocal) or detector grid
    laser: Optional[dict]       # None -> confocal
    patch_grid: dict            # lateral grid of the depth map
    depth: np.ndarray           # float32 [px, py] metres
    albedo: Optional[np.ndarray]  # float32 [px, py] in [0,1]; None -> 0.5
    mask: Optional[np.ndarray]  # uint8 [px, py]; None -> all present
    standoff_m: float
    bin_ps: float
    n_bins: int
    fwhm_ps: float
    cosines: bool = True
    seed: int = 0

    @property
    def n_scan(self) -> int:
        return self.relay["nx"] * self.relay["ny"]

    @property
    def n_laser(self) -> int:
        return 1 if self.laser is None else self.laser["nx"] * self.laser["ny"]

    @property
    def n_patch_total(self) -> int:
        return self.patch_grid["nx"] * self.patch_grid["ny"]

    def out_shape(self):
        r = self.relay
        if self.laser is None:
            return (r["nx"], r["ny"], self.n_bins)
        return (self.n_laser, r["nx"], r["ny"], self.n_bins)


def grid(nx: int, ny: int, half_x: float, half_y: float | None = None,
         cx: float = 0.0, cy: float = 0.0) -> dict:
    return dict(nx=int(nx), ny=int(ny), half_x=float(half_x),
                half_y=float(half_x if half_y is None else half_y),
                cx=float(cx), cy=float(cy))


def _smooth(x: np.ndarray, sigma_px: float) -> np.ndarray:
    return ndimage.gaussian_filter(x, sigma_px, mode="reflect")


def _minmax(x: np.ndarray) -> np.ndarray:
    lo, hi = float(x.min()), float(x.max())
    return (x - lo) / (hi - lo) if hi > lo else np.zeros_like(x)


def _blob_mask(rng: np.random.Generator, shape, sigma_px: float) -> np.ndarray:
    f = _smooth(rng.standard_normal(shape), sigma_px)
    return (f > np.median(f)).astype(np.uint8)


def cfg1(seed: int = 1) -> Scene:
    """Confocal plain: 32x32 scan on a 1x1 m wall, stand-off 1.0 m; 64x64
    patches at z = 0.5 m +/- 0.05 (smoothed), albedo U[0,1] masked by a random
    blob; T=512 bins of 16 ps; jitter FWHM 70 ps."""
    rng = np.random.default_rng(seed)
    n = 64
    z = _smooth(rng.uniform(-0.05, 0.05, (n, n)), 3.0)
    z = 0.45 + 0.10 * _minmax(z)
    albedo = rng.uniform(0.0, 1.0, (n, n))
    mask = _blob_mask(rng, (n, n), 8.0)
    return Scene("cfg1", grid(32, 32, 0.5), None, grid(n, n, 0.5),
                 z.astype(np.float32), albedo.astype(np.float32), mask,
                 standoff_m=1.0, bin_ps=16.0, n_bins=512, fwhm_ps=70.0, seed=seed)


def cfg2(seed: int = 2) -> Scene:
    """Confocal plain: 64x64 scan on a 2x2 m wall; 256x256 patches from a
    smooth random depth field in [0.4, 1.2] m with a binary mask, albedo
    U[0,1]; T=1024 bins of 8 ps; FWHM 50 ps.  No stand-off is given, so the
    calibrated (zero stand-off) convention applies."""
    rng = np.random.default_rng(seed)
    n = 256
    z = 0.4 + 0.8 * _minmax(_smooth(rng.standard_normal((n, n)), 16.0))
    mask_rng = np.random.default_rng([seed, 1])
    mask = _blob_mask(mask_rng, (n, n), 16.0)
    albedo = rng.uniform(0.0, 1.0, (n, n))
    return Scene("cfg2", grid(64, 64, 1.0), None, grid(n, n, 1.0),
                 z.astype(np.float32), albedo.astype(np.float32), mask,
                 standoff_m=0.0, bin_ps=8.0, n_bins=1024, fwhm_ps=50.0, seed=seed)


def cfg3(seed: int = 3, det: int = 128, las: int = 8, n_bins: int = 2048) -> Scene:
    """Non-confocal: 8x8 laser points x 128x128 detector points on a 2x2 m
    wall, stand-off 2.0 m; 128x128 patches from two overlapping seeded depth
    surfaces (front-most wins); T=2048 bins of 4 ps; FWHM 30 ps."""
    rng = np.random.default_rng(seed)
    n = 128
    z1 = 0.4 + 0.8 * _minmax(_smooth(rng.standard_normal((n, n)), 12.0))
    z2 = 0.4 + 0.8 * _minmax(_smooth(rng.standard_normal((n, n)), 12.0))
    m1 = _blob_mask(rng, (n, n), 12.0).astype(bool)
    m2 = _blob_mask(rng, (n, n), 12.0).astype(bool)
    a1 = rng.uniform(0.0, 1.0, (n, n))
    a2 = rng.uniform(0.0, 1.0, (n, n))
    z1m = np.where(m1, z1, np.inf)
    z2m = np.where(m2, z2, np.inf)
    front1 = z1m <= z2m
    depth = np.where(front1, z1m, z2m)
    albedo = np.where(front1, a1, a2)
    mask = (m1 | m2).astype(np.uint8)
    depth = np.where(mask.astype(bool), depth, 1.0)   # masked cells: any finite value
    return Scene("cfg3", grid(det, det, 1.0), grid(las, las, 1.0), grid(n, n, 1.0),
                 depth.astype(np.float32), albedo.astype(np.float32), mask,
                 standoff_m=2.0, bin_ps=4.0, n_bins=n_bins, fwhm_ps=30.0, seed=seed)


def cfg4_request(i: int, seed: int = 4, max_scan: int = 128, max_patch: int = 262144) -> Scene:
    """Request i of the batched serving mix (seed seed + i): confocal, scan
    size U{32..128}^2 on a 2x2 m wall, patch count U[4k, 262k] rounded to a
    square grid, T in {512, 1024, 2048}, bin 4-16 ps, FWHM 30-70 ps, depths in
    [0.2, 0.6] of the window's half path length so arrivals land in the window,
    albedo U[0,1], blob mask."""
    rng = np.random.default_rng(seed + i)
    ns = int(rng.integers(32, max_scan + 1))
    p = int(rng.integers(4096, max_patch + 1))
    npg = max(2, int(round(np.sqrt(p))))
    T = int(rng.choice([512, 1024, 2048]))
    bin_ps = float(rng.uniform(4.0, 16.0))
    fwhm = float(rng.uniform(30.0, 70.0))
    window_m = 299792458.0 * T * bin_ps * 1e-12
    zlo, zhi = 0.2 * window_m / 2, 0.6 * window_m / 2
    z = zlo + (zhi - zlo) * _minmax(_smooth(rng.standard_normal((npg, npg)), npg / 16.0))
    albedo = rng.uniform(0.0, 1.0, (npg, npg))
    mask = _blob_mask(rng, (npg, npg), npg / 16.0)
    return Scene(f"cfg4[{i}]", grid(ns, ns, 1.0), None, grid(npg, npg, 1.0),
                 z.astype(np.float32), albedo.astype(np.float32), mask,
                 standoff_m=0.0, bin_ps=bin_ps, n_bins=T, fwhm_ps=fwhm, seed=seed + i)


def cfg4_requests(n_requests: int = 256, seed: int = 4, max_scan: int = 128, max_patch: int = 262144):
    """The batched serving mix: requests 0 .. n_requests-1 of cfg4_request."""
    return [cfg4_request(i, seed, max_scan, max_patch) for i in range(n_requests)]


def cfg5(seed: int = 5) -> Scene:
    """Adjoint workload: confocal 128x128 scan on a 2x2 m wall, 128x128
    patches (no mask), T=1024 bins of 8 ps, FWHM 50 ps."""
    rng = np.random.default_rng(seed)
    n = 128
    z = 0.4 + 0.8 * _minmax(_smooth(rng.standard_normal((n, n)), 8.0))
    albedo = rng.uniform(0.0, 1.0, (n, n))
    return Scene("cfg5", grid(128, 128, 1.0), None, grid(n, n, 1.0),
                 z.astype(np.float32), albedo.astype(np.float32), None,
                 standoff_m=0.0, bin_ps=8.0, n_bins=1024, fwhm_ps=50.0, seed=seed)


def pshape(seed: int = 6) -> Scene:
    """Stand-in for the paper's dataset shape: 128x128 scan over 2x2 m,
    128x128 silhouette depth map, albedo 1, T=1024 bins of 32 ps, 70 ps FWHM."""
    rng = np.random.default_rng(seed)
    n = 128
    z = 0.5 + 1.0 * _minmax(_smooth(rng.standard_normal((n, n)), 10.0))
    mask = _blob_mask(rng, (n, n), 10.0)
    return Scene("pshape", grid(128, 128, 1.0), None, grid(n, n, 1.0),
                 z.astype(np.float32), np.ones((n, n), np.float32), mask,
                 standoff_m=0.0, bin_ps=32.0, n_bins=1024, fwhm_ps=70.0, seed=seed)


def tiny(seed: int = 100, scan=(4, 4), patches=(8, 8), n_bins: int = 64,
         bin_ps: float = 50.0, standoff_m: float = 0.0, fwhm_ps: float = 120.0,
         laser=None, half: float = 0.5, zlo: float = 0.3, zhi: float = 0.6,
         masked: bool = True, cosines: bool = True) -> Scene:
    """Small random scene for brute-force and high-precision checks."""
    rng = np.random.default_rng(seed)
    px, py = patches
    z = rng.uniform(zlo, zhi, (px, py))
    albedo = rng.uniform(0.05, 1.0, (px, py))
    mask = (rng.uniform(size=(px, py)) > 0.3).astype(np.uint8) if masked else None
    lg = None if laser is None else grid(laser[0], laser[1], half)
    return Scene(f"tiny{seed}", grid(scan[0], scan[1], half), lg, grid(px, py, half),
                 z.astype(np.float32), albedo.astype(np.float32), mask,
                 standoff_m=standoff_m, bin_ps=bin_ps, n_bins=n_bins, fwhm_ps=fwhm_ps,
                 cosines=cosines, seed=seed)


def by_name(name: str) -> Scene:
    return {"cfg1": cfg1, "cfg2": cfg2, "cfg3": cfg3, "cfg5": cfg5, "pshape": pshape}[name]()
