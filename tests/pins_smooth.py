"""Pins of the oracle's smooth forward and its gradient, each against
something other than the oracle's own formula:

  - a single patch, whose response is w * the normal density (scipy.stats),
    with w and u from the closed forms of the single-patch geometry;
  - mass: summed over bins, the smooth response equals the hard histogram's
    sum (a separate oracle function) when every arrival lies well inside the
    window (the Gaussian samples at unit spacing sum to 1 far below 1e-9);
  - the albedo gradient against central differences of the loss, which is
    quadratic in the albedo, so the difference is exact up to rounding;
  - the depth gradient against central differences with Richardson
    extrapolation on fp64 depth maps, at corners, borders, interior pixels
    and a masked pixel whose depth only enters its neighbours' normals.
Each takes the oracle library as argument so that a planted mistake in a
rebuilt copy can be checked against them."""
from __future__ import annotations

import math

import numpy as np

import oracle
import scenes

C = 299792458.0


def smooth_scene(seed, scan=(3, 3), patches=(6, 7), n_bins=512, bin_ps=20.0, fwhm_ps=60.0, standoff_m=0.0,
                 laser=None, cosines=True, masked=True, half=0.5):
    """Gently curved surface at about 0.5 m: arrivals well inside the window
    and no patch near grazing (so no cosine clamp is crossed by the finite
    differences)."""
    rng = np.random.default_rng(seed)
    px, py = patches
    x = np.linspace(-1, 1, px)[:, None]
    y = np.linspace(-1, 1, py)[None, :]
    ph = rng.uniform(0, 2 * np.pi, 3)
    z = 0.5 + 0.03 * np.sin(2.1 * x + ph[0]) * np.cos(1.7 * y + ph[1]) + 0.02 * np.sin(1.3 * x * y + ph[2])
    albedo = rng.uniform(0.2, 1.0, (px, py))
    mask = None
    if masked:
        mask = np.ones((px, py), np.uint8)
        mask[rng.integers(1, px - 1), rng.integers(1, py - 1)] = 0
    lg = None if laser is None else scenes.grid(laser[0], laser[1], half)
    return scenes.Scene(f"smooth{seed}", scenes.grid(scan[0], scan[1], half), lg, scenes.grid(px, py, half),
                        z.astype(np.float32), albedo.astype(np.float32), mask, standoff_m=standoff_m,
                        bin_ps=bin_ps, n_bins=n_bins, fwhm_ps=fwhm_ps, cosines=cosines, seed=seed)


def _sigma_bins(fwhm_ps, bin_ps):
    return fwhm_ps / (2.0 * math.sqrt(2.0 * math.log(2.0))) / bin_ps


def _loss(sc, y, depth64=None, albedo64=None, lib=None):
    rec = oracle.patches_f64(sc, depth64, albedo64, lib=lib)
    t = oracle.forward_smooth(sc, rec, lib=lib)
    return 0.5 * float(np.sum((t - y.reshape(t.shape)) ** 2))


def _target(sc, lib):
    """A second, different scene's smooth response as the target."""
    other = smooth_scene(sc.seed + 1000, scan=(sc.relay["nx"], sc.relay["ny"]),
                         patches=(sc.patch_grid["nx"], sc.patch_grid["ny"]), n_bins=sc.n_bins, bin_ps=sc.bin_ps,
                         fwhm_ps=sc.fwhm_ps, standoff_m=sc.standoff_m,
                         laser=None if sc.laser is None else (sc.laser["nx"], sc.laser["ny"]),
                         cosines=sc.cosines)
    other.depth = (other.depth + np.float32(0.004)).astype(np.float32)
    return oracle.forward_smooth(other, lib=lib)


def pin_smooth_single_patch(lib):
    from scipy.stats import norm
    for cosines in (True, False):
        for (cx, cy) in ((0.0, 0.0), (0.3, 0.4)):
            z, rho, half = 0.5, 0.8, 0.05
            sc = scenes.Scene("one", scenes.grid(1, 1, 0.5), None,
                              dict(nx=1, ny=1, half_x=half, half_y=half, cx=cx, cy=cy),
                              np.full((1, 1), z, np.float32), np.full((1, 1), rho, np.float32), None,
                              standoff_m=0.0, bin_ps=16.0, n_bins=600, fwhm_ps=70.0, cosines=cosines)
            t = oracle.forward_smooth(sc, lib=lib)[0]
            px, py = float(np.float32(cx)), float(np.float32(cy))
            r = math.sqrt(px * px + py * py + z * z)
            a = float(np.float32(rho)) * (2 * half) ** 2
            # normal (0, 0, -1): both cosines are z / r
            w = a * z ** 4 / r ** 8 if cosines else a / r ** 4
            u = 2.0 * r / (C * 16e-12)
            sig = _sigma_bins(70.0, 16.0)
            rs = math.ceil(6 * sig)
            k = np.arange(600)
            want = np.where(np.abs(k - math.floor(u)) <= rs, w * norm.pdf(k + 0.5 - u, scale=sig), 0.0)
            np.testing.assert_allclose(t, want, rtol=1e-11, atol=1e-14 * w)


def pin_smooth_mass(lib):
    for kw in (dict(seed=11), dict(seed=12, laser=(2, 2), standoff_m=0.3),
               dict(seed=13, cosines=False)):
        sc = smooth_scene(**kw)
        rec = oracle.patches_f64(sc, lib=lib)
        t = oracle.forward_smooth(sc, rec, lib=lib)
        o = oracle.forward(sc, rec, want_hist=True, want_tau=False, want_bins=True, lib=lib)
        rs = oracle.smooth_radius(sc.fwhm_ps, sc.bin_ps, lib=lib)
        b = o["bins"][o["bins"] != np.iinfo(np.int32).min]
        assert b.min() > rs + 1 and b.max() < sc.n_bins - rs - 2, "arrivals too close to the window edge"
        np.testing.assert_allclose(t.sum(axis=1), o["hist"].sum(axis=1), rtol=1e-8)


def pin_grad_albedo_fd(lib):
    for kw in (dict(seed=21), dict(seed=22, cosines=False, standoff_m=0.4)):
        sc = smooth_scene(**kw)
        y = _target(sc, lib)
        g = oracle.smooth_grad(sc, y, lib=lib)
        a0 = sc.albedo.astype(np.float64)
        h = 0.05
        for (i, j) in ((0, 0), (2, 3), (5, 6), (3, 0)):
            ap, am = a0.copy(), a0.copy()
            ap[i, j] += h
            am[i, j] -= h
            fd = (_loss(sc, y, albedo64=ap, lib=lib) - _loss(sc, y, albedo64=am, lib=lib)) / (2 * h)
            scale = np.abs(g["grad_albedo"]).max()
            assert abs(fd - g["grad_albedo"][i, j]) <= 1e-8 * scale + 1e-15, (kw, i, j, fd, g["grad_albedo"][i, j])


def _fd_richardson(sc, y, d0, i, j, h, lib):
    def cd(hh):
        dp, dm = d0.copy(), d0.copy()
        dp[i, j] += hh
        dm[i, j] -= hh
        return (_loss(sc, y, depth64=dp, lib=lib) - _loss(sc, y, depth64=dm, lib=lib)) / (2 * hh)
    return (4.0 * cd(h / 2) - cd(h)) / 3.0


def pin_grad_depth_fd(lib):
    for kw in (dict(seed=31), dict(seed=32, cosines=False), dict(seed=33, standoff_m=0.6, laser=(2, 1)),
               dict(seed=34, scan=(2, 4), patches=(5, 4))):
        sc = smooth_scene(**kw)
        y = _target(sc, lib)
        g = oracle.smooth_grad(sc, y, lib=lib)
        d0 = sc.depth.astype(np.float64)
        nx, ny = d0.shape
        pts = {(0, 0), (nx - 1, ny - 1), (0, ny // 2), (nx - 1, 1), (nx // 2, 0), (nx // 2, ny - 1),
               (nx // 2, ny // 2), (1, 1)}
        if sc.mask is not None:
            mi, mj = np.argwhere(sc.mask == 0)[0]
            pts.add((int(mi), int(mj)))
            assert sc.mask[mi, mj] == 0
        scale = np.abs(g["grad_depth"]).max()
        for (i, j) in sorted(pts):
            fd = _fd_richardson(sc, y, d0, i, j, 2e-5, lib)
            assert abs(fd - g["grad_depth"][i, j]) <= 2e-6 * scale, (kw, i, j, fd, g["grad_depth"][i, j], scale)


SMOOTH_PINS = [pin_smooth_single_patch, pin_smooth_mass, pin_grad_albedo_fd, pin_grad_depth_fd]


def pin_adjoint_records_fd(lib):
    """Adjoint identity on the records themselves: for a random upstream
    gradient G, sum(G * dtau_s/dq) by central differences of the smooth
    forward in each record field q (pz with Richardson; a and n enter
    polynomially of degree <= 2, so their differences are exact up to
    rounding) equals the record gradient."""
    rng = np.random.default_rng(5)
    for kw in (dict(seed=41), dict(seed=42, cosines=False, standoff_m=0.5), dict(seed=43, laser=(2, 2))):
        sc = smooth_scene(**kw)
        rec = oracle.patches_f64(sc, lib=lib)
        G = rng.standard_normal((sc.n_laser * sc.n_scan, sc.n_bins))
        present = np.nonzero(rec[:, 7])[0]
        sub = present[[0, len(present) // 2, len(present) - 1]]
        gr = oracle.adjoint_records(sc, G, rec, subset=sub, lib=lib)

        def dot(r):
            return float(np.sum(G * oracle.forward_smooth(sc, r, lib=lib)))

        for i, p in enumerate(sub):
            for field, h in ((2, 2e-5), (3, 1e-3), (4, 1e-2), (5, 1e-2), (6, 1e-2)):
                if field >= 4 and not sc.cosines:
                    assert gr[i, field] == 0.0
                    continue

                def cd(hh):
                    rp, rm = rec.copy(), rec.copy()
                    rp[p, field] += hh
                    rm[p, field] -= hh
                    return (dot(rp) - dot(rm)) / (2 * hh)
                fd = (4 * cd(h / 2) - cd(h)) / 3 if field == 2 else cd(h)
                scale = np.abs(gr[:, 2:7]).max()
                assert abs(fd - gr[i, field]) <= 2e-6 * scale, (kw, p, field, fd, gr[i, field])


SMOOTH_PINS.append(pin_adjoint_records_fd)
