"""Pins of the FP64 oracle: checks against what the paper and the mathematics
fix, independent of the oracle's own code.

Each ``pin_*`` function takes a loaded oracle library (so the mutation tests
can run the same pins against deliberately broken copies of the oracle) and
raises AssertionError on failure.  Kinds of pin used:
  * closed forms of the definition in special cases (single patch at normal
    and oblique incidence, stand-off legs, fronto-parallel plane integral);
  * library routines (numpy.gradient for normals, numpy.bincount for the
    histogram, scipy.ndimage.gaussian_filter1d for the jitter);
  * high-precision brute force (mpmath, 50 digits) on tiny scenes;
  * invariants (linearity in albedo, energy under jitter, mirror symmetry,
    reciprocity of laser and detector legs).
"""
from __future__ import annotations

import json
import math
import os

import mpmath
import numpy as np
from scipy import ndimage

import oracle
import scenes

C_LIGHT = 299792458.0
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _f32(x):
    return float(np.float32(x))


def single_patch_scene(scan_c=(0.0, 0.0), patch_c=(0.0, 0.0), z=0.5, half=0.05,
                       bin_ps=16.0, T=4096, standoff=0.0, scan_n=(1, 1), scan_half=None,
                       cosines=True, albedo=0.7, depth_map=None):
    sh = half if scan_half is None else scan_half
    depth = np.full((1, 1), z, np.float32) if depth_map is None else depth_map
    pg = scenes.grid(depth.shape[0], depth.shape[1], half, half, patch_c[0], patch_c[1])
    return scenes.Scene("single", scenes.grid(scan_n[0], scan_n[1], sh, sh, scan_c[0], scan_c[1]),
                        None, pg, depth, np.full(depth.shape, albedo, np.float32), None,
                        standoff_m=standoff, bin_ps=bin_ps, n_bins=T, fwhm_ps=0.0,
                        cosines=cosines)


def _load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# Closed forms
# --------------------------------------------------------------------------
def pin_single_patch_normal(lib):
    """Patch straight in front of the scan point (Eq. (1) with cosines):
    arrival 2z/(c dt), weight a/z^4 with a = albedo * area."""
    g = _load_golden("single_patch.json")
    for case in g["normal_incidence"]:
        sc = single_patch_scene(z=case["z"], bin_ps=case["bin_ps"], half=case["half"],
                                albedo=case["albedo"])
        out = oracle.forward(sc, want_hist=True, want_tau=False, want_bins=True, lib=lib)
        H = out["hist"][0]
        k = case["bin"]
        assert out["bins"][0, 0] == k, (out["bins"][0, 0], k)
        nz = np.nonzero(H)[0]
        assert list(nz) == [k], nz
        area = (2 * case["half"]) ** 2
        z = _f32(case["z"])
        expect = _f32(case["albedo"]) * area / z ** 4
        assert abs(H[k] - expect) <= 1e-12 * expect, (H[k], expect)
        assert abs(H[k] / (_f32(case["albedo"]) * area) - case["weight_over_a"]) < 1e-5


def pin_single_patch_oblique(lib):
    """Scan point at (-0.3,-0.4), patch at (0,0,0.5) facing the wall:
    r = sqrt(0.5), every cosine = sqrt(0.5), so weight = a * (1/2)^2 / r^4 = a;
    without cosines weight = a / r^4 = 4a."""
    g = _load_golden("single_patch.json")["oblique"]
    for cos_on, ratio in ((True, g["weight_over_a_cos"]), (False, g["weight_over_a_nocos"])):
        sc = single_patch_scene(scan_c=(-0.3, -0.4), z=0.5, bin_ps=g["bin_ps"], cosines=cos_on)
        out = oracle.forward(sc, want_hist=True, want_tau=False, want_bins=True, lib=lib)
        assert out["bins"][0, 0] == g["bin"], out["bins"][0, 0]
        a = _f32(0.7) * (2 * 0.05) ** 2
        wx, wy = _f32(-0.3), _f32(-0.4)
        r = math.sqrt(wx * wx + wy * wy + 0.25)
        exact = a * ((0.5 / r) ** 4 if cos_on else 1.0) / r ** 4
        H = out["hist"][0]
        assert abs(H[g["bin"]] - exact) <= 1e-12 * exact
        assert abs(H[g["bin"]] / a - ratio) < 1e-6


def pin_standoff(lib):
    """Stand-off s = 1 m, scan point (0.5, 0.5) of a 2x2 grid over [-1,1]^2,
    patch right in front at depth 0.5: L = sqrt(1.5), the two device legs add
    2(L - s) to the path and weigh (s/L)^6 = 8/27 together."""
    g = _load_golden("single_patch.json")["standoff"]
    sc = single_patch_scene(scan_c=(0.0, 0.0), scan_n=(2, 2), scan_half=1.0,
                            patch_c=(0.5, 0.5), z=0.5, bin_ps=g["bin_ps"], standoff=1.0)
    out = oracle.forward(sc, want_hist=True, want_tau=False, want_bins=True, lib=lib)
    # scan index d = ix * ny + iy; (0.5, 0.5) is ix = iy = 1 -> d = 3
    assert out["bins"][3, 0] == g["bin"], out["bins"][:, 0]
    a = _f32(0.7) * 0.1 ** 2
    exact = a / 0.5 ** 4 * (1.0 / math.sqrt(1.5)) ** 6
    H = out["hist"][3]
    assert abs(H[g["bin"]] - exact) <= 1e-12 * exact, (H[g["bin"]], exact)
    assert abs(exact / (a / 0.5 ** 4) - 8.0 / 27.0) < 1e-12
    # the other three scan points see the patch obliquely: later arrivals
    assert all(out["bins"][d, 0] > g["bin"] for d in range(3))


def pin_layout(lib):
    """Output layout [x'][y'][t]: on a 2x4 scan grid each scan point's single
    arrival must match the closed-form distance to its own (x, y)."""
    sc = single_patch_scene(scan_c=(0.0, 0.0), scan_n=(2, 4), scan_half=0.4,
                            patch_c=(0.13, -0.21), z=0.45, bin_ps=2.0, T=8192)
    out = oracle.forward(sc, want_hist=False, want_tau=False, want_bins=True, lib=lib)
    px, py = _f32(0.13), _f32(-0.21)
    inv = 1.0 / (C_LIGHT * 2e-12)
    for ix in range(2):
        for iy in range(4):
            x = _f32(-0.4 + (ix + 0.5) * 0.4)
            y = _f32(-0.4 + (iy + 0.5) * 0.2)
            r = math.sqrt((px - x) ** 2 + (py - y) ** 2 + _f32(0.45) ** 2)
            assert out["bins"][ix * 4 + iy, 0] == math.floor(2 * r * inv), (ix, iy)


def plane_closed_form(z, bin_ps, T, cosines, rho=1.0):
    """Per-bin integral of an infinite fronto-parallel plane (confocal, s=0):
    bin k holds radii r in [k b/2, (k+1) b/2), b = c dt; with cosines the
    integrand is rho z^4 / r^8 (four cosines z/r, 1/r^4), without it rho / r^4;
    dA = 2 pi r dr."""
    b = C_LIGHT * bin_ps * 1e-12
    H = np.zeros(T)
    for k in range(T):
        lo, hi = max(k * b / 2, z), (k + 1) * b / 2
        if hi <= z:
            continue
        if cosines:
            H[k] = math.pi * rho * z ** 4 / 3 * (lo ** -6 - hi ** -6)
        else:
            H[k] = math.pi * rho * (lo ** -2 - hi ** -2)
    return H


def plane_scene(n, W=1.0, z=0.5, bin_ps=16.0, T=512, cosines=True, fwhm=0.0):
    depth = np.full((n, n), z, np.float32)
    return scenes.Scene("plane", scenes.grid(1, 1, W), None, scenes.grid(n, n, W), depth,
                        np.ones((n, n), np.float32), None, standoff_m=0.0, bin_ps=bin_ps,
                        n_bins=T, fwhm_ps=fwhm, cosines=cosines)


def _valid_bins(W, z, bin_ps, T):
    b = C_LIGHT * bin_ps * 1e-12
    rmax = math.sqrt(W * W + z * z)
    return np.array([k for k in range(T) if (k + 1) * b / 2 <= rmax and (k + 1) * b / 2 > z])


def pin_plane(lib, sizes=(256, 1024), fwhm=70.0):
    """Discrete plane converges to the closed-form integral (raw and jittered),
    with the error falling as the patch grid is refined."""
    W, z, bin_ps, T = 1.0, 0.5, 16.0, 512
    errs = {}
    for cos_on in (True, False):
        exact = plane_closed_form(z, bin_ps, T, cos_on)
        valid = _valid_bins(W, z, bin_ps, T)
        for n in sizes:
            sc = plane_scene(n, W, z, bin_ps, T, cos_on, fwhm)
            out = oracle.forward(sc, want_hist=True, want_tau=True, lib=lib)
            H = out["hist"][0]
            e_raw = np.linalg.norm(H[valid] - exact[valid]) / np.linalg.norm(exact[valid])
            tp = oracle.taps(fwhm, bin_ps, lib=lib)
            R = len(tp) // 2
            ex_j = np.convolve(exact, tp, mode="same")
            vj = valid[(valid >= valid.min() + R) & (valid <= valid.max() - R)]
            tau = out["tau"][0]
            e_j = np.linalg.norm(tau[vj] - ex_j[vj]) / np.linalg.norm(ex_j[vj])
            errs[(cos_on, n)] = (e_raw, e_j)
    for cos_on in (True, False):
        e_small = errs[(cos_on, sizes[0])]
        e_big = errs[(cos_on, sizes[-1])]
        assert e_big[0] <= 2.5e-2, errs
        assert e_big[1] <= 3e-3, errs
        assert e_small[0] / e_big[0] >= 4.0, errs
    return errs


# --------------------------------------------------------------------------
# Library routines
# --------------------------------------------------------------------------
def pin_normals_gradient(lib):
    """Normals and areas equal what numpy.gradient (central differences,
    one-sided at the border) gives; a tilted plane has the exact normal."""
    sc = scenes.tiny(seed=7, patches=(9, 6), masked=False)
    rec = oracle.patches(sc, lib=lib).reshape(9, 6, 8)
    g = sc.patch_grid
    hx, hy = 2 * g["half_x"] / g["nx"], 2 * g["half_y"] / g["ny"]
    D = sc.depth.astype(np.float64)
    gx = np.gradient(D, hx, axis=0, edge_order=1)
    gy = np.gradient(D, hy, axis=1, edge_order=1)
    ln = np.sqrt(1 + gx ** 2 + gy ** 2)
    np.testing.assert_allclose(rec[..., 4], gx / ln, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(rec[..., 5], gy / ln, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(rec[..., 6], -1 / ln, rtol=1e-13)
    np.testing.assert_allclose(rec[..., 3], sc.albedo.astype(np.float64) * hx * hy * ln, rtol=1e-13)
    # positions: cell centres
    xs = g["cx"] - g["half_x"] + (np.arange(9) + 0.5) * hx
    np.testing.assert_allclose(rec[:, 0, 0], xs.astype(np.float32), rtol=0, atol=0)
    # tilted plane D = 0.5 + 0.25 x: normal (0.25, 0, -1)/sqrt(1.0625)
    pg = scenes.grid(8, 8, 0.5)
    xs8 = (-0.5 + (np.arange(8) + 0.5) / 8).astype(np.float32)
    tilt = (0.5 + 0.25 * xs8[:, None] + 0 * xs8[None, :]).astype(np.float32)
    sc2 = scenes.Scene("tilt", pg, None, pg, tilt, None, None, 0.0, 16.0, 64, 0.0)
    rec2 = oracle.patches(sc2, lib=lib).reshape(8, 8, 8)
    inner = rec2[1:-1, 1:-1]
    L = math.sqrt(1 + 0.25 ** 2)
    np.testing.assert_allclose(inner[..., 4], 0.25 / L, rtol=2e-6)
    np.testing.assert_allclose(inner[..., 6], -1 / L, rtol=2e-6)
    np.testing.assert_allclose(inner[..., 3], 0.5 * (1 / 8) ** 2 * L, rtol=2e-6)   # null albedo -> 0.5


def pin_jitter_taps(lib):
    """Taps: length 2 ceil(2 sigma) + 1 (Section 2), sum 1, and the sigma they
    encode has FWHM = 2 sqrt(2 ln 2) sigma; the jittered trace equals
    scipy.ndimage.gaussian_filter1d with zero padding."""
    for fwhm, bin_ps in ((70.0, 16.0), (50.0, 8.0), (30.0, 4.0), (70.0, 32.0), (120.0, 50.0)):
        tp = oracle.taps(fwhm, bin_ps, lib=lib)
        R = len(tp) // 2
        # sigma recovered from the tap ratio g1/g0 = exp(-1/(2 sigma^2))
        sigma = math.sqrt(-1.0 / (2.0 * math.log(tp[R + 1] / tp[R])))
        # FWHM of exp(-x^2/(2 sigma^2)): the two half-maximum points
        half_width = mpmath.findroot(lambda x: mpmath.exp(-x ** 2 / (2 * sigma ** 2)) - 0.5, sigma)
        assert abs(2 * float(half_width) * bin_ps - fwhm) < 1e-8 * fwhm
        assert len(tp) == 2 * math.ceil(2 * sigma - 1e-12) + 1
        assert abs(tp.sum() - 1.0) < 1e-14
        np.testing.assert_allclose(tp, tp[::-1], rtol=0, atol=0)
    g = _load_golden("jitter_taps.json")
    for case in g["cases"]:
        tp = oracle.taps(case["fwhm_ps"], case["bin_ps"], lib=lib)
        assert len(tp) == 2 * case["R"] + 1
        assert abs(tp[case["R"]] - case["g0"]) < 1e-9
    # convolution = library filter with zero padding (mode='constant')
    sc = scenes.tiny(seed=11, n_bins=96, fwhm_ps=150.0)
    out = oracle.forward(sc, want_hist=True, want_tau=True, lib=lib)
    tp = oracle.taps(sc.fwhm_ps, sc.bin_ps, lib=lib)
    R = len(tp) // 2
    sigma = sc.fwhm_ps / (2 * math.sqrt(2 * math.log(2))) / sc.bin_ps
    ref = ndimage.gaussian_filter1d(out["hist"], sigma, axis=-1, mode="constant", cval=0.0,
                                    truncate=R / sigma)
    np.testing.assert_allclose(out["tau"], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def _mp_pair(px, py, pz, n, a, wl, wd, s, c, cosines, inv_prec):
    """Weight and exact arrival of one pair, from vector geometry in mpmath."""
    p = mpmath.matrix([px, py, pz])
    def leg(w):
        v = mpmath.matrix([w[0], w[1], 0]) - p          # patch -> wall
        r = mpmath.norm(v)
        e = v / r
        cos_w = -e[2]                                    # wall normal +z; patch -> wall is -e
        cos_p = max(mpmath.mpf(0), n[0] * e[0] + n[1] * e[1] + n[2] * e[2])
        return r, cos_w, cos_p
    rl, cwl, cpl = leg(wl)
    rd, cwd, cpd = leg(wd)
    def stand(w):
        if s == 0:
            return mpmath.mpf(0), mpmath.mpf(1)
        Ldev = mpmath.sqrt((w[0] - c[0]) ** 2 + (w[1] - c[1]) ** 2 + s ** 2)
        return Ldev - s, (s / Ldev) ** 3
    ol, gl = stand(wl)
    od, gd = stand(wd)
    u = (rl + rd + ol + od) * inv_prec
    w = a * gl * gd / (rl ** 2 * rd ** 2)
    if cosines:
        w = w * cwl * cpl * cpd * cwd
    return u, w


def pin_mpmath_bruteforce(lib, seeds=(101, 102, 103), nonconfocal=True):
    """50-digit brute force on tiny scenes: exact bins floor(u) and histogram
    (accumulated with numpy.bincount) agree with the oracle."""
    mpmath.mp.dps = 50
    cases = []
    for sd in seeds:
        cases.append(scenes.tiny(seed=sd, scan=(3, 2), patches=(5, 4), n_bins=48, bin_ps=40.0,
                                 standoff_m=0.0 if sd % 2 else 0.8))
    if nonconfocal:
        cases.append(scenes.tiny(seed=104, scan=(2, 3), patches=(4, 4), n_bins=64, bin_ps=40.0,
                                 laser=(2, 2), standoff_m=0.6))
        cases.append(scenes.tiny(seed=105, scan=(2, 2), patches=(4, 3), n_bins=64, bin_ps=40.0,
                                 laser=(1, 2), standoff_m=0.0, cosines=False))
    for sc in cases:
        rec = oracle.patches(sc, lib=lib)
        out = oracle.forward(sc, rec, want_hist=True, want_tau=False, want_bins=True, lib=lib)
        g = sc.patch_grid
        hx, hy = 2 * g["half_x"] / g["nx"], 2 * g["half_y"] / g["ny"]
        D = sc.depth.astype(np.float64)
        gx = np.gradient(D, hx, axis=0) if g["nx"] > 1 else np.zeros_like(D)
        gy = np.gradient(D, hy, axis=1) if g["ny"] > 1 else np.zeros_like(D)
        xs = [np.float32(g["cx"] - g["half_x"] + (i + 0.5) * hx) for i in range(g["nx"])]
        ys = [np.float32(g["cy"] - g["half_y"] + (j + 0.5) * hy) for j in range(g["ny"])]
        rg = sc.relay
        rxs = [np.float32(rg["cx"] - rg["half_x"] + (i + 0.5) * 2 * rg["half_x"] / rg["nx"]) for i in range(rg["nx"])]
        rys = [np.float32(rg["cy"] - rg["half_y"] + (j + 0.5) * 2 * rg["half_y"] / rg["ny"]) for j in range(rg["ny"])]
        if sc.laser is None:
            lpts = None
        else:
            lgd = sc.laser
            lxs = [np.float32(lgd["cx"] - lgd["half_x"] + (i + 0.5) * 2 * lgd["half_x"] / lgd["nx"]) for i in range(lgd["nx"])]
            lys = [np.float32(lgd["cy"] - lgd["half_y"] + (j + 0.5) * 2 * lgd["half_y"] / lgd["ny"]) for j in range(lgd["ny"])]
            lpts = [(float(x), float(y)) for x in lxs for y in lys]
        dpts = [(float(x), float(y)) for x in rxs for y in rys]
        inv_prec = 1 / (mpmath.mpf(C_LIGHT) * mpmath.mpf(sc.bin_ps) * mpmath.mpf("1e-12"))
        T = sc.n_bins
        S = len(dpts)
        L = 1 if lpts is None else len(lpts)
        for h in range(L * S):
            l, d = divmod(h, S)
            wd = dpts[d]
            wl = wd if lpts is None else lpts[l]
            ks, ws = [], []
            for ix in range(g["nx"]):
                for iy in range(g["ny"]):
                    pidx = ix * g["ny"] + iy
                    present = (sc.mask is None or sc.mask[ix, iy]) and sc.albedo[ix, iy] > 0
                    if not present:
                        assert out["bins"][h, pidx] == np.iinfo(np.int32).min
                        continue
                    ln = math.sqrt(1 + gx[ix, iy] ** 2 + gy[ix, iy] ** 2)
                    n = (mpmath.mpf(gx[ix, iy] / ln), mpmath.mpf(gy[ix, iy] / ln), mpmath.mpf(-1 / ln))
                    area = hx * hy * (ln if sc.cosines else 1.0)
                    a = mpmath.mpf(float(sc.albedo[ix, iy])) * mpmath.mpf(area)
                    u, w = _mp_pair(mpmath.mpf(float(xs[ix])), mpmath.mpf(float(ys[iy])),
                                    mpmath.mpf(float(D[ix, iy])), n, a, wl, wd,
                                    mpmath.mpf(sc.standoff_m), (rg["cx"], rg["cy"]),
                                    sc.cosines, inv_prec)
                    k = int(mpmath.floor(u))
                    frac = u - k
                    if min(frac, 1 - frac) > mpmath.mpf("1e-9"):
                        assert out["bins"][h, pidx] == k, (sc.name, h, pidx, out["bins"][h, pidx], k)
                    if 0 <= k < T:
                        ks.append(k)
                        ws.append(float(w))
            Hm = np.bincount(np.array(ks, np.int64), weights=np.array(ws), minlength=T)[:T]
            np.testing.assert_allclose(out["hist"][h], Hm, rtol=1e-12, atol=1e-12 * max(Hm.max(), 1e-300))


# --------------------------------------------------------------------------
# Invariants
# --------------------------------------------------------------------------
def pin_linearity(lib):
    """Amplitudes scale with albedo (Section 2, albedo discussion): the
    operator is linear in albedo; scaling by 2 is exact in fp64."""
    s1 = scenes.tiny(seed=21, scan=(4, 4), patches=(12, 12), n_bins=128, bin_ps=30.0,
                     standoff_m=0.5, masked=False)
    a1 = s1.albedo.copy()
    a2 = np.random.default_rng(5).uniform(0.1, 1.0, a1.shape).astype(np.float32)
    t1 = oracle.forward(s1, lib=lib)["tau"]
    s1.albedo = a2
    t2 = oracle.forward(s1, lib=lib)["tau"]
    mix = (0.5 * a1 + 0.25 * a2).astype(np.float32)
    s1.albedo = mix
    tm = oracle.forward(s1, lib=lib)["tau"]
    # the fp32 mix of albedos is what the operator sees: compare against it
    ref = 0.5 * t1 + 0.25 * t2
    assert np.linalg.norm(tm - ref) <= 1e-6 * np.linalg.norm(ref)
    s1.albedo = (2 * a1).astype(np.float32)
    t4 = oracle.forward(s1, lib=lib)["tau"]
    np.testing.assert_array_equal(t4, 2 * t1)


def pin_energy(lib):
    """Jitter conserves each trace's energy when every arrival lies at least
    R bins inside the window (normalised taps, zero padding)."""
    sc = scenes.tiny(seed=31, scan=(3, 3), patches=(10, 10), n_bins=512, bin_ps=20.0,
                     fwhm_ps=200.0, zlo=0.3, zhi=0.5)
    out = oracle.forward(sc, want_hist=True, want_tau=True, want_bins=True, lib=lib)
    R = len(oracle.taps(sc.fwhm_ps, sc.bin_ps, lib=lib)) // 2
    b = out["bins"]
    pres = b != np.iinfo(np.int32).min
    assert b[pres].min() >= R and b[pres].max() < sc.n_bins - R, (b[pres].min(), b[pres].max())
    np.testing.assert_allclose(out["tau"].sum(1), out["hist"].sum(1), rtol=1e-12)
    # and lowers the peak
    assert np.all(out["tau"].max(1) <= out["hist"].max(1))


def pin_mirror(lib):
    """Mirroring the scene in x mirrors the bins exactly (power-of-two grids
    make the cell-centred coordinates exactly antisymmetric)."""
    sc = scenes.tiny(seed=41, scan=(4, 4), patches=(8, 8), n_bins=96, bin_ps=25.0,
                     standoff_m=0.7)
    out = oracle.forward(sc, want_tau=True, want_bins=True, lib=lib)
    sm = scenes.tiny(seed=41, scan=(4, 4), patches=(8, 8), n_bins=96, bin_ps=25.0, standoff_m=0.7)
    sm.depth = sc.depth[::-1].copy()
    sm.albedo = sc.albedo[::-1].copy()
    sm.mask = sc.mask[::-1].copy()
    om = oracle.forward(sm, want_tau=True, want_bins=True, lib=lib)
    tau = out["tau"].reshape(4, 4, -1)
    taum = om["tau"].reshape(4, 4, -1)
    np.testing.assert_allclose(taum, tau[::-1], rtol=1e-12, atol=1e-14 * tau.max())
    bins = out["bins"].reshape(4, 4, 8, 8)
    binsm = om["bins"].reshape(4, 4, 8, 8)
    np.testing.assert_array_equal(binsm, bins[::-1, :, ::-1, :])
    # x and y are not interchangeable unless the scene is transposed too
    st = scenes.tiny(seed=41, scan=(4, 4), patches=(8, 8), n_bins=96, bin_ps=25.0, standoff_m=0.7)
    st.depth, st.albedo, st.mask = sc.depth.T.copy(), sc.albedo.T.copy(), sc.mask.T.copy()
    ot = oracle.forward(st, want_tau=True, lib=lib)["tau"].reshape(4, 4, -1)
    np.testing.assert_allclose(ot, tau.transpose(1, 0, 2), rtol=1e-12, atol=1e-14 * tau.max())


def pin_reciprocity(lib):
    """With laser and detector grids equal, swapping the laser and detector
    points leaves every histogram unchanged; the diagonal equals confocal."""
    sc = scenes.tiny(seed=51, scan=(3, 3), patches=(6, 6), n_bins=128, bin_ps=30.0,
                     laser=(3, 3), standoff_m=0.9)
    sc.laser = dict(sc.relay)
    tau = oracle.forward(sc, lib=lib)["tau"].reshape(9, 9, -1)
    np.testing.assert_allclose(tau, tau.transpose(1, 0, 2), rtol=1e-12, atol=1e-14 * tau.max())
    conf = scenes.tiny(seed=51, scan=(3, 3), patches=(6, 6), n_bins=128, bin_ps=30.0,
                       standoff_m=0.9)
    tc = oracle.forward(conf, lib=lib)["tau"]
    np.testing.assert_allclose(tau[np.arange(9), np.arange(9)], tc, rtol=1e-13, atol=0)


def pin_presence(lib):
    """A null albedo means 0.5 (Section 2 depth-to-volume mapping); masked,
    zero-albedo and non-positive-depth patches are absent."""
    sc = scenes.tiny(seed=61, patches=(4, 4), masked=False)
    sc.albedo = None
    rec = oracle.patches(sc, lib=lib)
    g = sc.patch_grid
    hx = 2 * g["half_x"] / g["nx"]
    assert np.all(rec[:, 7] == 1)
    ln = np.sqrt(1 + rec[:, 4] ** 2 / rec[:, 6] ** 2 + rec[:, 5] ** 2 / rec[:, 6] ** 2)
    np.testing.assert_allclose(rec[:, 3], 0.5 * hx * hx * ln, rtol=1e-12)
    sc.albedo = np.ones((4, 4), np.float32)
    sc.albedo[0, 0] = 0.0
    sc.depth = sc.depth.copy()
    sc.depth[1, 1] = -0.2
    sc.depth[2, 2] = np.nan
    sc.mask = np.ones((4, 4), np.uint8)
    sc.mask[3, 3] = 0
    rec = oracle.patches(sc, lib=lib).reshape(4, 4, 8)
    absent = {(0, 0), (1, 1), (2, 2), (3, 3)}
    for ix in range(4):
        for iy in range(4):
            assert rec[ix, iy, 7] == (0 if (ix, iy) in absent else 1)


def pin_backfacing(lib):
    """Lambertian cosines clamp at zero: a steep patch (slope 2 along x) lit
    from behind contributes nothing, lit from the front it contributes the
    closed-form weight.  Non-confocal, so each leg's clamp is seen alone."""
    h = 0.125                                   # patch spacing: 3 cells over [-0.1875, 0.1875]
    z0 = 0.5
    depth = np.array([[z0 - 2 * h], [z0], [z0 + 2 * h]], np.float32)   # D_x = 2
    mask = np.array([[0], [1], [0]], np.uint8)
    pg = scenes.grid(3, 1, 1.5 * h, 0.5 * h)
    n = np.array([2.0, 0.0, -1.0]) / math.sqrt(5.0)
    for lx, dx in ((-0.4, 0.4), (0.4, -0.4), (0.4, 0.3)):
        sc = scenes.Scene("steep", scenes.grid(1, 1, 0.01, 0.01, dx, 0.0),
                          scenes.grid(1, 1, 0.01, 0.01, lx, 0.0), pg, depth,
                          np.full((3, 1), 0.6, np.float32), mask, standoff_m=0.0,
                          bin_ps=4.0, n_bins=4096, fwhm_ps=0.0)
        H = oracle.forward(sc, want_hist=True, want_tau=False, lib=lib)["hist"][0]
        p = np.array([0.0, 0.0, z0])
        wl, wd = np.array([_f32(lx), 0, 0]), np.array([_f32(dx), 0, 0])
        rl, rd = np.linalg.norm(wl - p), np.linalg.norm(wd - p)
        cpl = max(0.0, n @ (wl - p) / rl)
        cpd = max(0.0, n @ (wd - p) / rd)
        a = _f32(0.6) * h * h * math.sqrt(5.0)
        expect = a * (z0 / rl) * cpl * cpd * (z0 / rd) / (rl * rl * rd * rd)
        if lx < 0 or dx < 0:
            assert expect == 0.0 and not H.any(), H.sum()
        else:
            assert expect > 0 and abs(H.sum() - expect) <= 1e-9 * expect, (H.sum(), expect)


FAST_PINS = [pin_backfacing, pin_single_patch_normal, pin_single_patch_oblique, pin_standoff, pin_layout,
             pin_normals_gradient, pin_jitter_taps, pin_linearity, pin_energy, pin_mirror,
             pin_reciprocity, pin_presence]
