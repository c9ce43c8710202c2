"""Pins of the oracle's fp32 error model (CPU): the per-histogram tolerance
of the GPU parity tests comes from it, so it is checked against what it
claims to bound.

  * counts: the per-bin pair count equals numpy.bincount of the oracle's own
    bins (pinned to 50-digit mpmath elsewhere) over the in-window pairs;
  * bound: perturbing every record normal component by a relative amount of
    at most e1 and every patch factor a by at most e0 moves each bin of the
    raw histogram by no more than the model's bound (random draws on scenes
    with steep, grazing surfaces, confocal and non-confocal);
  * sharpness: on a single grazing patch placed so that every coordinate
    difference is a sum of magnitudes (patch and wall point on opposite
    sides of each axis), the perturbation that pushes each leg's cosine
    numerator by exactly e1 times the sum of its terms' moduli reaches the
    bound (so it is not vacuous, and every term of it counts);
  * without cosines the bound is e0 times the weight.
"""
from __future__ import annotations

import numpy as np

import oracle
import scenes

E0, E1 = 2e-6, 16 * 2.0 ** -24


def _steep_scene(seed, laser=None, standoff=0.0):
    """Tiny scene whose depth map has steep slopes (patches seen nearly
    edge-on from much of the wall)."""
    sc = scenes.tiny(seed=seed, scan=(5, 4), patches=(12, 10), n_bins=256, bin_ps=16.0, fwhm_ps=0.0,
                     laser=laser, standoff_m=standoff, masked=False)
    rng = np.random.default_rng(seed)
    x = np.linspace(-1, 1, 12)[:, None]
    y = np.linspace(-1, 1, 10)[None, :]
    sc.depth = (0.6 + 0.35 * np.sin(3.0 * x + 1.7 * y + rng.uniform(0, 6)) * np.cos(2.0 * y)).astype(np.float32)
    return sc


def _perturbed(rec, rng, e0, e1):
    r = rec.copy()
    r[:, 4:7] *= 1.0 + rng.uniform(-e1, e1, (r.shape[0], 3))
    r[:, 3] *= 1.0 + rng.uniform(-e0, e0, r.shape[0])
    return r


def pin_error_counts(lib):
    for sc in (_steep_scene(1201), _steep_scene(1202, laser=(2, 3), standoff=0.4)):
        rec = oracle.patches(sc, lib)
        m = oracle.error_model(sc, rec, lib=lib)
        bins = oracle.forward(sc, rec, want_tau=False, want_bins=True, lib=lib)["bins"]
        present = rec[:, 7] != 0
        T = sc.n_bins
        for h in range(bins.shape[0]):
            b = bins[h][present]
            b = b[(b >= 0) & (b < T)]
            np.testing.assert_array_equal(m["count"][h], np.bincount(b, minlength=T)[:T].astype(np.float64))


def pin_error_bound_holds(lib):
    for sc in (_steep_scene(1203), _steep_scene(1204, laser=(3, 2), standoff=0.7), _steep_scene(1205)):
        rec = oracle.patches(sc, lib)
        H = oracle.forward(sc, rec, want_hist=True, want_tau=False, lib=lib)["hist"]
        err = oracle.error_model(sc, rec, lib=lib)["err"]
        assert H.any()
        rng = np.random.default_rng(sc.seed)
        worst = 0.0
        for _ in range(6):
            Hp = oracle.forward(sc, _perturbed(rec, rng, E0, E1), want_hist=True, want_tau=False, lib=lib)["hist"]
            d = np.abs(Hp - H)
            slack = 1e-12 * np.abs(H) + 1e-300
            assert np.all(d <= err + slack), f"{sc.name}: {np.max(d - err)}"
            nz = err > 0
            worst = max(worst, float(np.max(d[nz] / err[nz])))
        # random perturbations reach a fair share of the bound somewhere
        assert worst > 0.05, worst


def pin_error_bound_sharp(lib):
    """One patch tilted to a few milliradians of grazing from the scan
    point: the adversarial perturbation reaches the bound within 1e-6."""
    for tilt in (3e-3, 2e-2):
        sc = scenes.tiny(seed=1206, scan=(1, 1), patches=(1, 1), n_bins=4096, bin_ps=8.0, fwhm_ps=0.0,
                         masked=False)
        sc.relay = scenes.grid(1, 1, 0.3, 0.3, 0.4, -0.1)
        sc.patch_grid = scenes.grid(1, 1, 0.05, 0.05, 0.0, 0.0)
        sc.depth = np.full((1, 1), 0.5, np.float32)
        rec = oracle.patches(sc, lib)
        wx, wy = oracle.grid_coords(sc.relay, lib)
        p = rec[0, :3]
        d = p - np.array([wx[0], wy[0], 0.0])
        # a unit normal (towards the wall) at `tilt` radians from grazing
        e = -d / np.linalg.norm(d)
        t = np.cross(e, [0.0, 1.0, 0.0])
        t /= np.linalg.norm(t)
        n = np.sin(tilt) * e + np.cos(tilt) * t
        rec[0, 4:7] = n
        err = oracle.error_model(sc, rec, e0=0.0, lib=lib)["err"]
        H = oracle.forward(sc, rec, want_hist=True, want_tau=False, lib=lib)["hist"]
        k = int(np.nonzero(H[0])[0][0])
        terms = n * d
        r = rec.copy()
        r[0, 4:7] = n * (1.0 + E1 * np.sign(terms) * np.sign(terms.sum()))
        Hp = oracle.forward(sc, r, want_hist=True, want_tau=False, lib=lib)["hist"]
        ratio = abs(Hp[0, k] - H[0, k]) / err[0, k]
        assert abs(ratio - 1.0) < 1e-6, (tilt, ratio)


def pin_error_no_cosines(lib):
    sc = _steep_scene(1207)
    sc.cosines = False
    rec = oracle.patches(sc, lib)
    H = oracle.forward(sc, rec, want_hist=True, want_tau=False, lib=lib)["hist"]
    err = oracle.error_model(sc, rec, e0=3e-6, e1=1.0, lib=lib)["err"]
    np.testing.assert_allclose(err, 3e-6 * H, rtol=1e-12, atol=0)


def pin_error_gain(lib):
    """The stand-off weight: 1 without stand-off; with it, the histogram sum
    of a lone patch without cosines times r_l^2 r_d^2 / a, and the closed
    form 8/27 for the scan point (0.5, 0.5) with s = 1 m (device at the
    origin's wall normal: L = sqrt(1.5), (s / L)^3 per leg, two legs)."""
    sc = scenes.tiny(seed=1208, scan=(2, 2), patches=(4, 4), n_bins=64, laser=(2, 1))
    assert np.all(oracle.error_model(sc, lib=lib)["gain"] == 1.0)
    sc = scenes.tiny(seed=1209, scan=(2, 2), patches=(1, 1), n_bins=8192, bin_ps=8.0, fwhm_ps=0.0,
                     masked=False, standoff_m=1.0, cosines=False)
    sc.relay = scenes.grid(2, 2, 1.0)
    sc.patch_grid = scenes.grid(1, 1, 0.05, 0.05, 0.1, -0.2)
    sc.depth = np.full((1, 1), 0.5, np.float32)
    rec = oracle.patches(sc, lib)
    g = oracle.error_model(sc, rec, lib=lib)["gain"]
    np.testing.assert_allclose(g, 8.0 / 27.0, rtol=1e-12)
    H = oracle.forward(sc, rec, want_hist=True, want_tau=False, lib=lib)["hist"]
    wx, wy = oracle.grid_coords(sc.relay, lib)
    for h in range(4):
        r2 = (rec[0, 0] - wx[h // 2]) ** 2 + (rec[0, 1] - wy[h % 2]) ** 2 + rec[0, 2] ** 2
        np.testing.assert_allclose(g[h], H[h].sum() * r2 * r2 / rec[0, 3], rtol=1e-12)


ERROR_PINS = [pin_error_counts, pin_error_bound_holds, pin_error_bound_sharp, pin_error_no_cosines, pin_error_gain]
