"""Pins of the numpy oracle of the paper's FFT (light-cone) forward route:

  - R_z after the pairwise means has the closed form 1 / (J M) at coarse
    sample (J^2 - 1) // M (the paper's 1 / sqrt(i) fold, M^2 -> M means);
  - the time resampling covers every fine v-sample exactly once (rows are
    means, columns add up to one coarse sample);
  - the FFT convolution equals a brute-force linear convolution (loops);
  - a single patch arrives in the same time bin (+-1) as in the direct
    operator at many lateral offsets, on 1 m and 2 m walls;
  - whole scenes correlate with the direct operator above 0.9 (the paper's
    route is a quantised discretisation of Eq. (1) without cosines);
  - linearity in albedo.
Each takes the module under test as argument (so a mutated copy can be
checked against them)."""
from __future__ import annotations

import numpy as np

import oracle
import scenes


def lct_scene(N=32, M=512, bin_ps=16.0, seed=3, half=0.5, masked=True, zlo=0.3, zhi=0.8, fwhm_ps=60.0):
    rng = np.random.default_rng(seed)
    z = zlo + (zhi - zlo) * scenes._minmax(scenes._smooth(rng.standard_normal((N, N)), N / 8))
    alb = rng.uniform(0.2, 1.0, (N, N))
    mask = scenes._blob_mask(rng, (N, N), N / 8) if masked else None
    return scenes.Scene(f"lct{seed}", scenes.grid(N, N, half), None, scenes.grid(N, N, half), z.astype(np.float32),
                        alb.astype(np.float32), mask, standoff_m=0.0, bin_ps=bin_ps, n_bins=M, fwhm_ps=fwhm_ps,
                        cosines=False, seed=seed)


def pin_rz_closed_form(L):
    for M in (1, 2, 8, 64):
        R = L.rz_matrix(M)
        want = np.zeros((M, M))
        for J in range(1, M + 1):
            want[(J * J - 1) // M, J - 1] = (1.0 / J) / M
        np.testing.assert_array_equal(R, want)


def pin_rt_coverage(L):
    for M in (1, 4, 16, 256):
        R = L.rt_matrix(M)
        np.testing.assert_allclose(R.sum(axis=1), 1.0, rtol=1e-14)
        span = 2 * np.arange(M) + 1.0
        np.testing.assert_allclose((R * span[:, None]).sum(axis=0), float(M), rtol=1e-14)


def pin_fft_convolution_brute_force(L):
    sc = lct_scene(N=3, M=4, bin_ps=400.0, half=0.5, zlo=0.05, zhi=0.2, masked=False, fwhm_ps=0.0)
    _, parts = L.forward(sc, jitter=False, return_parts=True)
    N, M = 3, 4
    P = L.psf(N, M, parts["slope"])
    RV = parts["RV"]
    want = np.zeros((N, N, M))
    for xo in range(N):
        for yo in range(N):
            for c in range(M):
                acc = 0.0
                for x in range(N):
                    for y in range(N):
                        for u in range(c + 1):
                            acc += RV[x, y, u] * P[(xo - x) % (2 * N), (yo - y) % (2 * N), c - u]
                want[xo, yo, c] = acc
    assert np.abs(want).max() > 0
    np.testing.assert_allclose(parts["conv"], want, rtol=1e-10, atol=1e-12 * np.abs(want).max())


def pin_single_patch_timing(L):
    for half, D0 in ((0.5, 0.5), (1.0, 0.8)):
        N, M = 32, 512
        z = np.ones((N, N), np.float32)
        z[N // 2, N // 2] = D0
        mask = np.zeros((N, N), np.uint8)
        mask[N // 2, N // 2] = 1
        sc = scenes.Scene("one", scenes.grid(N, N, half), None, scenes.grid(N, N, half), z,
                          np.ones((N, N), np.float32), mask, standoff_m=0.0, bin_ps=16.0, n_bins=M, fwhm_ps=0.0,
                          cosines=False)
        lt = L.forward(sc, jitter=False)
        d = oracle.forward(sc)["tau"].reshape(lt.shape)
        for (dx, dy) in ((0, 0), (4, 0), (0, 5), (3, 3), (10, 7), (-9, 4), (-14, -12)):
            x, y = N // 2 + dx, N // 2 + dy
            if not d[x, y].any():
                continue
            assert abs(int(np.argmax(lt[x, y])) - int(np.argmax(d[x, y]))) <= 1, (half, dx, dy)


def pin_correlation_with_direct(L):
    for kw in (dict(), dict(half=1.0, zlo=0.5, zhi=1.1), dict(masked=False, seed=4)):
        sc = lct_scene(**kw)
        lt = L.forward(sc)
        d = oracle.forward(sc)["tau"]
        r = float(np.corrcoef(lt.ravel(), d.ravel())[0, 1])
        assert r > 0.9, (kw, r)


def pin_taps_match_direct(L):
    """The jitter taps equal the direct operator's (its C oracle, pinned to
    scipy's Gaussian filter)."""
    for fwhm, dt in ((60.0, 16.0), (70.0, 32.0), (30.0, 4.0), (0.0, 8.0), (250.0, 3.0)):
        np.testing.assert_allclose(L.taps(fwhm, dt), oracle.taps(fwhm, dt), rtol=1e-13, atol=1e-16)


def pin_linear_in_albedo(L):
    sc = lct_scene(N=16, M=256, bin_ps=32.0, seed=5)
    a = L.forward(sc)
    sc2 = lct_scene(N=16, M=256, bin_ps=32.0, seed=5)
    sc2.albedo = (sc2.albedo * 2).astype(np.float32)
    np.testing.assert_allclose(L.forward(sc2), 2 * a, rtol=1e-9, atol=1e-12 * np.abs(a).max())


# cheapest first
LCT_PINS = [pin_rz_closed_form, pin_rt_coverage, pin_taps_match_direct, pin_fft_convolution_brute_force,
            pin_linear_in_albedo, pin_single_patch_timing, pin_correlation_with_direct]
