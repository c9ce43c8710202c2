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
  - linearity in albedo;
  - the absolute amplitude: a plane's windowed response equals the direct
    operator's times the ratio the discretisation of Eq. (3) predicts.
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


def pin_plane_amplitude(L):
    """Absolute scale against the direct operator.  For a uniform plane at
    depth z (albedo rho, no cosines, s = 0), Eq. (3) and Eq. (1) both give
    tau = pi rho / r^3 per unit of path, so the direct histogram of time bin
    j is pi rho (r_lo^-2 - r_hi^-2) = pi rho (2j + 1) / (dz^2 j^2 (j + 1)^2),
    dz = c dt / 2.  The route, on its grid, puts the plane at layer
    J0 = floor(z / dz) + 1 with the fold weight 1 / J0 and the means 1 / M,
    its cone holds about pi M dz^2 / cell^2 lattice cells per coarse sample
    (cell = 2 w / N), and each time bin J = j + 1 is divided by (J dz)^3:
        tau_route / tau_direct = N^2 dz j^2 / (4 w^2 J0 (j + 1) (2 j + 1)).
    Summed over the bins whose annulus stays on the plane seen from its
    centre (which evens out the lattice count), the route's output equals
    that ratio times the direct oracle's within 5% on three grids; a
    constant-factor mistake in the fold, the means, the time resampling or
    the v^(3/2) scaling does not."""
    c = 299792458.0
    for (N, M, dt, w, j0) in ((64, 512, 16.0, 1.0, 300), (96, 1024, 8.0, 1.0, 600), (64, 512, 16.0, 0.5, 200)):
        dz = c * dt * 1e-12 / 2.0
        z0 = (j0 + 0.5) * dz
        sc = scenes.Scene("plane", scenes.grid(N, N, w), None, scenes.grid(N, N, w),
                          np.full((N, N), z0, np.float32), np.ones((N, N), np.float32), None, standoff_m=0.0,
                          bin_ps=dt, n_bins=M, fwhm_ps=0.0, cosines=False)
        lt = L.forward(sc, jitter=False)
        d = oracle.forward(sc, want_hist=True, want_tau=False)["hist"].reshape(N, N, M)
        xc, J0 = N // 2, j0 + 1
        jmax = int(np.sqrt(z0 ** 2 + (0.5 * w) ** 2) / dz)
        js = np.arange(j0 + 4, jmax)
        K = N * N * dz * js ** 2 / (4.0 * w * w * J0 * (js + 1) * (2 * js + 1))
        ratio = lt[xc, xc, js].sum() / (K * d[xc, xc, js]).sum()
        assert abs(ratio - 1.0) < 0.05, (N, M, dt, w, ratio)


# cheapest first
LCT_PINS = [pin_rz_closed_form, pin_rt_coverage, pin_taps_match_direct, pin_fft_convolution_brute_force,
            pin_linear_in_albedo, pin_single_patch_timing, pin_correlation_with_direct, pin_plane_amplitude]
