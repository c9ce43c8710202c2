"""The moment form of the smooth response (the GPU's k_smooth_mom), checked on
the host: with t = f - 1/2, the Taylor series sum_m (-t)^m / m! N^(m)(d)
(m <= 7 at support radius 12, m <= 5 at 16 and 20),
N^(m)(d) = N(d) (-1/sigma)^m He_m(d / sigma), reproduces the direct Gaussian
samples N(d + 1/2 - f) over the support |d| <= ceil(6 sigma) to the stated
bound for every sub-bin offset, at the widths that take that kernel (the
narrowest, sigma just above 11/6 bins, included)."""
import math

import numpy as np
import pytest


def hermite_e(n, x):
    """Probabilists' Hermite polynomial He_n by its three-term recurrence."""
    h0, h1 = np.ones_like(x), x
    if n == 0:
        return h0
    for k in range(1, n):
        h0, h1 = h1, x * h1 - k * h0
    return h1


def moment_kernels(sigma, rs, n_moments=8):
    d = np.arange(-rs, rs + 1, dtype=np.float64)
    g = np.exp(-0.5 * (d / sigma) ** 2) / (sigma * math.sqrt(2 * math.pi))
    return d, [g * (-1.0 / sigma) ** m * hermite_e(m, d / sigma) / math.factorial(m) for m in range(n_moments)]


# moments per radius as the kernel takes them, and the bound each must meet
MOMENTS = {12: (8, 7e-8), 16: (6, 1.2e-6), 20: (6, 1.2e-6)}


@pytest.mark.parametrize("fwhm_ps,bin_ps", [(70.0, 16.0), (50.0, 8.0), (30.0, 4.0), (43.19, 10.0), (47.12, 8.0)])
def test_moment_series_matches_direct_samples(fwhm_ps, bin_ps):
    sigma = fwhm_ps / (2 * math.sqrt(2 * math.log(2))) / bin_ps
    rs = math.ceil(6 * sigma)
    assert rs in MOMENTS
    n_moments, bound = MOMENTS[rs]
    d, K = moment_kernels(sigma, rs, n_moments=n_moments)
    worst = 0.0
    for f in np.linspace(0.0, 1.0, 101, endpoint=False):
        t = f - 0.5
        direct = np.exp(-0.5 * ((d + 0.5 - f) / sigma) ** 2) / (sigma * math.sqrt(2 * math.pi))
        series = sum((-t) ** m * K[m] for m in range(len(K)))
        worst = max(worst, np.linalg.norm(series - direct) / np.linalg.norm(direct))
    assert worst <= bound


def test_moment_series_shifted_histogram():
    """A set of arrivals binned into moment rows and convolved gives the
    histogram of the direct sum (sigma = 2.65 bins, Rs = 16)."""
    sigma, rs, T = 50.0 / (2 * math.sqrt(2 * math.log(2))) / 8.0, 16, 128
    rng = np.random.default_rng(7)
    u = rng.uniform(-10.0, T + 10.0, 500)
    w = rng.uniform(0.1, 1.0, 500)
    direct = np.zeros(T)
    for ui, wi in zip(u, w):
        k0 = math.floor(ui)
        for k in range(max(0, k0 - rs), min(T, k0 + rs + 1)):
            x = k + 0.5 - ui
            direct[k] += wi * math.exp(-0.5 * (x / sigma) ** 2) / (sigma * math.sqrt(2 * math.pi))
    d, K = moment_kernels(sigma, rs)
    H = np.zeros((len(K), T + 2 * rs))
    for ui, wi in zip(u, w):
        k0 = math.floor(ui)
        if k0 + rs < 0 or k0 - rs > T - 1:
            continue
        t = (ui - k0) - 0.5
        for m in range(len(K)):
            H[m, k0 + rs] += wi * (-t) ** m
    series = np.zeros(T)
    for k in range(T):
        for m in range(len(K)):
            for j, dd in enumerate(d.astype(int)):
                series[k] += H[m, k - dd + rs] * K[m][j]
    assert np.linalg.norm(series - direct) <= 1e-7 * np.linalg.norm(direct)


# correlation rows per radius as the adjoint takes them
ADJ_ROWS = {12: 9, 16: 7, 20: 7}


@pytest.mark.parametrize("fwhm_ps,bin_ps", [(70.0, 16.0), (43.19, 10.0), (50.0, 8.0), (47.12, 8.0), (30.0, 4.0)])
def test_adjoint_series_matches_direct_sums(fwhm_ps, bin_ps):
    """The adjoint's two sums over the support, G0 = sum_k g N(x) and
    G1 = sum_k g (x / sigma^2) N(x), x = k + 1/2 - u, from the correlations
    C_m[k0] = sum_d g[k0 + d] K_m(d), m < n: G0 = sum_{m<=n-2} (-t)^m C_m,
    G1 = -sum_{m<=n-2} (-t)^m (m + 1) C_{m+1} (n = 9 at radius 12, 7 at 16
    and 20)."""
    sigma = fwhm_ps / (2 * math.sqrt(2 * math.log(2))) / bin_ps
    rs = math.ceil(6 * sigma)
    n = ADJ_ROWS[rs]
    d, K = moment_kernels(sigma, rs, n_moments=n)
    rng = np.random.default_rng(11)
    g = rng.standard_normal(2 * rs + 1)              # upstream gradient over the support of one pair
    C = [float(np.dot(g, K[m])) for m in range(n)]
    worst0 = worst1 = 0.0
    for f in np.linspace(0.0, 1.0, 51, endpoint=False):
        t = f - 0.5
        x = d + 0.5 - f
        N = np.exp(-0.5 * (x / sigma) ** 2) / (sigma * math.sqrt(2 * math.pi))
        G0 = float(np.dot(g, N))
        G1 = float(np.dot(g, x / sigma ** 2 * N))
        s0 = sum((-t) ** m * C[m] for m in range(n - 1))
        s1 = -sum((-t) ** m * (m + 1) * C[m + 1] for m in range(n - 1))
        scale0 = float(np.linalg.norm(g) * np.linalg.norm(N))
        scale1 = float(np.linalg.norm(g) * np.linalg.norm(x / sigma ** 2 * N))
        worst0 = max(worst0, abs(s0 - G0) / scale0)
        worst1 = max(worst1, abs(s1 - G1) / scale1)
    assert worst0 <= 1e-6
    assert worst1 <= 3e-6
