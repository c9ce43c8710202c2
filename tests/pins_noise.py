"""Pins of the oracle's Poisson noise (Algorithm 1 step 2.4):

  - the Philox4x64-10 blocks equal numpy's own Philox bit generator (whose
    zero-key, zero-counter block is the published known-answer vector);
  - the exp / log / log-factorial recipes against the C library within a
    few ulp;
  - below lambda = 10 every count equals the inversion of scipy's Poisson
    CDF at the uniform drawn from numpy's Philox (exact, ties aside);
  - above, the counts follow scipy's Poisson law (chi-square, mean and
    variance), and lambda = 0 gives 0;
  - the frame variance and sigma_n against numpy; noisy values are integer
    multiples of 1 / sigma_n with the right mean."""
from __future__ import annotations

import math

import numpy as np

import oracle

SEED = 0x1234ABCD


def _numpy_block(ctr, key):
    c = [int(x) for x in ctr]
    assert c[0] >= 1
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array([c[0] - 1, c[1], c[2], c[3]], dtype=np.uint64))
    return bg.random_raw(4).astype(np.uint64)


def pin_philox_vs_numpy(lib):
    m = np.uint64(0xFFFFFFFFFFFFFFFF)
    z = np.random.Philox(key=np.array([0, 0], dtype=np.uint64), counter=np.array([m, m, m, m], dtype=np.uint64))
    np.testing.assert_array_equal(oracle.philox4x64([0, 0, 0, 0], [0, 0], lib=lib), z.random_raw(4))
    rng = np.random.default_rng(3)
    for _ in range(20):
        ctr = [int(rng.integers(1, 2**63)), int(rng.integers(0, 2**63)), int(rng.integers(0, 2**32)), 0]
        key = [int(rng.integers(0, 2**63)), oracle.NOISE_KEY1]
        np.testing.assert_array_equal(oracle.philox4x64(ctr, key, lib=lib), _numpy_block(ctr, key))


def pin_exp_log_recipes(lib):
    xs = np.concatenate([-np.logspace(-12, np.log10(700), 400), [0.0, -1e-300]])
    for x in xs:
        assert abs(lib.oracle_nx_exp(x) - math.exp(x)) <= 1e-15 * math.exp(x), x
    for x in np.concatenate([np.logspace(-300, 300, 400), [1.0, 2.0, 0.5, 10.0]]):
        v = lib.oracle_nx_log(x)
        assert abs(v - math.log(x)) <= 4e-16 * max(1.0, abs(math.log(x))), x
    for k in list(range(0, 60)) + [100, 1000, 12345, 10**6, 10**9]:
        v = lib.oracle_nx_logfact(float(k))
        assert abs(v - math.lgamma(k + 1.0)) <= 1e-14 * max(1.0, math.lgamma(k + 1.0)), k


def _uniform(i, t, seed=SEED):
    """Uniform t of element i (i >= 1) from numpy's Philox, as documented."""
    blk = _numpy_block([i, t // 4, 0, 0], [seed, oracle.NOISE_KEY1])
    return float(int(blk[t % 4]) >> 11) / 2.0 ** 53


def pin_inversion_exact(lib):
    from scipy.stats import poisson
    lams = [1e-3, 0.3, 1.0, 2.5, 6.0, 9.99]
    n = 300
    for lam in lams:
        k = oracle.poisson_counts(np.full(n, lam), SEED, lib=lib)
        for i in range(1, n):
            u = _uniform(i, 0)
            kk = 0
            while u > poisson.cdf(kk, lam):
                kk += 1
            if abs(u - poisson.cdf(kk, lam)) < 1e-13 or (kk > 0 and abs(u - poisson.cdf(kk - 1, lam)) < 1e-13):
                continue   # a tie within rounding of the CDF: either count is correct
            assert k[i] == kk, (lam, i, k[i], kk)


def _chi2_p(k, lam):
    from scipy.stats import chi2, poisson
    lo, hi = int(poisson.ppf(1e-5, lam)), int(poisson.ppf(1 - 1e-5, lam))
    edges = np.unique(np.linspace(lo, hi + 1, min(80, hi - lo + 2)).astype(np.int64))
    obs = np.histogram(k, bins=np.concatenate([[-1], edges, [np.iinfo(np.int64).max]]))[0]
    cdf = np.concatenate([[0.0], poisson.cdf(edges - 1, lam), [1.0]])
    exp = k.size * np.diff(cdf)
    keep = exp > 5
    stat = float(np.sum((obs[keep] - exp[keep]) ** 2 / exp[keep]))
    return float(chi2.sf(stat, keep.sum() - 1))


def pin_ptrs_distribution(lib):
    """Rejection sampling corrects most mistakes in its proposal only in
    part: a million draws just above the switch point resolve a shifted
    proposal (chi-square p ~ 1e-27) while the correct sampler passes."""
    for lam, n in ((10.0, 1000000), (12.0, 1000000), (37.5, 200000), (1000.0, 60000), (2.5e5, 60000)):
        k = oracle.poisson_counts(np.full(n, lam), SEED + 1, lib=lib)
        assert k.min() >= 0
        z_mean = (k.mean() - lam) / math.sqrt(lam / n)
        assert abs(z_mean) < 5, (lam, z_mean)
        assert abs(k.var() / lam - 1.0) < 5 * math.sqrt(2.0 / n) + 0.01, lam
        assert _chi2_p(k, lam) > 1e-4, lam
    assert not oracle.poisson_counts(np.zeros(100), SEED, lib=lib).any()


def pin_noise_scale_and_output(lib):
    rng = np.random.default_rng(9)
    tau = (rng.gamma(0.3, 2.0, (37, 41)) * (rng.uniform(size=(37, 41)) < 0.6)).astype(np.float32)
    for nr in (0.0, 2.0, 15.0, 25.0):
        mean, var, sn = oracle.noise_scale(tau, nr, lib=lib)
        t64 = tau.astype(np.float64)
        assert abs(mean - t64.mean()) <= 1e-14 * abs(t64.mean())
        assert abs(var - t64.var()) <= 1e-13 * t64.var()
        assert abs(sn - t64.var() / 10 ** (nr / 10)) <= 1e-13 * sn
    _, _, sn = oracle.noise_scale(tau, 2.0, lib=lib)
    big = np.tile(tau, (20, 20))
    out = oracle.poisson_noise(big, sn, SEED, lib=lib)
    cnt = out.astype(np.float64) * sn
    assert np.all(np.abs(cnt - np.round(cnt)) <= 1e-6 * np.maximum(1.0, cnt))
    lam = big.astype(np.float64) * sn
    z = (np.round(cnt).sum() - lam.sum()) / math.sqrt(lam.sum())
    assert abs(z) < 5, z
    assert not oracle.poisson_noise(big, 0.0, SEED, lib=lib).any()


NOISE_PINS = [pin_philox_vs_numpy, pin_exp_log_recipes, pin_inversion_exact, pin_ptrs_distribution,
              pin_noise_scale_and_output]
