"""Writes the closed-form fixtures under tests/golden/ (50-digit mpmath).

Nothing here calls the HIP library or the oracle: every value is the closed
form of the paper's definitions evaluated on the fp32-rounded inputs the
operator sees.  Sources:
  * arrival and weight of a single patch: Section 2, Eq. (1) -- the delta
    puts a patch at distance r into the bin of path 2r, weight rho/r^4 (times
    four Lambertian cosines when enabled);
  * stand-off legs: device at distance s on the wall normal through the grid
    centre, path (L - s) and weight (s/L)^3 per leg;
  * jitter taps: Section 2, sigma = FWHM / (2 sqrt(2 ln 2)), kernel length
    2 ceil(2 sigma) + 1, normalised.
Run: python tests/golden/make_golden.py
"""
import json
import os

import mpmath
import numpy as np

mpmath.mp.dps = 50
C = mpmath.mpf(299792458)
HERE = os.path.dirname(os.path.abspath(__file__))


def f32(x):
    return mpmath.mpf(float(np.float32(x)))


def bin_of(path_m, bin_ps):
    return int(mpmath.floor(path_m / (C * mpmath.mpf(bin_ps) * mpmath.mpf("1e-12"))))


def single_patch():
    out = {"source": "Section 2, Eq. (1): single patch closed forms", "normal_incidence": []}
    for z, bin_ps in ((0.5, 16.0), (0.5, 8.0), (0.8, 8.0), (0.45, 4.0)):
        zz = f32(z)
        out["normal_incidence"].append(dict(z=z, bin_ps=bin_ps, half=0.05, albedo=0.7,
                                            bin=bin_of(2 * zz, bin_ps),
                                            weight_over_a=float(1 / zz ** 4)))
    wx, wy, z = f32(-0.3), f32(-0.4), f32(0.5)
    r = mpmath.sqrt(wx ** 2 + wy ** 2 + z ** 2)
    out["oblique"] = dict(bin_ps=16.0, bin=bin_of(2 * r, 16.0),
                          weight_over_a_cos=float((z / r) ** 4 / r ** 4),
                          weight_over_a_nocos=float(1 / r ** 4))
    s = mpmath.mpf(1)
    L = mpmath.sqrt(mpmath.mpf("0.25") + mpmath.mpf("0.25") + s * s)
    out["standoff"] = dict(bin_ps=16.0, bin=bin_of(2 * f32(0.5) + 2 * (L - s), 16.0),
                           weight_factor=float((s / L) ** 6))
    return out


def jitter_taps():
    cases = []
    for fwhm, bin_ps in ((70.0, 16.0), (50.0, 8.0), (30.0, 4.0), (70.0, 32.0)):
        sigma = mpmath.mpf(fwhm) / (2 * mpmath.sqrt(2 * mpmath.log(2))) / mpmath.mpf(bin_ps)
        R = int(mpmath.ceil(2 * sigma))
        g = [mpmath.exp(-mpmath.mpf(j * j) / (2 * sigma ** 2)) for j in range(-R, R + 1)]
        cases.append(dict(fwhm_ps=fwhm, bin_ps=bin_ps, sigma_bins=float(sigma), R=R,
                          g0=float(g[R] / sum(g))))
    return {"source": "Section 2, temporal jitter: sigma = FWHM/(2 sqrt(2 ln 2)), k = 2 ceil(2 sigma)+1",
            "cases": cases}


if __name__ == "__main__":
    for name, obj in (("single_patch.json", single_patch()), ("jitter_taps.json", jitter_taps())):
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(obj, f, indent=1)
        print(name, json.dumps(obj)[:300])
