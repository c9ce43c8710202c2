"""The pins have teeth: plant one plausible mistake at a time in a copy of
the oracle's source (CPU only), rebuild it, and check that at least one pin
fails on the broken copy."""
import os

import pytest

import oracle
import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "nlos_oracle.c")

# (name, text in the oracle source, planted replacement)
MUTANTS = [
    ("drop_patch_cosine", "cw_l * cp_l * cp_d * cw_d", "cw_l * cp_l * cw_d"),
    ("drop_wall_cosine", "cw_l * cp_l * cp_d * cw_d", "cp_l * cp_d * cw_d"),
    ("inverse_square_to_inverse", "(r_l * r_l * r_d * r_d)", "(r_l * r_d)"),
    ("normal_faces_away", "o[6] = -1.0 / len;", "o[6] = 1.0 / len;"),
    ("normal_x_sign", "o[4] = gx / len;", "o[4] = -gx / len;"),
    ("no_cosine_clamp", "if (cp_l < 0.0) cp_l = 0.0;", ""),
    ("round_not_floor", "floor(u)", "floor(u + 0.5)"),
    ("single_leg_path", "((r_l + r_d) + o) * inv", "((r_d + r_d) + o) * inv"),
    ("drop_standoff_path", "const double o = o_l + o_d;", "const double o = 0.0;"),
    ("drop_standoff_weight", "H[k] += w * g_l * g_d;", "H[k] += w;"),
    ("standoff_weight_square", "*weight = (s / L) * (s / L) * (s / L);", "*weight = (s / L) * (s / L);"),
    ("taps_unnormalised", "taps[j] /= sum;", "taps[j] /= 1.0;"),
    ("fwhm_without_factor_2", "fwhm_ps / (2.0 * sqrt(2.0 * log(2.0)))", "fwhm_ps / sqrt(2.0 * log(2.0))"),
    ("radius_ceil_sigma", "(int32_t)ceil(2.0 * sigma)", "(int32_t)ceil(sigma)"),
    ("projected_area_with_cosines", "(cosines ? len : 1.0)", "1.0"),
    ("grid_not_cell_centred", "((double)i + 0.5) * step", "((double)i) * step"),
    ("scan_xy_swapped", "const double wdx = rx[d / rg->ny], wdy = rx[rg->nx + d % rg->ny];",
     "const double wdx = rx[d % rg->ny], wdy = rx[rg->nx + d / rg->ny];"),
    ("jitter_wraps_around", "if (src >= 0 && src < T) acc += taps[j + R] * H[src];",
     "acc += taps[j + R] * H[(src + T) % T];"),
    ("gate_at_zero", "*offset = L - s;", "*offset = L;"),
    ("half_central_difference", "/ (2.0 * h);", "/ h;"),
]


# planted mistakes in the smooth forward and its gradient, checked against
# the smooth pins
SMOOTH_MUTANTS = [
    ("smooth_unnormalised", "/ (sigma * sqrt(2.0 * ORACLE_PI))", ""),
    ("smooth_no_half_offset", "((double)k + 0.5) - u", "((double)k) - u"),
    ("smooth_support_2_sigma", "ceil(6.0 * smooth_sigma", "ceil(2.0 * smooth_sigma"),
    ("smooth_sigma_fwhm", "return fwhm_ps / (2.0 * sqrt(2.0 * log(2.0))) / bin_ps;", "return fwhm_ps / bin_ps;"),
    ("grad_arrival_sign", "gpz += G0 * dw_dpz + w * G1 * du_dpz;", "gpz += G0 * dw_dpz - w * G1 * du_dpz;"),
    ("grad_drop_arrival", "gpz += G0 * dw_dpz + w * G1 * du_dpz;", "gpz += G0 * dw_dpz;"),
    ("grad_one_leg_arrival", "*du_dpz = inv * (pz / r_l + pz / r_d);", "*du_dpz = inv * (pz / r_l);"),
    ("grad_drop_normal_projection", "const double dL_dgx = o8[4] / len - dot * gx / l3",
     "const double dL_dgx = o8[4] / len"),
    ("grad_drop_area_term", "+ o8[3] * rho * hx * hy * gy / len;", ";"),
    ("grad_border_stencil", "if (ix == 0) { grad_depth[idx + ny] += dL_dgx / hx; grad_depth[idx] -= dL_dgx / hx; }",
     "if (ix == 0) { grad_depth[idx + ny] += dL_dgx / (2.0 * hx); grad_depth[idx] -= dL_dgx / (2.0 * hx); }"),
    ("grad_albedo_projected_area", "grad_albedo[idx] = o8[3] * hx * hy * (prm->cosines ? len : 1.0);",
     "grad_albedo[idx] = o8[3] * hx * hy;"),
    ("grad_drop_patch_cosine_depth", "- pz * pz * q[6] * c_d - pz * pz * c_l * q[6]", ""),
    ("grad_normal_sign", "dw_dn[0] = q[3] * gg * k * (-alx * c_d - adx * c_l);",
     "dw_dn[0] = q[3] * gg * k * (alx * c_d - adx * c_l);"),
    ("grad_inverse_square_power", "- F * (4.0 * pz / rl2 + 4.0 * pz / rd2);", "- F * (2.0 * pz / rl2 + 2.0 * pz / rd2);"),
]


def _run_smooth_pins(lib):
    import pins_smooth
    failures = []
    for pin in pins_smooth.SMOOTH_PINS:
        try:
            pin(lib)
        except Exception as e:  # noqa: BLE001 - any failure counts
            failures.append((pin.__name__, type(e).__name__))
    return failures


@pytest.mark.parametrize("name,old,new", SMOOTH_MUTANTS, ids=[m[0] for m in SMOOTH_MUTANTS])
def test_smooth_mutant_is_caught(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    path = str(tmp_path / "mut.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    so = str(tmp_path / "libmut.so")
    oracle.compile_library(path, so)
    failures = _run_smooth_pins(oracle.load(so))
    assert failures, f"mutant {name} passed every smooth pin"
    print(name, "caught by", failures)


NOISE_MUTANTS = [
    ("philox_multiplier", "0xD2E7470EE14C6C93ull", "0xD2E7470EE14C6C95ull"),
    ("philox_weyl", "k1 += 0xBB67AE8584CAA73Bull;", "k1 += 0xBB67AE8584CAA73Dull;"),
    ("uniform_word", "return (double)(o[t % 4] >> 11)", "return (double)(o[(t + 1) % 4] >> 11)"),
    ("inversion_off_by_one", "while (u > F && k < 1000) {", "while (u >= F - 1e-3 && k < 1000) {"),
    ("ptrs_shift", "* U + lam + 0.43);", "* U + lam + 0.93);"),
    ("ptrs_squeeze_only", "if (lhs <= rhs) return (int64_t)kd;", "return (int64_t)kd;"),
    ("exp_short_series", "for (int k = 1; k <= 13; ++k) {", "for (int k = 1; k <= 5; ++k) {"),
    ("logfact_no_half_log", "+ 0.5 * oracle_nx_log(2.0 * ORACLE_PI * k)", "+ oracle_nx_log(2.0 * ORACLE_PI * k)"),
    ("variance_sample", "const double var = n > 0 ? v / (double)n : 0.0;",
     "const double var = n > 1 ? v / (double)(n - 1) : 0.0;"),
    ("noise_db_scale", "out[2] = var / pow(10.0, nr_db / 10.0);", "out[2] = var / pow(10.0, nr_db / 20.0);"),
]


def _run_noise_pins(lib):
    import pins_noise
    failures = []
    for pin in pins_noise.NOISE_PINS:
        try:
            pin(lib)
        except Exception as e:  # noqa: BLE001 - any failure counts
            failures.append((pin.__name__, type(e).__name__))
    return failures


@pytest.mark.parametrize("name,old,new", NOISE_MUTANTS, ids=[m[0] for m in NOISE_MUTANTS])
def test_noise_mutant_is_caught(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    path = str(tmp_path / "mut.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    so = str(tmp_path / "libmut.so")
    oracle.compile_library(path, so)
    failures = _run_noise_pins(oracle.load(so))
    assert failures, f"mutant {name} passed every noise pin"
    print(name, "caught by", failures)


# planted mistakes in the fp32 error model (the GPU tests' tolerance),
# checked against its own pins
ERROR_MUTANTS = [
    ("error_drop_cross_term", "K * (dc_l * c_d + c_l * dc_d + dc_l * dc_d)", "K * (dc_l * c_d + c_l * dc_d)"),
    ("error_one_leg", "K * (dc_l * c_d + c_l * dc_d + dc_l * dc_d)", "K * (dc_l * c_d)"),
    ("error_dc_over_r2", "fabs(q[6] * pz)) / r_l;", "fabs(q[6] * pz)) / (r_l * r_l);"),
    ("error_dc_signed_terms",
     "e1 * (fabs(q[4]) * (fabs(px) + fabs(wdx)) + fabs(q[5]) * (fabs(py) + fabs(wdy)) + fabs(q[6] * pz))",
     "e1 * fabs(q[4] * adx + q[5] * ady + q[6] * pz)"),
    ("error_drop_e0", "e = e0 * (K * c_l * c_d) + K *", "e = K *"),
    ("error_count_all_pairs", "if (!(kf >= 0.0 && kf < (double)T)) continue;\n            const int32_t k = (int32_t)kf;",
     "const int32_t k = kf < 0.0 ? 0 : (kf >= (double)T ? T - 1 : (int32_t)kf);"),
]


def _run_error_pins(lib):
    import pins_error
    failures = []
    for pin in pins_error.ERROR_PINS:
        try:
            pin(lib)
        except Exception as e:  # noqa: BLE001 - any failure counts
            failures.append((pin.__name__, type(e).__name__))
    return failures


@pytest.mark.parametrize("name,old,new", ERROR_MUTANTS, ids=[m[0] for m in ERROR_MUTANTS])
def test_error_mutant_is_caught(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    path = str(tmp_path / "mut.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    so = str(tmp_path / "libmut.so")
    oracle.compile_library(path, so)
    failures = _run_error_pins(oracle.load(so))
    assert failures, f"mutant {name} passed every error-model pin"
    print(name, "caught by", failures)


def _run_pins(lib):
    failures = []
    for pin in pins.FAST_PINS:
        try:
            pin(lib)
        except Exception as e:  # noqa: BLE001 - any failure counts
            failures.append((pin.__name__, type(e).__name__))
    try:
        pins.pin_mpmath_bruteforce(lib, seeds=(101, 102), nonconfocal=True)
    except Exception as e:  # noqa: BLE001
        failures.append(("pin_mpmath_bruteforce", type(e).__name__))
    return failures


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    bad = src.replace(old, new)
    path = str(tmp_path / "mut.c")
    with open(path, "w") as f:
        f.write(bad)
    so = str(tmp_path / "libmut.so")
    oracle.compile_library(path, so)
    lib = oracle.load(so)
    failures = _run_pins(lib)
    assert failures, f"mutant {name} passed every pin"
    print(name, "caught by", failures)


def test_unmutated_passes_all(olib):
    assert _run_pins(olib) == []
