"""Pins of the FFT-route oracle (CPU), and planted mistakes in a copy of it."""
import importlib.util
import os

import pytest

import pins_lct
from oracle import lct

SRC = lct.__file__


@pytest.mark.parametrize("pin", pins_lct.LCT_PINS, ids=[p.__name__ for p in pins_lct.LCT_PINS])
def test_lct_pin(pin):
    pin(lct)


LCT_MUTANTS = [
    ("no_fold_weight", "fine[J * J - 1, J - 1] = 1.0 / J", "fine[J * J - 1, J - 1] = 1.0"),
    ("sum_not_mean", "mtx = 0.5 * (mtx[0::2] + mtx[1::2])", "mtx = (mtx[0::2] + mtx[1::2])"),
    ("cone_not_truncated", "    cone[:, :, M:] = 0.0\n", ""),
    ("cone_slope_not_4", "(4.0 * slope) ** 2", "(2.0 * slope) ** 2"),
    ("cone_not_centred", "return np.roll(cone, shift=(-N, -N), axis=(0, 1))", "return cone"),
    ("depth_layer_round", "j = np.floor(np.where(present, D, 0.0) / dz)", "j = np.round(np.where(present, D, 0.0) / dz)"),
    ("no_v_scaling", "/ v ** 1.5", "/ v ** 0.5"),
    ("time_point_sampling", "R[j, c] = ov / (2 * j + 1)", "R[j, c] = float(c == (hi - 1) // M)"),
    ("jitter_sigma", "sigma = fwhm_ps / (2.0 * math.sqrt(2.0 * math.log(2.0))) / bin_ps",
     "sigma = fwhm_ps / math.sqrt(2.0 * math.log(2.0)) / bin_ps"),
    # constant-factor mistakes that every scale-free pin lets through
    ("v_scaling_times_2", "/ v ** 1.5", "/ (2.0 * v ** 1.5)"),
    ("time_bins_summed", "R[j, c] = ov / (2 * j + 1)", "R[j, c] = ov / (2 * j + 1) * 2.0"),
    ("v_unit_scaled", "v = (J * dz) ** 2", "v = (J * dz * 1.25) ** 2"),
    ("cone_scaled", "cone = (res == res.min(axis=2, keepdims=True)).astype(np.float64)",
     "cone = 0.5 * (res == res.min(axis=2, keepdims=True)).astype(np.float64)"),
]


@pytest.mark.parametrize("name,old,new", LCT_MUTANTS, ids=[m[0] for m in LCT_MUTANTS])
def test_lct_mutant_is_caught(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    path = tmp_path / "lct_mut.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"lct_mut_{name}", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    failures = []
    for pin in pins_lct.LCT_PINS:
        try:
            pin(mod)
        except Exception as e:  # noqa: BLE001 - any failure counts
            failures.append((pin.__name__, type(e).__name__))
            break               # one failing pin is enough
    assert failures, f"mutant {name} passed every LCT pin"
    print(name, "caught by", failures)
