"""The FP64 oracle against closed forms, library routines, high-precision
brute force and invariants (no GPU)."""
import pytest

import pins


@pytest.mark.parametrize("pin", pins.FAST_PINS, ids=lambda f: f.__name__)
def test_pin(olib, pin):
    pin(olib)


def test_pin_mpmath_bruteforce(olib):
    pins.pin_mpmath_bruteforce(olib)


def test_pin_plane(olib):
    errs = pins.pin_plane(olib, sizes=(256, 1024))
    print(errs)


@pytest.mark.slow
def test_pin_plane_fine(olib):
    errs = pins.pin_plane(olib, sizes=(1024, 4096))
    for cos_on in (True, False):
        assert errs[(cos_on, 4096)][0] <= 3e-3, errs
