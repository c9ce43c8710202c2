"""Pins of the oracle's fp32 error model (CPU)."""
import pytest

import pins_error


@pytest.mark.parametrize("pin", pins_error.ERROR_PINS, ids=[p.__name__ for p in pins_error.ERROR_PINS])
def test_error_pin(olib, pin):
    pin(olib)
