"""Pins of the oracle's smooth forward and gradient (CPU)."""
import pytest

import pins_smooth


@pytest.mark.parametrize("pin", pins_smooth.SMOOTH_PINS, ids=[p.__name__ for p in pins_smooth.SMOOTH_PINS])
def test_smooth_pin(olib, pin):
    pin(olib)
