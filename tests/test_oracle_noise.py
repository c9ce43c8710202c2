"""Pins of the oracle's Poisson noise (CPU)."""
import pytest

import pins_noise


@pytest.mark.parametrize("pin", pins_noise.NOISE_PINS, ids=[p.__name__ for p in pins_noise.NOISE_PINS])
def test_noise_pin(olib, pin):
    pin(olib)
