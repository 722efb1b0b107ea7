"""The oracle's pins, run on the built oracle (see tests/oracle_pins.py)."""
import pytest

import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(P.default_lib())
