"""The oracle against facts fixed outside it (see oracle_pins.py for the list)."""
import pytest

import oracle as O
from oracle_pins import PINS


@pytest.fixture(scope="module")
def lib():
    O.build()
    return O.load()


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(lib, pin):
    pin(lib)
