"""The oracle against brute force, the paper's worked example, closed forms and invariants."""
import pytest

import oracle
from tests import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(pin):
    oracle.use_library(None)
    pin(oracle)
