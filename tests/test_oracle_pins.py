"""The CPU oracle against its pins (see tests/pins.py for what each checks)."""
import pytest

import oracle
import pins


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(None)
