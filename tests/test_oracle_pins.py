"""The oracle against its pins (CPU only)."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle_pins as pins  # noqa: E402


@pytest.mark.parametrize("name,check", pins.ALL_PINS, ids=[n for n, _ in pins.ALL_PINS])
def test_pin(orc, name, check):
    check(orc)


def test_edt_exhaustive_4x5(orc):
    """All 2^20 masks of a 4x5 frame against brute force."""
    pins.pin_edt_exhaustive(orc, 4, 5)


def test_edt_exhaustive_5x3(orc):
    pins.pin_edt_exhaustive(orc, 5, 3)
