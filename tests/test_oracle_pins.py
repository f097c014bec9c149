"""The CPU oracle pinned to closed forms, exact arithmetic and invariants."""
import pytest

import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    fails = pin()
    assert not fails, "\n".join(fails[:20])
