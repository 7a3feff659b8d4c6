"""The oracle against facts outside itself (see pins.py)."""
import pytest

import oracle
import pins


@pytest.fixture(scope="module")
def O():
    return oracle.default()


@pytest.mark.parametrize("check", pins.ALL, ids=[c.__name__ for c in pins.ALL])
def test_pin(O, check):
    check(O)
