"""The FP64 oracle against the paper's stated numbers, closed forms, textbook
routines and invariants (no GPU)."""
import pytest

import oracle
import pins


@pytest.fixture(scope="module")
def orc():
    return oracle._load()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(orc, pin):
    pin(orc)


def test_polar_rejects_bad_input(orc):
    import numpy as np
    with pytest.raises(ValueError):
        orc.polar(np.zeros((3, 5)))          # M < N
    with pytest.raises(FloatingPointError):
        orc.polar(np.zeros((4, 4)))          # ||A||_F = 0
    with pytest.raises(FloatingPointError):
        orc.polar(np.full((4, 4), np.nan))
    with pytest.raises(ValueError):
        orc.polar_2x2(np.array([[1.0, 2.0], [2.0, 4.0]]))   # singular
