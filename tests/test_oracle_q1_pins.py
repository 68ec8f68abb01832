"""The 2-D (bilinear quadrilateral) oracle against its pins (see oracle_q1_pins.py)."""
import numpy as np
import pytest

import oracle
from paper_2111_05651_amd import inputs
from tests import oracle_q1_pins as P


@pytest.fixture(scope="module")
def lib():
    oracle.build()
    return oracle.load()


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(lib, pin):
    pin(lib)


def test_q1_validate_codes(lib):
    m = inputs.make_quad_mesh(3, jitter=True, seed=3)
    assert oracle.q1_validate(m.npoin, m.lnods, m.coord, lib=lib) == (oracle.OR_OK, -1)
    bad = m.lnods.copy()
    bad[4, 1] = m.npoin
    assert oracle.q1_validate(m.npoin, bad, m.coord, lib=lib) == (oracle.OR_ERANGE, 4)
    bow = m.lnods.copy()
    bow[6] = bow[6][[0, 2, 1, 3]]          # a crossed ("bow-tie") quadrilateral
    st, e = oracle.q1_validate(m.npoin, bow, m.coord, lib=lib)
    assert st == oracle.OR_EDEGENERATE and e == 6
