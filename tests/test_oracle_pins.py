"""The CPU oracle against its pins (see oracle_pins.py for what pins each part)."""
import pytest

import oracle
from tests import oracle_pins as P


@pytest.fixture(scope="module")
def lib():
    oracle.build()
    return oracle.load()


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(lib, pin):
    pin(lib)


def test_validate_codes(lib):
    import numpy as np
    from paper_2111_05651_amd import inputs
    m = inputs.make_mesh(2, jitter=True, seed=3)
    assert oracle.validate(m.npoin, m.lnods, m.coord, lib=lib) == (oracle.OR_OK, -1)
    bad = m.lnods.copy()
    bad[5, 2] = m.npoin
    assert oracle.validate(m.npoin, bad, m.coord, lib=lib) == (oracle.OR_ERANGE, 5)
    flat = m.coord.copy()
    flat[m.lnods[7]] = flat[m.lnods[7][0]]     # collapse element 7 to a point
    st, e = oracle.validate(m.npoin, m.lnods, flat, lib=lib)
    assert st == oracle.OR_EDEGENERATE and e <= 7
