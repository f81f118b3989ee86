"""The readings of the pressure / velocity reconstruction (R1) against the
paper's Laplace test (Sec. III.A: static droplet in a periodic box of 5R,
density ratio 1000, M = 0.166, W = 4), on the NumPy twin of the CPU
reference: the committed evidence behind the choice of reading and behind
viscosity set 2 being reported as not reproduced.

* set 1 (air 1.67e-1, water 1.10e-2): the adopted reading keeps the droplet
  and builds the pressure jump sigma / R;
* set 2 (air 5.56e-3, water 3.67e-4): every reading weighed diverges within
  a few hundred steps, and so does the adopted reading with the
  density-weighted viscous term, the bulk term or the omega term of the
  pressure left out (diagnostic builds): no single term is the cause.
"""
import numpy as np
import pytest

from oracle import readings as RD
from oracle.twin import READINGS

pytestmark = pytest.mark.slow


def test_adopted_reading_holds_set1():
    div, dp, umax = RD.run(8.0, 1e-2, *RD.SETS[1], 1500, "pstar")
    assert div is None
    assert umax < 1e-4
    # the jump is still building after 1500 steps; within 10% of sigma / R
    assert 0.9 < dp < 1.1


@pytest.mark.parametrize("reading", READINGS)
def test_set2_diverges_under_every_reading(reading):
    div, _, _ = RD.run(8.0, 1e-2, *RD.SETS[2], 1000, reading)
    assert div is not None and div <= 1000


@pytest.mark.parametrize("terms", [("stress_density",), ("bulk",), ("omega",)])
def test_set2_divergence_is_not_one_term(terms):
    div, _, _ = RD.run(8.0, 1e-2, *RD.SETS[2], 1200, "pstar", terms)
    assert div is not None
