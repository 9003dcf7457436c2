"""Pins of the prior table: the hand-evaluated default table, the k = 0
special case in closed form, and the shape of the energy."""
import math

import numpy as np
import pytest

from oracle import ref


def test_default_table_values():
    # gamma 3, sigma 1, beta 0.02: unrounded -14.384, -9.207, -2.206, -0.185,
    # -0.0056, ... (hand evaluation of the ELAS prior energy, shifted so that
    # far candidates cost 0)
    lut = ref.prior_lut(ref.params(disp_max=127))
    assert list(lut[:6]) == [-14, -9, -2, 0, 0, 0]
    assert np.all(lut[3:] == 0)
    assert len(lut) == 128


@pytest.mark.parametrize("gamma,beta", [(3.0, 0.02), (1.0, 0.05), (10.0, 0.001), (0.5, 0.1)])
def test_zero_offset_closed_form(gamma, beta):
    # at k = 0 exp(0) = 1, so the energy is -ln((gamma + 1) / gamma) / beta
    p = ref.params(gamma=gamma, beta=beta, disp_max=15)
    lut = ref.prior_lut(p)
    g, b = float(np.float32(gamma)), float(np.float32(beta))
    assert lut[0] == round(-math.log1p(1.0 / g) / b)


@pytest.mark.parametrize("sigma", [0.5, 1.0, 2.0, 4.0])
def test_shape_monotone_nonpositive_vanishing(sigma):
    lut = ref.prior_lut(ref.params(sigma=sigma, disp_max=255))
    assert np.all(np.diff(lut) >= 0)       # cost grows with distance from the plane
    assert np.all(lut <= 0)
    assert lut[-1] == 0                      # far from the plane: no preference
    # wider sigma keeps the bonus further out
    assert np.count_nonzero(lut) >= 1


def test_wider_sigma_reaches_further():
    a = ref.prior_lut(ref.params(sigma=1.0, disp_max=63))
    b = ref.prior_lut(ref.params(sigma=3.0, disp_max=63))
    assert np.count_nonzero(b) > np.count_nonzero(a)
    assert a[0] == b[0]                      # the k = 0 value does not depend on sigma
