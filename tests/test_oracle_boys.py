"""Pins of the oracle's Boys function (Eq. boys) against closed forms and library routines."""
import math

import numpy as np
import pytest
import scipy.special as sp

from oracle import oracle as O

XS = [0.0, 1e-12, 1e-6, 1e-3, 0.1, 0.5, 1.0, 2.5, 7.0, 15.0, 29.9, 36.0, 49.999, 50.0, 50.001, 80.0, 1e3, 1e6]


@pytest.mark.parametrize("m", range(0, 9))
def test_boys_vs_confluent_hypergeometric(m):
    # F_m(x) = 1F1(m+1/2; m+3/2; -x) / (2m+1), evaluated by mpmath at 40 digits
    import mpmath as mp
    mp.mp.dps = 40
    for x in XS:
        ref = float(mp.hyp1f1(mp.mpf(m) + 0.5, mp.mpf(m) + 1.5, -mp.mpf(x)) / (2 * m + 1))
        v = O.boys(m, x)
        assert abs(v - ref) <= 1e-15 * abs(ref), (m, x, v, ref)


@pytest.mark.parametrize("m", range(0, 9))
def test_boys_vs_incomplete_gamma(m):
    # F_m(x) = Gamma(m+1/2) P(m+1/2, x) / (2 x^{m+1/2})  for x > 0
    for x in XS[1:]:
        ref = math.gamma(m + 0.5) * sp.gammainc(m + 0.5, x) / (2.0 * x ** (m + 0.5))
        v = O.boys(m, x)
        assert abs(v - ref) <= 1e-13 * abs(ref), (m, x, v, ref)


def test_boys_f0_erf_closed_form():
    for x in XS[1:]:
        ref = 0.5 * math.sqrt(math.pi / x) * math.erf(math.sqrt(x))
        assert abs(O.boys(0, x) - ref) <= 2e-15 * ref


def test_boys_at_zero():
    for m in range(12):
        assert O.boys(m, 0.0) == pytest.approx(1.0 / (2 * m + 1), rel=1e-16, abs=0)


def test_boys_recurrence_identity():
    # (2m+1) F_m = 2x F_{m+1} + e^{-x}, from integrating Eq. boys by parts
    for m in range(8):
        for x in XS:
            lhs = (2 * m + 1) * O.boys(m, x)
            rhs = 2 * x * O.boys(m + 1, x) + math.exp(-x)
            assert abs(lhs - rhs) <= 4e-15 * abs(lhs)


def test_boys_quadrature_of_definition():
    # brute force: Gauss-Legendre on the defining integral (numpy nodes carry ~1e-14 error)
    y, wq = np.polynomial.legendre.leggauss(200)
    y = 0.5 * (y + 1.0)
    wq = 0.5 * wq
    for m in range(5):
        for x in [0.3, 4.0, 20.0, 45.0]:
            ref = float(np.sum(wq * y ** (2 * m) * np.exp(-x * y * y)))
            assert abs(O.boys(m, x) - ref) <= 5e-14 * ref
