"""Pins of the oracle's Aitken stopping rule (Sec. 3.4, eqs. 24-26).

For a linearly convergent sequence l^(k) = L - c r^k, Aitken's extrapolation
is exact: l_inf = L at every step, so the gap |l_inf^(k+1) - l^(k+1)| equals
c r^(k+1) and the stopping iteration has a closed form."""
import math

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("L,c,r,tol", [(-1234.5, 10.0, 0.5, 1e-6), (10.0, 3.0, 0.9, 1e-3),
                                       (-5e4, 200.0, 0.2, 1e-6)])
def test_geometric_sequence_closed_form(L, c, r, tol):
    k = np.arange(200)
    trace = L - c * r ** k
    # first index i >= 2 with c r^i < tol; the fit has then run i + 1 E-steps
    i = max(2, math.floor(math.log(tol / c) / math.log(r)) + 1)
    assert i < 190
    while c * r ** i >= tol:
        i += 1
    while i > 2 and c * r ** (i - 1) < tol:
        i -= 1
    assert oracle.aitken_iterations(trace, tol) == i + 1


def test_aitken_extrapolation_is_exact_on_geometric():
    # the value the rule compares against: l_inf of eq. (25) equals the limit
    L, c, r = 7.0, 2.0, 0.6
    l = [L - c * r ** k for k in range(3)]
    a = (l[2] - l[1]) / (l[1] - l[0])
    assert abs(a - r) < 1e-12
    linf = l[1] + (l[2] - l[1]) / (1 - a)
    assert abs(linf - L) < 1e-12


def test_special_cases():
    assert oracle.aitken_iterations([1.0, 1.0, 2.0], 1e-6) == 2          # unchanged value stops
    assert oracle.aitken_iterations([1.0, float("nan"), 2.0], 1e-6) == 2  # non-finite stops
    assert oracle.aitken_iterations([0.0, 1.0, 2.0, 3.0, 4.0], 1e-6) == 5  # a = 1: never
    assert oracle.aitken_iterations([0.0, 1.0, 1.5, 1.75], 0.0) == 4       # tol 0: all
    # l^(k) = l^(k-1) is caught by the unchanged rule first
    assert oracle.aitken_iterations([3.0, 2.0, 2.0], 1.0) == 3
    # increasing, slowing: stops once the extrapolated gap is small
    trace = [-100.0, -50.0, -25.0, -12.5, -6.25]
    # (a geometric sequence, L = 0, c = 100, r = 1/2: the gap at index k is 100 / 2^k)
    assert oracle.aitken_iterations(trace, 13.0) == 4
    assert oracle.aitken_iterations(trace, 7.0) == 5
    assert oracle.aitken_iterations(trace, 6.0) == 5
