"""Structural pin of the recursive Gaussian's coefficient recipe (Young and
van Vliet 1995, the spatial filter of the paper's experiments, Sec. 3), for
both independently typed copies: the oracle's and the library's host code.

The recipe builds the causal denominator A(z) = b0 - b1 z^-1 - b2 z^-2 - b3 z^-3
from one cubic P(s) = a + b s + c s^2 + d s^3 evaluated at the backward
difference s = q (1 - z^-1):
    b0 = P(q),  b1 = b q + 2 c q^2 + 3 d q^3,  b2 = -(c q^2 + 3 d q^3),
    b3 = d q^3,  and the DC gain B = 1 - (b1 + b2 + b3)/b0 = a / b0.
Writing the normalised denominator 1 - r1 z^-1 - r2 z^-2 - r3 z^-3 (r_k =
b_k/b0) in powers of w = 1 - z^-1 gives the coefficients
    E0 = 1 - r1 - r2 - r3,  E1 = r1 + 2 r2 + 3 r3,  E2 = -(r2 + 3 r3),  E3 = r3,
which must equal (a, b q, c q^2, d q^3) / P(q).  From the returned numbers
the test recovers q by solving E3 P(q) = d q^3 (q^3 / P(q) increases with q),
then checks P(q) E0 = a, P(q) E1 = b q and P(q) E2 = c q^2.  The published
constants are rounded to about six digits, so the identities hold to that
rounding: the residue is at most 1e-5 q^2 + 5e-6 q^3; a slip in any digit
above that rounding in b0, b1, b2 or b3 breaks one of the three checks (the
last test plants such slips in a copy of the recipe).

Parity unpinned: q(sigma) (the published two-branch fit) and P's own four
constants are typed from the cited paper in both copies and checked only by
the shape tests of test_oracle_yvv (Gaussian-like impulse response).
"""
import numpy as np
import pytest

import oracle
from paper_1105_4204_amd import _native as nat

# P(s) = a + b s + c s^2 + d s^3, the cubic the recipe starts from
A_, B_, C_, D_ = 1.57825, 2.44413, 1.4281, 0.422205

SIGMAS = [0.5, 0.8, 1.0, 1.7, 2.0, 2.4, 2.5, 3.0, 5.0, 7.5, 10.0, 16.0, 20.0, 32.0, 50.0, 64.0]


def _check_structure(coeffs, s):
    Bgain, r1, r2, r3 = coeffs
    E0 = 1.0 - r1 - r2 - r3
    E1 = r1 + 2.0 * r2 + 3.0 * r3
    E2 = -(r2 + 3.0 * r3)
    E3 = r3
    assert abs(Bgain - E0) <= 1e-12, (s, Bgain, E0)
    P = lambda x: A_ + B_ * x + C_ * x * x + D_ * x ** 3
    lo, hi = 0.0, 1e4            # bisection on q^3 / P(q) = E3 / d
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid ** 3 / P(mid) < E3 / D_:
            lo = mid
        else:
            hi = mid
    q = 0.5 * (lo + hi)
    b0 = P(q)
    tol = 1.5e-5 * (q * q + q ** 3) + 1e-11 * b0
    assert abs(E0 * b0 - A_) <= tol, ("b0 / gain structure", s, E0 * b0, A_)
    assert abs(E1 * b0 - B_ * q) <= tol, ("b1 structure", s, E1 * b0, B_ * q)
    assert abs(E2 * b0 - C_ * q * q) <= tol, ("b2 structure", s, E2 * b0, C_ * q * q)
    return q


@pytest.mark.parametrize("s", SIGMAS)
def test_oracle_recipe_is_backward_difference_cubic(s):
    _check_structure(oracle.yvv_coeffs(s), s)


@pytest.mark.parametrize("s", SIGMAS)
def test_library_recipe_is_backward_difference_cubic(s):
    q = _check_structure(nat.yvv_coeffs(s), s)
    # the two copies agree to rounding
    lib = np.array(nat.yvv_coeffs(s))
    orc = np.array(oracle.yvv_coeffs(s))
    assert np.max(np.abs(lib - orc)) <= 1e-13, (s, lib, orc)
    assert q > 0


def test_structure_check_catches_digit_slips():
    """The check itself, on the recipe typed here with one digit changed at a
    time (each constant of b1, b2, b3, b0 in turn): every slip fails at some
    sigma of the sweep."""
    def recipe(s, k):
        q = 0.98711 * s - 0.96330 if s >= 2.5 else 3.97156 - 4.14554 * np.sqrt(1 - 0.26891 * s)
        c = [1.57825, 2.44413, 1.4281, 0.422205, 2.44413, 2.85619, 1.26661, 1.4281, 1.26661,
             0.422205]
        if k is not None:
            c[k] += 2e-4 * (1 if k % 2 else -1)
        b0 = c[0] + c[1] * q + c[2] * q * q + c[3] * q ** 3
        b1 = c[4] * q + c[5] * q * q + c[6] * q ** 3
        b2 = -(c[7] * q * q + c[8] * q ** 3)
        b3 = c[9] * q ** 3
        return (1 - (b1 + b2 + b3) / b0, b1 / b0, b2 / b0, b3 / b0)

    for s in SIGMAS:
        _check_structure(recipe(s, None), s)
    for k in range(10):
        caught = False
        for s in SIGMAS:
            try:
                _check_structure(recipe(s, k), s)
            except AssertionError:
                caught = True
                break
        assert caught, k
