"""Pins of the oracle's range kernel, degree rule and spatial kernel.

Each test checks the oracle against something fixed by the paper or by
mathematics, never against a retyped copy of its own formula:
 - Table 1's estimate row (stored in tests/golden, cited there);
 - the binomial expansion of cos^N (Sec. 2.3), computed here from math.comb;
 - the Gaussian limit eq. (convergence)/(convergence1) and its leading
   Taylor correction (Sec. 2.4 proof);
 - the degree bound of Sec. 2.5 (sign change exactly at the bound);
 - the discrete-uniform variance of iterated boxes and numpy.convolve.
"""
import math
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _binomial_phi(s, N, sigma_r):
    """Sec. 2.3: cos^N(t) = sum_n 2^-N C(N,n) exp(j(2n-N)t), real part."""
    alpha = 1.0 / (sigma_r * math.sqrt(N))
    s = np.asarray(s, dtype=np.float64)
    acc = np.zeros_like(s)
    for n in range(N + 1):
        acc += math.comb(N, n) * np.cos((2 * n - N) * alpha * s)
    return acc / 2.0 ** N


def test_table1_estimate_row():
    rows = np.loadtxt(os.path.join(GOLD, "table1_degree_estimate.txt"))
    for sigma, est in rows:
        assert oracle.range_degree(255.0, sigma) == int(est)


def test_degree_rule_other_T():
    # gamma sigma = 1 exactly -> N = 1; just below -> 2
    T = 100.0
    s1 = 2 * T / math.pi
    assert oracle.range_degree(T, s1 * 1.0000001) == 1
    assert oracle.range_degree(T, s1 * 0.99) == 2
    with pytest.raises(ValueError):
        oracle.range_degree(0.0, 10.0)


@pytest.mark.parametrize("N,sigma_r", [(1, 200.0), (2, 150.0), (5, 80.0), (30, 30.0),
                                       (31, 29.0), (66, 20.0), (264, 10.0)])
def test_binomial_identity(N, sigma_r):
    s = np.linspace(-255.0, 255.0, 2001)
    got = oracle.phi(s, N, sigma_r)
    ref = _binomial_phi(s, N, sigma_r)
    assert np.max(np.abs(got - ref)) <= 1e-13


def test_single_cosine_case():
    # N = 1 is the plain cosine kernel of eq. (cosine) with gamma -> 1/sigma_r
    s = np.linspace(-255, 255, 101)
    np.testing.assert_allclose(oracle.phi(s, 1, 300.0), np.cos(s / 300.0), rtol=0, atol=1e-15)


def test_zero_degree_is_constant():
    assert oracle.phi(123.0, 0, 10.0) == 1.0


@pytest.mark.parametrize("sigma_r", [10.0, 25.0, 60.0])
def test_gaussian_limit_leading_correction(sigma_r):
    """N (G - phi_N) -> G (s/sigma)^4 / 12 (log cos x = -x^2/2 - x^4/12 - ...)."""
    s = np.linspace(-3 * sigma_r, 3 * sigma_r, 61)
    G = np.exp(-s ** 2 / (2 * sigma_r ** 2))
    lead = G * (s / sigma_r) ** 4 / 12.0
    prev = None
    for N in (1_000, 10_000, 100_000):
        dev = N * (G - oracle.phi(s, N, sigma_r)) - lead
        err = np.max(np.abs(dev))
        # next Taylor order is O(1/N); rounding of cos^N contributes ~N^2 eps
        assert err < 50.0 / N + 1e-14 * N * N
        if prev is not None:
            assert err < prev  # converges
        prev = err


def test_gaussian_limit_bound_at_practical_N():
    """0 <= G - phi_N <= 0.2/N on [-255,255] once N meets the degree bound."""
    sigma_r = 25.0
    s = np.linspace(-255, 255, 5101)
    G = np.exp(-s ** 2 / (2 * sigma_r ** 2))
    for N in (oracle.range_degree(255.0, sigma_r), 100, 1000):
        d = G - oracle.phi(s, N, sigma_r)
        assert d.min() >= -1e-15
        assert d.max() <= 0.2 / N


@pytest.mark.parametrize("sigma_r", [10.0, 20.0, 30.0, 47.0])
def test_degree_bound_sign_change(sigma_r):
    """Sec. 2.5: N >= (gamma sigma)^-2 keeps alpha*T <= pi/2 (phi >= 0,
    monotone on [0, T]); with fewer terms alpha*T > pi/2."""
    T = 255.0
    N = oracle.range_degree(T, sigma_r)
    s = np.linspace(0.0, T, 4001)
    ph = oracle.phi(s, N, sigma_r)
    assert ph.min() >= 0.0
    assert np.all(np.diff(ph) <= 1e-300)
    # one fewer term: the cosine argument passes pi/2 before s = T
    Nm = N - 1
    if Nm >= 1:
        c = math.cos(T / (sigma_r * math.sqrt(Nm)))
        assert c < 0
        ph_m = oracle.phi(np.array([T]), Nm, sigma_r)[0]
        if Nm % 2 == 1:   # odd power of a negative cosine (may underflow to -0.0)
            assert math.copysign(1.0, ph_m) < 0


def test_exact_bound_zero_at_T():
    # sigma_r chosen so that (2T/(pi sigma_r))^2 = N exactly: phi(T) ~ cos(pi/2)^N
    T, N = 255.0, 16
    sigma_r = 2 * T / (math.pi * math.sqrt(N))
    assert abs(oracle.phi(T, N, sigma_r)) < 1e-200
    assert oracle.phi(0.0, N, sigma_r) == 1.0


@pytest.mark.parametrize("radii", [[0], [1], [5], [2, 3], [9, 9, 10], [5, 5, 6], [29, 29, 30], [1, 0, 2, 4]])
def test_spatial_kernel(radii):
    k = oracle.spatial_kernel(radii)
    ref = np.array([1.0])
    for r in radii:
        ref = np.convolve(ref, np.ones(2 * r + 1))
    assert k.shape == ref.shape
    np.testing.assert_array_equal(k, ref)
    assert k.sum() == np.prod([2 * r + 1 for r in radii])
    t = np.arange(k.size) - (k.size - 1) / 2
    var = float((k * t * t).sum() / k.sum())
    assert abs(var - sum(((2 * r + 1) ** 2 - 1) / 12.0 for r in radii)) < 1e-9
    np.testing.assert_array_equal(k, k[::-1])
