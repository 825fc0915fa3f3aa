"""Pins of the oracle's recursive Gaussian spatial kernel (the two-pass
recursive filter of Young and van Vliet, 1995, which the paper's experiments
use for the spatial averaging, Sec. 3) and of the direct filter with an
explicit separable kernel.

 - the impulse response of the two passes has the closed-form transfer
   function B^2 / |A(e^{jw})|^2, A(z) = 1 - a1 z^-1 - a2 z^-2 - a3 z^-3, at
   every frequency (a wrong tap, sign or direction in either pass breaks it);
 - unit DC gain, symmetry, positivity and a Gaussian shape: the response stays
   within 10% of a sampled Gaussian of the requested sigma (the published
   filter is an approximation; 6% from sigma = 2 on), with a standard
   deviation between sigma and 1.25 sigma (its tails are exponential);
 - the direct filter with an explicit kernel reduces to the pinned box
   filter for box taps, and equals the O(1) method, eq. (final-form) with
   library correlations of the auxiliary images, for the recursive kernel.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_1105_4204_amd import synth

SIGMAS = [0.5, 1.0, 2.0, 3.0, 5.0, 10.0, 20.0]


@pytest.mark.parametrize("s", SIGMAS)
def test_impulse_response_has_closed_form_transfer_function(s):
    B, a1, a2, a3 = oracle.yvv_coeffs(s)
    D = int(40 * s) + 100
    k = oracle.yvv_kernel(s, D)
    d = np.arange(-D, D + 1)
    for w in np.linspace(0.0, math.pi, 17):
        K = float(np.sum(k * np.cos(w * d)))
        z = np.exp(-1j * w)
        ref = B * B / abs(1.0 - a1 * z - a2 * z ** 2 - a3 * z ** 3) ** 2
        assert abs(K - ref) <= 1e-10, (s, w, K, ref)


@pytest.mark.parametrize("s", SIGMAS)
def test_impulse_response_is_gaussian_like(s):
    D = int(40 * s) + 100
    k = oracle.yvv_kernel(s, D)
    d = np.arange(-D, D + 1, dtype=np.float64)
    assert abs(k.sum() - 1.0) < 1e-9
    assert np.max(np.abs(k - k[::-1])) < 1e-15
    core = k[np.abs(d) <= 10 * s]                 # beyond, the tail is at rounding level
    assert np.all(core > 0.0)
    # decreasing away from the centre over the bulk (the complex pole pair
    # leaves a small ripple in the far tail at large sigma)
    bulk = k[D:D + int(3 * s) + 2]
    assert np.all(np.diff(bulk) < 0.0)
    g = np.exp(-d * d / (2 * s * s))
    g /= g.sum()
    assert np.max(np.abs(k - g)) < 0.10 * g.max(), s
    if s >= 2.0:
        assert np.max(np.abs(k - g)) < 0.06 * g.max(), s
    # the exponential tails carry more second moment than a Gaussian's
    sd = math.sqrt(float(np.sum(k * d * d)))
    assert s <= sd <= 1.25 * s


def test_coefficients_reject_small_sigma():
    with pytest.raises(ValueError):
        oracle.yvv_coeffs(0.4)


def test_explicit_kernel_with_box_taps_is_box_filter():
    f = synth.piecewise_smooth(21, 17, seed=5, n_shapes=3).astype(np.float64)
    k = np.ones(2 * 3 + 1)
    got = oracle.forward_kernel(f, 25.0, 43, k)
    ref = oracle.forward(f, 25.0, 43, [3])
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-11)
    idx = np.array([0, 5, 100, 356])
    np.testing.assert_allclose(oracle.forward_kernel(f, 25.0, 43, k, idx=idx),
                               ref.reshape(-1)[idx], rtol=1e-13, atol=1e-11)


@pytest.mark.parametrize("shape,sigma_r,N,s", [((19, 23), 30.0, 30, 2.0), ((14, 16), 25.0, 43, 3.5)])
def test_direct_equals_final_form_with_recursive_kernel(shape, sigma_r, N, s):
    f = synth.piecewise_smooth(*shape, seed=31, n_shapes=3).astype(np.float64)
    D = max(shape)
    k = oracle.yvv_kernel(s, D)
    k2 = np.outer(k, k)
    alpha = 1.0 / (sigma_r * math.sqrt(N))
    num = np.zeros(shape, dtype=np.complex128)
    den = np.zeros(shape, dtype=np.complex128)

    def corr(u):
        return (ndimage.correlate(u.real, k2, mode="constant")
                + 1j * ndimage.correlate(u.imag, k2, mode="constant"))

    for n in range(N + 1):
        c = math.comb(N, n) / 2.0 ** N
        w = (2 * n - N) * alpha
        h = np.exp(1j * w * f)
        d = c * np.exp(-1j * w * f)
        num += d * corr(f * h)
        den += d * corr(h)
    got, eta = oracle.forward_kernel(f, sigma_r, N, k, return_eta=True)
    np.testing.assert_allclose(got, (num / den).real, rtol=1e-9, atol=1e-8)
    np.testing.assert_allclose(eta, den.real, rtol=1e-9, atol=1e-14)
