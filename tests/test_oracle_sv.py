"""Pins of the oracle's space-variant filter (Sec. 4, space-variant extension):
a unit box of half-width r(x) around each pixel, fixed raised-cosine range
kernel.

 - a constant radius map reduces to the (separately pinned) fixed single-box
   filter, and a map made of two radii picks each pixel from the two
   fixed-radius results;
 - N = 0 reduces to the clipped box mean, checked against
   scipy.ndimage.uniform_filter ratios (a library routine);
 - eq. (final-form) with the binomial expansion of Sec. 2.3, evaluated with
   box sums read from summed-area tables (numpy cumsum), equals the direct
   sum: the method is exact for any kernel whose averages it can form;
 - radius 0 is the identity, constants are preserved, and out(x) depends on
   f only inside its own box.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_1105_4204_amd import synth


def _rmap(shape, seed, rmax):
    return np.random.default_rng(seed).integers(0, rmax + 1, size=shape).astype(np.int32)


@pytest.mark.parametrize("shape,r", [((11, 13), 0), ((11, 13), 2), ((7, 20), 5), ((5, 4), 9)])
def test_constant_radius_is_fixed_box(shape, r):
    f = synth.piecewise_smooth(*shape, seed=4, n_shapes=2).astype(np.float64)
    got = oracle.forward_sv(f, 25.0, 43, np.full(shape, r, np.int32))
    ref = oracle.forward(f, 25.0, 43, [r])
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-11)


def test_two_radius_map_selects_per_pixel():
    shape = (16, 19)
    f = synth.piecewise_smooth(*shape, seed=9, n_shapes=3).astype(np.float64)
    mask = np.random.default_rng(1).random(shape) < 0.5
    rmap = np.where(mask, 1, 4).astype(np.int32)
    got = oracle.forward_sv(f, 20.0, 66, rmap)
    ref = np.where(mask, oracle.forward(f, 20.0, 66, [1]), oracle.forward(f, 20.0, 66, [4]))
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-11)


@pytest.mark.parametrize("shape,rmax", [((13, 17), 3), ((1, 25), 6), ((20, 2), 4)])
def test_zero_degree_is_clipped_box_mean(shape, rmax):
    rng = np.random.default_rng(5)
    f = rng.uniform(0, 255, size=shape)
    rmap = _rmap(shape, 6, rmax)
    got = oracle.forward_sv(f, 10.0, 0, rmap)
    ref = np.empty_like(f)
    for r in range(rmax + 1):
        w = 2 * r + 1
        mean = (ndimage.uniform_filter(f, w, mode="constant")
                / ndimage.uniform_filter(np.ones_like(f), w, mode="constant"))
        ref[rmap == r] = mean[rmap == r]
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-10)


def _sat_box(u, rmap):
    """Box sums of half-width rmap[x] around each x, zero outside the image,
    from a summed-area table S[a, b] = sum of u[:a, :b]."""
    H, W = u.shape
    S = np.zeros((H + 1, W + 1), dtype=u.dtype)
    S[1:, 1:] = np.cumsum(np.cumsum(u, axis=0), axis=1)
    i, j = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    i0 = np.clip(i - rmap, 0, H)
    i1 = np.clip(i + rmap + 1, 0, H)
    j0 = np.clip(j - rmap, 0, W)
    j1 = np.clip(j + rmap + 1, 0, W)
    return S[i1, j1] - S[i0, j1] - S[i1, j0] + S[i0, j0]


@pytest.mark.parametrize("shape,sigma_r,N,rmax", [
    ((17, 23), 30.0, 30, 4),
    ((14, 12), 25.0, 43, 6),
    ((9, 15), 12.0, 181, 3),
])
def test_direct_equals_final_form_with_summed_area_tables(shape, sigma_r, N, rmax):
    f = synth.piecewise_smooth(*shape, seed=12, n_shapes=3).astype(np.float64)
    rmap = _rmap(shape, 13, rmax)
    alpha = 1.0 / (sigma_r * math.sqrt(N))
    num = np.zeros(shape, dtype=np.complex128)
    den = np.zeros(shape, dtype=np.complex128)
    for n in range(N + 1):
        c = math.comb(N, n) / 2.0 ** N
        w = (2 * n - N) * alpha
        h = np.exp(1j * w * f)
        d = c * np.exp(-1j * w * f)
        num += d * _sat_box(f * h, rmap)
        den += d * _sat_box(h, rmap)
    got, eta = oracle.forward_sv(f, sigma_r, N, rmap, return_eta=True)
    np.testing.assert_allclose(got, (num / den).real, rtol=1e-9, atol=1e-8)
    np.testing.assert_allclose(eta, den.real, rtol=1e-9, atol=1e-12)


def test_identity_constant_and_locality():
    shape = (12, 14)
    f = synth.piecewise_smooth(*shape, seed=21, n_shapes=3).astype(np.float64)
    assert np.array_equal(oracle.forward_sv(f, 20.0, 66, np.zeros(shape, np.int32)), f)
    c = np.full(shape, 97.25)
    np.testing.assert_allclose(oracle.forward_sv(c, 20.0, 66, _rmap(shape, 2, 5)), c,
                               rtol=1e-14)
    rmap = _rmap(shape, 3, 3)
    base = oracle.forward_sv(f, 20.0, 66, rmap)
    i, j = 6, 7
    r = int(rmap[i, j])
    g = f.copy()
    g[i, min(j + r + 1, shape[1] - 1)] += 50.0   # just outside the box of (i, j)
    g[min(i + r + 1, shape[0] - 1), j] += 50.0
    if j + r + 1 < shape[1] and i + r + 1 < shape[0]:
        assert oracle.forward_sv(g, 20.0, 66, rmap)[i, j] == base[i, j]
    g = f.copy()
    g[i, j + min(r, 1)] += 50.0                  # inside it
    if r > 0:
        assert oracle.forward_sv(g, 20.0, 66, rmap)[i, j] != base[i, j]


def test_rejects_negative_radius():
    f = np.zeros((3, 3))
    r = np.zeros((3, 3), np.int32)
    r[1, 1] = -1
    with pytest.raises(ValueError):
        oracle.forward_sv(f, 20.0, 4, r)
