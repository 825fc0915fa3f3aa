"""Pins of the oracle's gradient dL/df.

 - central finite differences of the oracle's own forward (a different code
   path: only the filter definition, no derivative), at two step sizes;
 - the dot-product test <J v, u> = <v, J^T u> with J v from finite
   differences along a random direction;
 - on a constant image phi' vanishes at 0 and the gradient is the adjoint of
   the normalised spatial filter, checked with scipy.ndimage.correlate.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_1105_4204_amd import synth


@pytest.mark.parametrize("shape,sigma_r,N,radii", [
    ((9, 11), 30.0, 30, [2]),
    ((10, 8), 25.0, 43, [1, 1, 2]),
    ((7, 12), 20.0, 66, [1, 2]),
    ((1, 15), 60.0, 8, [3]),
])
def test_grad_vs_finite_differences(shape, sigma_r, N, radii):
    f = synth.salt(*shape, seed=7).astype(np.float64)
    rng = np.random.default_rng(1)
    G = rng.normal(size=shape)
    g = oracle.grad(f, sigma_r, N, radii, G)
    fd = np.zeros_like(f)
    fd2 = np.zeros_like(f)
    for p in range(f.size):
        for h, dst in ((1e-3, fd), (5e-4, fd2)):
            fp = f.copy(); fp.reshape(-1)[p] += h
            fm = f.copy(); fm.reshape(-1)[p] -= h
            dst.reshape(-1)[p] = np.sum(G * (oracle.forward(fp, sigma_r, N, radii)
                                             - oracle.forward(fm, sigma_r, N, radii))) / (2 * h)
    scale = np.abs(g).max()
    np.testing.assert_allclose(fd, fd2, rtol=0, atol=1e-6 * scale)
    np.testing.assert_allclose(g, fd, rtol=0, atol=1e-6 * scale)


def test_dot_product():
    shape, sigma_r, N, radii = (8, 9), 25.0, 43, [1, 1]
    f = synth.rectangles(*shape, seed=4).astype(np.float64)
    rng = np.random.default_rng(2)
    u = rng.normal(size=shape)
    v = rng.normal(size=shape)
    h = 1e-4
    Jv = (oracle.forward(f + h * v, sigma_r, N, radii) - oracle.forward(f - h * v, sigma_r, N, radii)) / (2 * h)
    JTu = oracle.grad(f, sigma_r, N, radii, u)
    lhs, rhs = float(np.sum(Jv * u)), float(np.sum(v * JTu))
    assert abs(lhs - rhs) <= 1e-6 * (abs(lhs) + abs(rhs))


def test_constant_image_is_adjoint_of_normalised_filter():
    shape, radii = (10, 13), [1, 2]
    f = np.full(shape, 77.0)
    rng = np.random.default_rng(3)
    G = rng.normal(size=shape)
    k = np.array([1.0])
    for r in radii:
        k = np.convolve(k, np.ones(2 * r + 1))
    k2 = np.outer(k, k)
    eta = ndimage.correlate(np.ones(shape), k2, mode="constant")
    ref = ndimage.correlate(G / eta, k2, mode="constant")   # w is symmetric
    g = oracle.grad(f, 30.0, 30, radii, G)
    np.testing.assert_allclose(g, ref, rtol=1e-12, atol=1e-12)


def test_ssd_helpers_consistent():
    shape, sigma_r, N, radii = (12, 10), 25.0, 43, [1, 1, 1]
    f = synth.piecewise_smooth(*shape, seed=4000, n_shapes=2).astype(np.float64)
    t = synth.piecewise_smooth(*shape, seed=5000, n_shapes=2).astype(np.float64)
    idx = np.array([0, 17, 55, 119])
    g = oracle.ssd_grad_at(f, t, sigma_r, N, radii, idx)
    fd = oracle.ssd_loss_fd(f, t, sigma_r, N, radii, idx, h=1e-3)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-6 * np.abs(g).max())
