#!/usr/bin/env python3
"""Derives the polynomial coefficients of cis_small() in bf_tile.h.

cos x = 1 + x^2 P(x^2) (P of degree 4) and sin x = x + x^3 Q(x^2) (Q of
degree 3) on |x| <= pi/2, fitted by iteratively reweighted least squares on
Chebyshev nodes (weights grown where the error is largest, which drives the
fit toward the equioscillating minimax solution).  Truncation errors: about
2.5e-10 (cos) and 4.7e-9 (sin), far below the 6e-8 rounding unit of the
float32 evaluation.  Prints the float32 constants, highest power first, as
they appear in the kernel source.
"""
import numpy as np

HALF_PI = np.pi / 2


def _nodes(n=4000):
    k = np.arange(n)
    return HALF_PI * (0.5 + 0.5 * np.cos(np.pi * (k + 0.5) / n))


def _irls(A, b, iters=30):
    w = np.ones(len(b))
    for _ in range(iters):
        c, *_ = np.linalg.lstsq(A * w[:, None], b * w, rcond=None)
        e = np.abs(A @ c - b)
        w = w * (1 + e / e.max()) ** 2
        w /= w.max()
    return c


def coefficients():
    x = _nodes()
    cos_c = _irls(np.stack([x ** (2 * (j + 1)) for j in range(5)], 1), np.cos(x) - 1)
    sin_c = _irls(np.stack([x ** (2 * j + 3) for j in range(4)], 1), np.sin(x) - x)
    return ([float(np.float32(v)) for v in cos_c], [float(np.float32(v)) for v in sin_c])


def eval32(cos_c, sin_c, xv):
    """The kernel's float32 evaluation order (Horner in x^2, then fma)."""
    xv = np.asarray(xv, dtype=np.float32)
    x2 = (xv * xv).astype(np.float32)
    p = np.float32(cos_c[-1])
    for cj in cos_c[-2::-1]:
        p = (p * x2 + np.float32(cj)).astype(np.float32)
    c = (p * x2 + np.float32(1.0)).astype(np.float32)
    q = np.float32(sin_c[-1])
    for cj in sin_c[-2::-1]:
        q = (q * x2 + np.float32(cj)).astype(np.float32)
    s = ((q * x2) * xv + xv).astype(np.float32)
    return c, s


if __name__ == "__main__":
    cc, sc = coefficients()
    print("cos:", ", ".join(f"{v:.9e}f" for v in cc[::-1]))
    print("sin:", ", ".join(f"{v:.9e}f" for v in sc[::-1]))
