"""FP64 CPU oracle for the trigonometric bilateral filter.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The product path (the HIP library
and its Python binding) never imports or calls anything here, and this module
imports nothing from the product.

The numerics live in ``bf_oracle.c`` (plain C, double precision, OpenMP over
pixels): a brute-force window sum of the unbiased bilateral filter, eq. (BF) and
eq. (normalization), with the raised-cosine range kernel of Sec. 2.3 scaled as in
Sec. 2.5 / Algorithm 1 step 3, and the explicitly convolved iterated-box spatial
kernel.  Every entry point here is a thin ctypes marshaller over that library.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_range_degree.restype = ctypes.c_int64
    lib.oracle_range_degree.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.oracle_phi.restype = ctypes.c_double
    lib.oracle_phi.argtypes = [ctypes.c_double, ctypes.c_int64, ctypes.c_double]
    lib.oracle_spatial_kernel.restype = ctypes.c_int64
    lib.oracle_spatial_kernel.argtypes = [_i32p, ctypes.c_int32, _dp]
    lib.oracle_forward.restype = ctypes.c_int
    lib.oracle_forward.argtypes = [_dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                   ctypes.c_int64, _i32p, ctypes.c_int32, _dp, _dp]
    lib.oracle_forward_at.restype = ctypes.c_int
    lib.oracle_forward_at.argtypes = [_dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                      ctypes.c_int64, _i32p, ctypes.c_int32, _i64p,
                                      ctypes.c_int64, _dp, _dp]
    lib.oracle_grad_at.restype = ctypes.c_int
    lib.oracle_grad_at.argtypes = [_dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                   ctypes.c_int64, _i32p, ctypes.c_int32, _dp, _i64p,
                                   ctypes.c_int64, _dp]
    lib.oracle_forward_sv.restype = ctypes.c_int
    lib.oracle_forward_sv.argtypes = [_dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                      ctypes.c_int64, _i32p, _dp, _dp]
    lib.oracle_yvv_coeffs.restype = ctypes.c_int
    lib.oracle_yvv_coeffs.argtypes = [ctypes.c_double, _dp]
    lib.oracle_yvv_line.restype = ctypes.c_int
    lib.oracle_yvv_line.argtypes = [_dp, ctypes.c_int64, ctypes.c_double, _dp]
    lib.oracle_yvv_kernel.restype = ctypes.c_int
    lib.oracle_yvv_kernel.argtypes = [ctypes.c_double, ctypes.c_int64, _dp]
    lib.oracle_forward_kernel.restype = ctypes.c_int
    lib.oracle_forward_kernel.argtypes = [_dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                          ctypes.c_int64, _dp, ctypes.c_int64, _i64p,
                                          ctypes.c_int64, _dp, _dp]
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _radii(radii):
    r = np.ascontiguousarray(np.atleast_1d(radii), dtype=np.int32)
    return r


def num_threads() -> int:
    """OpenMP threads used by the oracle's parallel loops."""
    return int(_load().oracle_num_threads())


def range_degree(T: float, sigma_r: float) -> int:
    """N = ceil((gamma sigma_r)^-2), gamma = pi/2T (Algorithm 1 steps 1-2)."""
    n = int(_load().oracle_range_degree(float(T), float(sigma_r)))
    if n < 0:
        raise ValueError("T and sigma_r must be positive")
    return n


def phi(s, N: int, sigma_r: float):
    """Raised-cosine range kernel cos(s / (sigma_r sqrt N))^N (Sec. 2.3, 2.5)."""
    lib = _load()
    s = np.asarray(s, dtype=np.float64)
    out = np.empty_like(s)
    flat_in, flat_out = s.reshape(-1), out.reshape(-1)
    for t in range(flat_in.size):
        flat_out[t] = lib.oracle_phi(float(flat_in[t]), int(N), float(sigma_r))
    return out if out.ndim else float(out)


def spatial_kernel(radii) -> np.ndarray:
    """1-D composite kernel: explicit convolution of unit boxes of widths 2r+1."""
    r = _radii(radii)
    R = int(r.sum())
    k = np.empty(2 * R + 1, dtype=np.float64)
    if _load().oracle_spatial_kernel(r.ctypes.data_as(_i32p), r.size, k.ctypes.data_as(_dp)) < 0:
        raise ValueError("bad radii")
    return k


def forward(f, sigma_r: float, N: int, radii, return_eta: bool = False):
    """Direct FP64 bilateral filter of the whole image f (H x W)."""
    f = _f64(f)
    if f.ndim != 2:
        raise ValueError("f must be 2-D")
    H, W = f.shape
    r = _radii(radii)
    out = np.empty_like(f)
    eta = np.empty_like(f) if return_eta else None
    rc = _load().oracle_forward(f.ctypes.data_as(_dp), H, W, float(sigma_r), int(N),
                                r.ctypes.data_as(_i32p), r.size, out.ctypes.data_as(_dp),
                                eta.ctypes.data_as(_dp) if eta is not None else None)
    if rc != 0:
        raise ValueError("oracle_forward: bad arguments")
    return (out, eta) if return_eta else out


def forward_at(f, sigma_r: float, N: int, radii, idx, return_eta: bool = False):
    """Direct FP64 filter at flat pixel indices idx (row-major)."""
    f = _f64(f)
    H, W = f.shape
    r = _radii(radii)
    idx = np.ascontiguousarray(idx, dtype=np.int64).reshape(-1)
    out = np.empty(idx.size, dtype=np.float64)
    eta = np.empty(idx.size, dtype=np.float64) if return_eta else None
    rc = _load().oracle_forward_at(f.ctypes.data_as(_dp), H, W, float(sigma_r), int(N),
                                   r.ctypes.data_as(_i32p), r.size, idx.ctypes.data_as(_i64p),
                                   idx.size, out.ctypes.data_as(_dp),
                                   eta.ctypes.data_as(_dp) if eta is not None else None)
    if rc != 0:
        raise ValueError("oracle_forward_at: bad arguments")
    return (out, eta) if return_eta else out


def grad_at(f, sigma_r: float, N: int, radii, G, idx):
    """dL/df at flat indices idx for upstream gradient G = dL/dout (full image)."""
    f = _f64(f)
    H, W = f.shape
    G = _f64(G)
    if G.shape != f.shape:
        raise ValueError("G must match f")
    r = _radii(radii)
    idx = np.ascontiguousarray(idx, dtype=np.int64).reshape(-1)
    g = np.empty(idx.size, dtype=np.float64)
    rc = _load().oracle_grad_at(f.ctypes.data_as(_dp), H, W, float(sigma_r), int(N),
                                r.ctypes.data_as(_i32p), r.size, G.ctypes.data_as(_dp),
                                idx.ctypes.data_as(_i64p), idx.size, g.ctypes.data_as(_dp))
    if rc != 0:
        raise ValueError("oracle_grad_at: bad arguments")
    return g


def grad(f, sigma_r: float, N: int, radii, G):
    """Full-image dL/df (small images only: cost grows as (2R+1)^4 per pixel)."""
    f = _f64(f)
    idx = np.arange(f.size, dtype=np.int64)
    return grad_at(f, sigma_r, N, radii, G, idx).reshape(f.shape)


def window_pixels(H: int, W: int, R: int, idx) -> np.ndarray:
    """Flat indices of every pixel within Chebyshev distance R of any idx."""
    mask = np.zeros((H, W), dtype=bool)
    for p in np.asarray(idx, dtype=np.int64).reshape(-1):
        i, j = divmod(int(p), W)
        mask[max(0, i - R):min(H, i + R + 1), max(0, j - R):min(W, j + R + 1)] = True
    return np.flatnonzero(mask)


def ssd_grad_at(f, target, sigma_r: float, N: int, radii, idx):
    """d/df of sum((out - target)^2) at idx; out is the oracle's own forward."""
    f = _f64(f)
    H, W = f.shape
    R = int(_radii(radii).sum())
    near = window_pixels(H, W, R, idx)
    out_near = forward_at(f, sigma_r, N, radii, near)
    G = np.zeros((H, W), dtype=np.float64)
    G.reshape(-1)[near] = 2.0 * (out_near - _f64(target).reshape(-1)[near])
    return grad_at(f, sigma_r, N, radii, G, idx)


def ssd_loss_fd(f, target, sigma_r: float, N: int, radii, idx, h: float = 1e-3):
    """Central finite difference of sum((out - target)^2) at idx (FP64).

    Only the pixels within R of the perturbed pixel change, so each difference
    re-evaluates the oracle on that window alone.
    """
    f = _f64(f).copy()
    H, W = f.shape
    R = int(_radii(radii).sum())
    tgt = _f64(target).reshape(-1)
    res = np.empty(len(np.atleast_1d(idx)), dtype=np.float64)
    for t, p in enumerate(np.asarray(idx, dtype=np.int64).reshape(-1)):
        near = window_pixels(H, W, R, [p])
        flat = f.reshape(-1)
        v0 = flat[p]
        flat[p] = v0 + h
        lp = np.sum((forward_at(f, sigma_r, N, radii, near) - tgt[near]) ** 2)
        flat[p] = v0 - h
        lm = np.sum((forward_at(f, sigma_r, N, radii, near) - tgt[near]) ** 2)
        flat[p] = v0
        res[t] = (lp - lm) / (2.0 * h)
    return res


def forward_sv(f, sigma_r: float, N: int, rmap, return_eta: bool = False):
    """Space-variant filter (Sec. 4): unit box of half-width rmap[i, j] around
    each pixel, fixed raised-cosine range kernel; direct FP64 window sums."""
    f = _f64(f)
    if f.ndim != 2:
        raise ValueError("f must be 2-D")
    H, W = f.shape
    rm = np.ascontiguousarray(rmap, dtype=np.int32)
    if rm.shape != f.shape:
        raise ValueError("rmap must match f")
    out = np.empty_like(f)
    eta = np.empty_like(f) if return_eta else None
    rc = _load().oracle_forward_sv(f.ctypes.data_as(_dp), H, W, float(sigma_r), int(N),
                                   rm.ctypes.data_as(_i32p), out.ctypes.data_as(_dp),
                                   eta.ctypes.data_as(_dp) if eta is not None else None)
    if rc != 0:
        raise ValueError("oracle_forward_sv: bad arguments")
    return (out, eta) if return_eta else out


def yvv_coeffs(sigma_s: float):
    """(B, b1/b0, b2/b0, b3/b0) of the recursive Gaussian of Young and van
    Vliet (1995) for standard deviation sigma_s >= 0.5."""
    c = np.empty(4, dtype=np.float64)
    if _load().oracle_yvv_coeffs(float(sigma_s), c.ctypes.data_as(_dp)) != 0:
        raise ValueError("sigma_s must be >= 0.5")
    return tuple(float(x) for x in c)


def yvv_line(u, sigma_s: float) -> np.ndarray:
    """Causal then anticausal pass over a finite line, zero state at both ends."""
    u = _f64(u).reshape(-1)
    out = np.empty_like(u)
    if _load().oracle_yvv_line(u.ctypes.data_as(_dp), u.size, float(sigma_s),
                               out.ctypes.data_as(_dp)) != 0:
        raise ValueError("bad arguments")
    return out


def yvv_kernel(sigma_s: float, D: int) -> np.ndarray:
    """Impulse response of the two passes on an infinite line, taps -D..D."""
    k = np.empty(2 * int(D) + 1, dtype=np.float64)
    if _load().oracle_yvv_kernel(float(sigma_s), int(D), k.ctypes.data_as(_dp)) != 0:
        raise ValueError("bad arguments")
    return k


def forward_kernel(f, sigma_r: float, N: int, k, idx=None, return_eta: bool = False):
    """Direct FP64 filter with the separable spatial kernel k (x) k, k of odd
    length 2D+1 centred on tap D; at flat indices idx, or every pixel."""
    f = _f64(f)
    H, W = f.shape
    k = _f64(k).reshape(-1)
    if k.size % 2 != 1:
        raise ValueError("kernel length must be odd")
    D = (k.size - 1) // 2
    if idx is None:
        n, ip = H * W, None
    else:
        idx = np.ascontiguousarray(idx, dtype=np.int64).reshape(-1)
        n, ip = idx.size, idx.ctypes.data_as(_i64p)
    out = np.empty(n, dtype=np.float64)
    eta = np.empty(n, dtype=np.float64) if return_eta else None
    rc = _load().oracle_forward_kernel(f.ctypes.data_as(_dp), H, W, float(sigma_r), int(N),
                                       k.ctypes.data_as(_dp), D, ip, n, out.ctypes.data_as(_dp),
                                       eta.ctypes.data_as(_dp) if eta is not None else None)
    if rc != 0:
        raise ValueError("oracle_forward_kernel: bad arguments")
    if idx is None:
        out = out.reshape(H, W)
        eta = eta.reshape(H, W) if eta is not None else None
    return (out, eta) if return_eta else out
