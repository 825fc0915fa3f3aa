"""Randomised property sweep on the GPU: seeded random image sizes, box
counts, radii, degrees and image kinds, each compared over the whole image
with the FP64 oracle, forward on both evaluations and the adjoint on a
subset.  The cases come from a fixed seed, so a failure names a case that
reruns the same way.

Tolerances as in the other parity tests: forward |gpu - oracle| <= 1e-2 +
1e-4 |oracle| gray levels; adjoint |g - g_ref| <= 1e-3 max|g_ref| + 1e-3
|g_ref|.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1105_4204_amd import synth

pytestmark = pytest.mark.gpu

KINDS = ("smooth", "rect", "salt", "noise")


def _cases(n, seed, max_radius, max_total):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        nb = int(rng.integers(1, 5))
        radii = [int(rng.integers(0, max_radius + 1)) for _ in range(nb)]
        if sum(radii) > max_total:
            continue
        H = int(rng.integers(1, 161))
        W = int(rng.integers(1, 161))
        sr = float(np.exp(rng.uniform(np.log(6.0), np.log(250.0))))
        Nmin = oracle.range_degree(255.0, sr)
        # either the automatic degree or one above it
        N = 0 if rng.random() < 0.6 else int(Nmin + rng.integers(1, 40))
        out.append((H, W, sr, N, radii, KINDS[int(rng.integers(0, 4))], int(rng.integers(0, 10**6))))
    return out


def _img(kind, H, W, seed):
    if kind == "rect":
        return synth.rectangles(H, W, seed)
    if kind == "salt":
        return synth.salt(H, W, seed)
    if kind == "noise":
        return (np.random.default_rng(seed).random((H, W)) * 255.0).astype(np.float32)
    return synth.piecewise_smooth(H, W, seed, n_shapes=3)


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


FWD_FUSED = _cases(24, 2024, 12, 63)
FWD_STREAMED = _cases(24, 2025, 40, 120)
BWD = [c for c in _cases(16, 2026, 5, 10) if c[0] * c[1] <= 6000]


def _fwd(case, path):
    from paper_1105_4204_amd import ops
    H, W, sr, N, radii, kind, seed = case
    print(f"case {case} path {path}", flush=True)
    f = _img(kind, H, W, seed)
    Nuse = N or oracle.range_degree(255.0, sr)
    ref = oracle.forward(f, sr, Nuse, radii)
    out = ops.trig_forward(_cuda(f), 255.0, sr, radii, N=N, path=path)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref)
    print(f"max_abs {err.max():.3e}", flush=True)
    assert np.all(np.isfinite(got))
    assert np.all(err <= 1e-2 + 1e-4 * np.abs(ref))


@pytest.mark.parametrize("case", FWD_FUSED, ids=[f"{c[0]}x{c[1]}-N{c[3]}-r{c[4]}-{c[5]}"
                                                  for c in FWD_FUSED])
def test_random_forward_fused(case):
    _fwd(case, 1)


@pytest.mark.parametrize("case", FWD_STREAMED, ids=[f"{c[0]}x{c[1]}-N{c[3]}-r{c[4]}-{c[5]}"
                                                     for c in FWD_STREAMED])
def test_random_forward_streamed(case):
    _fwd(case, 2)


@pytest.mark.parametrize("path", [1, 2], ids=["fused", "streamed"])
@pytest.mark.parametrize("case", BWD, ids=[f"{c[0]}x{c[1]}-N{c[3]}-r{c[4]}-{c[5]}" for c in BWD])
def test_random_adjoint(case, path):
    from paper_1105_4204_amd import ops
    H, W, sr, N, radii, kind, seed = case
    print(f"case {case} path {path}", flush=True)
    f = _img(kind, H, W, seed)
    G = np.random.default_rng(seed + 1).standard_normal((H, W)).astype(np.float32)
    Nuse = N or oracle.range_degree(255.0, sr)
    ref = oracle.grad(f, sr, Nuse, radii, G.astype(np.float64))
    fg = _cuda(f)
    out, eta, aux = ops.trig_forward(fg, 255.0, sr, radii, N=N, return_aux=True, path=path)
    g = ops.trig_backward(fg, out, eta, aux, _cuda(G), 255.0, sr, radii, N=N, path=path)
    torch.cuda.synchronize()
    got = g.cpu().numpy().astype(np.float64)
    scale = max(np.abs(ref).max(), 1e-12)
    err = np.abs(got - ref)
    print(f"max_abs {err.max():.3e} scale {scale:.3e}", flush=True)
    assert np.all(np.isfinite(got))
    assert np.all(err <= 1e-3 * scale + 1e-3 * np.abs(ref))
