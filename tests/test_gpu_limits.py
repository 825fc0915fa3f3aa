"""GPU parity at the largest image sizes the library accepts: 2^20 pixels
along one axis and 2^31 pixels in total (46340 x 46340, 8.6 GB per plane).

The filter at a pixel depends only on f inside its window, so each sampled
pixel is checked against the FP64 oracle run on the crop of f that holds its
whole window (a crop edge is an image edge only where the image's is).
Tolerance as elsewhere: |out - ref| <= 1e-2 + 1e-4 |ref| gray levels; the
adjoint on the long row against the oracle's gradient at sampled pixels.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1105_4204_amd import synth

pytestmark = pytest.mark.gpu


def _ops():
    from paper_1105_4204_amd import ops
    return ops


def _crop_ref(f, i, j, R, sr, N, radii):
    H, W = f.shape
    i0, i1 = max(0, i - R), min(H, i + R + 1)
    j0, j1 = max(0, j - R), min(W, j + R + 1)
    crop = np.asarray(f[i0:i1, j0:j1], dtype=np.float64)
    return oracle.forward(crop, sr, N, radii)[i - i0, j - j0]


def _check(got, ref, what):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    err = np.abs(got - ref)
    print(f"{what}: max_abs={err.max():.3e} n={err.size}", flush=True)
    assert np.all(np.isfinite(got)), what
    assert np.all(err <= 1e-2 + 1e-4 * np.abs(ref)), what


@pytest.mark.parametrize("shape", [(1, 1 << 20), (1 << 20, 1)], ids=["row", "column"])
def test_longest_axis(shape):
    H, W = shape
    sr, radii = 30.0, [9, 9, 10]
    N = oracle.range_degree(255.0, sr)
    line = synth.piecewise_smooth(1, 1 << 20, seed=33, n_shapes=64).reshape(shape)
    ops = _ops()
    f = torch.from_numpy(np.ascontiguousarray(line)).cuda()
    out, eta, aux = ops.trig_forward(f, 255.0, sr, radii, return_aux=True)
    G = torch.randn(shape, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    gf = ops.trig_backward(f, out, eta, aux, G, 255.0, sr, radii)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    rng = np.random.default_rng(8)
    pos = [0, 1, 27, (1 << 20) - 1, (1 << 20) - 30] + list(rng.integers(0, 1 << 20, 40))
    ij = [(p, 0) if H > 1 else (0, p) for p in pos]
    R = sum(radii)
    _check([o[i, j] for i, j in ij], [_crop_ref(line, i, j, R, sr, N, radii) for i, j in ij],
           f"forward {shape}")
    # adjoint at a few pixels: its window reaches 2R (the pixels whose windows hold it)
    g = gf.cpu().numpy()
    Gn = G.cpu().numpy()
    for p in pos[:12]:
        i, j = (p, 0) if H > 1 else (0, p)
        lo, hi = max(0, p - 2 * R), min(1 << 20, p + 2 * R + 1)
        if H > 1:
            fc, Gc, k = line[lo:hi, :], Gn[lo:hi, :], (p - lo) * 1
        else:
            fc, Gc, k = line[:, lo:hi], Gn[:, lo:hi], p - lo
        ref = oracle.grad_at(np.asarray(fc, np.float64), sr, N, radii, Gc, np.array([k]))[0]
        assert abs(g[i, j] - ref) <= 1e-3 * max(abs(ref), 1.0) + 1e-3, (p, g[i, j], ref)


def test_largest_total_size():
    side = 46340                       # 46340^2 < 2^31 pixels
    sr, radii = 40.0, [5, 5, 6]
    N = oracle.range_degree(255.0, sr)
    gen = torch.Generator("cuda").manual_seed(12)
    f = torch.rand(side, side, device="cuda", generator=gen) * 255.0
    ops = _ops()
    out = ops.trig_forward(f, 255.0, sr, radii)
    torch.cuda.synchronize()
    rng = np.random.default_rng(13)
    pts = [(0, 0), (side - 1, side - 1), (0, side - 1), (side - 1, 0), (23170, 23170)]
    pts += [(int(a), int(b)) for a, b in zip(rng.integers(0, side, 20), rng.integers(0, side, 20))]
    R = sum(radii)
    got, ref = [], []
    for i, j in pts:
        i0, i1 = max(0, i - R), min(side, i + R + 1)
        j0, j1 = max(0, j - R), min(side, j + R + 1)
        crop = f[i0:i1, j0:j1].cpu().numpy().astype(np.float64)
        ref.append(oracle.forward(crop, sr, N, radii)[i - i0, j - j0])
        got.append(out[i, j].item())
    del f, out
    torch.cuda.empty_cache()
    _check(got, ref, "46340^2 sampled")
