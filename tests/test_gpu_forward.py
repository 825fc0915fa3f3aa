"""GPU parity of the fused O(1) forward kernel (and the direct-window kernel)
against the FP64 oracle.

Tolerance: |gpu - oracle| <= 1e-2 + 1e-4 |oracle| per pixel (1e-2 gray
levels absolute and 1e-4 relative, FP64 only in the final division).
Small cases compare every pixel; the full-size workloads compare sampled
pixels (random, image borders, and the smallest-eta pixels the GPU reports,
where the expansion cancels most).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1105_4204_amd import synth

pytestmark = pytest.mark.gpu

ATOL, RTOL = 1e-2, 1e-4


def _ops():
    from paper_1105_4204_amd import ops
    return ops


def _check(gpu, ref, what):
    gpu = np.asarray(gpu, dtype=np.float64)
    err = np.abs(gpu - ref)
    tol = ATOL + RTOL * np.abs(ref)
    bad = int((err > tol).sum())
    print(f"{what}: max_abs={err.max():.3e} max_rel={np.max(err / np.maximum(np.abs(ref), 1e-30)):.3e} "
          f"bad={bad}/{err.size}", flush=True)
    assert np.all(np.isfinite(gpu)), what
    assert bad == 0, what


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


SMALL = [
    # (H, W, sigma_r, N(0=auto), radii, generator)
    (64, 64, 30.0, 0, [5], "rect"),
    (97, 131, 20.0, 0, [3, 3, 4], "smooth"),
    (131, 97, 25.0, 0, [2, 2, 3], "smooth"),
    (50, 70, 25.0, 0, [1, 2], "salt"),
    (33, 45, 60.0, 9, [4], "rect"),
    (40, 41, 10.0, 0, [2, 2, 2], "smooth"),     # N = 264
    (23, 300, 45.0, 0, [1, 1, 1, 1], "smooth"),  # 4 boxes, N = 15
    (1, 200, 30.0, 0, [3], "rect"),
    (200, 1, 30.0, 0, [3], "rect"),
    (1, 1, 30.0, 0, [2], "rect"),
    (7, 5, 30.0, 31, [6, 6], "salt"),            # window larger than the image
    (60, 60, 30.0, 0, [0], "smooth"),            # radius 0: identity
    (129, 257, 15.0, 0, [7, 7, 8], "smooth"),    # several tiles and ragged tails
    (20, 30, 5.1, 1024, [2], "smooth"),          # the largest degree accepted
    (40, 50, 30.0, 0, [31, 31, 1], "smooth"),    # R = 63: the widest fused kernel
    # the smallest degrees, Table 1's estimate row: sigma_r = 200, 150, 100
    # give N = 1 (the single cosine of eq. (cosine): one odd pair, no centre
    # pair), N = 2 (centre pair and m = 2) and N = 3 (m = 1, 3)
    (48, 56, 200.0, 0, [2, 2, 3], "smooth"),
    (40, 44, 150.0, 0, [3], "salt"),
    (52, 47, 100.0, 0, [1, 2, 2], "smooth"),
    (70, 66, 200.0, 0, [5], "rect"),
]


def _img(kind, H, W, seed):
    if kind == "rect":
        return synth.rectangles(H, W, seed)
    if kind == "salt":
        return synth.salt(H, W, seed)
    return synth.piecewise_smooth(H, W, seed, n_shapes=4)


@pytest.mark.parametrize("path", [1, 2], ids=["fused", "streamed"])
@pytest.mark.parametrize("case", SMALL, ids=[f"{c[0]}x{c[1]}-sr{c[2]}-N{c[3]}-r{c[4]}" for c in SMALL])
def test_forward_small_full_parity(case, path):
    H, W, sr, N, radii, kind = case
    print(f"case {case} path {path}", flush=True)
    f = _img(kind, H, W, seed=H * 1000 + W)
    Nuse = N or oracle.range_degree(255.0, sr)
    ref, eta_ref = oracle.forward(f, sr, Nuse, radii, return_eta=True)
    out, eta = _ops().trig_forward(_cuda(f), 255.0, sr, radii, N=N, return_eta=True, path=path)
    torch.cuda.synchronize()
    _check(out.cpu().numpy(), ref, f"out {case}")
    e = eta.cpu().numpy().astype(np.float64)
    rel = np.abs(e - eta_ref) / eta_ref
    print(f"eta max rel {rel.max():.3e}", flush=True)
    assert rel.max() < 1e-3


def test_forward_deterministic():
    f = _cuda(synth.piecewise_smooth(300, 257, seed=9))
    a = _ops().trig_forward(f, 255.0, 20.0, [9, 9, 10])
    b = _ops().trig_forward(f, 255.0, 20.0, [9, 9, 10])
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_forward_tile_override_consistent():
    f = _cuda(synth.piecewise_smooth(150, 170, seed=3))
    a = _ops().trig_forward(f, 255.0, 25.0, [5, 5, 6])
    b = _ops().trig_forward(f, 255.0, 25.0, [5, 5, 6], tile=(21, 35))
    torch.cuda.synchronize()
    ref = oracle.forward(synth.piecewise_smooth(150, 170, seed=3), 25.0, 43, [5, 5, 6])
    _check(b.cpu().numpy(), ref, "tile 21x35")
    assert torch.max(torch.abs(a - b)).item() < 2e-2


def test_forward_fused_wide_kernel_tile_override():
    """R = 46 forced through the fused kernel (a tile shape is given, so the
    streamed passes are not taken): 36 x 36 tiles on the 128-sample line,
    against the oracle, and the evaluation the library picks unforced."""
    H, W, radii, sr = 90, 100, [15, 15, 16], 30.0
    f_np = synth.piecewise_smooth(H, W, seed=46, n_shapes=4)
    f = _cuda(f_np)
    a = _ops().trig_forward(f, 255.0, sr, radii, tile=(36, 36))
    b = _ops().trig_forward(f, 255.0, sr, radii)
    torch.cuda.synchronize()
    ref = oracle.forward(f_np, sr, oracle.range_degree(255.0, sr), radii)
    _check(a.cpu().numpy(), ref, "fused R=46 tile 36x36")
    _check(b.cpu().numpy(), ref, "default path R=46")


def test_config1_full_image():
    f = synth.config_image(1)
    N = oracle.range_degree(255.0, 30.0)
    assert N == 30
    ref = oracle.forward(f, 30.0, N, [5])
    out = _ops().trig_forward(_cuda(f), 255.0, 30.0, [5])
    torch.cuda.synchronize()
    _check(out.cpu().numpy(), ref, "config1 256x256 box r=5")


def _sample_idx(H, W, R, eta, n_rand, seed):
    rng = np.random.default_rng(seed)
    idx = set(rng.integers(0, H * W, size=n_rand).tolist())
    # every pixel within R of the border on a few random rows/cols
    for i in list(range(0, R + 1)) + list(range(H - R - 1, H)):
        for j in rng.integers(0, W, size=4):
            idx.add(int(i) * W + int(j))
    for j in list(range(0, R + 1)) + list(range(W - R - 1, W)):
        for i in rng.integers(0, H, size=4):
            idx.add(int(i) * W + int(j))
    # all pixels within R of the border on two random 64-pixel stretches
    # (one along the top edge, one along the right edge)
    c0 = int(rng.integers(0, max(W - 64, 1)))
    r0 = int(rng.integers(0, max(H - 64, 1)))
    for i in range(min(R + 1, H)):
        for j in range(c0, min(c0 + 64, W)):
            idx.add(i * W + j)
    for i in range(r0, min(r0 + 64, H)):
        for j in range(max(W - R - 1, 0), W):
            idx.add(i * W + j)
    for c in [0, W - 1, (H - 1) * W, H * W - 1]:
        idx.add(c)
    # where the expansion cancels most: smallest eta
    idx.update(np.argsort(eta.reshape(-1))[:1000].tolist())
    return np.array(sorted(idx), dtype=np.int64)


@pytest.mark.parametrize("path", [1, 2], ids=["fused", "streamed"])
@pytest.mark.parametrize("cfg", [2, 4])
def test_full_size_sampled_parity(cfg, path):
    if cfg == 2:
        f = synth.config_image(2)
        sr, radii = 20.0, [9, 9, 10]
    else:
        f = synth.diff_batch(1)[0][0]
        sr, radii = 25.0, [5, 5, 6]
    N = oracle.range_degree(255.0, sr)
    out, eta = _ops().trig_forward(_cuda(f), 255.0, sr, radii, return_eta=True, path=path)
    torch.cuda.synchronize()
    out, eta = out.cpu().numpy(), eta.cpu().numpy()
    H, W = f.shape
    idx = _sample_idx(H, W, sum(radii), eta, 65536, seed=cfg)
    ref, eta_ref = oracle.forward_at(f, sr, N, radii, idx, return_eta=True)
    _check(out.reshape(-1)[idx], ref, f"config{cfg} path {path} sampled ({idx.size} px)")
    rel = np.abs(eta.reshape(-1)[idx] - eta_ref) / eta_ref
    assert rel.max() < 1e-3


def test_direct_kernel_small_parity():
    f = synth.piecewise_smooth(60, 75, seed=5, n_shapes=3)
    for sr, radii in [(20.0, [3, 3, 4]), (30.0, [5])]:
        N = oracle.range_degree(255.0, sr)
        ref = oracle.forward(f, sr, N, radii)
        out = _ops().direct_forward(_cuda(f), 255.0, sr, radii)
        torch.cuda.synchronize()
        _check(out.cpu().numpy(), ref, f"direct sr={sr} r={radii}")


def test_direct_vs_o1_config2():
    f = _cuda(synth.config_image(2))
    a = _ops().trig_forward(f, 255.0, 20.0, [9, 9, 10])
    b = _ops().direct_forward(f, 255.0, 20.0, [9, 9, 10])
    torch.cuda.synchronize()
    d = torch.abs(a - b)
    print(f"O(1) vs direct: max {d.max().item():.3e} mean {d.mean().item():.3e}", flush=True)
    assert d.max().item() < 2e-2
