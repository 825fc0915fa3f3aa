"""GPU parity of the staged forward (spatial kernels wider than the fused
kernel's register line: sum of radii 63 < R <= 127) against the FP64 oracle,
including the 4096x4096, sigma_s = 30 (boxes 29, 29, 30), sigma_r = 10
(N = 264) workload on sampled pixels.  Tolerance as for the fused forward:
|gpu - oracle| <= 1e-2 + 1e-4 |oracle| per pixel."""
import numpy as np
import pytest
import torch

import oracle
from paper_1105_4204_amd import synth

pytestmark = pytest.mark.gpu


def _ops():
    from paper_1105_4204_amd import ops
    return ops


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _check(got, ref, what):
    err = np.abs(np.asarray(got, dtype=np.float64) - ref)
    tol = 1e-2 + 1e-4 * np.abs(ref)
    bad = int((err > tol).sum())
    print(f"{what}: max_abs={err.max():.3e} bad={bad}/{err.size}", flush=True)
    assert np.all(np.isfinite(got)), what
    assert bad == 0, what


CASES = [
    (150, 170, 30.0, 0, [25, 25, 25]),      # R = 75, N = 30
    (131, 97, 25.0, 0, [20, 22, 24]),       # R = 66, odd N = 43
    (70, 300, 20.0, 0, [31, 31, 31]),       # R = 93, taller than the image
    (1, 90, 40.0, 0, [30, 30, 10]),         # single row
    (40, 40, 12.0, 0, [31, 20, 20]),        # N = 184, image smaller than the halo
    (100, 260, 25.0, 0, [21, 21, 22]),      # R = 64: 128 outputs per horizontal line
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-r{c[4]}" for c in CASES])
def test_staged_small_full_parity(case):
    H, W, sr, N, radii = case
    print(f"case {case}", flush=True)
    f = synth.piecewise_smooth(H, W, seed=H * 3 + W, n_shapes=3)
    Nuse = N or oracle.range_degree(255.0, sr)
    ref, eta_ref = oracle.forward(f, sr, Nuse, radii, return_eta=True)
    out, eta = _ops().trig_forward(_cuda(f), 255.0, sr, radii, N=N, return_eta=True)
    torch.cuda.synchronize()
    _check(out.cpu().numpy(), ref, f"staged {case}")
    e = eta.cpu().numpy().astype(np.float64)
    assert np.allclose(e, eta_ref, rtol=2e-4, atol=1e-3 * eta_ref.max()), case


def test_staged_rejects_adjoint_sums():
    from paper_1105_4204_amd import _native as nat
    f = _cuda(synth.rectangles(64, 64, seed=1))
    with pytest.raises(nat.BFError) as e:
        _ops().trig_forward(f, 255.0, 20.0, [29, 29, 30], return_aux=True)
    assert e.value.code == 6


def test_wide_kernel_workload_sampled():
    """4096 x 4096 piecewise-smooth image (seed 3), sigma_s = 30 realised as
    boxes (29, 29, 30), sigma_r = 10, N = 264: 65536 random pixels, the 1000
    pixels of smallest eta, every pixel within R of the border on a 64-pixel
    stretch of the top and of the left edge, and the four corners, against
    the oracle."""
    from paper_1105_4204_amd import _native as nat
    f_np = synth.config_image(3)
    radii = nat.spatial_gaussian(30.0, 3)
    assert radii == [29, 29, 30]
    N = oracle.range_degree(255.0, 10.0)
    assert N == 264
    out, eta = _ops().trig_forward(_cuda(f_np), 255.0, 10.0, radii, return_eta=True)
    torch.cuda.synchronize()
    o = out.cpu().numpy().reshape(-1)
    e = eta.cpu().numpy().reshape(-1)
    rng = np.random.default_rng(33)
    H = W = 4096
    R = sum(radii)
    c0, r0 = int(rng.integers(0, W - 64)), int(rng.integers(0, H - 64))
    top = [i * W + j for i in range(R + 1) for j in range(c0, c0 + 64)]
    left = [i * W + j for i in range(r0, r0 + 64) for j in range(R + 1)]
    idx = np.unique(np.concatenate([rng.integers(0, H * W, size=65536), np.argsort(e)[:1000],
                                    np.array(top + left + [0, W - 1, (H - 1) * W, H * W - 1])]))
    ref = oracle.forward_at(f_np, 10.0, N, radii, idx)
    _check(o[idx], ref, "4096^2 sigma_s=30 N=264 sampled")
