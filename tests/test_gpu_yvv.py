"""GPU parity of the recursive-Gaussian forward (Young and van Vliet spatial
kernel, whole-line passes) against the FP64 oracle: the direct window sum
with the exact two-sided impulse response of the passes as spatial kernel.

Tolerance as for the box kernels: |out - ref| <= 1e-2 + 1e-4 |ref| gray
levels.  Small images use a kernel window covering the whole image (exact);
the 2048 x 2048 case is checked on sampled pixels with a window of 16 sigma
(the response beyond it holds under 1e-9 of the mass).
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


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _check(got, ref, what, atol=1e-2, rtol=1e-4):
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - ref)
    bad = int((err > atol + rtol * np.abs(ref)).sum())
    print(f"{what}: max_abs={err.max():.3e} bad={bad}/{err.size}", flush=True)
    assert np.all(np.isfinite(got)), what
    assert bad == 0, what


CASES = [   # H, W, sigma_r, N, sigma_s
    (60, 70, 20.0, 0, 2.0),
    (33, 100, 30.0, 0, 5.0),
    (48, 52, 20.0, 0, 10.0),
    (1, 80, 30.0, 0, 3.0),
    (70, 1, 30.0, 0, 1.0),
    (40, 45, 25.0, 0, 0.5),      # odd N = 43
    (37, 41, 12.0, 0, 3.0),      # N = 184: three launch chunks of pairs
    (64, 66, 60.0, 9, 20.0),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-sr{c[2]}-ss{c[4]}" for c in CASES])
def test_yvv_small_full_parity(case):
    H, W, sr, N, ss = case
    print(f"case {case}", flush=True)
    f = synth.piecewise_smooth(H, W, seed=2 * H + W, n_shapes=3)
    Nuse = N or oracle.range_degree(255.0, sr)
    k = oracle.yvv_kernel(ss, max(H, W))
    ref, eta_ref = oracle.forward_kernel(f, sr, Nuse, k, return_eta=True)
    out, eta = _ops().yvv_forward(_cuda(f), 255.0, sr, ss, N=N, return_eta=True)
    torch.cuda.synchronize()
    _check(out.cpu().numpy(), ref, f"yvv {case}")
    e = eta.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(e - eta_ref) <= 1e-3 * np.abs(eta_ref) + 1e-7), np.abs(e - eta_ref).max()


def test_yvv_constant_image_is_preserved():
    f = np.full((50, 67), 173.0, dtype=np.float32)
    out = _ops().yvv_forward(_cuda(f), 255.0, 20.0, 6.0)
    torch.cuda.synchronize()
    _check(out.cpu().numpy(), f.astype(np.float64), "constant")


def test_yvv_workspace_and_sigma_checks():
    from paper_1105_4204_amd import _native as nat
    ops = _ops()
    f = torch.zeros(32, 32, device="cuda")
    need = nat.yvv_workspace_bytes(32, 32, 255.0, 20.0)
    small = torch.empty(need // 4 - 1, device="cuda")
    with pytest.raises(nat.BFError, match="EINVAL"):
        ops.yvv_forward(f, 255.0, 20.0, 3.0, workspace=small)
    with pytest.raises(nat.BFError, match="ERANGE"):
        ops.yvv_forward(f, 255.0, 20.0, 0.25)
    with pytest.raises(nat.BFError, match="ERANGE"):
        ops.yvv_forward(f, 255.0, 20.0, 100.0)


def test_yvv_truncation_within_bound():
    """Truncated pairs (bf_range_truncate's bound with this kernel's centre
    tap and unit mass) against the exact FP64 oracle with the recursive
    kernel: within the requested tolerance plus the usual FP32 tolerance, at
    every pixel; and the truncation really drops pairs."""
    H, W, sr, ss, tol = 64, 64, 10.0, 4.0, 0.05
    f = synth.piecewise_smooth(H, W, seed=77, n_shapes=3)
    ops = _ops()
    full = ops.yvv_forward(_cuda(f), 255.0, sr, ss)
    cut = ops.yvv_forward(_cuda(f), 255.0, sr, ss, trunc_tol=tol)
    torch.cuda.synchronize()
    N = oracle.range_degree(255.0, sr)
    ref = oracle.forward_kernel(f, sr, N, oracle.yvv_kernel(ss, max(H, W)))
    err = np.abs(cut.cpu().numpy().astype(np.float64) - ref)
    print(f"truncated vs oracle: max {err.max():.3e} (tol {tol})", flush=True)
    assert np.all(err <= tol + 1e-2 + 1e-4 * np.abs(ref))
    assert not torch.equal(full, cut)


def test_yvv_2048_sampled_and_deterministic():
    H = W = 2048
    ss, sr = 10.0, 20.0
    f = synth.config_image(2)
    ops = _ops()
    fg = _cuda(f)
    out = ops.yvv_forward(fg, 255.0, sr, ss)
    out2 = ops.yvv_forward(fg, 255.0, sr, ss)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)
    got = out.cpu().numpy().reshape(-1)
    N = oracle.range_degree(255.0, sr)
    rng = np.random.default_rng(17)
    idx = list(rng.integers(0, H * W, 24))
    idx += [0, W - 1, (H - 1) * W, H * W - 1, 1000 * W + 1000, 5 * W + 2040]
    idx = np.array(idx, dtype=np.int64)
    ref = oracle.forward_kernel(f, sr, N, oracle.yvv_kernel(ss, int(16 * ss)), idx=idx)
    _check(got[idx], ref, "yvv 2048 sampled")
