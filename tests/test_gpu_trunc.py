"""GPU checks of term truncation with an error bound (bf_range_truncate):
the truncated filter stays within bound + the usual FP32 tolerance of the
exact FP64 oracle, in the fused and the streamed evaluations, the batch honours a
per-image tolerance bit for bit, and the adjoint of the truncated forward is
what autograd returns."""
import numpy as np
import pytest
import torch

import oracle
from paper_1105_4204_amd import synth

pytestmark = pytest.mark.gpu


def _mods():
    from paper_1105_4204_amd import _native as nat
    from paper_1105_4204_amd import batch, ops
    return nat, ops, batch


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _check(got, ref, bound, what):
    err = np.abs(np.asarray(got, dtype=np.float64) - ref)
    tol = bound + 1e-2 + 1e-4 * np.abs(ref)
    print(f"{what}: max_abs={err.max():.3e} bound={bound:.3e}", flush=True)
    assert np.all(err <= tol), what


@pytest.mark.parametrize("tol", [0.05, 1.0])
def test_truncated_small_full(tol):
    nat, ops, _ = _mods()
    H, W, sr, radii = 70, 90, 15.0, [4, 4, 5]
    N = oracle.range_degree(255.0, sr)
    Q, bound = nat.range_truncate(N, 255.0, radii, tol)
    assert Q < len(nat.range_coeffs(N))
    f = synth.salt(H, W, seed=11)
    ref = oracle.forward(f, sr, N, radii)
    out = ops.trig_forward(_cuda(f), 255.0, sr, radii, trunc_tol=tol)
    full = ops.trig_forward(_cuda(f), 255.0, sr, radii)
    torch.cuda.synchronize()
    _check(out.cpu().numpy(), ref, bound, f"trunc {tol} Q={Q}")
    assert not torch.equal(out, full)


def test_truncated_2048_sampled():
    nat, ops, _ = _mods()
    f_np = synth.config_image(2)
    radii, sr = [9, 9, 10], 20.0
    N = oracle.range_degree(255.0, sr)
    Q, bound = nat.range_truncate(N, 255.0, radii, 1e-2)
    out, eta = ops.trig_forward(_cuda(f_np), 255.0, sr, radii, return_eta=True, trunc_tol=1e-2)
    torch.cuda.synchronize()
    o = out.cpu().numpy().reshape(-1)
    e = eta.cpu().numpy().reshape(-1)
    rng = np.random.default_rng(21)
    idx = np.concatenate([rng.integers(0, o.size, size=48), np.argsort(e)[:16]])
    ref = oracle.forward_at(f_np, sr, N, radii, idx)
    _check(o[idx], ref, bound, f"2048^2 trunc 1e-2 Q={Q}")


def test_truncated_wide_kernel_sampled():
    """The 4096^2, sigma_s = 30, N = 264 workload through the streamed passes with
    truncation at 1e-2 gray (48 of 133 pairs)."""
    nat, ops, _ = _mods()
    f_np = synth.config_image(3)
    radii, sr = [29, 29, 30], 10.0
    N = oracle.range_degree(255.0, sr)
    Q, bound = nat.range_truncate(N, 255.0, radii, 1e-2)
    out, eta = ops.trig_forward(_cuda(f_np), 255.0, sr, radii, return_eta=True, trunc_tol=1e-2)
    torch.cuda.synchronize()
    o = out.cpu().numpy().reshape(-1)
    e = eta.cpu().numpy().reshape(-1)
    rng = np.random.default_rng(22)
    idx = np.concatenate([rng.integers(0, o.size, size=32), np.argsort(e)[:8]])
    ref = oracle.forward_at(f_np, sr, N, radii, idx)
    _check(o[idx], ref, bound, f"4096^2 wide trunc 1e-2 Q={Q}")


def test_truncated_adjoint_and_batch():
    nat, ops, batch = _mods()
    H, W, sr, radii, tol = 96, 80, 20.0, [3, 3, 4], 0.05
    f_np = synth.piecewise_smooth(H, W, seed=31, n_shapes=3)
    t_np = synth.piecewise_smooth(H, W, seed=32, n_shapes=3)
    f = _cuda(f_np).requires_grad_(True)
    out = ops.bf_trig(f, 255.0, sr, radii, trunc_tol=tol)
    ((out - _cuda(t_np)) ** 2).sum().backward()
    fd = _cuda(f_np)
    o2, e2, x2 = ops.trig_forward(fd, 255.0, sr, radii, return_aux=True, trunc_tol=tol)
    g2 = ops.trig_backward(fd, o2, e2, x2, 2.0 * (o2 - _cuda(t_np)), 255.0, sr, radii,
                           trunc_tol=tol)
    o3, e3, x3 = ops.trig_forward(fd, 255.0, sr, radii, return_aux=True)
    g3 = ops.trig_backward(fd, o3, e3, x3, 2.0 * (o3 - _cuda(t_np)), 255.0, sr, radii)
    torch.cuda.synchronize()
    assert torch.equal(f.grad, g2)
    scale = float(g3.abs().max())
    assert float((g2 - g3).abs().max()) <= 0.05 * scale
    # batch with a per-image tolerance equals the single-image kernels
    specs = [dict(H=H, W=W, radii=radii, sigma_r=sr, trunc_tol=tol),
             dict(H=50, W=70, radii=[2, 2, 3], sigma_r=30.0)]
    fs = [fd, _cuda(synth.rectangles(50, 70, seed=5))]
    ts = [_cuda(t_np), _cuda(synth.rectangles(50, 70, seed=6))]
    plan = batch.BatchPlan(specs, path=1)   # the fused tiles: bit-equal to the single image
    bo, be, bg, bl = plan.allocate()
    plan.bind(fs, ts, bo, be, bg, bl)
    plan.launch()
    plan.check()
    torch.cuda.synchronize()
    # the batch runs the fused tiles: compare with the single-image fused kernels
    o5, e5, x5 = ops.trig_forward(fd, 255.0, sr, radii, return_aux=True, trunc_tol=tol, path=1)
    g5 = ops.trig_backward(fd, o5, e5, x5, 2.0 * (o5 - _cuda(t_np)), 255.0, sr, radii,
                           trunc_tol=tol, path=1)
    torch.cuda.synchronize()
    assert torch.equal(bo[0], o5)
    assert torch.equal(bg[0], g5)
    o4 = ops.trig_forward(fs[1], 255.0, 30.0, [2, 2, 3], path=1)
    torch.cuda.synchronize()
    assert torch.equal(bo[1], o4)
