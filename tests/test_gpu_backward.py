"""GPU parity of the adjoint (the fused tile kernel and the streamed passes)
against the FP64 oracle.

The oracle's gradient is the exact derivative of the direct window sum; it is
itself pinned by finite differences in test_oracle_grad.  Tolerance (the
paper gives none for the gradient; derived from the FP32 arithmetic of the
forward, whose outputs feed the adjoint): per pixel
|g - g_ref| <= 1e-3 * max|g_ref| + 1e-3 * |g_ref|.
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


def _check(g, ref, what):
    g = np.asarray(g, dtype=np.float64)
    scale = np.abs(ref).max()
    err = np.abs(g - ref)
    tol = 1e-3 * scale + 1e-3 * np.abs(ref)
    bad = int((err > tol).sum())
    print(f"{what}: max_abs={err.max():.3e} scale={scale:.3e} bad={bad}/{err.size}", flush=True)
    assert np.all(np.isfinite(g)), what
    assert bad == 0, what


CASES = [
    (24, 31, 30.0, 0, [2]),
    (29, 22, 25.0, 0, [1, 1, 2]),       # odd N = 43
    (20, 26, 20.0, 0, [2, 2, 3]),       # even N = 66
    (16, 40, 60.0, 9, [3]),
    (1, 50, 30.0, 0, [3]),
    (18, 18, 12.0, 0, [1, 1, 1]),       # N = 181
    # extended tiles wider than 120 samples: the 128-sample line variants,
    # g from global memory (W, R multiples of 4) and g staged in LDS
    (24, 28, 25.0, 0, [16, 18, 18]),    # R = 52, extended tile 128 x 128
    (30, 30, 30.0, 0, [15, 17, 18]),    # R = 50, extended tile 128 x 124
    # the smallest degrees (Table 1's estimate row): N = 1, 2, 3
    (26, 30, 200.0, 0, [2, 2, 3]),
    (22, 27, 150.0, 0, [3]),
    (25, 24, 100.0, 0, [1, 2, 2]),
]


@pytest.mark.parametrize("path", [1, 2], ids=["fused", "streamed"])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-sr{c[2]}-r{c[4]}" for c in CASES])
def test_backward_small_full_parity(case, path):
    H, W, sr, N, radii = case
    print(f"case {case} path {path}", flush=True)
    f = synth.piecewise_smooth(H, W, seed=H + 7 * W, n_shapes=3)
    G = np.random.default_rng(H * W).normal(size=(H, W))
    Nuse = N or oracle.range_degree(255.0, sr)
    ref = oracle.grad(f, sr, Nuse, radii, G)
    ops = _ops()
    fg = _cuda(f)
    out, eta, aux = ops.trig_forward(fg, 255.0, sr, radii, N=N, return_aux=True, path=path)
    gf = ops.trig_backward(fg, out, eta, aux, _cuda(G), 255.0, sr, radii, N=N, path=path)
    torch.cuda.synchronize()
    _check(gf.cpu().numpy(), ref, f"grad {case} path {path}")


def test_autograd_matches_explicit_backward():
    f_np = synth.rectangles(40, 36, seed=3)
    t_np = synth.rectangles(40, 36, seed=4)
    ops = _ops()
    f = _cuda(f_np).requires_grad_(True)
    out = ops.bf_trig(f, 255.0, 25.0, (2, 2, 3))
    loss = ((out - _cuda(t_np)) ** 2).sum()
    loss.backward()
    fd = _cuda(f_np)
    o2, e2, x2 = ops.trig_forward(fd, 255.0, 25.0, [2, 2, 3], return_aux=True)
    g2 = ops.trig_backward(fd, o2, e2, x2, 2.0 * (o2 - _cuda(t_np)), 255.0, 25.0, [2, 2, 3])
    torch.cuda.synchronize()
    assert torch.equal(f.grad, g2)


def _seam_border_idx(H, W, tile, rng, n_per):
    """Pixels on the seams of a tile grid (rows and columns tile-1 and tile of
    every seam), on the image borders and at the corners."""
    idx = set()
    for s in range(tile, max(H, W), tile):
        for i in (s - 1, s):
            if i < H:
                for j in rng.integers(0, W, size=n_per):
                    idx.add(int(i) * W + int(j))
            if i < W:
                for r in rng.integers(0, H, size=n_per):
                    idx.add(int(r) * W + int(i))
    for i in (0, 1, H - 2, H - 1):
        for j in rng.integers(0, W, size=n_per):
            idx.add(i * W + int(j))
    for j in (0, 1, W - 2, W - 1):
        for i in rng.integers(0, H, size=n_per):
            idx.add(int(i) * W + j)
    for i, j in ((0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (tile - 1, tile - 1),
                 (tile, tile), (tile - 1, tile), (2 * tile - 1, 2 * tile)):
        idx.add(i * W + j)
    return idx


@pytest.mark.parametrize("path", [1, 2], ids=["fused", "streamed"])
def test_config2_adjoint_sampled(path):
    """The adjoint of the benchmarked step at its own size: 2048 x 2048,
    boxes 9, 9, 10 (R = 28), sigma_r = 20 (N = 66): the fused kernel's
    global-g variant on 64 x 64 tiles with the 120-sample line, and the
    streamed passes.  Upstream gradient G: seeded N(0, 1) noise (independent
    of the GPU).  Compared with the oracle's exact gradient on more than 256
    pixels: random ones, the 64 pixels of smallest eta (where the expansion
    cancels most), the pixels of largest local contrast, the seams of the
    64 x 64 tile grid (rows and columns 63/64, 127/128, ...), the image
    borders and the corners."""
    f = synth.config_image(2)
    H, W = f.shape
    radii, sr = [9, 9, 10], 20.0
    N = oracle.range_degree(255.0, sr)
    assert N == 66
    G = np.random.default_rng(2048).normal(size=(H, W))
    ops = _ops()
    fg = _cuda(f)
    out, eta, aux = ops.trig_forward(fg, 255.0, sr, radii, return_aux=True, path=path)
    gf = ops.trig_backward(fg, out, eta, aux, _cuda(G), 255.0, sr, radii, path=path)
    torch.cuda.synchronize()
    g = gf.cpu().numpy().reshape(-1)
    e = eta.cpu().numpy().reshape(-1)
    rng = np.random.default_rng(2049)
    idx = set(rng.integers(0, H * W, size=96).tolist())
    idx |= _seam_border_idx(H, W, 64, rng, 2)
    idx |= set(np.argsort(e)[:64].tolist())
    from scipy import ndimage
    contrast = np.abs(f - ndimage.uniform_filter(f.astype(np.float64), 2 * sum(radii) + 1))
    idx |= set(np.argsort(contrast.reshape(-1))[-32:].tolist())
    idx = np.array(sorted(idx), dtype=np.int64)
    assert idx.size >= 256
    ref = oracle.grad_at(f, sr, N, radii, G, idx)
    _check(g[idx], ref, f"config2 adjoint path {path} ({idx.size} px)")


def test_config4_ssd_gradient_vs_fd_and_oracle():
    """Batch of 16 512x512 images, sigma_s = 6 (boxes 5,5,6), sigma_r = 25
    (N = 43); loss = SSD to a second seeded image; dL/df on 32 random pixels
    of image 0 against FP64 central differences and the oracle gradient; the
    other 15 images checked against the oracle on 4 pixels each."""
    fb, tb = synth.diff_batch(16)
    radii, sr = [5, 5, 6], 25.0
    N = oracle.range_degree(255.0, sr)
    ops = _ops()
    grads = []
    for i in range(16):
        f = _cuda(fb[i])
        out, eta, aux = ops.trig_forward(f, 255.0, sr, radii, return_aux=True)
        grads.append(ops.trig_backward(f, out, eta, aux, 2.0 * (out - _cuda(tb[i])), 255.0, sr,
                                       radii))
    torch.cuda.synchronize()
    rng = np.random.default_rng(44)
    idx = rng.integers(0, 512 * 512, size=32)
    g0 = grads[0].cpu().numpy().reshape(-1)[idx]
    fd = oracle.ssd_loss_fd(fb[0], tb[0], sr, N, radii, idx, h=1e-3)
    fd2 = oracle.ssd_loss_fd(fb[0], tb[0], sr, N, radii, idx, h=5e-4)
    ref = oracle.ssd_grad_at(fb[0], tb[0], sr, N, radii, idx)
    scale = np.abs(ref).max()
    assert np.max(np.abs(fd - fd2)) <= 1e-6 * scale + 1e-6
    assert np.max(np.abs(ref - fd)) <= 1e-6 * scale + 1e-6
    _check(g0, ref, "config4 image 0 (32 px) vs oracle")
    _check(g0, fd, "config4 image 0 (32 px) vs FD")
    # 64 more pixels on each of the 16 images (1024 + 32 in all): random
    # ones, the 64 x 64 tile seams, the borders and corners
    for i in range(16):
        seams = np.array(sorted(_seam_border_idx(512, 512, 64, rng, 1)), dtype=np.int64)
        ii = set(rng.choice(seams, size=40, replace=False).tolist())
        while len(ii) < 64:
            ii.add(int(rng.integers(0, 512 * 512)))
        ii = np.array(sorted(ii), dtype=np.int64)
        ref_i = oracle.ssd_grad_at(fb[i], tb[i], sr, N, radii, ii)
        gi = grads[i].cpu().numpy().reshape(-1)[ii]
        _check(gi, ref_i, f"config4 image {i} ({ii.size} px)")


def test_backward_deterministic():
    f = _cuda(synth.piecewise_smooth(200, 190, seed=5))
    ops = _ops()
    out, eta, aux = ops.trig_forward(f, 255.0, 20.0, [9, 9, 10], return_aux=True)
    G = torch.randn_like(f)
    a = ops.trig_backward(f, out, eta, aux, G, 255.0, 20.0, [9, 9, 10])
    b = ops.trig_backward(f, out, eta, aux, G, 255.0, 20.0, [9, 9, 10])
    torch.cuda.synchronize()
    assert torch.equal(a, b)


# The adjoint reads g from global memory (one LDS plane, larger tiles) when W
# and R are multiples of 4 and f is 16-byte aligned; these cases take that path.
GG_CASES = [
    (36, 48, 25.0, 0, [1, 1, 2]),
    (33, 68, 30.0, 0, [4]),
    (20, 8, 20.0, 0, [2, 2]),
]


@pytest.mark.parametrize("case", GG_CASES, ids=[f"{c[0]}x{c[1]}-r{c[4]}" for c in GG_CASES])
def test_backward_global_g_full_parity(case):
    H, W, sr, N, radii = case
    assert W % 4 == 0 and sum(radii) % 4 == 0
    print(f"case {case}", flush=True)
    f = synth.piecewise_smooth(H, W, seed=H + 11 * W, n_shapes=3)
    G = np.random.default_rng(H + W).normal(size=(H, W))
    Nuse = N or oracle.range_degree(255.0, sr)
    ref = oracle.grad(f, sr, Nuse, radii, G)
    ops = _ops()
    fg = _cuda(f)
    out, eta, aux = ops.trig_forward(fg, 255.0, sr, radii, N=N, return_aux=True, path=1)
    gf = ops.trig_backward(fg, out, eta, aux, _cuda(G), 255.0, sr, radii, N=N, path=1)
    torch.cuda.synchronize()
    _check(gf.cpu().numpy(), ref, f"grad gg {case}")


def test_backward_both_g_paths_agree_and_match_oracle():
    """The same 130 x 200 image (R = 8) through both adjoint variants: an
    aligned tensor takes the global-g kernel (64 x 64 tiles), a view shifted
    by one float (not 16-byte aligned) the LDS-g kernel (smaller tiles).  Both
    must match the oracle on sampled pixels, borders included, and each other
    to rounding."""
    H, W, sr, radii = 130, 200, 20.0, [2, 3, 3]
    f = synth.piecewise_smooth(H, W, seed=91, n_shapes=4)
    G = np.random.default_rng(92).normal(size=(H, W))
    ops = _ops()
    fa = _cuda(f)
    big = torch.empty(H * W + 1, device="cuda")
    fm = big[1:].view(H, W)
    fm.copy_(fa)
    assert fa.data_ptr() % 16 == 0 and fm.data_ptr() % 16 != 0
    grads = []
    for fx in (fa, fm):
        out, eta, aux = ops.trig_forward(fx, 255.0, sr, radii, return_aux=True, path=1)
        grads.append(ops.trig_backward(fx, out, eta, aux, _cuda(G), 255.0, sr, radii, path=1))
    torch.cuda.synchronize()
    g0, g1 = grads[0].cpu().numpy(), grads[1].cpu().numpy()
    scale = np.abs(g0).max()
    assert np.max(np.abs(g0 - g1)) <= 1e-4 * scale
    N = oracle.range_degree(255.0, sr)
    rng = np.random.default_rng(93)
    idx = list(rng.integers(0, H * W, 24)) + [0, W - 1, (H - 1) * W, H * W - 1, 64 * W + 64,
                                              63 * W + 127, 100 * W + 196]
    idx = np.array(idx, dtype=np.int64)
    ref = oracle.grad_at(f, sr, N, radii, G, idx)
    _check(g0.reshape(-1)[idx], ref, "global-g sampled")
    _check(g1.reshape(-1)[idx], ref, "LDS-g sampled")


@pytest.mark.parametrize("path", [1, 2], ids=["fused", "streamed"])
def test_backward_without_forward_sums(path):
    """The adjoint called with only (f, out, eta, grad_out), aux NULL: the
    library recomputes the forward's sums with the same evaluation, so the
    gradient equals the one computed from the forward's own sums bit for bit,
    and matches the oracle over the whole image."""
    ops = _ops()
    H, W, sr, radii = 70, 90, 25.0, [3, 3, 4]
    f_np = synth.piecewise_smooth(H, W, seed=41, n_shapes=3)
    G_np = np.random.default_rng(42).standard_normal((H, W)).astype(np.float32)
    f, G = _cuda(f_np), _cuda(G_np)
    out, eta, aux = ops.trig_forward(f, 255.0, sr, radii, return_aux=True, path=path)
    g_aux = ops.trig_backward(f, out, eta, aux, G, 255.0, sr, radii, path=path)
    g_none = ops.trig_backward(f, out, eta, None, G, 255.0, sr, radii, path=path)
    torch.cuda.synchronize()
    assert torch.equal(g_aux, g_none)
    N = oracle.range_degree(255.0, sr)
    ref = oracle.grad(f_np.astype(np.float64), sr, N, radii, G_np.astype(np.float64))
    _check(g_none.cpu().numpy(), ref, f"aux NULL {H}x{W} path {path}")
