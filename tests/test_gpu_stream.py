"""GPU parity of the streamed passes (whole-line column and row passes whose
cost does not depend on the kernel width) against the FP64 oracle.

Forward: small images pixel by pixel, across box counts, radii up to 150 per
box, odd and even degrees, several pair chunks and column segments; the
4096x4096, sigma_s = 30 (boxes 29, 29, 30), sigma_r = 10 (N = 264) workload
and a 2048x2048 image at sigma_s = 100 on sampled pixels.  Tolerance as for
the fused forward: |gpu - oracle| <= 1e-2 + 1e-4 |oracle| per pixel.
Adjoint: kernels the fused tiles cannot hold, every pixel against the
oracle's exact gradient, tolerance 1e-3 max|g_ref| + 1e-3 |g_ref|."""
import numpy as np
import pytest
import torch

import oracle
from paper_1105_4204_amd import synth

pytestmark = pytest.mark.gpu

STREAMED = 2


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
    # H, W, sigma_r, N (0 = automatic), radii
    (150, 170, 30.0, 0, [25, 25, 25]),      # R = 75, N = 30
    (131, 97, 25.0, 0, [20, 22, 24]),       # R = 66, odd N = 43
    (70, 300, 20.0, 0, [31, 31, 31]),       # R = 93, taller kernel than the image
    (1, 90, 40.0, 0, [30, 30, 10]),         # single row
    (90, 1, 40.0, 0, [3, 30, 10]),          # single column
    (40, 40, 12.0, 0, [31, 20, 20]),        # N = 184, image smaller than the halo
    (100, 261, 25.0, 0, [21, 21, 22]),      # W not a multiple of 4
    (96, 80, 20.0, 0, [2, 2, 3]),           # narrow kernel through the streamed path
    (77, 64, 30.0, 0, [5]),                 # one box
    (64, 77, 30.0, 0, [4, 9]),              # two boxes
    (70, 66, 30.0, 0, [3, 5, 7, 9]),        # four boxes (merged taps +-2)
    (80, 72, 20.0, 0, [50, 50, 51]),        # R = 151
    (120, 90, 60.0, 0, [100, 100, 100]),    # R = 300, equal radii (four taps)
    (64, 64, 20.0, 67, [7, 0, 7]),          # explicit odd N, a zero radius
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-r{c[4]}" for c in CASES])
def test_stream_small_full_parity(case):
    H, W, sr, N, radii = case
    print(f"case {case}", flush=True)
    f = synth.piecewise_smooth(H, W, seed=H * 3 + W, n_shapes=3)
    Nuse = N or oracle.range_degree(255.0, sr)
    ref, eta_ref = oracle.forward(f, sr, Nuse, radii, return_eta=True)
    out, eta = _ops().trig_forward(_cuda(f), 255.0, sr, radii, N=N, return_eta=True,
                                   path=STREAMED)
    torch.cuda.synchronize()
    _check(out.cpu().numpy(), ref, f"streamed {case}")
    e = eta.cpu().numpy().astype(np.float64)
    assert np.allclose(e, eta_ref, rtol=2e-4, atol=1e-4 * eta_ref.max()), case


def test_stream_salt_tiny_eta():
    """Isolated 0/255 outliers on a mid-grey field: eta at the outliers falls
    towards w(0), where the expansion cancels most."""
    f = synth.salt(96, 112, seed=5)
    radii, sr = [15, 15, 16], 12.0
    N = oracle.range_degree(255.0, sr)
    ref = oracle.forward(f, sr, N, radii)
    out = _ops().trig_forward(_cuda(f), 255.0, sr, radii, path=STREAMED)
    torch.cuda.synchronize()
    _check(out.cpu().numpy(), ref, "streamed salt")


def test_stream_chunks_match_one_chunk():
    """A workspace for one or three pairs (many chunks, den and num carried
    between them) gives the result of the recommended workspace to float
    rounding of the partial sums, and both match the oracle."""
    from paper_1105_4204_amd import _native as nat
    H, W, sr, radii = 73, 130, 15.0, [12, 12, 13]
    f = synth.piecewise_smooth(H, W, seed=9, n_shapes=3)
    N = oracle.range_degree(255.0, sr)
    ref = oracle.forward(f, sr, N, radii)
    fd = _cuda(f)
    full = _ops().trig_forward(fd, 255.0, sr, radii, path=STREAMED)
    for pairs in (1, 3):
        ws = torch.empty(nat.stream_workspace_bytes(H, W, pairs), dtype=torch.uint8,
                         device="cuda")
        got = _ops().trig_forward(fd, 255.0, sr, radii, path=STREAMED, workspace=ws)
        torch.cuda.synchronize()
        _check(got.cpu().numpy(), ref, f"streamed, {pairs}-pair chunks")
        d = np.abs(got.cpu().numpy() - full.cpu().numpy()).max()
        assert d < 2e-3, (pairs, d)


def test_stream_matches_fused_where_both_run():
    """Both evaluations of the same eq. (final-form) on a kernel the fused
    tiles hold: equal to well inside the oracle tolerance."""
    f = synth.piecewise_smooth(200, 230, seed=4, n_shapes=4)
    fd = _cuda(f)
    radii, sr = [9, 9, 10], 20.0
    a = _ops().trig_forward(fd, 255.0, sr, radii, path=1)
    b = _ops().trig_forward(fd, 255.0, sr, radii, path=STREAMED)
    torch.cuda.synchronize()
    d = np.abs(a.cpu().numpy() - b.cpu().numpy()).max()
    print(f"fused vs streamed: {d:.3e}", flush=True)
    assert d < 5e-3


def test_stream_deterministic_and_library_workspace():
    """The C call without opts (library workspace) equals the torch-workspace
    call bit for bit, and repeated calls are bit-identical."""
    import ctypes
    from paper_1105_4204_amd import _native as nat
    H, W = 150, 140
    f = _cuda(synth.piecewise_smooth(H, W, seed=12, n_shapes=3))
    radii = [40, 40, 41]
    a = _ops().trig_forward(f, 255.0, 20.0, radii)
    out = torch.empty_like(f)
    spec = nat.SpatialSpec.of(radii)
    torch.cuda.synchronize()
    nat.check(nat.lib().bf_trig_forward(ctypes.c_void_p(f.data_ptr()), H, W, 255.0, 20.0,
                                        ctypes.byref(spec), ctypes.c_void_p(out.data_ptr())),
              "bf_trig_forward")
    torch.cuda.synchronize()   # the call ran on the null stream
    b = _ops().trig_forward(f, 255.0, 20.0, radii)
    torch.cuda.synchronize()
    assert torch.equal(a, out)
    assert torch.equal(a, b)


def test_stream_aux_and_eta_match_fused():
    """The adjoint's sums P, Q and eta from the streamed passes equal the fused
    kernel's to float rounding (both evaluate the same expansion)."""
    H, W, sr, radii = 150, 140, 20.0, [9, 9, 10]
    f = _cuda(synth.piecewise_smooth(H, W, seed=31, n_shapes=4))
    a = _ops().trig_forward(f, 255.0, sr, radii, return_aux=True, path=1)
    b = _ops().trig_forward(f, 255.0, sr, radii, return_aux=True, path=STREAMED)
    torch.cuda.synchronize()
    for k, name in ((0, "out"), (1, "eta"), (2, "aux")):
        x, y = a[k].cpu().numpy().astype(np.float64), b[k].cpu().numpy().astype(np.float64)
        rel = np.abs(x - y).max() / np.abs(x).max()
        print(f"{name}: max rel {rel:.3e}", flush=True)
        assert rel < 2e-5, name


def _grad_check(g, ref, what):
    g = np.asarray(g, dtype=np.float64)
    scale = np.abs(ref).max()
    err = np.abs(g - ref)
    tol = 1e-3 * scale + 1e-3 * np.abs(ref)
    bad = int((err > tol).sum())
    print(f"{what}: max_abs={err.max():.3e} scale={scale:.3e} bad={bad}/{err.size}", flush=True)
    assert np.all(np.isfinite(g)), what
    assert bad == 0, what


ADJ_CASES = [
    (40, 46, 25.0, 0, [20, 22, 24]),     # R = 66, odd N = 43
    (34, 30, 20.0, 0, [50, 50, 51]),     # R = 151, kernel wider than the image
    (1, 60, 30.0, 0, [30, 30, 10]),      # single row
    (36, 28, 12.0, 0, [31, 20, 20]),     # N = 184
    (30, 33, 30.0, 0, [3, 5, 7, 9]),     # four boxes
]


@pytest.mark.parametrize("case", ADJ_CASES, ids=[f"{c[0]}x{c[1]}-r{c[4]}" for c in ADJ_CASES])
def test_stream_adjoint_wide_full_parity(case):
    """The streamed adjoint on kernels the fused tiles cannot hold (R > 63 or
    a radius above 31), against the oracle's exact gradient at every pixel,
    with the adjoint's sums from the streamed forward (the library's choice)."""
    H, W, sr, N, radii = case
    print(f"case {case}", flush=True)
    f = synth.piecewise_smooth(H, W, seed=H + 5 * W, n_shapes=3)
    G = np.random.default_rng(H * W + 1).normal(size=(H, W))
    Nuse = N or oracle.range_degree(255.0, sr)
    ref = oracle.grad(f, sr, Nuse, radii, G)
    fg = _cuda(f)
    out, eta, aux = _ops().trig_forward(fg, 255.0, sr, radii, N=N, return_aux=True)
    gf = _ops().trig_backward(fg, out, eta, aux, _cuda(G), 255.0, sr, radii, N=N)
    torch.cuda.synchronize()
    _grad_check(gf.cpu().numpy(), ref, f"streamed adjoint {case}")


# Three boxes, at pair counts (N // 2 + 1 = 4 .. 34) that give every group size
# of the column pass: forward 4 to 8, adjoint 4 to 7, one or several groups
# per column (pairs: group size forward / adjoint):
# 4: 4/4, 5: 5/5, 6: 6/6, 7: 7/7, 8: 8/4 (two groups), 9: 5/5 (two),
# 13: 7/7 (two), 16: 8/6 (two / three), 24: 8/6, 34: 7/7 (five).
GROUP_N = [6, 8, 10, 12, 14, 16, 24, 30, 46, 66]
GROUP_N_ADJ = [6, 8, 10, 12, 24, 30]


@pytest.mark.parametrize("N", GROUP_N)
def test_three_box_group_sizes_forward(N):
    """Every pixel against the oracle at each group size of the forward
    column pass (sigma_r 120: these degrees are all valid)."""
    H, W, sr, radii = 37, 70, 120.0, [4, 4, 5]
    print(f"N {N}", flush=True)
    f = synth.piecewise_smooth(H, W, seed=N + 11, n_shapes=3)
    ref, eta_ref = oracle.forward(f, sr, N, radii, return_eta=True)
    out, eta = _ops().trig_forward(_cuda(f), 255.0, sr, radii, N=N, return_eta=True,
                                   path=STREAMED)
    torch.cuda.synchronize()
    _check(out.cpu().numpy(), ref, f"group sizes, N {N}")
    e = eta.cpu().numpy().astype(np.float64)
    assert np.allclose(e, eta_ref, rtol=2e-4, atol=1e-4 * eta_ref.max()), N


@pytest.mark.parametrize("N", GROUP_N_ADJ)
def test_three_box_group_sizes_adjoint(N):
    """Every pixel of the adjoint against the oracle's exact gradient at each
    group size of the adjoint column pass."""
    H, W, sr, radii = 24, 40, 120.0, [4, 4, 5]
    print(f"N {N}", flush=True)
    f = synth.piecewise_smooth(H, W, seed=N + 13, n_shapes=3)
    G = np.random.default_rng(N).normal(size=(H, W))
    ref = oracle.grad(f, sr, N, radii, G)
    fg = _cuda(f)
    out, eta, aux = _ops().trig_forward(fg, 255.0, sr, radii, N=N, return_aux=True,
                                        path=STREAMED)
    gf = _ops().trig_backward(fg, out, eta, aux, _cuda(G), 255.0, sr, radii, N=N, path=STREAMED)
    torch.cuda.synchronize()
    _grad_check(gf.cpu().numpy(), ref, f"group sizes adjoint, N {N}")


def test_stream_adjoint_chunks():
    """The streamed adjoint and the forward's sums with one-pair chunks (the
    partial sums carried between chunks) against the recommended workspace."""
    from paper_1105_4204_amd import _native as nat
    H, W, sr, radii = 61, 70, 15.0, [12, 12, 13]
    f = _cuda(synth.piecewise_smooth(H, W, seed=19, n_shapes=3))
    G = torch.from_numpy(np.random.default_rng(20).normal(size=(H, W)).astype(np.float32)).cuda()
    ws = torch.empty(nat.stream_workspace_bytes(H, W, 1), dtype=torch.uint8, device="cuda")
    o1, e1, x1 = _ops().trig_forward(f, 255.0, sr, radii, return_aux=True, path=STREAMED)
    o2, e2, x2 = _ops().trig_forward(f, 255.0, sr, radii, return_aux=True, path=STREAMED,
                                     workspace=ws)
    g1 = _ops().trig_backward(f, o1, e1, x1, G, 255.0, sr, radii, path=STREAMED)
    g2 = _ops().trig_backward(f, o1, e1, x1, G, 255.0, sr, radii, path=STREAMED, workspace=ws)
    torch.cuda.synchronize()
    for a, b, name in ((x1, x2, "aux"), (g1, g2, "grad")):
        rel = (a - b).abs().max().item() / a.abs().max().item()
        print(f"{name}: chunked vs one chunk, max rel {rel:.3e}", flush=True)
        assert rel < 1e-5, name


def _sampled(f_np, sr, N, radii, out, eta, what, seed, nrand=65536):
    o = out.cpu().numpy().reshape(-1)
    e = eta.cpu().numpy().reshape(-1)
    rng = np.random.default_rng(seed)
    H, W = f_np.shape
    R = sum(radii)
    c0, r0 = int(rng.integers(0, W - 64)), int(rng.integers(0, H - 64))
    top = [i * W + j for i in range(min(R + 1, H)) for j in range(c0, c0 + 64)]
    left = [i * W + j for i in range(r0, r0 + 64) for j in range(min(R + 1, W))]
    idx = np.unique(np.concatenate([rng.integers(0, H * W, size=nrand), np.argsort(e)[:1000],
                                    np.array(top + left + [0, W - 1, (H - 1) * W, H * W - 1])]))
    ref = oracle.forward_at(f_np, sr, N, radii, idx)
    _check(o[idx], ref, what)


def test_wide_kernel_workload_sampled():
    """4096 x 4096 piecewise-smooth image (seed 3), sigma_s = 30 realised as
    boxes (29, 29, 30), sigma_r = 10, N = 264, through the library's choice
    (the streamed passes): 65536 random pixels, the 1000 pixels of smallest
    eta, every pixel within R of the border on a 64-pixel stretch of the top
    and of the left edge, and the four corners, against the oracle."""
    from paper_1105_4204_amd import _native as nat
    f_np = synth.config_image(3)
    radii = nat.spatial_gaussian(30.0, 3)
    assert radii == [29, 29, 30]
    N = oracle.range_degree(255.0, 10.0)
    assert N == 264
    out, eta = _ops().trig_forward(_cuda(f_np), 255.0, 10.0, radii, return_eta=True)
    torch.cuda.synchronize()
    _sampled(f_np, 10.0, N, radii, out, eta, "4096^2 sigma_s=30 N=264 sampled", 33)


def test_sigma_s_100_sampled():
    """2048 x 2048 (seed 2), sigma_s = 100 as boxes (99, 99, 100), R = 298,
    sigma_r = 20 (N = 66): the same sampling with 8192 random pixels (each
    oracle pixel sums a 599 x 599 window)."""
    from paper_1105_4204_amd import _native as nat
    f_np = synth.config_image(2)
    radii = nat.spatial_gaussian(100.0, 3)
    assert radii == [99, 99, 100], radii
    N = oracle.range_degree(255.0, 20.0)
    out, eta = _ops().trig_forward(_cuda(f_np), 255.0, 20.0, radii, return_eta=True)
    torch.cuda.synchronize()
    _sampled(f_np, 20.0, N, radii, out, eta, "2048^2 sigma_s=100 N=66 sampled", 34, 8192)


def test_four_boxes_many_pairs_in_one_chunk():
    """Four boxes (three pairs per column-pass group) with more than 192 pairs
    in one chunk: 68 groups, beyond the 64 the argument table once held."""
    from paper_1105_4204_amd import ops
    H, W, sr, N, radii = 24, 40, 8.0, 420, [1, 1, 2, 2]
    f = synth.piecewise_smooth(H, W, seed=424, n_shapes=3)
    print(f"case {H}x{W} N={N} radii={radii}", flush=True)
    ref = oracle.forward(f, sr, N, radii)
    out = ops.trig_forward(torch.from_numpy(f).cuda(), 255.0, sr, radii, N=N, path=2)
    torch.cuda.synchronize()
    err = np.abs(out.cpu().numpy().astype(np.float64) - ref)
    print(f"max_abs {err.max():.3e}", flush=True)
    assert np.all(err <= 1e-2 + 1e-4 * np.abs(ref))


def test_stream_forward_and_adjoint_captured_in_a_graph():
    """The streamed forward (with eta and the adjoint's sums) and adjoint,
    given a caller workspace, allocate and synchronise nothing: captured into
    a HIP graph and replayed three times, with eager work on the outputs
    between replays, they reproduce the eager results bit for bit."""
    from paper_1105_4204_amd import _native as nat
    from paper_1105_4204_amd import ops
    H, W, sr, radii = 150, 230, 20.0, [4, 4, 5]
    f = torch.from_numpy(synth.piecewise_smooth(H, W, seed=808, n_shapes=4)).cuda()
    G = torch.randn(H, W, device="cuda", generator=torch.Generator("cuda").manual_seed(9))
    nws = nat.stream_workspace_bytes(H, W, 8)          # several chunks
    ws = torch.empty(nws, dtype=torch.uint8, device="cuda")
    kw = dict(path=2, workspace=ws)
    o1, e1, x1 = ops.trig_forward(f, 255.0, sr, radii, return_aux=True, **kw)
    g1 = ops.trig_backward(f, o1, e1, x1, G, 255.0, sr, radii, **kw)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):       # warm-up off the capture stream
        ops.trig_forward(f, 255.0, sr, radii, return_aux=True, **kw)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        o, e, x = ops.trig_forward(f, 255.0, sr, radii, return_aux=True, **kw)
        g = ops.trig_backward(f, o, e, x, G, 255.0, sr, radii, **kw)
    for rep in range(3):
        for t in (o, e, x, g):
            t.fill_(-1.0)
        graph.replay()
        torch.cuda.synchronize()
        print(f"replay {rep}", flush=True)
        assert torch.equal(o, o1) and torch.equal(e, e1), rep
        assert torch.equal(x, x1) and torch.equal(g, g1), rep
