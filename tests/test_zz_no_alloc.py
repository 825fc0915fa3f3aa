"""The allocation-free forward, bf_trig_forward_noalloc, called through the C
ABI: its streamed passes use the library's static 64 MiB device scratch.
Two calls in a row, the second on a smaller image, each equal bit for bit to
bf_trig_forward_ex given a caller workspace of the same 64 MiB (the same
chunks of pairs), and within the forward tolerance of the FP64 oracle
(|gpu - oracle| <= 1e-2 + 1e-4 |oracle|).  An image whose pair does not fit
the scratch falls back to the fused kernel (equal to it bit for bit), or is
rejected with BF_ERANGE when the streamed passes are forced."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1105_4204_amd import _native as nat
from paper_1105_4204_amd import synth

pytestmark = pytest.mark.gpu

SCRATCH = 64 << 20


def _ptr(x):
    return ctypes.c_void_p(x.data_ptr()) if x is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _noalloc(f, sr, radii, path=0, workspace=None):
    H, W = f.shape
    out, eta = torch.empty_like(f), torch.empty_like(f)
    spec = nat.SpatialSpec.of(radii)
    opts = nat.make_opts(_stream(), 0, _ptr(eta), path=path,
                         workspace=_ptr(workspace) if workspace is not None else None,
                         workspace_bytes=workspace.numel() if workspace is not None else 0)
    st = nat.lib().bf_trig_forward_noalloc(_ptr(f), H, W, 255.0, float(sr), ctypes.byref(spec),
                                           _ptr(out), ctypes.byref(opts))
    return st, out, eta


def _forward_ex(f, sr, radii, path, workspace=None):
    H, W = f.shape
    out, eta = torch.empty_like(f), torch.empty_like(f)
    spec = nat.SpatialSpec.of(radii)
    opts = nat.make_opts(_stream(), 0, _ptr(eta), path=path,
                         workspace=_ptr(workspace) if workspace is not None else None,
                         workspace_bytes=workspace.numel() if workspace is not None else 0)
    nat.check(nat.lib().bf_trig_forward_ex(_ptr(f), H, W, 255.0, float(sr), ctypes.byref(spec),
                                           _ptr(out), ctypes.byref(opts)), "bf_trig_forward_ex")
    return out, eta


def test_noalloc_two_calls_match_forward_ex_and_oracle():
    ws = torch.empty(SCRATCH, dtype=torch.uint8, device="cuda")
    cases = [(300, 280, 10.0, [29, 29, 30], 61),   # N = 264: pairs in several chunks
             (150, 130, 25.0, [40, 40, 41], 62)]   # smaller, after the first
    for H, W, sr, radii, seed in cases:
        print(f"case {H}x{W} sr={sr} radii={radii}", flush=True)
        f_np = synth.piecewise_smooth(H, W, seed=seed, n_shapes=3)
        f = torch.from_numpy(f_np).cuda()
        st, out, eta = _noalloc(f, sr, radii)
        assert st == 0, nat.lib().bf_last_error()
        ref_out, ref_eta = _forward_ex(f, sr, radii, 2, ws)
        torch.cuda.synchronize()
        assert torch.equal(out, ref_out)
        assert torch.equal(eta, ref_eta)
        N = oracle.range_degree(255.0, sr)
        idx = np.random.default_rng(seed).integers(0, H * W, size=400)
        idx = np.concatenate([idx, np.argsort(eta.cpu().numpy().reshape(-1))[:50]])
        ref = oracle.forward_at(f_np, sr, N, radii, idx)
        got = out.cpu().numpy().reshape(-1)[idx].astype(np.float64)
        err = np.abs(got - ref)
        print(f"  max_abs vs oracle {err.max():.3e}", flush=True)
        assert np.all(err <= 1e-2 + 1e-4 * np.abs(ref))


def test_noalloc_fallback_and_errors():
    # one pair of a 2048 x 2048 image needs 16 H Wp + 24 H W > 64 MiB: the
    # fused kernel (radii <= 31) runs instead
    f = torch.from_numpy(synth.config_image(2)).cuda()
    st, out, eta = _noalloc(f, 20.0, [9, 9, 10])
    assert st == 0, nat.lib().bf_last_error()
    ref_out, ref_eta = _forward_ex(f, 20.0, [9, 9, 10], 1)
    torch.cuda.synchronize()
    assert torch.equal(out, ref_out) and torch.equal(eta, ref_eta)
    st, _, _ = _noalloc(f, 20.0, [9, 9, 10], path=2)          # streamed forced
    assert st == 2 and b"static scratch" in nat.lib().bf_last_error()
    st, _, _ = _noalloc(f, 20.0, [29, 29, 30])                 # neither fits
    assert st == 2
    small = torch.from_numpy(synth.piecewise_smooth(40, 40, seed=3)).cuda()
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    st, _, _ = _noalloc(small, 20.0, [9, 9, 10], workspace=ws)
    assert st == 1
    torch.cuda.synchronize()
