"""PyTorch-facing calls of the trigonometric bilateral filter.

PyTorch supplies device memory and the current HIP stream; every value is
computed by the HIP kernels of libbftrig.so through the C ABI (see
``_native``).  Inputs must be contiguous float32 CUDA (HIP) tensors.
"""
from __future__ import annotations

import ctypes

import torch

from . import _native as nat


def _stream_ptr():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_img(x: torch.Tensor, name: str):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP tensor")
    if x.dtype != torch.float32 or x.dim() != 2 or not x.is_contiguous():
        raise TypeError(f"{name} must be a contiguous 2-D float32 tensor, got "
                        f"{x.dtype} {tuple(x.shape)}")


def _ptr(x):
    return ctypes.c_void_p(x.data_ptr()) if x is not None else None


def _stream_workspace(f, H, W, T, sigma_r, radii, N, path, tile, workspace):
    """(tensor, bytes) of the streamed passes' workspace: the caller's, else
    one of the size the library recommends for this degree from torch's
    allocator (none where the fused kernel runs)."""
    if tile is not None or path == nat.PATH_FUSED:
        return None, 0
    if workspace is not None:
        return workspace, workspace.numel() * workspace.element_size()
    if path == nat.PATH_AUTO:
        nws = nat.workspace_bytes_ex(H, W, T, sigma_r, N, radii)
    else:
        n = N or nat.range_degree(T, sigma_r)
        nws = nat.stream_workspace_bytes(H, W, min(n // 2 + 1, 256))
    if not nws:
        return None, 0
    return torch.empty(nws, device=f.device, dtype=torch.uint8), nws


def trig_forward(f: torch.Tensor, T: float, sigma_r: float, radii, N: int = 0,
                 return_eta: bool = False, tile=None, out: torch.Tensor | None = None,
                 return_aux: bool = False, trunc_tol: float = 0.0, path: int = nat.PATH_AUTO,
                 workspace: torch.Tensor | None = None):
    """O(1) raised-cosine bilateral filter of a 2-D image: the fused tile
    kernel, or the streamed whole-line passes (the library's choice unless
    `path` forces one).  The streamed passes' workspace comes from torch's
    allocator (`workspace`, else a fresh buffer of the recommended size).

    Returns out, or (out, eta) with return_eta, or (out, eta, aux) with
    return_aux, where aux (2 x H x W) holds the sums the backward needs."""
    _check_img(f, "f")
    H, W = f.shape
    out = torch.empty_like(f) if out is None else out
    eta = torch.empty_like(f) if (return_eta or return_aux) else None
    aux = torch.empty((2, H, W), device=f.device, dtype=f.dtype) if return_aux else None
    spec = nat.SpatialSpec.of(radii)
    ws, nws = _stream_workspace(f, H, W, T, sigma_r, radii, N, path, tile, workspace)
    opts = nat.make_opts(_stream_ptr(), N, _ptr(eta), tile, _ptr(aux), _ptr(ws), nws, trunc_tol,
                         path)
    nat.check(nat.lib().bf_trig_forward_ex(_ptr(f), H, W, float(T), float(sigma_r),
                                           ctypes.byref(spec), _ptr(out), ctypes.byref(opts)),
              "bf_trig_forward_ex")
    if return_aux:
        return out, eta, aux
    return (out, eta) if return_eta else out


def check_range(f: torch.Tensor, T: float) -> int:
    """Number of pixels of f outside [0, T] or NaN (the input precondition of
    the filter, which the kernels do not test); synchronises the stream."""
    _check_img(f, "f")
    H, W = f.shape
    count = torch.empty(1, dtype=torch.int32, device=f.device)
    nat.check(nat.lib().bf_check_range(_ptr(f), H, W, float(T), _ptr(count), _stream_ptr()),
              "bf_check_range")
    return int(count.item()) & 0xFFFFFFFF


def direct_forward(f: torch.Tensor, T: float, sigma_r: float, radii, N: int = 0,
                   return_eta: bool = False):
    """Direct-window (O((2R+1)^2) per pixel) filter on the GPU."""
    _check_img(f, "f")
    H, W = f.shape
    out = torch.empty_like(f)
    eta = torch.empty_like(f) if return_eta else None
    spec = nat.SpatialSpec.of(radii)
    opts = nat.make_opts(_stream_ptr(), N, _ptr(eta))
    nat.check(nat.lib().bf_direct_forward(_ptr(f), H, W, float(T), float(sigma_r),
                                          ctypes.byref(spec), _ptr(out), ctypes.byref(opts)),
              "bf_direct_forward")
    return (out, eta) if return_eta else out


def sv_forward(f: torch.Tensor, radius: torch.Tensor, T: float, sigma_r: float,
               rmax: int | None = None, N: int = 0, trunc_tol: float = 0.0,
               return_eta: bool = False):
    """Space-variant filter: unit box of half-width radius[i, j] (int32, clamped
    to [0, rmax]) around each pixel, fixed raised-cosine range kernel.  rmax
    defaults to radius.max() (one device-to-host read)."""
    _check_img(f, "f")
    H, W = f.shape
    if (not isinstance(radius, torch.Tensor) or not radius.is_cuda
            or radius.dtype != torch.int32 or tuple(radius.shape) != (H, W)
            or not radius.is_contiguous()):
        raise TypeError("radius must be a contiguous H x W int32 CUDA tensor")
    if rmax is None:
        rmax = int(radius.max().item())
    out = torch.empty_like(f)
    eta = torch.empty_like(f) if return_eta else None
    opts = nat.make_opts(_stream_ptr(), N, _ptr(eta), trunc_tol=trunc_tol)
    nat.check(nat.lib().bf_sv_forward(_ptr(f), _ptr(radius), H, W, float(T), float(sigma_r),
                                      int(rmax), _ptr(out), ctypes.byref(opts)),
              "bf_sv_forward")
    return (out, eta) if return_eta else out


def yvv_forward(f: torch.Tensor, T: float, sigma_r: float, sigma_s: float, N: int = 0,
                trunc_tol: float = 0.0, return_eta: bool = False,
                workspace: torch.Tensor | None = None):
    """Forward filter with the recursive Gaussian spatial kernel (Young and
    van Vliet) of standard deviation sigma_s, over whole image lines.  The
    workspace (bf_yvv_workspace_bytes) is allocated here unless given."""
    _check_img(f, "f")
    H, W = f.shape
    need = nat.yvv_workspace_bytes(H, W, T, sigma_r, N)
    if workspace is None:
        workspace = torch.empty((need + 3) // 4, dtype=torch.float32, device=f.device)
    out = torch.empty_like(f)
    eta = torch.empty_like(f) if return_eta else None
    opts = nat.make_opts(_stream_ptr(), N, _ptr(eta), workspace=_ptr(workspace),
                         workspace_bytes=workspace.numel() * workspace.element_size(),
                         trunc_tol=trunc_tol)
    nat.check(nat.lib().bf_yvv_forward(_ptr(f), H, W, float(T), float(sigma_r), float(sigma_s),
                                       _ptr(out), ctypes.byref(opts)),
              "bf_yvv_forward")
    return (out, eta) if return_eta else out


def trig_backward(f, out, eta, aux, grad_out, T: float, sigma_r: float, radii, N: int = 0,
                  tile=None, trunc_tol: float = 0.0, path: int = nat.PATH_AUTO,
                  workspace: torch.Tensor | None = None):
    """grad_f = J^T grad_out for the forward that produced (out, eta, aux):
    the fused adjoint tiles or the streamed passes, as for the forward.  With
    aux None the library recomputes the forward's sums itself (one more
    forward, in its own workspace)."""
    for x, n in ((f, "f"), (out, "out"), (eta, "eta"), (grad_out, "grad_out")):
        _check_img(x, n)
    H, W = f.shape
    if aux is not None and (not isinstance(aux, torch.Tensor) or not aux.is_cuda
                            or aux.dtype != torch.float32 or tuple(aux.shape) != (2, H, W)
                            or not aux.is_contiguous()):
        raise TypeError("aux must be the contiguous 2 x H x W float32 tensor of the forward")
    gf = torch.empty_like(f)
    spec = nat.SpatialSpec.of(radii)
    ws, nws = _stream_workspace(f, H, W, T, sigma_r, radii, N, path, tile, workspace)
    opts = nat.make_opts(_stream_ptr(), N, None, tile, None, _ptr(ws), nws, trunc_tol, path)
    nat.check(nat.lib().bf_trig_backward(_ptr(f), _ptr(out), _ptr(eta), _ptr(aux),
                                         _ptr(grad_out), H, W, float(T), float(sigma_r),
                                         ctypes.byref(spec), _ptr(gf), ctypes.byref(opts)),
              "bf_trig_backward")
    return gf


class BFTrig(torch.autograd.Function):
    """Autograd wrapper: forward saves (f, out, eta, aux); backward calls the
    hand-written adjoint kernel.  T, sigma_r, radii and N are constants."""

    @staticmethod
    def forward(ctx, f, T, sigma_r, radii, N, trunc_tol):
        f = f.contiguous()
        if ctx.needs_input_grad[0]:
            out, eta, aux = trig_forward(f, T, sigma_r, radii, N, return_aux=True,
                                         trunc_tol=trunc_tol)
            ctx.save_for_backward(f, out, eta, aux)
        else:
            out = trig_forward(f, T, sigma_r, radii, N, trunc_tol=trunc_tol)
        ctx.params = (T, sigma_r, tuple(radii), N, trunc_tol)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        f, out, eta, aux = ctx.saved_tensors
        T, sigma_r, radii, N, trunc_tol = ctx.params
        gf = trig_backward(f, out, eta, aux, grad_out.contiguous(), T, sigma_r, radii, N,
                           trunc_tol=trunc_tol)
        return gf, None, None, None, None, None


def bf_trig(f: torch.Tensor, T: float = 255.0, sigma_r: float = 30.0, radii=(5,), N: int = 0,
            trunc_tol: float = 0.0):
    """Differentiable O(1) bilateral filter of a 2-D float32 image (trunc_tol > 0:
    drop outer cosine pairs within that many gray levels, bf_range_truncate)."""
    return BFTrig.apply(f, float(T), float(sigma_r), tuple(int(r) for r in radii), int(N),
                        float(trunc_tol))
