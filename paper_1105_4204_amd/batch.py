"""Batched persistent launch over many images of different sizes and
parameters (C ABI bf_batch_*), capturable into a HIP graph.

``BatchPlan(specs)`` fixes sizes and parameters; ``bind`` attaches torch
tensors (allocated by the caller or by ``allocate``); ``launch`` enqueues the
forward, per-image SSD loss and adjoint of every image as one persistent
kernel on the current stream.  All arithmetic runs in libbftrig.
"""
from __future__ import annotations

import ctypes

import torch

from . import _native as nat


def _spec_desc(s) -> nat.ImageDesc:
    d = nat.ImageDesc()
    d.H, d.W = int(s["H"]), int(s["W"])
    d.T = float(s.get("T", 255.0))
    d.sigma_r = float(s["sigma_r"])
    d.N = int(s.get("N", 0))
    radii = s.get("radii")
    if radii is None:
        radii = nat.spatial_gaussian(float(s["sigma_s"]), int(s.get("n_boxes", 3)))
    d.spatial = nat.SpatialSpec.of(radii)
    th, tw = s.get("tile") or (0, 0)
    bh, bw = s.get("bwd_tile") or (0, 0)
    d.tile_h, d.tile_w, d.bwd_tile_h, d.bwd_tile_w = int(th), int(tw), int(bh), int(bw)
    d.trunc_tol = float(s.get("trunc_tol", 0.0))
    return d


class BatchPlan:
    """A plan for one fixed list of images; see include/bf_trig.h."""

    def __init__(self, specs, tuner=None, path=nat.PATH_AUTO):
        """path: PATH_AUTO (the streamed passes when every image is within
        their limits, else the persistent fused-tile kernel), PATH_FUSED or
        PATH_STREAMED.  The tuner's tiles apply to the fused kernel only."""
        specs = [dict(s) for s in specs]
        if tuner is not None:
            for s in specs:
                s.setdefault("tile", tuner.tile_for(s, "fwd"))
                s.setdefault("bwd_tile", tuner.tile_for(s, "bwd"))
        self.specs = specs
        arr = (nat.ImageDesc * len(specs))(*[_spec_desc(s) for s in specs])
        self._descs = arr
        h = ctypes.c_void_p()
        nat.check(nat.lib().bf_batch_plan_create_ex(arr, len(specs), int(path), ctypes.byref(h)),
                  "bf_batch_plan_create_ex")
        self.path = path
        self._h = h
        self._bound = None

    def __len__(self):
        return len(self.specs)

    def allocate(self, device="cuda", backward=True):
        """Output tensors matching the plan (out, eta, grad_f, loss)."""
        out = [torch.empty(s["H"], s["W"], device=device) for s in self.specs]
        eta = [torch.empty_like(o) for o in out]
        gf = [torch.empty_like(o) for o in out] if backward else None
        loss = torch.empty(len(self.specs), device=device)
        return out, eta, gf, loss

    def bind(self, f, target=None, out=None, eta=None, grad_f=None, loss=None):
        n = len(self.specs)

        def arr(xs, name, required):
            if xs is None:
                if required:
                    raise ValueError(f"{name} is required")
                return None
            if len(xs) != n:
                raise ValueError(f"{name}: expected {n} tensors")
            for x, s in zip(xs, self.specs):
                if (not x.is_cuda or x.dtype != torch.float32 or not x.is_contiguous()
                        or tuple(x.shape) != (s["H"], s["W"])):
                    raise TypeError(f"{name}: need contiguous float32 CUDA tensors of the "
                                    "planned shapes")
            return (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])

        pf = arr(f, "f", True)
        pt = arr(target, "target", False)
        po = arr(out, "out", True)
        pe = arr(eta, "eta", False)
        pg = arr(grad_f, "grad_f", False)
        ploss = ctypes.c_void_p(loss.data_ptr()) if loss is not None else None
        nat.check(nat.lib().bf_batch_bind(self._h, pf, pt, po, pe, pg, ploss), "bf_batch_bind")
        # keep the tensors alive while bound
        self._bound = (f, target, out, eta, grad_f, loss)

    def launch(self, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream()
        nat.check(nat.lib().bf_batch_launch(self._h, ctypes.c_void_p(s.cuda_stream)),
                  "bf_batch_launch")

    def launch_stage(self, stage: int, stream=None):
        """One stage of launch() (bf_batch_launch_stage), for per-stage timing."""
        s = stream if stream is not None else torch.cuda.current_stream()
        nat.check(nat.lib().bf_batch_launch_stage(self._h, int(stage),
                                                  ctypes.c_void_p(s.cuda_stream)),
                  "bf_batch_launch_stage")

    def streamed(self) -> bool:
        """Whether the plan runs the streamed passes (else the fused tiles)."""
        return nat.lib().bf_batch_plan_path(self._h) == nat.PATH_STREAMED

    def check(self):
        nat.check(nat.lib().bf_batch_check(self._h), "bf_batch_check")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            nat.lib().bf_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def capture(plan: BatchPlan, warmup: int = 1) -> torch.cuda.CUDAGraph:
    """Capture plan.launch() into a graph (after `warmup` eager launches)."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(warmup):
            plan.launch(s)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch()
    return g


def trig_forward_channels(img: torch.Tensor, T: float, sigma_r: float, radii, N: int = 0,
                          trunc_tol: float = 0.0, path: int = nat.PATH_AUTO) -> torch.Tensor:
    """Channel-wise filter of a C x H x W image (e.g. RGB, each channel filtered
    on its own as in the paper's colour experiments), run as the C items of one
    batched launch (`path` as for BatchPlan).  Returns a C x H x W tensor;
    synchronises the current stream before it returns (the plan is released)."""
    if img.dim() != 3 or not img.is_cuda or img.dtype != torch.float32:
        raise TypeError("img must be a C x H x W float32 CUDA tensor")
    img = img.contiguous()
    C, H, W = img.shape
    spec = dict(H=H, W=W, T=float(T), sigma_r=float(sigma_r), N=int(N),
                radii=[int(r) for r in radii], trunc_tol=float(trunc_tol))
    plan = BatchPlan([spec] * C, path=path)
    out = torch.empty_like(img)
    plan.bind([img[c] for c in range(C)], out=[out[c] for c in range(C)])
    plan.launch()
    torch.cuda.current_stream().synchronize()   # the plan's tables outlive the launch
    plan.close()
    return out
