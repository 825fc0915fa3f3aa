#!/usr/bin/env python3
"""Benchmark of the O(1) trigonometric bilateral filter on one MI355X.

One step = one pass of the whole hot path over one batch of synthetic input.
Default (headline) workload: the ragged batch of 256 float32 images (H, W ~
U{64..1024}, sigma_s ~ U[2,16] as three boxes, sigma_r ~ U[10,60], each image
with its own degree N), forward + per-image SSD loss + adjoint, one persistent
kernel replayed from a HIP graph with autotuned tiles.  `value` is that step's
Mpixel/s (forward+backward).

The same JSON line carries the single-image workloads as extras: 256^2 box
r = 5 forward; 2048^2 sigma_s = 10, sigma_r = 20 (N = 66) forward and
forward+backward with the direct-window GPU filter beside it; 16 x 512^2
forward+backward; 4096^2 sigma_s = 30, sigma_r = 10 (N = 264) forward; a
sigma_s sweep at fixed N; the recursive-Gaussian and space-variant kernels.
Every timed kernel's time comes from HIP events on its launch stream; the
roofline of the headline's kernel (and of the extras' dominant kernels) uses
the algorithmic operation counts per pixel; the FP64 oracle is timed on the
host cores over a bounded sample of the headline workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X vector FP32 (FMA = 2 flops)
PEAK_HBM_GBS = 8000.0         # MI355X HBM3E

METRIC = "Megapixels/s fwd and fwd+bwd at stated N vs direct GPU filter; % HBM peak"

BATCH_DESC = ("256 ragged f32 images, H,W~U{64..1024}, sigma_s~U[2,16] (3 boxes), "
              "sigma_r~U[10,60] (per-image N), same piecewise-smooth generator; forward + "
              "per-image SSD loss + backward in one persistent kernel replayed from a HIP "
              "graph, autotuned tiles")

WORKLOADS = {
    "config2": dict(H=2048, W=2048, sigma_s=10.0, sigma_r=20.0, gen="smooth", seed=2,
                    desc="2048x2048 f32 piecewise-smooth (discs+rectangles, ramps, N(0,15^2) noise), "
                         "sigma_s=10 as 3 boxes (9,9,10), T=255, sigma_r=20, N=66"),
    "config1": dict(H=256, W=256, radii=[5], sigma_r=30.0, gen="rect", seed=1,
                    desc="256x256 f32 12 rectangles over a ramp + N(0,10^2), box r=5, T=255, "
                         "sigma_r=30, N=30"),
    "config3": dict(H=4096, W=4096, sigma_s=30.0, sigma_r=10.0, gen="smooth", seed=3,
                    desc="4096x4096 f32 piecewise-smooth, sigma_s=30 as 3 boxes (29,29,30), T=255, "
                         "sigma_r=10, N=264 (staged wide-kernel path, forward only)"),
    "config4": dict(H=512, W=512, sigma_s=6.0, sigma_r=25.0, gen="smooth", seed=4000,
                    desc="512x512 f32 piecewise-smooth, sigma_s=6 as 3 boxes (5,5,6), T=255, "
                         "sigma_r=25, N=43"),
}

# HBM bytes per launch of the fused kernels measured with rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE (separate runs), each scaled by the factor that
# maps the same counter of a plain copy kernel onto its known size (FETCH_SIZE
# x 2.0, WRITE_SIZE x 1.0 for a 512 MiB device copy); valid only for the
# kernel sources they were taken on (hash of TILE_SOURCES).  Record:
# profiles/bf_tile_kernels_2048x2048_N66_hbm_traffic.md.
_TILE_PROFILE = "profiles/bf_tile_kernels_2048x2048_N66_hbm_traffic.md"
MEASURED_TRAFFIC = {
    ("bf_tile_kernel<kForward,false>", "config2"): {"bytes": 51079993, "src": "9da9b8efdfe2",
                                                    "profile": _TILE_PROFILE},
    ("bf_tile_kernel<kForward,true>", "config2"): {"bytes": 101592485, "src": "9da9b8efdfe2",
                                                   "profile": _TILE_PROFILE},
    ("bf_tile_kernel<kBackward,false>", "config2"): {"bytes": 217940168, "src": "9da9b8efdfe2",
                                                     "profile": _TILE_PROFILE},
}
TILE_SOURCES = ("bf_tile.h", "bf_box.h", "bf_tile.hip")


def _src_hash(names=TILE_SOURCES) -> str:
    h = hashlib.sha1()
    for name in names:
        with open(os.path.join(ROOT, "paper_1105_4204_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def copy_calibration(mib: int = 512, reps: int = 3):
    """A plain device copy of `mib` MiB (torch's copy kernel), for scaling the
    FETCH_SIZE / WRITE_SIZE counters: each launch reads and writes exactly
    mib MiB."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4, "reps": reps,
                      "src_hash": _src_hash()}), flush=True)


def fwd_flops_per_pixel(N: int, nb: int, aux: bool = False) -> int:
    """Algorithmic FP32 flops per output pixel of one forward (FMA = 2).

    Per cosine pair with m > 0: phase step z <- z*u (complex multiply, 6),
    modulated products g*C, g*S (2), four channels filtered by nb boxes in two
    directions with running sums (4 * nb * 2 * 2), demodulation and
    accumulation into num and den (4 FMA = 8).  With the auxiliary sums P, Q
    of the adjoint, four more FMAs (8).  The centre pair (m = 0, even N)
    filters two channels (1, g) and accumulates 2 * 2.
    """
    pairs = N // 2 + 1
    full = pairs - (0 if N % 2 else 1)
    per_pair = 6 + 2 + 16 * nb + 8 + (8 if aux else 0)
    centre = 0 if N % 2 else (8 * nb + 4)
    return full * per_pair + centre


def bwd_flops_per_pixel(N: int, nb: int) -> int:
    """Algorithmic flops per pixel of the adjoint (FMA = 2).

    Per pair with m > 0: phase step of Y = A Z (6), modulated products h*Re Y,
    h*Im Y (2), four channels filtered by nb boxes in two directions
    (4 * nb * 2 * 2), four coefficients (C - ma g S, S + ma g C: 4 each; ma S,
    ma C: 1 each) and four accumulations (4 * 2).  The centre pair filters A
    alone (4 * nb + 2).  Plus the per-pixel closing term a (A P - B Q) (6).
    """
    pairs = N // 2 + 1
    full = pairs - (0 if N % 2 else 1)
    per_pair = 6 + 2 + 16 * nb + 10 + 8
    centre = 0 if N % 2 else (4 * nb + 2)
    return full * per_pair + centre + 6


def sigma_s_sweep(f, T, sr, sigmas=(2.0, 4.0, 6.0, 10.0, 16.0, 20.0, 30.0),
                  direct_sigmas=(2.0, 10.0, 30.0), reps=3):
    """Forward Mpixel/s at fixed sigma_r (fixed N) across spatial widths: the
    O(1) filter's cost should not grow with sigma_s (the fused kernel up to
    R = 63, the staged wide-kernel path beyond), while the direct-window
    filter's grows with the window area."""
    import torch

    from paper_1105_4204_amd import _native, ops
    H, W = f.shape
    res = []
    for ss in sigmas:
        radii = _native.spatial_gaussian(ss, 3)
        ops.trig_forward(f, T, sr, radii)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            ops.trig_forward(f, T, sr, radii)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        row = {"sigma_s": ss, "radii": radii, "R": sum(radii),
               "path": "staged" if _native.workspace_bytes(H, W, radii) else "fused",
               "fwd_ms": round(ms, 3), "fwd_mpix_s": round(H * W / 1e6 / (ms / 1e3), 1)}
        if ss in direct_sigmas:
            ops.direct_forward(f, T, sr, radii)
            torch.cuda.synchronize()
            e0.record()
            ops.direct_forward(f, T, sr, radii)
            e1.record()
            torch.cuda.synchronize()
            dms = e0.elapsed_time(e1)
            row["direct_ms"] = round(dms, 3)
            row["direct_mpix_s"] = round(H * W / 1e6 / (dms / 1e3), 1)
        res.append(row)
    return res


def wide_config_bench(reps=2):
    """The wide-kernel, many-term workload: 4096x4096 (same generator, seed
    3), sigma_s = 30 as boxes (29, 29, 30), sigma_r = 10 (N = 264), forward
    only, through the staged path; in full and with term truncation at 1e-2
    gray (pairs kept and the error bound reported)."""
    import torch

    from paper_1105_4204_amd import _native, ops, synth
    f = torch.from_numpy(synth.config_image(3)).to("cuda:0")
    H, W = f.shape
    radii = _native.spatial_gaussian(30.0, 3)
    sr, T = 10.0, 255.0
    N = _native.range_degree(T, sr)
    res = {"workload": "4096x4096 f32 piecewise-smooth, sigma_s=30 as 3 boxes "
                       f"{tuple(radii)}, T=255, sigma_r=10, N={N}, forward",
           "path": "staged" if _native.workspace_bytes(H, W, radii) else "fused",
           "pairs": len(_native.range_coeffs(N)),
           "nonzero_pairs": sum(1 for c in _native.range_coeffs(N) if c != 0.0)}
    for key, tol in (("full", 0.0), ("trunc_1e-2", 1e-2)):
        ops.trig_forward(f, T, sr, radii, trunc_tol=tol)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            ops.trig_forward(f, T, sr, radii, trunc_tol=tol)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        row = {"fwd_ms": round(ms, 2), "fwd_mpix_s": round(H * W / 1e6 / (ms / 1e3), 1)}
        if tol == 0:
            row["roofline"] = roofline_of(res["path"] + " forward", ms,
                                          ops_per_pixel(N, len(radii), "fwd") * H * W,
                                          fwd_flops_per_pixel(N, len(radii)) * H * W)
        if tol > 0:
            q, bound = _native.range_truncate(N, T, radii, tol)
            row.update({"pairs_kept": q, "error_bound_gray": bound})
        res[key] = row
    return res


def yvv_bytes_per_pixel(npairs: int) -> int:
    """Algorithmic HBM bytes per pixel of the recursive-Gaussian forward.

    Per pair and channel (4 channels): vertical pass writes the causal output
    and rewrites it anticausally (read + write), horizontal pass reads it,
    writes and rereads its causal output (6 x 4 B).  Per group of 2 pairs: f
    read by both passes (8 B), den and num partial planes written and reduced
    (16 B).  Per launch chunk of up to 40 pairs: den and num read-modify-written
    (16 B); then the division reads them and writes out (12 B).
    """
    groups = (npairs + 1) // 2
    chunks = (groups + 19) // 20
    return npairs * 4 * 24 + groups * 24 + chunks * 16 + 12


def other_spatial_kernels(f, T, sr, reps=3):
    """The two other spatial kernels at fixed sigma_r: the recursive Gaussian
    (whole-line passes, HBM-bound) across sigma_s, and the space-variant box
    (summed-area tables) across radius bounds."""
    import torch

    from paper_1105_4204_amd import _native, ops, synth
    H, W = f.shape
    mpix = H * W / 1e6

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    N = _native.range_degree(T, sr)
    npairs = len(_native.range_coeffs(N))
    ws = torch.empty(_native.yvv_workspace_bytes(H, W, T, sr) // 4 + 1, device=f.device)
    yv = []
    for ss in (2.0, 10.0, 30.0):
        ms = timed(lambda: ops.yvv_forward(f, T, sr, ss, workspace=ws))
        byts = yvv_bytes_per_pixel(npairs) * H * W
        yv.append({"sigma_s": ss, "ms": round(ms, 3), "mpix_s": round(mpix / (ms / 1e3), 1),
                   "algorithmic_GB": round(byts / 1e9, 2),
                   "achieved_GBs": round(byts / (ms / 1e3) / 1e9, 1),
                   "hbm_frac": round(byts / (ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4)})
    del ws
    sv = []
    for rmax in (2, 8, 16, 28):
        rm = torch.from_numpy(synth.radius_map(H, W, seed=2, rmax=rmax)).to(f.device)
        ms = timed(lambda: ops.sv_forward(f, rm, T, sr, rmax=rmax))
        sv.append({"rmax": rmax, "ms": round(ms, 3), "mpix_s": round(mpix / (ms / 1e3), 1)})
    return {"recursive_gaussian": yv, "space_variant_box": sv}


def ops_per_pixel(N: int, nb: int, mode: str) -> int:
    """Algorithmic VALU operations per output pixel, the count the hot-path
    scope fixes for the roofline: forward (floor(N/2)+1)(12 + 16 nb) (phase
    step 4, channel products 2, box adds 4 channels x 2 directions x 2 per box,
    demodulation 6), adjoint (floor(N/2)+1)(20 + 32 nb)."""
    pairs = N // 2 + 1
    if mode == "fwd":
        return pairs * (12 + 16 * nb)
    return pairs * (20 + 32 * nb)


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def _timed(fn, reps, stream):
    """Mean ms of fn() over reps runs, HIP events on `stream` around each."""
    import numpy as np
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for e0, e1 in evs:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in evs]))


def roofline_of(kernel, kms, ops_launch, builder_flops=None, traffic=None, traffic_from=None):
    achieved = ops_launch / (kms / 1e3) / 1e12
    r = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
         "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
         "traffic": traffic, "kernel": kernel, "kernel_ms": round(kms, 4),
         "ops_per_launch": int(ops_launch),
         "count": "algorithmic ops per pixel: fwd (floor(N/2)+1)(12+16 nb), "
                  "bwd (floor(N/2)+1)(20+32 nb)"}
    if builder_flops is not None:
        ach_b = builder_flops / (kms / 1e3) / 1e12
        r["builder_count"] = {"flops_per_launch": int(builder_flops),
                              "achieved": round(ach_b, 3),
                              "frac": round(ach_b / PEAK_FP32_TFLOPS, 4)}
    if traffic_from:
        r["traffic_from"] = traffic_from
    return r


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter runs, valid
    only while the kernel sources hash to what they were taken on."""
    tr = MEASURED_TRAFFIC.get((kernel, workload))
    if tr and tr["src"] == _src_hash(tr.get("sources", TILE_SOURCES)):
        return tr["bytes"], (f"rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (copy-calibrated), "
                             f"{tr['profile']}, sources {tr['src']}")
    return None, None


def headline_batch(steps, warmup):
    """The headline step: the 256-image ragged batch, forward + SSD loss +
    adjoint, one graph replay per step."""
    import numpy as np
    import torch

    from paper_1105_4204_amd import _native, autotune, batch, synth
    specs = synth.ragged_batch_specs(256, seed=5)
    fs, ts = synth.ragged_batch_images(specs)
    f = [torch.from_numpy(x).cuda() for x in fs]
    t = [torch.from_numpy(x).cuda() for x in ts]
    del fs, ts
    tuner = autotune.Tuner(reps=2, probe_tiles=(8, 32))
    t0 = time.perf_counter()
    for s in specs:
        tuner.tune(s, "fwd")
        tuner.tune(s, "bwd")
    tune_s = time.perf_counter() - t0
    plan = batch.BatchPlan(specs, tuner=tuner)
    out, eta, gf, loss = plan.allocate()
    plan.bind(f, t, out, eta, gf, loss)
    g = batch.capture(plan)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    start.record(stream)
    for e0, e1 in evs:
        e0.record(stream)
        g.replay()
        e1.record(stream)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    plan.check()
    ms_step = start.elapsed_time(end) / steps
    kms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    px = sum(s["H"] * s["W"] for s in specs)
    ops = 0
    bflops = 0
    Ns = []
    for s in specs:
        radii = _native.spatial_gaussian(s["sigma_s"], 3)
        N = _native.range_degree(255.0, s["sigma_r"])
        Ns.append(N)
        hw = s["H"] * s["W"]
        ops += hw * (ops_per_pixel(N, 3, "fwd") + ops_per_pixel(N, 3, "bwd"))
        bflops += hw * (fwd_flops_per_pixel(N, 3, aux=True) + bwd_flops_per_pixel(N, 3))
    traffic, tfrom = measured_traffic("bf_batch_kernel", "batch")
    roof = roofline_of("bf_batch_kernel", kms, ops, bflops, traffic, tfrom)
    alg_bytes = px * (20 + 28 + 4)   # forward with eta and sums, adjoint, target read
    hbm = {"algorithmic_bytes_per_step": alg_bytes,
           "achieved_GBs": round(alg_bytes / (ms_step / 1e3) / 1e9, 2),
           "peak_GBs": PEAK_HBM_GBS,
           "frac": round(alg_bytes / (ms_step / 1e3) / 1e9 / PEAK_HBM_GBS, 5)}
    return {"ms_step": ms_step, "kernel_ms": kms, "pixels": px, "wall": wall, "roofline": roof,
            "hbm": hbm, "N_mean": float(np.mean(Ns)), "N_range": [int(min(Ns)), int(max(Ns))],
            "autotune": {"keys": len(tuner.table), "seconds": round(tune_s, 1)},
            "specs": specs}


def image_step(f, target, T, sr, radii, reps, stream, label, workload):
    """Forward (inference), and forward with the adjoint's sums + adjoint of
    the SSD loss, on one image; per-kernel times from HIP events."""
    import torch

    from paper_1105_4204_amd import _native, ops
    H, W = f.shape
    N = _native.range_degree(T, sr)
    nb = len(radii)
    out_buf = torch.empty_like(f)
    ops.trig_forward(f, T, sr, radii, out=out_buf)
    fwd_ms = _timed(lambda: ops.trig_forward(f, T, sr, radii, out=out_buf), reps, stream)
    res = {"workload": workload, "N": N, "radii": list(radii), "fwd_ms": round(fwd_ms, 4),
           "fwd_mpix_s": round(H * W / 1e3 / fwd_ms, 1)}
    path = "staged" if _native.workspace_bytes(H, W, radii) else "fused"
    res["path"] = path
    if path == "fused":
        holder = {}

        def fwd_aux():
            holder["r"] = ops.trig_forward(f, T, sr, radii, return_aux=True)

        fwd_aux()
        aux_ms = _timed(fwd_aux, reps, stream)
        o, e, x = holder["r"]
        gout = 2.0 * (o - target)
        bwd_ms = _timed(lambda: ops.trig_backward(f, o, e, x, gout, T, sr, radii), reps, stream)
        step = aux_ms + bwd_ms
        res.update({"fwd_aux_ms": round(aux_ms, 4), "bwd_ms": round(bwd_ms, 4),
                    "fwd_bwd_ms": round(step, 4),
                    "fwd_bwd_mpix_s": round(H * W / 1e3 / step, 1)})
        name = "bf_tile_kernel<kBackward,false>"
        traffic, tfrom = measured_traffic(name, label)
        res["roofline_bwd"] = roofline_of(name, bwd_ms, ops_per_pixel(N, nb, "bwd") * H * W,
                                          bwd_flops_per_pixel(N, nb) * H * W, traffic, tfrom)
        name = "bf_tile_kernel<kForward,false>"
        traffic, tfrom = measured_traffic(name, label)
        res["roofline_fwd"] = roofline_of(name, fwd_ms, ops_per_pixel(N, nb, "fwd") * H * W,
                                          fwd_flops_per_pixel(N, nb) * H * W, traffic, tfrom)
    else:
        res["roofline_fwd"] = roofline_of("staged passes", fwd_ms,
                                          ops_per_pixel(N, nb, "fwd") * H * W,
                                          fwd_flops_per_pixel(N, nb) * H * W)
    return res


def config4_bench(reps, stream):
    """16 images of 512^2, sigma_s = 6 (boxes 5, 5, 6), sigma_r = 25 (N = 43):
    forward with the adjoint's sums + adjoint of the SSD loss, image by image."""
    import torch

    from paper_1105_4204_amd import _native, ops, synth
    fb, tb = synth.diff_batch(16)
    fs = [torch.from_numpy(x).cuda() for x in fb]
    ts = [torch.from_numpy(x).cuda() for x in tb]
    radii, sr, T = [5, 5, 6], 25.0, 255.0
    N = _native.range_degree(T, sr)

    def step():
        for f, t in zip(fs, ts):
            o, e, x = ops.trig_forward(f, T, sr, radii, return_aux=True)
            ops.trig_backward(f, o, e, x, 2.0 * (o - t), T, sr, radii)

    step()
    ms = _timed(step, reps, stream)
    px = 16 * 512 * 512
    ops_launch = px * (ops_per_pixel(N, 3, "fwd") + ops_per_pixel(N, 3, "bwd"))
    return {"workload": "16 x 512x512 f32 piecewise-smooth, sigma_s=6 as 3 boxes (5,5,6), "
                        "sigma_r=25, N=43, SSD loss, forward (with the adjoint's sums) + "
                        "adjoint per image",
            "N": N, "ms": round(ms, 3), "fwd_bwd_mpix_s": round(px / 1e3 / ms, 1),
            "step_ops_frac_of_fp32_peak": round(ops_launch / (ms / 1e3) / 1e12 /
                                               PEAK_FP32_TFLOPS, 4)}


def batch_cpu_baseline(specs, budget_s=20.0, n_images=8, fwd_px=2048, grad_px=8):
    """The FP64 oracle on the host cores over a bounded sample of the headline
    workload: for each of the first n_images images of the ragged batch, the
    forward at fwd_px random pixels and the SSD-loss gradient (brute force,
    which re-evaluates the forward around each pixel) at grad_px random pixels;
    per-pixel times extrapolated to all pixels of those images."""
    import numpy as np

    import oracle
    from paper_1105_4204_amd import _native, synth
    rng = np.random.default_rng(123)
    t_fwd = t_grad = 0.0
    px_total = 0.0
    t_total_est = 0.0
    used = 0
    for s in specs[:n_images]:
        f, t = synth.ragged_batch_images([s])
        f, t = f[0], t[0]
        H, W = f.shape
        radii = _native.spatial_gaussian(s["sigma_s"], 3)
        N = oracle.range_degree(255.0, s["sigma_r"])
        idx = rng.integers(0, H * W, size=fwd_px)
        a = time.perf_counter()
        oracle.forward_at(f, s["sigma_r"], N, radii, idx)
        b = time.perf_counter()
        gidx = rng.integers(0, H * W, size=grad_px)
        oracle.ssd_grad_at(f, t, s["sigma_r"], N, radii, gidx)
        c = time.perf_counter()
        t_fwd += b - a
        t_grad += c - b
        per_px = (b - a) / fwd_px + (c - b) / grad_px
        px_total += H * W
        t_total_est += per_px * H * W
        used += 1
        if t_fwd + t_grad > budget_s:
            break
    return {"value": px_total / t_total_est / 1e6, "unit": "Mpix/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"first {used} images of the ragged batch ({int(px_total)} px): FP64 forward "
                      f"at {fwd_px} random px and brute-force SSD gradient at {grad_px} random px "
                      f"per image, per-pixel times extrapolated to all their pixels (forward "
                      f"{t_fwd:.1f} s, gradient {t_grad:.1f} s)",
            "host": host_cpu()}


def progress(msg):
    """One progress line on stderr (stdout carries the single JSON line)."""
    print(f"# bench: {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batch",
                    choices=["batch", "config1", "config2", "config3", "config4"],
                    help="the headline workload (default: the ragged batch)")
    ap.add_argument("--no-extras", action="store_true",
                    help="time the headline workload only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-direct", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the sigma_s sweep")
    ap.add_argument("--no-other", action="store_true",
                    help="skip the recursive-Gaussian and space-variant timings")
    ap.add_argument("--no-wide", action="store_true",
                    help="skip the 4096x4096, sigma_s=30, N=264 forward")
    ap.add_argument("--only-other", action="store_true",
                    help="only time the recursive-Gaussian and space-variant paths on the "
                         "2048^2 image (for counter runs); prints their JSON and exits")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 512 MiB device copy (counter calibration) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark measures one GPU: the filter would shard by image "
                                   "(batches) or by row strips with an R-row halo (single "
                                   "images), but no multi-GPU path is built; run with --gpus 1"}),
              flush=True)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return

    import torch

    from paper_1105_4204_amd import _native, ops, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    T = 255.0

    if args.only_other:
        wl = WORKLOADS["config2"]
        f = torch.from_numpy(synth.config_image(2)).to(dev)
        print(json.dumps({"workload": wl["desc"], "sigma_r": wl["sigma_r"],
                          "other_spatial_kernels": other_spatial_kernels(f, T, wl["sigma_r"])}),
              flush=True)
        return

    line = {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic"}
    extras = {}
    cpu = None
    if args.workload == "batch":
        progress("headline: 256-image ragged batch")
        hb = headline_batch(args.steps, args.warmup)
        progress(f"headline: {hb['ms_step']:.2f} ms per step")
        value = hb["pixels"] / 1e3 / hb["ms_step"]
        line.update({"value": round(value, 3), "unit": "Mpix/s",
                     "ms_per_step": round(hb["ms_step"], 4),
                     "config": {"workload": BATCH_DESC, "images": 256,
                                "pixels": hb["pixels"], "N_mean": round(hb["N_mean"], 1),
                                "N_range": hb["N_range"], "T": T, "step": "fwd+bwd"},
                     "roofline": hb["roofline"], "hbm": hb["hbm"],
                     "autotune": hb["autotune"], "wall_s_timed": round(hb["wall"], 3)})
        if not args.no_cpu_baseline:
            progress("oracle on the host cores")
            cpu = batch_cpu_baseline(hb["specs"])
    else:
        wl = WORKLOADS[args.workload]
        if args.workload == "config4":
            r4 = config4_bench(args.steps, stream)
            line.update({"value": r4["fwd_bwd_mpix_s"], "unit": "Mpix/s",
                         "ms_per_step": r4["ms"], "config": {"workload": r4["workload"]}})
        else:
            f_np = synth.config_image(int(args.workload[-1]))
            f = torch.from_numpy(f_np).to(dev)
            tgt = torch.from_numpy(synth.piecewise_smooth(*f_np.shape, seed=wl["seed"] + 1000)
                                   ).to(dev)
            radii = wl.get("radii") or _native.spatial_gaussian(wl["sigma_s"], 3)
            r = image_step(f, tgt, T, wl["sigma_r"], radii, args.steps, stream, args.workload,
                           wl["desc"])
            ms = r.get("fwd_bwd_ms", r["fwd_ms"])
            line.update({"value": round(f.numel() / 1e3 / ms, 3), "unit": "Mpix/s",
                         "ms_per_step": round(ms, 4),
                         "config": {"workload": wl["desc"],
                                    "step": "fwd+bwd" if "fwd_bwd_ms" in r else "fwd"},
                         "roofline": r.get("roofline_bwd", r["roofline_fwd"]), "detail": r})

    if not args.no_extras:
        # 2048^2, the paper's nearest Table-2 setting
        wl = WORKLOADS["config2"]
        f2_np = synth.config_image(2)
        f2 = torch.from_numpy(f2_np).to(dev)
        t2 = torch.from_numpy(synth.piecewise_smooth(2048, 2048, seed=wl["seed"] + 1000)).to(dev)
        radii2 = _native.spatial_gaussian(wl["sigma_s"], 3)
        progress("extras: 2048^2")
        if args.workload != "config2":
            extras["config2"] = image_step(f2, t2, T, wl["sigma_r"], radii2, args.steps, stream,
                                           "config2", wl["desc"])
        if not args.no_direct:
            ops.direct_forward(f2, T, wl["sigma_r"], radii2)
            dms = _timed(lambda: ops.direct_forward(f2, T, wl["sigma_r"], radii2), 3, stream)
            extras["direct_gpu_config2"] = {"ms": round(dms, 3),
                                            "mpix_s": round(f2.numel() / 1e3 / dms, 1)}
        progress("extras: 256^2 and 16 x 512^2")
        if args.workload != "config1":
            wl1 = WORKLOADS["config1"]
            f1 = torch.from_numpy(synth.config_image(1)).to(dev)
            extras["config1"] = image_step(f1, f1, T, wl1["sigma_r"], wl1["radii"], args.steps,
                                           stream, "config1", wl1["desc"])
            for k in ("fwd_aux_ms", "bwd_ms", "fwd_bwd_ms", "fwd_bwd_mpix_s", "roofline_bwd"):
                extras["config1"].pop(k, None)   # forward only for this workload
        if args.workload != "config4":
            extras["config4"] = config4_bench(max(2, args.steps // 4), stream)
        progress("extras: sigma_s sweep, other kernels, 4096^2")
        if not args.no_sweep:
            extras["sigma_s_sweep"] = sigma_s_sweep(f2, T, wl["sigma_r"])
        if not args.no_other:
            extras["other_spatial_kernels"] = other_spatial_kernels(f2, T, wl["sigma_r"])
        if not args.no_wide and args.workload != "config3":
            extras["config3"] = wide_config_bench()
        del f2, t2
    line.update(extras)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
