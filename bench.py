#!/usr/bin/env python3
"""Benchmark of the O(1) trigonometric bilateral filter on one MI355X.

One step = one pass of the hot path over one synthetic image: the fused
forward kernel (degree, coefficients, phase recurrence, modulation, iterated-
box running sums, demodulation, FP64 division) followed by the fused adjoint
kernel for an SSD loss gradient.  Default workload: a 2048 x 2048 float32
piecewise-smooth image, spatial Gaussian sigma_s = 10 as three boxes of radii
9, 9, 10, sigma_r = 20 (N = 66), T = 255.

Prints ONE JSON line.  `value` is forward+backward Mpixel/s; the same line
carries forward-only Mpixel/s, the direct-window GPU filter's Mpixel/s on the
same image, HBM figures, the roofline of the dominant kernel (timed with HIP
events on the launch stream) and the FP64 oracle timed on the host cores over
a bounded sample of the same workload.
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
MEASURED_TRAFFIC = {
    ("bf_tile_kernel<kForward,false>", "config2"): {"bytes": 51079993, "src": "9da9b8efdfe2"},
    ("bf_tile_kernel<kForward,true>", "config2"): {"bytes": 101592485, "src": "9da9b8efdfe2"},
    ("bf_tile_kernel<kBackward,false>", "config2"): {"bytes": 217940168, "src": "9da9b8efdfe2"},
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


def batch_bench(reps: int = 3):
    """256 ragged images (H, W ~ U{64..1024}, sigma_s ~ U[2,16], sigma_r ~
    U[10,60]): forward, per-image SSD loss and adjoint in one graph replay."""
    import torch

    from paper_1105_4204_amd import batch, synth
    from paper_1105_4204_amd import autotune
    specs = synth.ragged_batch_specs(256, seed=5)
    fs, ts = synth.ragged_batch_images(specs)
    f = [torch.from_numpy(x).cuda() for x in fs]
    t = [torch.from_numpy(x).cuda() for x in ts]
    del fs, ts
    # tiles from the autotuner (cached per device, mode, radii and N bucket;
    # tuning happens here, before the timed replays)
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
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    plan.check()
    ms = e0.elapsed_time(e1) / reps
    px = sum(s["H"] * s["W"] for s in specs)
    return {"images": len(specs), "pixels": px, "ms": round(ms, 3),
            "mpix_s_fwd_bwd": round(px / 1e6 / (ms / 1e3), 3),
            "autotune": {"keys": len(tuner.table), "seconds": round(tune_s, 1)},
            "desc": "256 ragged images, H,W~U{64..1024}, sigma_s~U[2,16] (3 boxes), "
                    "sigma_r~U[10,60] (per-image N), fwd + SSD loss + bwd, one persistent "
                    "kernel replayed from a HIP graph, tiles from the autotuner"}


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


def cpu_baseline(f, sigma_r, N, radii, budget_s=12.0, max_rows=1024):
    import numpy as np
    import oracle
    H, W = f.shape
    rows = 0
    t_total = 0.0
    r0 = H // 2 - max_rows // 2
    while rows < max_rows and t_total < budget_s:
        idx = (np.arange(16 * W, dtype=np.int64) + (r0 + rows) * W)
        t0 = time.perf_counter()
        oracle.forward_at(f, sigma_r, N, radii, idx)
        t_total += time.perf_counter() - t0
        rows += 16
    px = rows * W
    return {"value": px / t_total / 1e6, "unit": "Mpix/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{rows} full rows ({px} px) of the {H}x{W} image, rows {r0}..{r0 + rows - 1}, "
                      f"FP64 direct window sum, {t_total:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="config2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-direct", action="store_true")
    ap.add_argument("--fwd-only", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the sigma_s sweep (and the wide-kernel configuration)")
    ap.add_argument("--no-other", action="store_true",
                    help="skip the recursive-Gaussian and space-variant timings")
    ap.add_argument("--no-wide", action="store_true",
                    help="skip the 4096x4096, sigma_s=30, N=264 forward")
    ap.add_argument("--only-other", action="store_true",
                    help="only time the recursive-Gaussian and space-variant paths (for "
                         "counter runs); prints their JSON and exits")
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

    import numpy as np
    import torch

    from paper_1105_4204_amd import _native, ops, synth

    wl = WORKLOADS[args.workload]
    H, W = wl["H"], wl["W"]
    if wl["gen"] == "rect":
        f_np = synth.rectangles(H, W, seed=wl["seed"])
    else:
        f_np = synth.piecewise_smooth(H, W, seed=wl["seed"])
    t_np = synth.piecewise_smooth(H, W, seed=wl["seed"] + 1000)
    radii = wl.get("radii") or _native.spatial_gaussian(wl["sigma_s"], 3)
    sr, T = wl["sigma_r"], 255.0
    N = _native.range_degree(T, sr)
    nb = len(radii)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    f = torch.from_numpy(f_np).to(dev)
    if args.only_other:
        print(json.dumps({"workload": wl["desc"], "sigma_r": sr,
                          "other_spatial_kernels": other_spatial_kernels(f, T, sr)}), flush=True)
        return
    target = torch.from_numpy(t_np).to(dev)
    stream = torch.cuda.current_stream()
    do_bwd = not args.fwd_only
    try:
        ops.trig_forward(f, T, sr, radii, return_aux=True)
    except _native.BFError as e:
        if e.code == 6:
            do_bwd = False
        else:
            raise

    # the training step: forward (with the sums the adjoint needs) + adjoint
    # of the SSD loss; events on the launch stream around each kernel
    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        if do_bwd:
            out, eta, aux = ops.trig_forward(f, T, sr, radii, return_aux=True)
        else:
            out = ops.trig_forward(f, T, sr, radii)
        if ev is not None:
            ev[1].record(stream)
        if do_bwd:
            g = 2.0 * (out - target)
            if ev is not None:
                ev[2].record(stream)
            gf = ops.trig_backward(f, out, eta, aux, g, T, sr, radii)
            if ev is not None:
                ev[3].record(stream)
            return gf
        return out

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for k in range(args.steps):
        step(evs[k])
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(end)
    ms_step = total_ms / args.steps
    step_fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    bwd_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in evs])) if do_bwd else None

    # inference forward alone (no auxiliary sums)
    out_buf = torch.empty_like(f)
    ops.trig_forward(f, T, sr, radii, out=out_buf)
    torch.cuda.synchronize()
    fevs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    for k in range(args.steps):
        fevs[k][0].record(stream)
        ops.trig_forward(f, T, sr, radii, out=out_buf)
        fevs[k][1].record(stream)
    torch.cuda.synchronize()
    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in fevs]))

    mpix = H * W / 1e6
    value = mpix / (ms_step / 1e3)
    fwd_mpix = mpix / (fwd_ms / 1e3)

    direct = None
    if not args.no_direct:
        ops.direct_forward(f, T, sr, radii)
        torch.cuda.synchronize()
        d0, d1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 3
        d0.record(stream)
        for _ in range(reps):
            ops.direct_forward(f, T, sr, radii)
        d1.record(stream)
        torch.cuda.synchronize()
        direct_ms = d0.elapsed_time(d1) / reps
        direct = {"ms": direct_ms, "mpix_s": mpix / (direct_ms / 1e3),
                  "fwd_speedup_vs_direct": direct_ms / fwd_ms}

    # dominant kernel of the step: the forward with auxiliary sums or the adjoint
    fwd_flops = fwd_flops_per_pixel(N, nb) * H * W
    dom = ("bf_tile_kernel<kForward,false>", fwd_ms, fwd_flops)
    if do_bwd:
        dom = ("bf_tile_kernel<kForward,true>", step_fwd_ms,
               fwd_flops_per_pixel(N, nb, aux=True) * H * W)
        if bwd_ms > step_fwd_ms:
            dom = ("bf_tile_kernel<kBackward,false>", bwd_ms, bwd_flops_per_pixel(N, nb) * H * W)
    name, kms, kflops = dom
    achieved = kflops / (kms / 1e3) / 1e12
    tr = MEASURED_TRAFFIC.get((name, args.workload))
    traffic = tr["bytes"] if tr and tr["src"] == _src_hash() else None
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": traffic, "kernel": name, "kernel_ms": round(kms, 4),
                "flops_per_launch": kflops}
    fwd_bytes = 8 * H * W        # inference: read f, write out
    fwd_aux_bytes = 20 * H * W   # training: read f; write out, eta, P, Q
    bwd_bytes = 28 * H * W       # read f, out, eta, P, Q, grad_out; write grad_f
    step_bytes = (fwd_aux_bytes + bwd_bytes) if do_bwd else fwd_bytes
    hbm = {"algorithmic_bytes_per_step": step_bytes,
           "achieved_GBs": round(step_bytes / (ms_step / 1e3) / 1e9, 2),
           "peak_GBs": PEAK_HBM_GBS,
           "frac": round(step_bytes / (ms_step / 1e3) / 1e9 / PEAK_HBM_GBS, 5),
           "dominant_kernel_measured_GBs": (round(traffic / (kms / 1e3) / 1e9, 2)
                                            if traffic is not None else None),
           "note": "ALU-bound: 2(N+1) filtered channels per pixel stay in registers and LDS"}

    batch_res = None
    if not args.no_batch and do_bwd and args.workload == "config2":
        batch_res = batch_bench()

    sweep = None
    if not args.no_sweep and args.workload == "config2":
        sweep = sigma_s_sweep(f, T, sr)

    other = None
    if not args.no_other and args.workload == "config2":
        other = other_spatial_kernels(f, T, sr)

    wide = None
    if not args.no_wide and not args.no_sweep and args.workload == "config2":
        wide = wide_config_bench()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(f_np, sr, N, radii)

    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "H": H, "W": W, "radii": radii, "sigma_r": sr,
                   "T": T, "N": N, "step": "fwd+bwd" if do_bwd else "fwd"},
        "fwd_mpix_s": round(fwd_mpix, 3),
        "fwd_ms": round(fwd_ms, 4),
        "fwd_aux_ms": round(step_fwd_ms, 4) if do_bwd else None,
        "bwd_ms": round(bwd_ms, 4) if bwd_ms is not None else None,
        "fwd_bwd_mpix_s": round(value, 3) if do_bwd else None,
        "direct_gpu": direct,
        "hbm": hbm,
        "roofline": roofline,
        "batch": batch_res,
        "sigma_s_sweep": sweep,
        "other_spatial_kernels": other,
        "wide_kernel_config": wide,
        "cpu_baseline": cpu,
        "wall_s_timed": round(wall, 3),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
