#!/usr/bin/env python3
"""Benchmark of the O(1) trigonometric bilateral filter on one MI355X.

One step = one pass of the whole hot path over one batch of synthetic input.
Default (headline) workload: the ragged batch of 256 float32 images (H, W ~
U{64..1024}, sigma_s ~ U[2,16] as three boxes, sigma_r ~ U[10,60], each image
with its own degree N), forward + per-image SSD loss + adjoint, replayed from
a HIP graph of the batch plan's launches (the streamed passes over all
images).  `value` is that step's Mpixel/s (forward+backward).

The same JSON line carries the single-image workloads as extras: 256^2 box
r = 5 forward; 2048^2 sigma_s = 10, sigma_r = 20 (N = 66) forward and
forward+backward with the fused tile kernel and the direct-window GPU filter
beside it; 16 x 512^2 forward+backward as a batch; 4096^2 sigma_s = 30,
sigma_r = 10 (N = 264) forward; a sigma_s sweep at fixed N; the
recursive-Gaussian and space-variant kernels.  Every kernel time comes from
HIP events on its launch stream; the roofline of the headline's dominant
kernel uses the algorithmic operation counts per pixel; the FP64 oracle is
timed on the host cores over a bounded sample of the headline workload.
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
              "per-image SSD loss + backward, the batch plan's launches (streamed column and "
              "row passes over all images) replayed from a HIP graph")

WORKLOADS = {
    "config2": dict(H=2048, W=2048, sigma_s=10.0, sigma_r=20.0, gen="smooth", seed=2,
                    desc="2048x2048 f32 piecewise-smooth (discs+rectangles, ramps, N(0,15^2) noise), "
                         "sigma_s=10 as 3 boxes (9,9,10), T=255, sigma_r=20, N=66"),
    "config1": dict(H=256, W=256, radii=[5], sigma_r=30.0, gen="rect", seed=1,
                    desc="256x256 f32 12 rectangles over a ramp + N(0,10^2), box r=5, T=255, "
                         "sigma_r=30, N=30"),
    "config3": dict(H=4096, W=4096, sigma_s=30.0, sigma_r=10.0, gen="smooth", seed=3,
                    desc="4096x4096 f32 piecewise-smooth, sigma_s=30 as 3 boxes (29,29,30), T=255, "
                         "sigma_r=10, N=264, forward"),
    "config4": dict(H=512, W=512, sigma_s=6.0, sigma_r=25.0, gen="smooth", seed=4000,
                    desc="16 x 512x512 f32 piecewise-smooth, sigma_s=6 as 3 boxes (5,5,6), T=255, "
                         "sigma_r=25, N=43, SSD loss, forward + backward as one batch"),
}

# HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE
# (separate runs), each scaled by the factor that maps the same counter of a
# plain device copy onto its known size (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0
# for a 512 MiB copy); valid only for the kernel sources they were taken on
# (hash of STREAM_SOURCES).  Record: profiles/bf_sb_kernels_ragged256_hbm_traffic.md.
_SB_PROFILE = "profiles/bf_sb_kernels_ragged256_hbm_traffic.md"
MEASURED_TRAFFIC = {
    ("bf_sb_v<3,7,1> (adjoint column pass, groups of 4 to 7 pairs)", "ragged256"):
        {"bytes": 33267732297, "src": "86fe931f85cd", "profile": _SB_PROFILE},
    ("bf_sb_v<3,8,0> (forward column pass, groups of 4 to 8 pairs)", "ragged256"):
        {"bytes": 29166826038, "src": "86fe931f85cd", "profile": _SB_PROFILE},
}
STREAM_SOURCES = ("bf_stream.hip", "bf_tile.h")


def _src_hash(names=STREAM_SOURCES) -> str:
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


def ops_per_pixel(N: int, nb: int, mode: str) -> int:
    """Algorithmic VALU operations per output pixel, the count the hot-path
    scope fixes for the roofline: forward (floor(N/2)+1)(12 + 16 nb) (phase
    step 4, channel products 2, box adds 4 channels x 2 directions x 2 per box,
    demodulation 6), adjoint (floor(N/2)+1)(20 + 32 nb).  Each of the two
    streamed passes (column, row) filters one direction: half of it each."""
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


def roofline_of(kernel, kms, ops_launch, traffic=None, traffic_from=None, count=None):
    achieved = ops_launch / (kms / 1e3) / 1e12
    r = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
         "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
         "traffic": traffic, "kernel": kernel, "kernel_ms": round(kms, 4),
         "ops_per_launch": int(ops_launch),
         "count": count or "algorithmic ops per pixel: fwd (floor(N/2)+1)(12+16 nb), "
                           "bwd (floor(N/2)+1)(20+32 nb)"}
    if traffic_from:
        r["traffic_from"] = traffic_from
    if traffic:
        r["traffic_GBs"] = round(traffic / (kms / 1e3) / 1e9, 1)
        r["traffic_hbm_frac"] = round(traffic / (kms / 1e3) / 1e9 / PEAK_HBM_GBS, 4)
    return r


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter runs, valid
    only while the kernel sources hash to what they were taken on."""
    tr = MEASURED_TRAFFIC.get((kernel, workload))
    if tr and tr["src"] == _src_hash(tr.get("sources", STREAM_SOURCES)):
        return tr["bytes"], (f"rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (copy-calibrated), "
                             f"{tr['profile']}, sources {tr['src']}")
    return None, None


ROW_LINES = (3, 5, 7, 9, 11, 13, 15, 17, 19, 21, 23, 25, 27, 29, 31, 33, 37, 41, 45, 49, 57, 65,
             69, 73, 81)


def line_lanes(W: int, R: int) -> int:
    """Samples per lane of the row pass the library instantiates for a row of
    W pixels and total radius R (W rounded up to 4 plus R on each side, over
    64 lanes): the row passes launch once per distinct value."""
    need = (((W + 3) & ~3) + 2 * R + 63) // 64
    return next(e for e in ROW_LINES if e >= need)


STAGES = ("forward column pass", "forward row pass", "loss and adjoint weights",
          "adjoint column pass", "adjoint row pass")
STAGE_KERNELS = ("bf_sb_v<3,8,0> (forward column pass, groups of 4 to 8 pairs)",
                 "bf_sb_h<E,0,true> (forward row pass, one launch per line length E)",
                 "bf_sb_lossab + bf_sb_lossred",
                 "bf_sb_v<3,7,1> (adjoint column pass, groups of 4 to 7 pairs)",
                 "bf_sb_h<E,1,false> (adjoint row pass, one launch per line length E)")


def batch_step(specs, fs, ts, steps, warmup, path=0, tuner=None):
    """One plan over the images; `steps` graph replays timed by HIP events on
    the replay stream, then each stage of the launch timed on its own (eager,
    events on the same stream)."""
    import numpy as np
    import torch

    from paper_1105_4204_amd import batch
    f = [torch.from_numpy(x).cuda() for x in fs]
    t = [torch.from_numpy(x).cuda() for x in ts]
    plan = batch.BatchPlan(specs, tuner=tuner, path=path)
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
    res = {"ms_step": ms_step, "wall": wall,
           "replay_ms": float(np.mean([a.elapsed_time(b) for a, b in evs]))}
    if plan.path != 1 and plan.streamed():
        reps = max(2, min(steps, 5))
        stage_ms = [0.0] * 5
        for _ in range(reps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
            ev[0].record(stream)
            for k in range(5):
                plan.launch_stage(k, stream)
                ev[k + 1].record(stream)
            torch.cuda.synchronize()
            for k in range(5):
                stage_ms[k] += ev[k].elapsed_time(ev[k + 1]) / reps
        res["stage_ms"] = stage_ms
    del g
    plan.close()
    return res


def headline_batch(steps, warmup):
    """The headline step: the 256-image ragged batch, forward + SSD loss +
    adjoint; the roofline of its dominant stage (one kernel: the column pass
    of one direction) from the algorithmic operation count of its half of the
    filter."""
    import numpy as np

    from paper_1105_4204_amd import _native, synth
    specs = synth.ragged_batch_specs(256, seed=5)
    fs, ts = synth.ragged_batch_images(specs)
    res = batch_step(specs, fs, ts, steps, warmup)
    px = sum(s["H"] * s["W"] for s in specs)
    ops_half = {"fwd": 0, "bwd": 0}
    Ns = []
    for s in specs:
        radii = _native.spatial_gaussian(s["sigma_s"], 3)
        N = _native.range_degree(255.0, s["sigma_r"])
        Ns.append(N)
        hw = s["H"] * s["W"]
        ops_half["fwd"] += hw * ops_per_pixel(N, 3, "fwd") // 2
        ops_half["bwd"] += hw * ops_per_pixel(N, 3, "bwd") // 2
    st = res["stage_ms"]
    # the column passes are one launch each (every image has 3 boxes); the
    # row passes one launch per line length, each shorter than a column pass:
    # the dominant kernel is the slower column pass
    k = 0 if st[0] >= st[3] else 3
    mode = "fwd" if k == 0 else "bwd"
    name = STAGE_KERNELS[k]
    row_launches = len({line_lanes(s["W"],
                                   sum(_native.spatial_gaussian(s["sigma_s"], 3)))
                        for s in specs})
    traffic, tfrom = measured_traffic(name, "ragged256")
    roof = roofline_of(name, st[k], ops_half[mode], traffic, tfrom,
                       count=f"half of the {mode} algorithmic ops per pixel (one of the two "
                             "separable passes): fwd (floor(N/2)+1)(12+16 nb)/2, "
                             "bwd (floor(N/2)+1)(20+32 nb)/2, summed over the 256 images")
    step_ops = 2 * (ops_half["fwd"] + ops_half["bwd"])
    step_roof = {"achieved": round(step_ops / (res["ms_step"] / 1e3) / 1e12, 3),
                 "frac": round(step_ops / (res["ms_step"] / 1e3) / 1e12 / PEAK_FP32_TFLOPS, 4)}
    alg_bytes = px * (20 + 28 + 4)   # forward with eta and sums, adjoint, target read
    pair_px = sum(s["H"] * s["W"] * (_native.range_degree(255.0, s["sigma_r"]) // 2 + 1)
                  for s in specs)
    hbm = {"algorithmic_bytes_per_step": alg_bytes,
           "achieved_GBs": round(alg_bytes / (res["ms_step"] / 1e3) / 1e9, 2),
           "peak_GBs": PEAK_HBM_GBS,
           "frac": round(alg_bytes / (res["ms_step"] / 1e3) / 1e9 / PEAK_HBM_GBS, 5),
           "plane_bytes_per_step": 64 * pair_px,
           "plane_GBs": round(64 * pair_px / (res["ms_step"] / 1e3) / 1e9, 1),
           "plane_note": "the column-filtered channels the streamed passes keep in device "
                         "memory: 16 B per pixel and pair written and read, forward and adjoint"}
    roof["row_pass_launches"] = row_launches
    return {"ms_step": res["ms_step"], "wall": res["wall"], "pixels": px, "roofline": roof,
            "step_roofline": step_roof, "hbm": hbm, "N_mean": float(np.mean(Ns)),
            "N_range": [int(min(Ns)), int(max(Ns))],
            "stages": {STAGES[i]: round(st[i], 3) for i in range(5)},
            "specs": specs, "fs": fs, "ts": ts}


def image_step(f, target, T, sr, radii, reps, stream, workload, path=0):
    """Forward (inference), and forward with the adjoint's sums + adjoint of
    the SSD loss, on one image; times from HIP events on the stream."""
    import torch

    from paper_1105_4204_amd import _native, ops
    H, W = f.shape
    N = _native.range_degree(T, sr)
    nb = len(radii)
    out_buf = torch.empty_like(f)
    ws = None
    if path != 1:
        nws = _native.workspace_bytes_ex(H, W, T, sr, 0, radii) or \
            _native.stream_workspace_bytes(H, W, N // 2 + 1)
        ws = torch.empty(nws, dtype=torch.uint8, device=f.device)
    kw = dict(path=path, workspace=ws)
    ops.trig_forward(f, T, sr, radii, out=out_buf, **kw)
    fwd_ms = _timed(lambda: ops.trig_forward(f, T, sr, radii, out=out_buf, **kw), reps, stream)
    res = {"workload": workload, "N": N, "radii": list(radii), "path": "fused" if path == 1 else
           "streamed" if _native.workspace_bytes(H, W, radii) or path == 2 else "fused",
           "fwd_ms": round(fwd_ms, 4), "fwd_mpix_s": round(H * W / 1e3 / fwd_ms, 1)}
    holder = {}

    def fwd_aux():
        holder["r"] = ops.trig_forward(f, T, sr, radii, return_aux=True, **kw)

    fwd_aux()
    aux_ms = _timed(fwd_aux, reps, stream)
    o, e, x = holder["r"]
    gout = 2.0 * (o - target)
    bwd_ms = _timed(lambda: ops.trig_backward(f, o, e, x, gout, T, sr, radii, **kw), reps,
                    stream)
    step = aux_ms + bwd_ms
    res.update({"fwd_aux_ms": round(aux_ms, 4), "bwd_ms": round(bwd_ms, 4),
                "fwd_bwd_ms": round(step, 4), "fwd_bwd_mpix_s": round(H * W / 1e3 / step, 1)})
    res["roofline_fwd"] = roofline_of("forward (both passes)" if path != 1 else
                                      "bf_tile_kernel<kForward,false>", fwd_ms,
                                      ops_per_pixel(N, nb, "fwd") * H * W)
    res["roofline_bwd"] = roofline_of("adjoint (both passes)" if path != 1 else
                                      "bf_tile_kernel<kBackward,false>", bwd_ms,
                                      ops_per_pixel(N, nb, "bwd") * H * W)
    return res


def sigma_s_sweep(f, T, sr, sigmas=(2.0, 4.0, 6.0, 10.0, 16.0, 20.0, 30.0, 50.0, 100.0),
                  direct_sigmas=(2.0, 10.0, 30.0), reps=3):
    """Forward time at fixed sigma_r (fixed N) across spatial widths: the O(1)
    filter's cost should not grow with sigma_s (the streamed passes; the fused
    tiles beside them while they hold the kernel), while the direct-window
    filter's grows with the window area."""
    import torch

    from paper_1105_4204_amd import _native, ops
    H, W = f.shape
    stream = torch.cuda.current_stream()
    res = []
    for ss in sigmas:
        radii = _native.spatial_gaussian(ss, 3)
        nws = _native.workspace_bytes_ex(H, W, T, sr, 0, radii)
        ws = torch.empty(nws, dtype=torch.uint8, device=f.device) if nws else None
        ops.trig_forward(f, T, sr, radii, workspace=ws)
        ms = _timed(lambda: ops.trig_forward(f, T, sr, radii, workspace=ws), reps, stream)
        row = {"sigma_s": ss, "radii": radii, "R": sum(radii),
               "path": "streamed" if nws else "fused",
               "fwd_ms": round(ms, 3), "fwd_mpix_s": round(H * W / 1e3 / ms, 1)}
        if sum(radii) <= 63 and max(radii) <= 31 and ss <= 16:
            ops.trig_forward(f, T, sr, radii, path=1)
            fms = _timed(lambda: ops.trig_forward(f, T, sr, radii, path=1), reps, stream)
            row["fused_fwd_ms"] = round(fms, 3)
        if ss in direct_sigmas:
            ops.direct_forward(f, T, sr, radii)
            dms = _timed(lambda: ops.direct_forward(f, T, sr, radii), 1, stream)
            row["direct_ms"] = round(dms, 3)
            row["direct_mpix_s"] = round(H * W / 1e3 / dms, 1)
        res.append(row)
        del ws
    base = [r["fwd_ms"] for r in res if r["sigma_s"] == 10.0][0]
    for r in res:
        r["ratio_to_sigma_s_10"] = round(r["fwd_ms"] / base, 3)
    return res


def wide_config_bench(reps=2):
    """The wide-kernel, many-term workload: 4096x4096 (same generator, seed
    3), sigma_s = 30 as boxes (29, 29, 30), sigma_r = 10 (N = 264), forward
    only; in full and with term truncation at 1e-2 gray (pairs kept and the
    error bound reported)."""
    import torch

    from paper_1105_4204_amd import _native, ops, synth
    f = torch.from_numpy(synth.config_image(3)).to("cuda:0")
    H, W = f.shape
    radii = _native.spatial_gaussian(30.0, 3)
    sr, T = 10.0, 255.0
    N = _native.range_degree(T, sr)
    nws = _native.workspace_bytes_ex(H, W, T, sr, 0, radii)
    ws = torch.empty(nws, dtype=torch.uint8, device=f.device)
    stream = torch.cuda.current_stream()
    res = {"workload": WORKLOADS["config3"]["desc"], "path": "streamed",
           "pairs": len(_native.range_coeffs(N)),
           "nonzero_pairs": sum(1 for c in _native.range_coeffs(N) if c != 0.0),
           "workspace_bytes": nws}
    for key, tol in (("full", 0.0), ("trunc_1e-2", 1e-2)):
        ops.trig_forward(f, T, sr, radii, trunc_tol=tol, workspace=ws)
        ms = _timed(lambda: ops.trig_forward(f, T, sr, radii, trunc_tol=tol, workspace=ws),
                    reps, stream)
        row = {"fwd_ms": round(ms, 2), "fwd_mpix_s": round(H * W / 1e3 / ms, 1)}
        if tol == 0:
            row["roofline"] = roofline_of("forward (both passes)", ms,
                                          ops_per_pixel(N, len(radii), "fwd") * H * W)
            pair_bytes = 32 * H * W * res["nonzero_pairs"]
            row["plane_GBs"] = round(pair_bytes / (ms / 1e3) / 1e9, 1)
        else:
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
    stream = torch.cuda.current_stream()
    N = _native.range_degree(T, sr)
    npairs = len(_native.range_coeffs(N))
    ws = torch.empty(_native.yvv_workspace_bytes(H, W, T, sr) // 4 + 1, device=f.device)
    yv = []
    for ss in (2.0, 10.0, 30.0):
        ops.yvv_forward(f, T, sr, ss, workspace=ws)
        ms = _timed(lambda: ops.yvv_forward(f, T, sr, ss, workspace=ws), reps, stream)
        byts = yvv_bytes_per_pixel(npairs) * H * W
        yv.append({"sigma_s": ss, "ms": round(ms, 3), "mpix_s": round(mpix / (ms / 1e3), 1),
                   "algorithmic_GB": round(byts / 1e9, 2),
                   "achieved_GBs": round(byts / (ms / 1e3) / 1e9, 1),
                   "hbm_frac": round(byts / (ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4)})
    del ws
    sv = []
    for rmax in (2, 8, 16, 28):
        rm = torch.from_numpy(synth.radius_map(H, W, seed=2, rmax=rmax)).to(f.device)
        ops.sv_forward(f, rm, T, sr, rmax=rmax)
        ms = _timed(lambda: ops.sv_forward(f, rm, T, sr, rmax=rmax), reps, stream)
        sv.append({"rmax": rmax, "ms": round(ms, 3), "mpix_s": round(mpix / (ms / 1e3), 1)})
    return {"recursive_gaussian": yv, "space_variant_box": sv}


def config4_bench(steps):
    """16 images of 512^2, sigma_s = 6 (boxes 5, 5, 6), sigma_r = 25 (N = 43):
    forward + SSD loss + adjoint as one batch (graph replay)."""
    from paper_1105_4204_amd import _native, synth
    fb, tb = synth.diff_batch(16)
    specs = [dict(H=512, W=512, radii=[5, 5, 6], sigma_r=25.0) for _ in range(16)]
    res = batch_step(specs, list(fb), list(tb), steps, 2)
    N = _native.range_degree(255.0, 25.0)
    px = 16 * 512 * 512
    ops_step = px * (ops_per_pixel(N, 3, "fwd") + ops_per_pixel(N, 3, "bwd"))
    ms = res["ms_step"]
    return {"workload": WORKLOADS["config4"]["desc"], "N": N, "ms": round(ms, 3),
            "fwd_bwd_mpix_s": round(px / 1e3 / ms, 1),
            "step_ops_frac_of_fp32_peak": round(ops_step / (ms / 1e3) / 1e12 / PEAK_FP32_TFLOPS, 4),
            "stages_ms": [round(x, 3) for x in res.get("stage_ms", [])]}


def colour_bench(reps=5):
    """A 3 x 2048 x 2048 colour image (the colour generator, seed 9), each
    channel filtered on its own as one item of a forward-only batch plan
    (sigma_s = 10 as boxes 9, 9, 10, sigma_r = 20, N = 66); launches timed
    with HIP events on the stream."""
    import torch

    from paper_1105_4204_amd import batch, synth
    img = torch.from_numpy(synth.colour(2048, 2048, seed=9)).cuda()
    C, H, W = img.shape
    spec = dict(H=H, W=W, T=255.0, sigma_r=20.0, radii=[9, 9, 10])
    plan = batch.BatchPlan([spec] * C)
    out = torch.empty_like(img)
    plan.bind([img[c] for c in range(C)], out=[out[c] for c in range(C)])
    stream = torch.cuda.current_stream()
    plan.launch()
    ms = _timed(lambda: plan.launch(), reps, stream)
    plan.check()
    plan.close()
    return {"workload": "3 x 2048x2048 f32 colour (per-channel gain, offset, noise), boxes 9, 9, 10, "
                        "sigma_r=20, N=66, channel-wise forward as one batch",
            "ms": round(ms, 3), "mpix_s": round(H * W / 1e3 / ms, 1),
            "channel_mpix_s": round(C * H * W / 1e3 / ms, 1)}


def batch_cpu_baseline(specs, fs, ts, budget_s=30.0, n_images=8, fwd_px=32768, grad_px=128):
    """The FP64 oracle on the host cores over a bounded sample of the headline
    workload: for each of the first n_images images of the ragged batch, the
    forward at fwd_px random pixels and the SSD-loss gradient (brute force,
    which re-evaluates the forward around each pixel) at grad_px random pixels;
    per-pixel times extrapolated to all pixels of those images."""
    import numpy as np

    import oracle
    from paper_1105_4204_amd import _native
    rng = np.random.default_rng(123)
    t_fwd = t_grad = 0.0
    px_total = 0.0
    t_total_est = 0.0
    used = 0
    for s, f, t in list(zip(specs, fs, ts))[:n_images]:
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
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[1])
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
    ap.add_argument("--no-fused-batch", action="store_true",
                    help="skip the persistent fused-tile batch timed beside the headline")
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
                     "roofline": hb["roofline"], "step_roofline": hb["step_roofline"],
                     "hbm": hb["hbm"], "stages_ms": hb["stages"],
                     "wall_s_timed": round(hb["wall"], 3)})
        if not args.no_extras and not args.no_fused_batch:
            progress("extras: the same batch through the persistent fused-tile kernel")
            from paper_1105_4204_amd import autotune
            tuner = autotune.Tuner(reps=2, probe_tiles=(8, 32))
            t0 = time.perf_counter()
            for s in hb["specs"]:
                tuner.tune(s, "fwd")
                tuner.tune(s, "bwd")
            tune_s = time.perf_counter() - t0
            fb = batch_step(hb["specs"], hb["fs"], hb["ts"], max(3, args.steps // 4), 2,
                            path=1, tuner=tuner)
            extras["batch_fused_persistent"] = {
                "ms": round(fb["ms_step"], 3), "mpix_s": round(hb["pixels"] / 1e3 / fb["ms_step"], 1),
                "autotune": {"keys": len(tuner.table), "seconds": round(tune_s, 1)}}
        if not args.no_cpu_baseline:
            progress("oracle on the host cores")
            cpu = batch_cpu_baseline(hb["specs"], hb["fs"], hb["ts"])
    else:
        wl = WORKLOADS[args.workload]
        if args.workload == "config4":
            r4 = config4_bench(args.steps)
            line.update({"value": r4["fwd_bwd_mpix_s"], "unit": "Mpix/s",
                         "ms_per_step": r4["ms"], "config": {"workload": r4["workload"]}})
        elif args.workload == "config3":
            r3 = wide_config_bench(args.steps)
            ms = r3["full"]["fwd_ms"]
            line.update({"value": r3["full"]["fwd_mpix_s"], "unit": "Mpix/s",
                         "ms_per_step": ms, "config": {"workload": r3["workload"],
                                                       "step": "fwd"},
                         "roofline": r3["full"]["roofline"], "detail": r3})
        else:
            f_np = synth.config_image(int(args.workload[-1]))
            f = torch.from_numpy(f_np).to(dev)
            tgt = torch.from_numpy(synth.piecewise_smooth(*f_np.shape, seed=wl["seed"] + 1000)
                                   ).to(dev)
            radii = wl.get("radii") or _native.spatial_gaussian(wl["sigma_s"], 3)
            r = image_step(f, tgt, T, wl["sigma_r"], radii, args.steps, stream, wl["desc"])
            ms = r["fwd_bwd_ms"] if args.workload == "config2" else r["fwd_ms"]
            line.update({"value": round(f.numel() / 1e3 / ms, 3), "unit": "Mpix/s",
                         "ms_per_step": round(ms, 4),
                         "config": {"workload": wl["desc"],
                                    "step": "fwd+bwd" if args.workload == "config2" else "fwd"},
                         "roofline": r["roofline_bwd"] if args.workload == "config2"
                         else r["roofline_fwd"], "detail": r})

    if not args.no_extras:
        wl = WORKLOADS["config2"]
        f2_np = synth.config_image(2)
        f2 = torch.from_numpy(f2_np).to(dev)
        t2 = torch.from_numpy(synth.piecewise_smooth(2048, 2048, seed=wl["seed"] + 1000)).to(dev)
        radii2 = _native.spatial_gaussian(wl["sigma_s"], 3)
        progress("extras: 2048^2")
        if args.workload != "config2":
            extras["config2"] = image_step(f2, t2, T, wl["sigma_r"], radii2, args.steps, stream,
                                           wl["desc"])
            extras["config2_fused_tiles"] = image_step(f2, t2, T, wl["sigma_r"], radii2,
                                                       args.steps, stream, wl["desc"], path=1)
        if not args.no_direct:
            ops.direct_forward(f2, T, wl["sigma_r"], radii2)
            dms = _timed(lambda: ops.direct_forward(f2, T, wl["sigma_r"], radii2), 3, stream)
            extras["direct_gpu_config2"] = {"ms": round(dms, 3),
                                            "mpix_s": round(f2.numel() / 1e3 / dms, 1)}
        progress("extras: 256^2 and 16 x 512^2")
        if args.workload != "config1":
            wl1 = WORKLOADS["config1"]
            f1 = torch.from_numpy(synth.config_image(1)).to(dev)
            r1 = image_step(f1, f1, T, wl1["sigma_r"], wl1["radii"], args.steps, stream,
                            wl1["desc"])
            extras["config1"] = {k: r1[k] for k in ("workload", "N", "radii", "path", "fwd_ms",
                                                    "fwd_mpix_s", "roofline_fwd")}
        if args.workload != "config4":
            extras["config4"] = config4_bench(max(3, args.steps // 4))
        extras["colour"] = colour_bench()
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
