"""Tile-shape autotuner for the fused kernels.

For a (spatial radii, degree N, mode) key it times a few candidate output
tiles of the fused forward / adjoint kernel and keeps the one with the least
time per pixel (median of several launches timed with HIP events).  Each
candidate runs on a probe image of exactly 16 x 32 of its own tiles, so that
every candidate fills the chip for two rounds of workgroups and none is
favoured by how its tiles happen to divide a fixed probe size.  Results are
cached in a JSON file (BF_TUNE_CACHE, default ~/.cache/bftrig/tune.json) keyed
by device name, so a batch plan reuses them without re-timing.  Candidates
are odd tile sides (odd LDS pitches) that fit the kernel's limits; invalid
ones are rejected by the library and skipped.
"""
from __future__ import annotations

import json
import os
import statistics

import torch

from . import _native as nat
from . import ops

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "bftrig", "tune.json")


class Tuner:
    def __init__(self, cache_path: str | None = None, reps: int = 5, probe_tiles=(16, 32)):
        self.path = cache_path or os.environ.get("BF_TUNE_CACHE", DEFAULT_CACHE)
        self.reps = reps
        self.probe_tiles = tuple(probe_tiles)
        self.table = {}
        if os.path.exists(self.path):
            try:
                with open(self.path) as fh:
                    self.table = json.load(fh)
            except (OSError, ValueError):
                self.table = {}

    @staticmethod
    def _radii(spec):
        r = spec.get("radii")
        if r is None:
            r = nat.spatial_gaussian(float(spec["sigma_s"]), int(spec.get("n_boxes", 3)))
        return [int(x) for x in r]

    def key(self, spec, mode):
        T = float(spec.get("T", 255.0))
        N = int(spec.get("N", 0)) or nat.range_degree(T, float(spec["sigma_r"]))
        nbucket = 1 << max(0, (N - 1).bit_length())          # N rounded up to a power of 2
        dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
        return f"v3|{dev}|{mode}|r={','.join(map(str, self._radii(spec)))}|N<={nbucket}"

    def candidates(self, R, mode):
        """Output tiles up to 64 x 64 whose extended sides fit a 128-long
        register line; the library rejects those over the LDS budget."""
        smax = min(64, 128 - 2 * R)
        if smax < 1:
            return []
        cands = []
        for th, tw in ((smax, smax), (smax, smax - 8), (smax - 8, smax), (smax, smax - 16),
                       (smax - 16, smax), (smax - 8, smax - 8), (smax - 16, smax - 16),
                       (smax, smax // 2), (smax // 2, smax)):
            if th >= 1 and tw >= 1 and (th, tw) not in cands:
                cands.append((th, tw))
        return cands

    def _time(self, fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(self.reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return statistics.median(ts)

    def tune(self, spec, mode="fwd"):
        k = self.key(spec, mode)
        if k in self.table:
            return tuple(self.table[k]["tile"])
        radii = self._radii(spec)
        R = sum(radii)
        T = float(spec.get("T", 255.0))
        sr = float(spec["sigma_r"])
        N = int(spec.get("N", 0))
        gen = torch.Generator(device="cuda").manual_seed(99)
        best = None
        for tile in self.candidates(R, mode):
            H, W = tile[0] * self.probe_tiles[0], tile[1] * self.probe_tiles[1]
            # a view one float into its buffer: not 16-byte aligned, so the
            # single-image adjoint stages g in LDS like the batch kernel does
            # (the global-g variant fits larger tiles than the batch can use)
            f = (torch.rand(H * W + 1, device="cuda", generator=gen) * T)[1:].view(H, W)
            try:
                if mode == "fwd":
                    # the batch's forward tiles also accumulate the adjoint's
                    # sums: time that variant
                    t = self._time(lambda: ops.trig_forward(f, T, sr, radii, N=N, tile=tile,
                                                            return_aux=True))
                else:
                    out, eta, aux = ops.trig_forward(f, T, sr, radii, N=N, return_aux=True)
                    G = torch.randn(H, W, device="cuda", generator=gen)
                    t = self._time(lambda: ops.trig_backward(f, out, eta, aux, G, T, sr, radii,
                                                             N=N, tile=tile))
            except nat.BFError:
                continue
            t /= H * W                      # time per output pixel
            if best is None or t < best[0]:
                best = (t, tile)
        if best is None:
            return (0, 0)
        self.table[k] = {"tile": list(best[1]), "ns_per_px": best[0] * 1e6}
        self.save()
        return best[1]

    def tile_for(self, spec, mode):
        k = self.key(spec, mode)
        if k in self.table:
            return tuple(self.table[k]["tile"])
        return None

    def save(self):
        os.makedirs(os.path.dirname(self.path), exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(self.table, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)
