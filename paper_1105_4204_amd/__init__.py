"""Constant-time trigonometric bilateral filter for AMD MI355X (gfx950).

The filter of Chaudhury, Sage and Unser ("Fast O(1) bilateral filtering using
trigonometric range kernels"): a raised-cosine range kernel expanded into
cosine pairs (Sec. 2.3), each pair's auxiliary images averaged by iterated
running box sums (Sec. 2.1), then demodulated and divided (eq. (final-form)).
All arithmetic runs in the hand-written HIP kernels of ``libbftrig.so``
(C ABI in ``include/bf_trig.h``); the Python layer only marshals arguments.

Submodules are imported lazily so that ``synth`` (input generators) works
without the native library or a GPU.
"""
import importlib

__all__ = ["bf_trig", "trig_forward", "trig_backward", "sv_forward", "yvv_forward",
           "direct_forward", "check_range", "BFTrig",
           "range_degree", "range_coeffs", "range_truncate", "spatial_gaussian", "BatchPlan",
           "trig_forward_channels", "synth"]

_LAZY = {
    "bf_trig": ("ops", "bf_trig"),
    "trig_forward": ("ops", "trig_forward"),
    "trig_backward": ("ops", "trig_backward"),
    "direct_forward": ("ops", "direct_forward"),
    "check_range": ("ops", "check_range"),
    "sv_forward": ("ops", "sv_forward"),
    "yvv_forward": ("ops", "yvv_forward"),
    "BFTrig": ("ops", "BFTrig"),
    "range_degree": ("_native", "range_degree"),
    "range_coeffs": ("_native", "range_coeffs"),
    "spatial_gaussian": ("_native", "spatial_gaussian"),
    "BatchPlan": ("batch", "BatchPlan"),
    "trig_forward_channels": ("batch", "trig_forward_channels"),
    "range_truncate": ("_native", "range_truncate"),
}


def __getattr__(name):
    if name in _LAZY:
        mod, attr = _LAZY[name]
        return getattr(importlib.import_module(f".{mod}", __name__), attr)
    if name in ("synth", "ops", "batch", "autotune", "_native", "build"):
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
