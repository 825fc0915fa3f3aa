"""ctypes binding of libbftrig.so (argument marshalling only).

Every function here forwards device pointers, sizes and the current HIP stream
to the C ABI declared in include/bf_trig.h; all arithmetic of the filter runs
in the library's HIP kernels.  Importing this module fails loudly when the
library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbftrig.so")

BF_MAX_BOXES = 4
BF_MAX_RADIUS = 256
PATH_AUTO, PATH_FUSED, PATH_STREAMED = 0, 1, 2
BF_MAX_DEGREE = 1024

STATUS = {0: "BF_OK", 1: "BF_EINVAL", 2: "BF_ERANGE", 3: "BF_ENOMEM", 4: "BF_EDEVICE",
          5: "BF_ECAPTURE", 6: "BF_EUNSUPPORTED"}

# exported symbols, in the order include/bf_trig.h declares them
EXPORTS = ["bf_range_degree", "bf_range_coeffs", "bf_range_truncate", "bf_spatial_gaussian",
           "bf_trig_workspace_bytes", "bf_trig_workspace_bytes_ex", "bf_trig_forward",
           "bf_trig_forward_ex", "bf_trig_forward_noalloc", "bf_trig_backward", "bf_sv_forward",
           "bf_yvv_coeffs", "bf_yvv_workspace_bytes", "bf_yvv_forward", "bf_direct_forward", "bf_check_range",
           "bf_batch_plan_create", "bf_batch_plan_create_ex", "bf_batch_bind", "bf_batch_launch", "bf_batch_launch_stage", "bf_batch_plan_path", "bf_batch_check",
           "bf_batch_plan_destroy", "bf_status_string", "bf_last_error"]


class BFError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)}: {detail}")


class SpatialSpec(ctypes.Structure):
    _fields_ = [("n_boxes", ctypes.c_int32), ("radius", ctypes.c_int32 * BF_MAX_BOXES)]

    @classmethod
    def of(cls, radii):
        radii = [int(r) for r in radii]
        if not 1 <= len(radii) <= BF_MAX_BOXES:
            raise ValueError(f"need 1..{BF_MAX_BOXES} box radii, got {radii}")
        s = cls()
        s.n_boxes = len(radii)
        for i, r in enumerate(radii):
            s.radius[i] = r
        return s

    def radii(self):
        return [int(self.radius[i]) for i in range(self.n_boxes)]


class Opts(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("N", ctypes.c_int32),
                ("eta_out", ctypes.c_void_p), ("tile_h", ctypes.c_int32),
                ("tile_w", ctypes.c_int32), ("aux_out", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_int64),
                ("trunc_tol", ctypes.c_float), ("path", ctypes.c_int32)]


class ImageDesc(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int64), ("W", ctypes.c_int64), ("T", ctypes.c_float),
                ("sigma_r", ctypes.c_float), ("N", ctypes.c_int32), ("spatial", SpatialSpec),
                ("tile_h", ctypes.c_int32), ("tile_w", ctypes.c_int32),
                ("bwd_tile_h", ctypes.c_int32), ("bwd_tile_w", ctypes.c_int32),
                ("trunc_tol", ctypes.c_float)]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m "
                          "paper_1105_4204_amd.build` (or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, f32, f64, vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double,
                              ctypes.c_void_p)
    sp = ctypes.POINTER(SpatialSpec)
    op = ctypes.POINTER(Opts)
    sig = {
        "bf_range_degree": [f64, f64, ctypes.POINTER(i32)],
        "bf_range_coeffs": [i32, ctypes.POINTER(f32), i32, ctypes.POINTER(i32)],
        "bf_range_truncate": [i32, f64, sp, f64, ctypes.POINTER(i32), ctypes.POINTER(f64)],
        "bf_spatial_gaussian": [f64, i32, sp],
        "bf_trig_workspace_bytes": [i64, i64, sp, ctypes.POINTER(i64)],
        "bf_trig_workspace_bytes_ex": [i64, i64, f32, f32, i32, sp, ctypes.POINTER(i64)],
        "bf_trig_forward": [vp, i64, i64, f32, f32, sp, vp],
        "bf_trig_forward_ex": [vp, i64, i64, f32, f32, sp, vp, op],
        "bf_trig_forward_noalloc": [vp, i64, i64, f32, f32, sp, vp, op],
        "bf_trig_backward": [vp, vp, vp, vp, vp, i64, i64, f32, f32, sp, vp, op],
        "bf_sv_forward": [vp, vp, i64, i64, f32, f32, i32, vp, op],
        "bf_yvv_coeffs": [f64, ctypes.POINTER(f64)],
        "bf_yvv_workspace_bytes": [i64, i64, f32, f32, i32, ctypes.POINTER(i64)],
        "bf_yvv_forward": [vp, i64, i64, f32, f32, f32, vp, op],
        "bf_direct_forward": [vp, i64, i64, f32, f32, sp, vp, op],
        "bf_check_range": [vp, i64, i64, f32, vp, vp],
        "bf_batch_plan_create": [ctypes.POINTER(ImageDesc), i32, ctypes.POINTER(vp)],
        "bf_batch_plan_create_ex": [ctypes.POINTER(ImageDesc), i32, i32, ctypes.POINTER(vp)],
        "bf_batch_bind": [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                          ctypes.POINTER(vp), ctypes.POINTER(vp), vp],
        "bf_batch_launch": [vp, vp],
        "bf_batch_launch_stage": [vp, i32, vp],
        "bf_batch_plan_path": [vp],
        "bf_batch_check": [vp],
        "bf_batch_plan_destroy": [vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = None if name == "bf_batch_plan_destroy" else ctypes.c_int
    L.bf_status_string.restype = ctypes.c_char_p
    L.bf_status_string.argtypes = [ctypes.c_int]
    L.bf_last_error.restype = ctypes.c_char_p
    L.bf_last_error.argtypes = []
    _lib = L
    return L


def check(code: int, where: str):
    if code != 0:
        detail = lib().bf_last_error().decode(errors="replace")
        raise BFError(code, where, detail)


def range_degree(T: float, sigma_r: float) -> int:
    n = ctypes.c_int32()
    check(lib().bf_range_degree(float(T), float(sigma_r), ctypes.byref(n)), "bf_range_degree")
    return int(n.value)


def range_coeffs(N: int):
    cap = N // 2 + 1
    buf = (ctypes.c_float * cap)()
    n = ctypes.c_int32()
    check(lib().bf_range_coeffs(int(N), buf, cap, ctypes.byref(n)), "bf_range_coeffs")
    return [float(buf[i]) for i in range(n.value)]


def spatial_gaussian(sigma_s: float, n_boxes: int = 3):
    s = SpatialSpec()
    check(lib().bf_spatial_gaussian(float(sigma_s), int(n_boxes), ctypes.byref(s)),
          "bf_spatial_gaussian")
    return s.radii()


def make_opts(stream=None, N=0, eta_out=None, tile=None, aux_out=None, workspace=None,
              workspace_bytes=0, trunc_tol=0.0, path=PATH_AUTO) -> Opts:
    o = Opts()
    o.stream = stream
    o.N = int(N)
    o.eta_out = eta_out
    o.tile_h, o.tile_w = (0, 0) if tile is None else (int(tile[0]), int(tile[1]))
    o.aux_out = aux_out
    o.workspace = workspace
    o.workspace_bytes = int(workspace_bytes)
    o.trunc_tol = float(trunc_tol)
    o.path = int(path)
    return o


def range_truncate(N: int, T: float, radii, tol: float):
    """(pairs kept, error bound in gray levels) for term truncation at tol."""
    n = ctypes.c_int32()
    b = ctypes.c_double()
    spec = SpatialSpec.of(radii)
    check(lib().bf_range_truncate(int(N), float(T), ctypes.byref(spec), float(tol),
                                  ctypes.byref(n), ctypes.byref(b)), "bf_range_truncate")
    return int(n.value), float(b.value)


def workspace_bytes(H: int, W: int, radii) -> int:
    """Recommended device workspace of the forward's streamed passes (0 where
    the library evaluates this geometry with the fused kernel)."""
    n = ctypes.c_int64()
    spec = SpatialSpec.of(radii)
    check(lib().bf_trig_workspace_bytes(int(H), int(W), ctypes.byref(spec), ctypes.byref(n)),
          "bf_trig_workspace_bytes")
    return int(n.value)


def stream_workspace_bytes(H: int, W: int, pairs: int) -> int:
    """Workspace of the streamed passes for chunks of `pairs` cosine pairs:
    four column-filtered planes per pair (pitch W rounded up to 64, to 4 below
    64), the
    partial sums and the adjoint's weights (the layout bf_trig_workspace_bytes
    documents)."""
    W = int(W)
    Wp = (W + 3) // 4 * 4 if W < 64 else (W + 63) // 64 * 64
    return 16 * int(pairs) * int(H) * Wp + 24 * int(H) * W


def workspace_bytes_ex(H: int, W: int, T: float, sigma_r: float, N: int, radii) -> int:
    """Recommended workspace of the streamed passes for this degree (every
    pair in one chunk up to 16 GiB of planes; 0 where the fused kernel runs)."""
    n = ctypes.c_int64()
    spec = SpatialSpec.of(radii)
    check(lib().bf_trig_workspace_bytes_ex(int(H), int(W), float(T), float(sigma_r), int(N),
                                           ctypes.byref(spec), ctypes.byref(n)),
          "bf_trig_workspace_bytes_ex")
    return int(n.value)


def yvv_coeffs(sigma_s: float):
    """(B, a1, a2, a3) of the library's recursive-Gaussian line passes."""
    c = (ctypes.c_double * 4)()
    check(lib().bf_yvv_coeffs(float(sigma_s), c), "bf_yvv_coeffs")
    return tuple(float(c[i]) for i in range(4))


def yvv_workspace_bytes(H: int, W: int, T: float, sigma_r: float, N: int = 0) -> int:
    b = ctypes.c_int64()
    check(lib().bf_yvv_workspace_bytes(int(H), int(W), float(T), float(sigma_r), int(N),
                                       ctypes.byref(b)), "bf_yvv_workspace_bytes")
    return int(b.value)
