// extern "C" entry points of libbftrig: argument validation, parameter
// derivation and dispatch to the HIP kernels.  Nothing here allocates on the
// single-image paths, so they may be captured into a hipGraph.
#include <cmath>

#include "bf_internal.h"

using namespace bf;

namespace {

struct Common {
    RangeParams rp;
    SpatialParams sp;
    hipStream_t stream;
};

bf_status prepare(const float* f, int64_t H, int64_t W, float T, float sigma_r,
                  const bf_spatial_spec* spec, const bf_opts* opts, Common* c) {
    bf_status st = check_image(f, H, W, "f");
    if (st != BF_OK) return st;
    st = make_spatial(spec, &c->sp);
    if (st != BF_OK) return st;
    st = make_range((double)T, (double)sigma_r, opts ? opts->N : 0, &c->rp);
    if (st != BF_OK) return st;
    if (opts && opts->trunc_tol != 0.0f) {
        st = truncate_pairs(&c->rp, c->sp, (double)T, (double)opts->trunc_tol, nullptr);
        if (st != BF_OK) return st;
    }
    c->stream = opts ? (hipStream_t)opts->stream : nullptr;
    return BF_OK;
}

}  // namespace

extern "C" {

bf_status bf_trig_forward_ex(const float* f, int64_t H, int64_t W, float T, float sigma_r,
                             const bf_spatial_spec* spatial_spec, float* out,
                             const bf_opts* opts) {
    Common c;
    bf_status st = prepare(f, H, W, T, sigma_r, spatial_spec, opts, &c);
    if (st != BF_OK) return st;
    st = check_image(out, H, W, "out");
    if (st != BF_OK) return st;
    const int64_t bytes = H * W * (int64_t)sizeof(float);
    float* eta = opts ? opts->eta_out : nullptr;
    float* aux = opts ? opts->aux_out : nullptr;
    if (overlaps(f, out, bytes) || overlaps(f, eta, bytes) || overlaps(out, eta, bytes) ||
        overlaps(f, bytes, aux, 2 * bytes) || overlaps(out, bytes, aux, 2 * bytes) ||
        overlaps(eta, bytes, aux, 2 * bytes)) {
        set_error("out / eta_out / aux_out must not overlap f or each other");
        return BF_EINVAL;
    }
    TileGeom g = {};
    const int req_h = opts ? opts->tile_h : 0, req_w = opts ? opts->tile_w : 0;
    st = plan_fwd_tiles(H, W, c.sp, req_h, req_w, &g);
    const bool fused_ok = st == BF_OK;
    const size_t need = staged_workspace_bytes(H, W);
    void* ws = opts ? opts->workspace : nullptr;
    const bool have_ws = ws && opts->workspace_bytes >= (int64_t)need;
    // the staged passes: where the fused kernel cannot hold the kernel width,
    // or where its shrunken tiles cost more (and a workspace is given, no
    // adjoint sums are requested and no tile shape was forced)
    const bool staged =
        staged_supported(c.sp) &&
        (!fused_ok || (have_ws && !aux && req_h <= 0 && req_w <= 0 &&
                       prefer_staged(H, W, c.sp, st, g)));
    if (staged) {
        if (aux) {
            set_error("R=%d: the adjoint's sums (aux_out) are only produced by the fused kernel "
                      "(R <= 63)", c.sp.R);
            return BF_EUNSUPPORTED;
        }
        if (!have_ws) {
            set_error("R=%d needs the staged path and a workspace of %zu bytes "
                      "(bf_trig_workspace_bytes)", c.sp.R, need);
            return BF_EINVAL;
        }
        if (overlaps(ws, (int64_t)need, f, bytes) || overlaps(ws, (int64_t)need, out, bytes) ||
            overlaps(ws, (int64_t)need, eta, bytes)) {
            set_error("workspace must not overlap the images");
            return BF_EINVAL;
        }
        if ((reinterpret_cast<uintptr_t>(ws) & 15) != 0) {
            set_error("the staged path's workspace must be 16-byte aligned");
            return BF_EINVAL;
        }
        return launch_staged(f, out, eta, H, W, c.rp, c.sp, ws, c.stream);
    }
    if (st != BF_OK) return st;
    return launch_fwd(f, out, eta, aux, H, W, c.rp, c.sp, g, c.stream);
}

bf_status bf_trig_workspace_bytes(int64_t H, int64_t W, const bf_spatial_spec* spatial_spec,
                                  int64_t* bytes_out) {
    if (!bytes_out) {
        set_error("bytes_out is NULL");
        return BF_EINVAL;
    }
    *bytes_out = 0;
    if (H <= 0 || W <= 0) {
        set_error("image size %lld x %lld must be positive", (long long)H, (long long)W);
        return BF_EINVAL;
    }
    SpatialParams sp;
    bf_status st = make_spatial(spatial_spec, &sp);
    if (st != BF_OK) return st;
    TileGeom g = {};
    st = plan_fwd_tiles(H, W, sp, 0, 0, &g);
    if (st != BF_OK && st != BF_EUNSUPPORTED) return st;
    if (prefer_staged(H, W, sp, st, g)) {
        *bytes_out = (int64_t)staged_workspace_bytes(H, W);
        return BF_OK;
    }
    return st;
}

bf_status bf_trig_forward(const float* f, int64_t H, int64_t W, float T, float sigma_r,
                          const bf_spatial_spec* spatial_spec, float* out) {
    return bf_trig_forward_ex(f, H, W, T, sigma_r, spatial_spec, out, nullptr);
}

bf_status bf_direct_forward(const float* f, int64_t H, int64_t W, float T, float sigma_r,
                            const bf_spatial_spec* spatial_spec, float* out,
                            const bf_opts* opts) {
    Common c;
    bf_status st = prepare(f, H, W, T, sigma_r, spatial_spec, opts, &c);
    if (st != BF_OK) return st;
    st = check_image(out, H, W, "out");
    if (st != BF_OK) return st;
    const int64_t bytes = H * W * (int64_t)sizeof(float);
    float* eta = opts ? opts->eta_out : nullptr;
    if (overlaps(f, out, bytes) || overlaps(f, eta, bytes) || overlaps(out, eta, bytes)) {
        set_error("out / eta_out must not overlap f or each other");
        return BF_EINVAL;
    }
    return launch_direct(f, out, eta, H, W, c.rp, c.sp, c.stream);
}

bf_status bf_check_range(const float* f, int64_t H, int64_t W, float T, uint32_t* count_dev,
                         void* stream) {
    bf_status st = check_image(f, H, W, "f");
    if (st != BF_OK) return st;
    if (!count_dev) {
        set_error("count_dev is NULL");
        return BF_EINVAL;
    }
    if (!(T > 0.0f) || !std::isfinite(T)) {
        set_error("T=%g must be positive and finite", (double)T);
        return BF_EINVAL;
    }
    return launch_check_range(f, H, W, T, count_dev, static_cast<hipStream_t>(stream));
}

bf_status bf_sv_forward(const float* f, const int32_t* radius, int64_t H, int64_t W, float T,
                        float sigma_r, int32_t rmax, float* out, const bf_opts* opts) {
    if (rmax < 0) {
        set_error("rmax=%d must be >= 0", rmax);
        return BF_EINVAL;
    }
    // the truncation bound (if asked for) is taken for the widest box
    bf_spatial_spec box = {};
    box.n_boxes = 1;
    box.radius[0] = rmax;
    Common c;
    bf_status st = prepare(f, H, W, T, sigma_r, &box, opts, &c);
    if (st != BF_OK) return st;
    st = check_image(out, H, W, "out");
    if (st != BF_OK) return st;
    st = check_image(radius, H, W, "radius");
    if (st != BF_OK) return st;
    const int64_t bytes = H * W * (int64_t)sizeof(float);
    float* eta = opts ? opts->eta_out : nullptr;
    if (overlaps(f, out, bytes) || overlaps(f, eta, bytes) || overlaps(out, eta, bytes) ||
        overlaps(radius, out, bytes) || overlaps(radius, eta, bytes)) {
        set_error("out / eta_out must not overlap f, radius or each other");
        return BF_EINVAL;
    }
    return launch_sv(f, radius, out, eta, H, W, rmax, c.rp, c.stream);
}

bf_status bf_yvv_workspace_bytes(int64_t H, int64_t W, float T, float sigma_r, int32_t N,
                                 int64_t* bytes_out) {
    if (!bytes_out) {
        set_error("bytes_out is NULL");
        return BF_EINVAL;
    }
    *bytes_out = 0;
    if (H <= 0 || W <= 0) {
        set_error("image size %lld x %lld must be positive", (long long)H, (long long)W);
        return BF_EINVAL;
    }
    RangeParams rp;
    bf_status st = make_range((double)T, (double)sigma_r, N, &rp);
    if (st != BF_OK) return st;
    *bytes_out = (int64_t)yvv_workspace_bytes(H, W, rp.npairs);
    return BF_OK;
}

bf_status bf_yvv_forward(const float* f, int64_t H, int64_t W, float T, float sigma_r,
                         float sigma_s, float* out, const bf_opts* opts) {
    bf_status st = check_image(f, H, W, "f");
    if (st != BF_OK) return st;
    st = check_image(out, H, W, "out");
    if (st != BF_OK) return st;
    YvvParams yp;
    st = make_yvv((double)sigma_s, &yp);
    if (st != BF_OK) return st;
    RangeParams rp;
    st = make_range((double)T, (double)sigma_r, opts ? opts->N : 0, &rp);
    if (st != BF_OK) return st;
    if (opts && opts->trunc_tol != 0.0f) {
        st = truncate_pairs_km(&rp, yp.k0, 1.0, (double)T, (double)opts->trunc_tol, nullptr);
        if (st != BF_OK) return st;
    }
    const int64_t bytes = H * W * (int64_t)sizeof(float);
    float* eta = opts ? opts->eta_out : nullptr;
    void* ws = opts ? opts->workspace : nullptr;
    const int64_t wsb = opts ? opts->workspace_bytes : 0;
    if (!ws) {
        set_error("the recursive-Gaussian forward needs opts->workspace (bf_yvv_workspace_bytes)");
        return BF_EINVAL;
    }
    if (overlaps(f, out, bytes) || overlaps(f, eta, bytes) || overlaps(out, eta, bytes) ||
        overlaps(ws, wsb, f, bytes) || overlaps(ws, wsb, out, bytes) ||
        overlaps(ws, wsb, eta, bytes)) {
        set_error("out / eta_out / workspace must not overlap f or each other");
        return BF_EINVAL;
    }
    return launch_yvv(f, out, eta, H, W, rp, yp, ws, (size_t)(wsb > 0 ? wsb : 0),
                      opts ? (hipStream_t)opts->stream : nullptr);
}

bf_status bf_trig_backward(const float* f, const float* out, const float* eta,
                           const float* aux, const float* grad_out, int64_t H, int64_t W,
                           float T, float sigma_r, const bf_spatial_spec* spatial_spec,
                           float* grad_f, const bf_opts* opts) {
    Common c;
    bf_status st = prepare(f, H, W, T, sigma_r, spatial_spec, opts, &c);
    if (st != BF_OK) return st;
    const void* bufs[5] = {out, eta, aux, grad_out, grad_f};
    const char* names[5] = {"out", "eta", "aux", "grad_out", "grad_f"};
    for (int i = 0; i < 5; ++i) {
        st = check_image(bufs[i], H, W, names[i]);
        if (st != BF_OK) return st;
    }
    const int64_t bytes = H * W * (int64_t)sizeof(float);
    const void* ins[5] = {f, out, eta, aux, grad_out};
    const int64_t sizes[5] = {bytes, bytes, bytes, 2 * bytes, bytes};
    for (int i = 0; i < 5; ++i) {
        if (overlaps(ins[i], sizes[i], grad_f, bytes)) {
            set_error("grad_f must not overlap the inputs");
            return BF_EINVAL;
        }
    }
    TileGeom g;
    st = plan_bwd_tiles(H, W, c.sp, opts ? opts->tile_h : 0, opts ? opts->tile_w : 0, &g, f);
    if (st != BF_OK) return st;
    return launch_bwd(f, out, eta, aux, grad_out, grad_f, H, W, c.rp, c.sp, g, c.stream);
}

}  // extern "C"
