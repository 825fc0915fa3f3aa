// extern "C" entry points of libbftrig: argument validation, parameter
// derivation and dispatch to the HIP kernels.  The single-image paths
// allocate nothing, except the streamed forward's workspace when the caller
// passes none (allocated once per device, outside stream capture).
#include <algorithm>
#include <cmath>
#include <mutex>

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

// Workspace of the streamed path for callers that pass none: one buffer per
// device, grown on demand (hipMalloc, never during stream capture) and kept
// until the process ends.  Calls on different streams are ordered through an
// event recorded after each use, so they never share it concurrently.
struct LibWorkspace {
    void* p = nullptr;
    size_t n = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};
constexpr int kMaxDevices = 64;
std::mutex g_ws_mu;
LibWorkspace g_ws[kMaxDevices];
thread_local int g_ws_dev = -1;

}  // namespace

namespace bf {

bf_status library_workspace(size_t need, hipStream_t stream, void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_error("no current HIP device for the library workspace");
        return BF_EDEVICE;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess) cs = hipStreamCaptureStatusNone;
    g_ws_mu.lock();   // held until library_workspace_done (or an error below)
    LibWorkspace& w = g_ws[dev];
    if (cs != hipStreamCaptureStatusNone) {
        g_ws_mu.unlock();
        set_error("the streamed path needs opts->workspace while the stream is being captured");
        return BF_ECAPTURE;
    }
    if (!w.done && hipEventCreateWithFlags(&w.done, hipEventDisableTiming) != hipSuccess) {
        w.done = nullptr;
        g_ws_mu.unlock();
        set_error("hipEventCreateWithFlags failed");
        return BF_EDEVICE;
    }
    if (w.n < need) {
        if (w.p) {
            if (hipDeviceSynchronize() != hipSuccess || hipFree(w.p) != hipSuccess) {
                g_ws_mu.unlock();
                set_error("freeing the library workspace failed");
                return BF_EDEVICE;
            }
            w.p = nullptr;
            w.n = 0;
            w.pending = false;
        }
        if (hipMalloc(&w.p, need) != hipSuccess) {
            w.p = nullptr;
            (void)hipGetLastError();
            g_ws_mu.unlock();
            set_error("allocating the %zu-byte library workspace failed", need);
            return BF_ENOMEM;
        }
        w.n = need;
    }
    if (w.pending && hipStreamWaitEvent(stream, w.done, 0) != hipSuccess) {
        g_ws_mu.unlock();
        set_error("hipStreamWaitEvent on the library workspace failed");
        return BF_EDEVICE;
    }
    g_ws_dev = dev;
    *out = w.p;
    return BF_OK;
}

bf_status library_workspace_done(hipStream_t stream) {
    LibWorkspace& w = g_ws[g_ws_dev];
    const bool ok = hipEventRecord(w.done, stream) == hipSuccess;
    w.pending = ok;
    g_ws_mu.unlock();
    if (!ok) {
        set_error("hipEventRecord on the library workspace failed");
        return BF_EDEVICE;
    }
    return BF_OK;
}

// The streamed passes with the caller's workspace (validated) or the
// library's own.
bf_status run_stream(int mode, const StreamIO& io, int64_t H, int64_t W, const Common& c,
                     const bf_opts* opts, int64_t bytes) {
    if (!stream_supported(W, c.sp)) {
        set_error("the streamed path handles W + 2R <= 5184 and a kernel mass below 2^31 "
                  "(W=%lld, R=%d)", (long long)W, c.sp.R);
        return BF_EUNSUPPORTED;
    }
    void* ws = opts ? opts->workspace : nullptr;
    size_t wsb = opts && opts->workspace_bytes > 0 ? (size_t)opts->workspace_bytes : 0;
    bf_status st = BF_OK;
    if (ws) {
        const void* imgs[9] = {io.f, io.out, io.eta, io.aux, io.fout, io.feta,
                               io.faux, io.gout, io.gf};
        const int64_t sizes[9] = {bytes, bytes, bytes, 2 * bytes, bytes, bytes,
                                  2 * bytes, bytes, bytes};
        for (int i = 0; i < 9; ++i) {
            if (imgs[i] && overlaps(ws, (int64_t)wsb, imgs[i], sizes[i])) {
                set_error("workspace must not overlap the images");
                return BF_EINVAL;
            }
        }
        if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) {
            set_error("the streamed path's workspace must be 256-byte aligned");
            return BF_EINVAL;
        }
        if (stream_chunk_pairs(H, W, wsb, c.rp.npairs) <= 0) {
            set_error("workspace of %zu bytes is below the %zu bytes of one cosine pair",
                      wsb, stream_workspace_bytes(H, W, 1));
            return BF_EINVAL;
        }
    } else {
        wsb = stream_default_workspace(H, W, c.rp.npairs);
        st = library_workspace(wsb, c.stream, &ws);
        if (st != BF_OK) return st;
    }
    st = launch_stream(mode, io, H, W, c.rp, c.sp, ws, wsb, c.stream);
    if (!(opts && opts->workspace)) {
        const bf_status st2 = library_workspace_done(c.stream);   // releases the lock
        if (st == BF_OK) st = st2;
    }
    return st;
}

}  // namespace bf

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
    const int path = opts ? opts->path : BF_PATH_AUTO;
    if (path != BF_PATH_AUTO && path != BF_PATH_FUSED && path != BF_PATH_STREAMED) {
        set_error("opts->path=%d is not one of BF_PATH_AUTO, BF_PATH_FUSED, BF_PATH_STREAMED",
                  path);
        return BF_EINVAL;
    }
    TileGeom g = {};
    const int req_h = opts ? opts->tile_h : 0, req_w = opts ? opts->tile_w : 0;
    const bf_status fst = plan_fwd_tiles(H, W, c.sp, req_h, req_w, &g);
    // the streamed passes: where the fused kernel cannot hold the kernel width,
    // or where its shrunken tiles cost more (no tile shape forced), or on request
    bool streamed;
    if (path == BF_PATH_FUSED || req_h > 0 || req_w > 0)
        streamed = false;
    else if (path == BF_PATH_STREAMED)
        streamed = true;
    else
        streamed = prefer_stream(H, W, c.sp, fst, g);
    if (!streamed) {
        if (fst != BF_OK) return fst;
        return launch_fwd(f, out, eta, aux, H, W, c.rp, c.sp, g, c.stream);
    }
    StreamIO io = {};
    io.f = f;
    io.out = out;
    io.eta = eta;
    io.aux = aux;
    return run_stream(kStreamFwd, io, H, W, c, opts, bytes);
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
    if (prefer_stream(H, W, sp, st, g)) {
        *bytes_out = (int64_t)stream_workspace_bytes(H, W, kStreamChunkPairs);
        return BF_OK;
    }
    if (st != BF_OK)
        set_error("neither the fused kernel nor the streamed passes handle W=%lld, R=%d",
                  (long long)W, sp.R);
    return st;
}

bf_status bf_trig_workspace_bytes_ex(int64_t H, int64_t W, float T, float sigma_r, int32_t N,
                                     const bf_spatial_spec* spatial_spec, int64_t* bytes_out) {
    bf_status st = bf_trig_workspace_bytes(H, W, spatial_spec, bytes_out);
    if (st != BF_OK || *bytes_out == 0) return st;
    RangeParams rp;
    st = make_range((double)T, (double)sigma_r, N, &rp);
    if (st != BF_OK) {
        *bytes_out = 0;
        return st;
    }
    *bytes_out = (int64_t)stream_default_workspace(H, W, rp.npairs);
    return BF_OK;
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

}  // extern "C"

namespace {

// The adjoint given the forward's sums P and Q (aux).
bf_status backward_with_sums(const float* f, const float* out, const float* eta,
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
    const int path = opts ? opts->path : BF_PATH_AUTO;
    if (path != BF_PATH_AUTO && path != BF_PATH_FUSED && path != BF_PATH_STREAMED) {
        set_error("opts->path=%d is not one of BF_PATH_AUTO, BF_PATH_FUSED, BF_PATH_STREAMED",
                  path);
        return BF_EINVAL;
    }
    const int req_h = opts ? opts->tile_h : 0, req_w = opts ? opts->tile_w : 0;
    TileGeom g = {};
    const bf_status fst = plan_bwd_tiles(H, W, c.sp, req_h, req_w, &g, f);
    bool streamed;
    if (path == BF_PATH_FUSED || req_h > 0 || req_w > 0)
        streamed = false;
    else if (path == BF_PATH_STREAMED)
        streamed = true;
    else
        streamed = prefer_stream(H, W, c.sp, fst, g);
    if (!streamed) {
        if (fst != BF_OK) return fst;
        return launch_bwd(f, out, eta, aux, grad_out, grad_f, H, W, c.rp, c.sp, g, c.stream);
    }
    StreamIO io = {};
    io.f = f;
    io.fout = out;
    io.feta = eta;
    io.faux = aux;
    io.gout = grad_out;
    io.gf = grad_f;
    return run_stream(kStreamBwd, io, H, W, c, opts, bytes);
}

}  // namespace

extern "C" {

bf_status bf_trig_backward(const float* f, const float* out, const float* eta,
                           const float* aux, const float* grad_out, int64_t H, int64_t W,
                           float T, float sigma_r, const bf_spatial_spec* spatial_spec,
                           float* grad_f, const bf_opts* opts) {
    if (aux)
        return backward_with_sums(f, out, eta, aux, grad_out, H, W, T, sigma_r, spatial_spec,
                                  grad_f, opts);
    // The caller kept only out and eta: P and Q come from a forward of the
    // library's own (they depend on f and the parameters alone), written with
    // a scratch copy of out into the library workspace, followed by the
    // streamed passes' planes unless the caller brings a workspace.
    Common c;
    bf_status st = prepare(f, H, W, T, sigma_r, spatial_spec, opts, &c);
    if (st != BF_OK) return st;
    const void* bufs[4] = {out, eta, grad_out, grad_f};
    const char* names[4] = {"out", "eta", "grad_out", "grad_f"};
    for (int i = 0; i < 4; ++i) {
        st = check_image(bufs[i], H, W, names[i]);
        if (st != BF_OK) return st;
    }
    const int64_t bytes = H * W * (int64_t)sizeof(float);
    const void* ins[4] = {f, out, eta, grad_out};
    for (int i = 0; i < 4; ++i) {
        if (overlaps(ins[i], bytes, grad_f, bytes)) {
            set_error("grad_f must not overlap the inputs");
            return BF_EINVAL;
        }
    }
    const int path = opts ? opts->path : BF_PATH_AUTO;
    if (path != BF_PATH_AUTO && path != BF_PATH_FUSED && path != BF_PATH_STREAMED) {
        set_error("opts->path=%d is not one of BF_PATH_AUTO, BF_PATH_FUSED, BF_PATH_STREAMED",
                  path);
        return BF_EINVAL;
    }
    const size_t plane = (size_t)bytes;
    const size_t sums = (3 * plane + 255) & ~(size_t)255;   // P, Q, scratch out
    const bool own_planes = !(opts && opts->workspace) && stream_supported(W, c.sp);
    const size_t planes = own_planes ? stream_default_workspace(H, W, c.rp.npairs) : 0;
    void* base = nullptr;
    st = library_workspace(sums + planes, c.stream, &base);
    if (st != BF_OK) return st;
    float* pq = static_cast<float*>(base);
    float* out2 = pq + 2 * (size_t)H * (size_t)W;
    bf_opts o = {};
    if (opts) o = *opts;
    o.eta_out = nullptr;
    o.aux_out = pq;
    if (own_planes) {
        o.workspace = static_cast<unsigned char*>(base) + sums;
        o.workspace_bytes = (int64_t)planes;
    }
    st = bf_trig_forward_ex(f, H, W, T, sigma_r, spatial_spec, out2, &o);
    if (st == BF_OK)
        st = backward_with_sums(f, out, eta, pq, grad_out, H, W, T, sigma_r, spatial_spec,
                                grad_f, &o);
    const bf_status st2 = library_workspace_done(c.stream);   // releases the lock
    return st == BF_OK ? st2 : st;
}

}  // extern "C"
