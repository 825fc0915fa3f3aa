// The forward for callers that cannot allocate device memory: the streamed
// passes take their workspace from a file-scope device array instead of a
// caller buffer or the library's own (hipMalloc'd) workspace.
#include <algorithm>
#include <mutex>

#include "bf_internal.h"

using bf::set_error;

namespace {

// 64 MiB per device, held from the module's load until the process ends.
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxScratchDevices];   // the array's device address, per device

// The array's address on the current device (the name itself is a host-side
// stand-in): looked up once per device, with that device current.
bf_status scratch_address(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) {
        set_error("no current HIP device for the static scratch");
        return BF_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            return BF_EDEVICE;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return BF_OK;
}

}  // namespace

extern "C" bf_status bf_trig_forward_noalloc(const float* f, int64_t H, int64_t W, float T,
                                             float sigma_r, const bf_spatial_spec* spatial_spec,
                                             float* out, const bf_opts* opts) {
    using namespace bf;
    if (opts && opts->workspace) {
        set_error("bf_trig_forward_noalloc takes no workspace (it uses the static scratch)");
        return BF_EINVAL;
    }
    const int path = opts ? opts->path : BF_PATH_AUTO;
    if (path != BF_PATH_AUTO && path != BF_PATH_FUSED && path != BF_PATH_STREAMED) {
        set_error("opts->path=%d is not one of BF_PATH_AUTO, BF_PATH_FUSED, BF_PATH_STREAMED",
                  path);
        return BF_EINVAL;
    }
    bf_status st = check_image(f, H, W, "f");
    if (st != BF_OK) return st;
    SpatialParams sp;
    st = make_spatial(spatial_spec, &sp);
    if (st != BF_OK) return st;
    bf_opts o = {};
    if (opts) o = *opts;
    const bool fits = stream_workspace_bytes(H, W, 1) <= kScratchBytes;
    bool streamed = false;
    if (path == BF_PATH_STREAMED) {
        if (!fits) {
            set_error("H=%lld, W=%lld: one cosine pair of the streamed passes needs %zu bytes; "
                      "the static scratch holds %zu", (long long)H, (long long)W,
                      stream_workspace_bytes(H, W, 1), kScratchBytes);
            return BF_ERANGE;
        }
        streamed = true;
    } else if (path == BF_PATH_AUTO && o.tile_h <= 0 && o.tile_w <= 0 &&
               stream_supported(W, sp)) {
        TileGeom g = {};
        const bf_status fst = plan_fwd_tiles(H, W, sp, 0, 0, &g);
        streamed = fits || fst != BF_OK;
        if (!fits && fst != BF_OK) {
            set_error("H=%lld, W=%lld, R=%d: the fused kernel cannot hold the spatial kernel "
                      "and one cosine pair of the streamed passes needs %zu bytes; the static "
                      "scratch holds %zu", (long long)H, (long long)W, sp.R,
                      stream_workspace_bytes(H, W, 1), kScratchBytes);
            return BF_ERANGE;
        }
    }
    if (streamed) {
        void* p = nullptr;
        st = scratch_address(&p);
        if (st != BF_OK) return st;
        o.workspace = p;
        o.workspace_bytes = (int64_t)kScratchBytes;
        o.path = BF_PATH_STREAMED;
    } else {
        o.path = BF_PATH_FUSED;
    }
    return bf_trig_forward_ex(f, H, W, T, sigma_r, spatial_spec, out, &o);
}
