// Host side of the single-image fused kernels: tile planning and launches.
// The kernels themselves are in bf_tile.h.
#include "bf_tile.h"

namespace bf {

bf_status plan_tiles(int mode, int64_t H, int64_t W, const SpatialParams& sp, int req_h,
                            int req_w, TileGeom* g) {
    const int R = sp.R;
    for (int k = 0; k < sp.nb; ++k) {
        if (sp.r[k] > kBoxMaxRadius) {
            set_error("box radius %d exceeds %d, the largest the register-line kernels handle",
                      sp.r[k], kBoxMaxRadius);
            return BF_EUNSUPPORTED;
        }
    }
    const int ext_max = kTileThreads * (mode == kForward ? ModeTraits<kForward>::kKMax
                                                         : ModeTraits<kBackward>::kKMax);
    const int nacc = mode == kForward ? ModeTraits<kForward>::kAcc : ModeTraits<kBackward>::kAcc;
    auto lds_of = [&](int th, int tw) {
        return tile_lds_floats(th, tw, th + 2 * R, tw + 2 * R, nacc) * sizeof(float);
    };
    auto fits = [&](int th, int tw) {
        const int eh = th + 2 * R, ew = tw + 2 * R;
        return th >= 1 && tw >= 1 && (int64_t)eh * ew <= ext_max && eh <= kLine && ew <= kLine &&
               tw <= kTileThreads - kColLane0 && lds_of(th, tw) <= 160 * 1024;
    };
    int th = req_h, tw = req_w;
    if (th <= 0 || tw <= 0) {
        // odd tile sides keep the extended pitches odd, so lanes striding by a
        // row or column of LDS hit distinct banks
        int side = 0;
        for (int s = 1; s <= kLine; s += 2)
            if (fits(s, s)) side = s;
        if (side == 0) {
            set_error("spatial radius R=%d too large for the fused tile kernels", R);
            return BF_EUNSUPPORTED;
        }
        th = tw = side;
        if (th > H) th = (int)(H | 1);
        if (tw > W) tw = (int)(W | 1);
        while (th < H && fits(th + 2, tw)) th += 2;
        while (tw < W && fits(th, tw + 2)) tw += 2;
    } else if (!fits(th, tw)) {
        set_error("tile %dx%d does not fit (R=%d)", th, tw, R);
        return BF_EINVAL;
    }
    g->TH = th;
    g->TW = tw;
    g->EH = th + 2 * R;
    g->EW = tw + 2 * R;
    g->tiles_y = (int)((H + th - 1) / th);
    g->tiles_x = (int)((W + tw - 1) / tw);
    g->lds_bytes = lds_of(th, tw);
    return BF_OK;
}

bf_status plan_fwd_tiles(int64_t H, int64_t W, const SpatialParams& sp, int req_h, int req_w,
                         TileGeom* g) {
    return plan_tiles(kForward, H, W, sp, req_h, req_w, g);
}

bf_status plan_bwd_tiles(int64_t H, int64_t W, const SpatialParams& sp, int req_h, int req_w,
                         TileGeom* g) {
    return plan_tiles(kBackward, H, W, sp, req_h, req_w, g);
}

void fill_tile_args(TileArgs& a, int64_t H, int64_t W, const RangeParams& rp,
                        const SpatialParams& sp, const TileGeom& g, int mode) {
    a.H = (int)H;
    a.W = (int)W;
    a.TH = g.TH;
    a.TW = g.TW;
    a.EH = g.EH;
    a.EW = g.EW;
    a.tiles_x = g.tiles_x;
    a.R = sp.R;
    a.nb = sp.nb;
    for (int k = 0; k < BF_MAX_BOXES; ++k) a.r[k] = sp.r[k];
    a.npairs = rp.npairs;
    a.odd = rp.odd;
    if (mode == kForward)
        a.nsteps = 4 * rp.npairs - (rp.odd ? 0 : 2);
    else
        a.nsteps = 8 * rp.npairs - (rp.odd ? 0 : 7);
    a.alpha = rp.alpha;
    a.alpha_f = (float)rp.alpha;
    a.two_alpha = (float)(2.0 * rp.alpha);
    a.center = rp.center;
    for (int q = 0; q < kMaxPairs; ++q) a.chat[q] = q < rp.npairs ? rp.chat[q] : 0.0f;
}

template <int MODE>
static bf_status launch_tile(const TileArgs& a, const TileGeom& g, hipStream_t stream,
                             const char* what) {
    const dim3 grid((unsigned)(g.tiles_x * g.tiles_y)), block(kTileThreads);
    (void)hipFuncSetAttribute((const void*)bf_tile_kernel<MODE>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds_bytes);
    hipLaunchKernelGGL(bf_tile_kernel<MODE>, grid, block, g.lds_bytes, stream, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s launch failed: %s", what, hipGetErrorString(e));
        return BF_EDEVICE;
    }
    return BF_OK;
}

bf_status launch_fwd(const float* f, float* out, float* eta, int64_t H, int64_t W,
                     const RangeParams& rp, const SpatialParams& sp, const TileGeom& g,
                     hipStream_t stream) {
    TileArgs a = {};
    a.f = f;
    a.out = out;
    a.eta = eta;
    fill_tile_args(a, H, W, rp, sp, g, kForward);
    return launch_tile<kForward>(a, g, stream, "forward");
}

bf_status launch_bwd(const float* f, const float* out, const float* eta, const float* gout,
                     float* gf, int64_t H, int64_t W, const RangeParams& rp,
                     const SpatialParams& sp, const TileGeom& g, hipStream_t stream) {
    TileArgs a = {};
    a.f = f;
    a.out = gf;
    a.fout = out;
    a.feta = eta;
    a.gout = gout;
    fill_tile_args(a, H, W, rp, sp, g, kBackward);
    return launch_tile<kBackward>(a, g, stream, "backward");
}

}  // namespace bf
