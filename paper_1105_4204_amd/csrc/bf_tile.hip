// Host side of the single-image fused kernels: tile planning and launches.
// The kernels themselves are in bf_tile.h.
#include <algorithm>

#include "bf_tile.h"

namespace bf {

static constexpr size_t kLdsLimit = 160 * 1024 - 256;   // LDS per workgroup on gfx950, less
                                                          // room for a persistent kernel's statics

bf_status plan_tiles(int mode, int64_t H, int64_t W, const SpatialParams& sp, int req_h,
                     int req_w, TileGeom* g, bool gg) {
    const int R = sp.R;
    for (int k = 0; k < sp.nb; ++k) {
        if (sp.r[k] > kBoxMaxRadius) {
            set_error("box radius %d exceeds %d, the largest the register-line kernels handle",
                      sp.r[k], kBoxMaxRadius);
            return BF_EUNSUPPORTED;
        }
    }
    const int side_max = std::min(kOutMax, kLine - 2 * R);
    if (side_max < 1) {
        set_error("spatial radius R=%d too large for the fused tile kernels (2R+1 > %d)", R,
                  kLine);
        return BF_EUNSUPPORTED;
    }
    auto lds_of = [&](int th, int tw) {
        return tile_lds_floats(mode, th, tw, R, gg) * sizeof(float);
    };
    auto fits = [&](int th, int tw) {
        return th >= 1 && tw >= 1 && th <= side_max && tw <= side_max &&
               lds_of(th, tw) <= kLdsLimit && (!gg || tw % 4 == 0);
    };
    int th = req_h, tw = req_w;
    if (th <= 0 || tw <= 0) {
        // Every tile costs about the same (each wave runs the whole line
        // program whatever its active lanes), so take the fewest tiles, then
        // the largest area.
        const int hmax = (int)std::min<int64_t>(side_max, H);
        const int wmax = (int)std::min<int64_t>(side_max, W);
        int64_t best_n = -1, best_area = -1;
        for (int h = hmax; h >= 1; --h) {
            int w = wmax;
            while (w >= 1 && !fits(h, w)) --w;
            if (w < 1) continue;
            const int64_t n = ((H + h - 1) / h) * ((W + w - 1) / w);
            const int64_t area = (int64_t)h * w;
            if (best_n < 0 || n < best_n || (n == best_n && area > best_area)) {
                best_n = n;
                best_area = area;
                th = h;
                tw = w;
            }
        }
        if (best_n < 0) {
            set_error("no tile fits for R=%d", R);
            return BF_EUNSUPPORTED;
        }
    } else if (!fits(th, tw)) {
        set_error("tile %dx%d does not fit (R=%d: sides <= %d, LDS <= %zu bytes)", th, tw, R,
                  side_max, kLdsLimit);
        return BF_EINVAL;
    }
    g->TH = th;
    g->TW = tw;
    g->EH = th + 2 * R;
    g->EW = tw + 2 * R;
    g->EWp = tile_pitch(g->EW);
    g->EHp = tile_pitch(g->EH);
    g->tiles_y = (int)((H + th - 1) / th);
    g->tiles_x = (int)((W + tw - 1) / tw);
    g->lds_bytes = lds_of(th, tw);
    g->gg = gg;
    // every lane of the single-image kernels runs its whole register line,
    // whatever part of it the tile uses, so extended tiles of at most 120
    // take the shorter line (about 6 % less work for R <= 28 at 64 x 64)
    g->line = (g->EH <= kLineShort && g->EW <= kLineShort) ? kLineShort : kLine;
    return BF_OK;
}

bf_status plan_fwd_tiles(int64_t H, int64_t W, const SpatialParams& sp, int req_h, int req_w,
                         TileGeom* g) {
    return plan_tiles(kForward, H, W, sp, req_h, req_w, g);
}

// The adjoint reads g from global memory (GG), freeing one LDS plane for
// larger tiles, when 16-byte row chunks line up with the image: W and R
// multiples of 4, f 16-byte aligned and the image under 2 GiB (32-bit buffer
// offsets); the tile width is then kept a multiple of 4 as well.  Otherwise
// g is staged in LDS.
bf_status plan_bwd_tiles(int64_t H, int64_t W, const SpatialParams& sp, int req_h, int req_w,
                         TileGeom* g, const float* f) {
    const bool gg_ok = W % 4 == 0 && sp.R % 4 == 0 && H * W * 4 < ((int64_t)1 << 31) &&
                       (reinterpret_cast<uintptr_t>(f) & 15) == 0 &&
                       (req_w <= 0 || req_w % 4 == 0);
    if (gg_ok && plan_tiles(kBackward, H, W, sp, req_h, req_w, g, true) == BF_OK) return BF_OK;
    return plan_tiles(kBackward, H, W, sp, req_h, req_w, g, false);
}

void fill_tile_args(TileArgs& a, int64_t H, int64_t W, const RangeParams& rp,
                    const SpatialParams& sp, const TileGeom& g, int mode) {
    a.H = (int)H;
    a.W = (int)W;
    a.TH = g.TH;
    a.TW = g.TW;
    a.EH = g.EH;
    a.EW = g.EW;
    a.EWp = g.EWp;
    a.EHp = g.EHp;
    a.tiles_x = g.tiles_x;
    a.R = sp.R;
    a.nb = sp.nb;
    for (int k = 0; k < BF_MAX_BOXES; ++k) a.r[k] = sp.r[k];
    a.npairs = rp.npairs;
    a.odd = rp.odd;
    // four channels per pair; the centre pair of an even degree has two
    // (forward: 1, g) or one (adjoint: A)
    a.nsteps = 4 * rp.npairs - (rp.odd ? 0 : (mode == kForward ? 2 : 3));
    a.alpha_f = (float)rp.alpha;
    a.two_alpha = (float)(2.0 * rp.alpha);
    a.center = rp.center;
    for (int q = 0; q < kMaxPairs; ++q) a.chat[q] = q < rp.npairs ? rp.chat[q] : 0.0f;
}

template <int MODE, bool AUX, bool GG = false>
static bf_status launch_tile(const TileArgs& a, const TileGeom& g, hipStream_t stream,
                             const char* what) {
    const dim3 grid((unsigned)(g.tiles_x * g.tiles_y)), block(kTileThreads);
    if (g.line == kLineShort) {
        (void)hipFuncSetAttribute((const void*)bf_tile_kernel<MODE, AUX, GG, kLineShort>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds_bytes);
        hipLaunchKernelGGL((bf_tile_kernel<MODE, AUX, GG, kLineShort>), grid, block,
                           g.lds_bytes, stream, a);
    } else {
        (void)hipFuncSetAttribute((const void*)bf_tile_kernel<MODE, AUX, GG>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds_bytes);
        hipLaunchKernelGGL((bf_tile_kernel<MODE, AUX, GG>), grid, block, g.lds_bytes, stream, a);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s launch failed: %s", what, hipGetErrorString(e));
        return BF_EDEVICE;
    }
    return BF_OK;
}

bf_status launch_fwd(const float* f, float* out, float* eta, float* aux, int64_t H, int64_t W,
                     const RangeParams& rp, const SpatialParams& sp, const TileGeom& g,
                     hipStream_t stream) {
    TileArgs a = {};
    a.f = f;
    a.out = out;
    a.eta = eta;
    a.aux = aux;
    fill_tile_args(a, H, W, rp, sp, g, kForward);
    if (aux) return launch_tile<kForward, true>(a, g, stream, "forward");
    return launch_tile<kForward, false>(a, g, stream, "forward");
}

bf_status launch_bwd(const float* f, const float* out, const float* eta, const float* aux,
                     const float* gout, float* gf, int64_t H, int64_t W, const RangeParams& rp,
                     const SpatialParams& sp, const TileGeom& g, hipStream_t stream) {
    TileArgs a = {};
    a.f = f;
    a.out = gf;
    a.fout = out;
    a.feta = eta;
    a.paux = aux;
    a.gout = gout;
    fill_tile_args(a, H, W, rp, sp, g, kBackward);
    if (g.gg) return launch_tile<kBackward, false, true>(a, g, stream, "backward");
    return launch_tile<kBackward, false>(a, g, stream, "backward");
}

}  // namespace bf
