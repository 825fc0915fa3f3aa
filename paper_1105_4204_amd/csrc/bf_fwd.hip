// Fused O(1) forward kernel of the trigonometric bilateral filter (gfx950).
//
// One workgroup owns an output tile of TH x TW pixels and the extended tile
// (TH + 2R) x (TW + 2R) around it.  For every cosine pair m of the raised
// cosine (Sec. 2.3) it builds the auxiliary images of eq. (final-form) on the
// extended tile -- C = cos(m a g), S = sin(m a g), gC, gS with g = f - T/2,
// zero outside the image -- filters each with the separable iterated-box
// kernel, and demodulates at the output pixels:
//     den += c_m (C F[C] + S F[S]),   num += c_m (C F[gC] + S F[gS]).
// After the last pair, out = T/2 + num / den (divided in FP64) and eta = den.
// The auxiliary images live only in LDS; nothing per-term reaches HBM.
//
// Phase: every thread keeps z = exp(j m a g) for its extended-tile pixels in
// registers and advances it by one complex multiply per pair,
// z <- z * exp(j 2 a g), starting from the centre term (m = 0, z = 1) or from
// m = 1 (z = exp(j a g)) for odd N.  exp(j 2 a g) is re-derived per pair from
// g (deterministically) instead of being stored, which halves the register
// state and costs only VALU cycles the LDS-bound passes leave idle.
//
// Filtering: each box stage is a running sum s += (x_enter - x_leave).  A lane
// marches one line (a row of the extended tile, then a column of the
// row-filtered tile); the stage-1 leaving value is re-read from the line
// itself, the later stages' leaving values come from per-lane ring buffers in
// LDS.  Rows are marched from the plane written by the phase owners, columns
// from the transposed buffer T written by the row march.
#include "bf_internal.h"

namespace bf {

constexpr int kFwdThreads = 256;
constexpr int kFwdKMax = 48;                          // extended pixels per thread
constexpr int kFwdExtMax = kFwdThreads * kFwdKMax;    // 12288
constexpr int kFwdLineMax = 256;                      // marching lanes per pass

struct FwdArgs {
    const float* f;
    float* out;
    float* eta;
    int H, W;
    int TH, TW, EH, EW, tiles_x;
    int R;
    int w[BF_MAX_BOXES];      // box widths 2r+1
    int ring_off[BF_MAX_BOXES];
    int ring_len;             // sum of widths of boxes 2..nb
    int nl;                   // lanes with a ring: max(EH, TW)
    int npairs, odd;
    float two_alpha;          // 2 a in float for the per-pair step factor
    double alpha;
    float center;
    float chat[kMaxPairs];
};

// LDS layout (floats): plane[EH*EW] | T[TW*EH] | ring[ring_len*nl] |
//                      cs[2*TH*TW] | acc[2*TH*TW]
__host__ __device__ inline size_t fwd_lds_floats(int TH, int TW, int EH, int EW, int ring_len,
                                                 int nl) {
    return (size_t)EH * EW + (size_t)TW * EH + (size_t)ring_len * nl + 4 * (size_t)TH * TW;
}

// One stage of a running box sum with its leaving value taken from a ring.
__device__ __forceinline__ float ring_stage(float v, float& s, float* ring, int& idx, int w,
                                            int nl) {
    float* rp = ring + idx * nl;
    const float lv = *rp;
    *rp = v;
    idx = (idx + 1 == w) ? 0 : idx + 1;
    s += (v - lv);
    return s;
}

template <int NB>
__device__ __forceinline__ float march_step(const float* line, int x, float& s0, float& s1,
                                            float& s2, float& s3, int& i1, int& i2, int& i3,
                                            float* ring, const FwdArgs& a, int lane) {
    const float e = line[x];
    const float l = (x >= a.w[0]) ? line[x - a.w[0]] : 0.0f;
    s0 += (e - l);
    float v = s0;
    if (NB > 1) v = ring_stage(v, s1, ring + a.ring_off[1] * a.nl + lane, i1, a.w[1], a.nl);
    if (NB > 2) v = ring_stage(v, s2, ring + a.ring_off[2] * a.nl + lane, i2, a.w[2], a.nl);
    if (NB > 3) v = ring_stage(v, s3, ring + a.ring_off[3] * a.nl + lane, i3, a.w[3], a.nl);
    return v;
}

template <int NB>
__global__ void __launch_bounds__(kFwdThreads)
bf_fwd_kernel(const FwdArgs a) {
    extern __shared__ float smem[];
    const int EH = a.EH, EW = a.EW, TH = a.TH, TW = a.TW, R = a.R;
    const int E = EH * EW;
    float* plane = smem;
    float* T = plane + (size_t)E;
    float* ring = T + (size_t)TW * EH;
    float* cs = ring + (size_t)a.ring_len * a.nl;
    float* acc = cs + 2 * (size_t)TH * TW;   // acc[0..THTW) = den, acc[THTW..) = num
    const int THTW = TH * TW;

    const int t = threadIdx.x;
    const int ty = blockIdx.x / a.tiles_x, tx = blockIdx.x - ty * a.tiles_x;
    const int i0 = ty * TH, j0 = tx * TW;          // output tile origin (image coords)
    const int ei0 = i0 - R, ej0 = j0 - R;          // extended tile origin
    const uint32_t magic = (uint32_t)((0x100000000ull + EW - 1) / EW);

    // ---- per-pixel phase state ---------------------------------------------
    float zr[kFwdKMax], zi[kFwdKMax], gv[kFwdKMax];
    uint64_t inimg = 0;
#pragma unroll
    for (int k = 0; k < kFwdKMax; ++k) {
        const int p = t + kFwdThreads * k;
        zr[k] = 0.0f;
        zi[k] = 0.0f;
        gv[k] = 0.0f;
        if (p < E) {
            const int ei = EW == 1 ? p : (int)__umulhi((uint32_t)p, magic);
            const int ej = p - ei * EW;
            const int gi = ei0 + ei, gj = ej0 + ej;
            if (gi >= 0 && gi < a.H && gj >= 0 && gj < a.W) {
                inimg |= (1ull << k);
                const float g = a.f[(size_t)gi * a.W + gj] - a.center;
                gv[k] = g;
                if (a.odd) {
                    double sn, cn;
                    sincos(a.alpha * (double)g, &sn, &cn);
                    zr[k] = (float)cn;
                    zi[k] = (float)sn;
                } else {
                    zr[k] = 1.0f;
                }
            }
        }
    }
    for (int o = t; o < 2 * THTW; o += kFwdThreads) acc[o] = 0.0f;

    for (int q = 0; q < a.npairs; ++q) {
        const bool center_term = (q == 0) && !a.odd;   // m = 0: S and gS vanish
        const float c = a.chat[q];
        if (q > 0) {
            // z <- z * exp(j 2 a g); the step factor is recomputed from g
#pragma unroll
            for (int k = 0; k < kFwdKMax; ++k) {
                if (inimg & (1ull << k)) {
                    float su, cu;
                    sincosf(a.two_alpha * gv[k], &su, &cu);
                    const float nr = zr[k] * cu - zi[k] * su;
                    const float ni = zr[k] * su + zi[k] * cu;
                    zr[k] = nr;
                    zi[k] = ni;
                }
            }
        }
        __syncthreads();   // previous pair's column march has finished with cs
        // C and S at the output pixels, read by the column march's demodulation
#pragma unroll
        for (int k = 0; k < kFwdKMax; ++k) {
            const int p = t + kFwdThreads * k;
            if (p < E) {
                const int ei = EW == 1 ? p : (int)__umulhi((uint32_t)p, magic);
                const int ej = p - ei * EW;
                const int oi = ei - R, oj = ej - R;
                if (oi >= 0 && oi < TH && oj >= 0 && oj < TW) {
                    cs[oi * TW + oj] = zr[k];
                    cs[THTW + oi * TW + oj] = zi[k];
                }
            }
        }
        const int nch = center_term ? 2 : 4;
        for (int ch = 0; ch < nch; ++ch) {
            // channel order: C, gC, S, gS  (C/S select the phase component,
            // the g variants multiply by g)
            const bool use_s = ch >= 2;
            const bool use_g = (ch & 1) != 0;
            // ---- phase owners write the auxiliary image of this channel ----
#pragma unroll
            for (int k = 0; k < kFwdKMax; ++k) {
                const int p = t + kFwdThreads * k;
                if (p < E) {
                    float v = use_s ? zi[k] : zr[k];
                    if (use_g) v *= gv[k];
                    plane[p] = v;   // zero outside the image: z = g = 0 there
                }
            }
            __syncthreads();
            // ---- row march: lane = extended row --------------------------
            if (t < EH) {
                const int lane = t;
                for (int qq = 0; qq < a.ring_len; ++qq) ring[qq * a.nl + lane] = 0.0f;
                float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
                int i1 = 0, i2 = 0, i3 = 0;
                const float* line = plane + (size_t)lane * EW;
                for (int x = 0; x < EW; ++x) {
                    const float v = march_step<NB>(line, x, s0, s1, s2, s3, i1, i2, i3, ring, a,
                                                   lane);
                    const int j = x - 2 * R;
                    if (j >= 0) T[(size_t)j * EH + lane] = v;
                }
            }
            __syncthreads();
            // ---- column march with demodulation: lane = output column ------
            if (t < TW) {
                const int lane = t;
                for (int qq = 0; qq < a.ring_len; ++qq) ring[qq * a.nl + lane] = 0.0f;
                float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
                int i1 = 0, i2 = 0, i3 = 0;
                const float* line = T + (size_t)lane * EH;
                const float* csel = cs + (use_s ? THTW : 0);
                float* dst = acc + (use_g ? THTW : 0);
                for (int y = 0; y < EH; ++y) {
                    const float v = march_step<NB>(line, y, s0, s1, s2, s3, i1, i2, i3, ring, a,
                                                   lane);
                    const int i = y - 2 * R;
                    if (i >= 0) {
                        const int o = i * TW + lane;
                        dst[o] += c * (csel[o] * v);
                    }
                }
            }
            // the next channel's plane write is fenced by the barrier at the
            // top of the channel loop's row march; the plane is not read by
            // the column march, so the owners may overwrite it right away.
        }
    }
    __syncthreads();
    // ---- ratio and store ------------------------------------------------------
    for (int o = t; o < THTW; o += kFwdThreads) {
        const int oi = o / TW, oj = o - oi * TW;
        const int gi = i0 + oi, gj = j0 + oj;
        if (gi < a.H && gj < a.W) {
            const float den = acc[o];
            const float num = acc[THTW + o];
            a.out[(size_t)gi * a.W + gj] = (float)((double)a.center + (double)num / (double)den);
            if (a.eta) a.eta[(size_t)gi * a.W + gj] = den;
        }
    }
}

bf_status plan_fwd_tiles(int64_t H, int64_t W, const SpatialParams& sp, int req_h, int req_w,
                         TileGeom* g) {
    const int R = sp.R;
    int ring_len = 0;
    for (int k = 1; k < sp.nb; ++k) ring_len += 2 * sp.r[k] + 1;
    auto lds_of = [&](int th, int tw) {
        const int eh = th + 2 * R, ew = tw + 2 * R;
        const int nl = eh > tw ? eh : tw;
        return fwd_lds_floats(th, tw, eh, ew, ring_len, nl) * sizeof(float);
    };
    auto fits = [&](int th, int tw) {
        const int eh = th + 2 * R, ew = tw + 2 * R;
        return th >= 1 && tw >= 1 && (int64_t)eh * ew <= kFwdExtMax && eh <= kFwdLineMax &&
               tw <= kFwdLineMax && lds_of(th, tw) <= 160 * 1024;
    };
    int th = req_h, tw = req_w;
    if (th <= 0 || tw <= 0) {
        // largest square-ish odd tile that fits, no larger than the image needs
        int side = 1;
        for (int s = 1; s <= kFwdLineMax; s += 2)
            if (fits(s, s)) side = s;
        th = tw = side;
        if (th > H) th = (int)(H | 1);
        if (tw > W) tw = (int)(W | 1);
        // widen the other side where the image is narrow
        while (th < H && fits(th + 2, tw)) th += 2;
        while (tw < W && fits(th, tw + 2)) tw += 2;
        if (!fits(th, tw)) {
            set_error("spatial radius R=%d too large for the fused forward tile", R);
            return BF_EUNSUPPORTED;
        }
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

bf_status launch_fwd(const float* f, float* out, float* eta, int64_t H, int64_t W,
                     const RangeParams& rp, const SpatialParams& sp, const TileGeom& g,
                     hipStream_t stream) {
    FwdArgs a;
    a.f = f;
    a.out = out;
    a.eta = eta;
    a.H = (int)H;
    a.W = (int)W;
    a.TH = g.TH;
    a.TW = g.TW;
    a.EH = g.EH;
    a.EW = g.EW;
    a.tiles_x = g.tiles_x;
    a.R = sp.R;
    int off = 0;
    for (int k = 0; k < BF_MAX_BOXES; ++k) {
        a.w[k] = 2 * sp.r[k] + 1;
        a.ring_off[k] = 0;
    }
    for (int k = 1; k < sp.nb; ++k) {
        a.ring_off[k] = off;
        off += a.w[k];
    }
    a.ring_len = off;
    a.nl = g.EH > g.TW ? g.EH : g.TW;
    a.npairs = rp.npairs;
    a.odd = rp.odd;
    a.alpha = rp.alpha;
    a.two_alpha = (float)(2.0 * rp.alpha);
    a.center = rp.center;
    for (int q = 0; q < kMaxPairs; ++q) a.chat[q] = q < rp.npairs ? rp.chat[q] : 0.0f;
    const dim3 grid((unsigned)(g.tiles_x * g.tiles_y)), block(kFwdThreads);
    const size_t lds = g.lds_bytes;
    static const void* kern[4] = {(const void*)bf_fwd_kernel<1>, (const void*)bf_fwd_kernel<2>,
                                  (const void*)bf_fwd_kernel<3>, (const void*)bf_fwd_kernel<4>};
    hipFuncSetAttribute(kern[sp.nb - 1], hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    switch (sp.nb) {
        case 1: hipLaunchKernelGGL(bf_fwd_kernel<1>, grid, block, lds, stream, a); break;
        case 2: hipLaunchKernelGGL(bf_fwd_kernel<2>, grid, block, lds, stream, a); break;
        case 3: hipLaunchKernelGGL(bf_fwd_kernel<3>, grid, block, lds, stream, a); break;
        default: hipLaunchKernelGGL(bf_fwd_kernel<4>, grid, block, lds, stream, a); break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("forward launch failed: %s", hipGetErrorString(e));
        return BF_EDEVICE;
    }
    return BF_OK;
}

}  // namespace bf
