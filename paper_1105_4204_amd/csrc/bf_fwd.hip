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
// The auxiliary images live only in LDS and registers; nothing per-term
// reaches HBM.
//
// Phase: every thread keeps z = exp(j m a g) for its extended-tile pixels in
// registers and advances it by one complex multiply per pair,
// z <- z * exp(j 2 a g), starting from the centre term (m = 0, z = 1) or from
// m = 1 (z = exp(j a g)) for odd N.  The step factor exp(j 2 a g) is
// re-evaluated per pair from g by its Taylor series (|2 a g| <= pi/2 when f
// lies in [0, T] and N meets the degree bound), deterministic and cheaper in
// registers than storing it.
//
// Filtering: the separable iterated-box kernel is applied by lanes that hold
// one whole line in registers (bf_box.h): a row of the extended tile for the
// horizontal pass, then a column of the row-filtered tile for the vertical
// pass, each box stage a running sum s += (x_enter - x_leave) with
// compile-time indices.  LDS carries only the bulk hand-offs: the phase owners
// write the auxiliary image of one channel (plane), row lanes write their
// results transposed (T, double-buffered), column lanes demodulate into the
// accumulators.  Rows of channel c and columns of channel c-1 run at the same
// time on different waves.
#include "bf_box.h"
#include "bf_internal.h"

namespace bf {

constexpr int kFwdThreads = 256;
constexpr int kFwdKMax = 48;                          // extended pixels per thread
constexpr int kFwdExtMax = kFwdThreads * kFwdKMax;    // 12288
constexpr int kFwdLine = 128;                         // register line length (rows, cols)
constexpr int kColLane0 = 128;                        // first thread of the column waves
constexpr int kColLaneEnd = 256;
constexpr int kPad = kFwdLine;                        // LDS slack after each line buffer
constexpr int kChunk = 8;                             // outputs stored per uniform guard

struct FwdArgs {
    const float* f;
    float* out;
    float* eta;
    int H, W;
    int TH, TW, EH, EW, tiles_x;
    int R;
    int nb;
    int r[BF_MAX_BOXES];      // box radii (<= kBoxMaxRadius)
    int npairs, odd, nsteps;
    float two_alpha;          // 2a: the per-pair phase step per unit intensity
    double alpha;
    float center;
    float chat[kMaxPairs];
};

// LDS layout (floats): plane[EH*EW + kPad] | T0 | T1 | cs | acc, where
// T0/T1 hold (TW + kChunk) columns of EH plus kPad, and cs/acc hold two
// planes of (TH + kChunk) rows of TW each.  The pads let every lane load a
// whole kFwdLine-long line and store whole chunks of kChunk unconditionally;
// the values past a line's end only reach outputs that are discarded.
__host__ __device__ inline size_t fwd_t_stride(int TW, int EH) {
    return (size_t)(TW + kChunk) * EH + kPad;
}
__host__ __device__ inline size_t fwd_cs_plane(int TH, int TW) {
    return (size_t)(TH + kChunk) * TW;
}
__host__ __device__ inline size_t fwd_lds_floats(int TH, int TW, int EH, int EW) {
    return (size_t)EH * EW + kPad + 2 * fwd_t_stride(TW, EH) + 4 * fwd_cs_plane(TH, TW);
}

// exp(j x) for |x| <= pi/2 by the Taylor series of cos (to x^14) and sin (to
// x^13); truncation error below 1e-9 on that interval.
__device__ __forceinline__ void cis_small(float x, float& c, float& s) {
    const float x2 = x * x;
    float pc = -1.0f / 87178291200.0f;                 // -1/14!
    pc = fmaf(pc, x2, 1.0f / 479001600.0f);            //  1/12!
    pc = fmaf(pc, x2, -1.0f / 3628800.0f);             // -1/10!
    pc = fmaf(pc, x2, 1.0f / 40320.0f);                //  1/8!
    pc = fmaf(pc, x2, -1.0f / 720.0f);                 // -1/6!
    pc = fmaf(pc, x2, 1.0f / 24.0f);                   //  1/4!
    pc = fmaf(pc, x2, -0.5f);                          // -1/2!
    c = fmaf(pc, x2, 1.0f);
    float ps = 1.0f / 6227020800.0f;                   //  1/13!
    ps = fmaf(ps, x2, -1.0f / 39916800.0f);            // -1/11!
    ps = fmaf(ps, x2, 1.0f / 362880.0f);               //  1/9!
    ps = fmaf(ps, x2, -1.0f / 5040.0f);                // -1/7!
    ps = fmaf(ps, x2, 1.0f / 120.0f);                  //  1/5!
    ps = fmaf(ps, x2, -1.0f / 6.0f);                   // -1/3!
    s = fmaf(ps * x2, x, x);
}

__global__ void __launch_bounds__(kFwdThreads)
bf_fwd_kernel(const FwdArgs a) {
    extern __shared__ float smem[];
    const int EH = a.EH, EW = a.EW, TH = a.TH, TW = a.TW, R = a.R;
    const int E = EH * EW;
    const int THTW = TH * TW;
    float* plane = smem;
    float* Tbuf = plane + (size_t)E + kPad;           // two transposed buffers
    const size_t tstride = fwd_t_stride(TW, EH);
    const int CSP = (int)fwd_cs_plane(TH, TW);        // cs/acc plane stride
    float* cs = Tbuf + 2 * tstride;
    float* acc = cs + 2 * (size_t)CSP;                // acc[0..) = den, acc[CSP..) = num

    const int t = threadIdx.x;
    const int ty = blockIdx.x / a.tiles_x, tx = blockIdx.x - ty * a.tiles_x;
    const int i0 = ty * TH, j0 = tx * TW;             // output tile origin (image coords)
    const int ei0 = i0 - R, ej0 = j0 - R;             // extended tile origin
    const uint32_t magic = (uint32_t)((0x100000000ull + EW - 1) / EW);

    // ---- per-pixel phase state --------------------------------------------------
    float zr[kFwdKMax], zi[kFwdKMax], gv[kFwdKMax];
    uint64_t inimg = 0, inout = 0;
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
            if (ei >= R && ei < R + TH && ej >= R && ej < R + TW) inout |= (1ull << k);
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
    for (int o = t; o < 2 * CSP; o += kFwdThreads) acc[o] = 0.0f;

    // The channel steps of all pairs form one sequence s = 0, 1, ...; step s
    // writes the plane of channel s, then row lanes filter it into T[s & 1]
    // while column lanes filter channel s-1 out of T[(s-1) & 1].  Channel
    // order within a pair: C, gC, S, gS (the centre pair has only C and gC).
    int q = 0, ch = 0;             // channel of step s
    int pq = -1, pch = 0;          // channel of step s-1 (column lanes)
    const int nsteps = a.nsteps;
    for (int s = 0; s <= nsteps; ++s) {
        const bool have_row = s < nsteps;
        if (have_row) {
            if (ch == 0 && q > 0) {
                // next pair: z <- z * exp(j 2 a g)
#pragma unroll
                for (int k = 0; k < kFwdKMax; ++k) {
                    if (inimg & (1ull << k)) {
                        float cu, su;
                        cis_small(a.two_alpha * gv[k], cu, su);
                        const float nr = zr[k] * cu - zi[k] * su;
                        const float ni = zr[k] * su + zi[k] * cu;
                        zr[k] = nr;
                        zi[k] = ni;
                    }
                }
            }
            const bool use_s = ch >= 2;
            const bool use_g = (ch & 1) != 0;
#pragma unroll
            for (int k = 0; k < kFwdKMax; ++k) {
                const int p = t + kFwdThreads * k;
                if (p < E) {
                    float v = use_s ? zi[k] : zr[k];
                    if (use_g) v *= gv[k];
                    plane[p] = v;   // zero outside the image: z = g = 0 there
                }
            }
            if (ch == 1) {
                // C and S of this pair at the output pixels; the column lanes
                // of the previous pair finished with them at the last barrier
                int tt = t;
                asm volatile("" : "+v"(tt));
#pragma unroll
                for (int k = 0; k < kFwdKMax; ++k) {
                    if (inout & (1ull << k)) {
                        const int p = tt + kFwdThreads * k;
                        const int ei = EW == 1 ? p : (int)__umulhi((uint32_t)p, magic);
                        const int o = (ei - R) * TW + (p - ei * EW - R);
                        cs[o] = zr[k];
                        cs[CSP + o] = zi[k];
                    }
                }
            }
        }
        __syncthreads();
        // One code path for both passes: a row lane (t < kColLane0) filters
        // extended row t of channel s into T[s & 1]; a column lane filters
        // column t - kColLane0 of channel s-1 out of T[(s-1) & 1].
        const bool is_row = t < kColLane0;
        const bool active = is_row ? (have_row && t < EH)
                                   : (pq >= 0 && t < kColLaneEnd && t - kColLane0 < TW);
        if (active) {
            const int lane = is_row ? t : t - kColLane0;
            const float* src = is_row ? plane + (size_t)lane * EW
                                      : Tbuf + (size_t)((s - 1) & 1) * tstride + (size_t)lane * EH;
            float v[kFwdLine];
#pragma unroll
            for (int x = 0; x < kFwdLine; ++x) v[x] = src[x];
            for (int b = 0; b < a.nb; ++b) box_dispatch<kFwdLine>(v, a.r[b]);
            if (is_row) {
                float* dst = Tbuf + (size_t)(s & 1) * tstride + lane;
#pragma unroll
                for (int j0 = 0; j0 < kFwdLine; j0 += kChunk) {
                    if (j0 < TW) {   // uniform; a chunk may spill into the pad
#pragma unroll
                        for (int jj = 0; jj < kChunk; ++jj) dst[(size_t)(j0 + jj) * EH] = v[j0 + jj];
                    }
                }
            } else {
                const float c = a.chat[pq];
                const float* csel = cs + ((pch >= 2) ? CSP : 0) + lane;
                float* dst = acc + ((pch & 1) ? CSP : 0) + lane;
#pragma unroll
                for (int i0 = 0; i0 < kFwdLine; i0 += kChunk) {
                    if (i0 < TH) {   // uniform; rows past TH land in the pad
#pragma unroll
                        for (int ii = 0; ii < kChunk; ++ii)
                            dst[(i0 + ii) * TW] += c * (csel[(i0 + ii) * TW] * v[i0 + ii]);
                    }
                }
            }
        }
        __syncthreads();
        // advance the step counters (uniform)
        pq = have_row ? q : -1;
        pch = ch;
        if (have_row) {
            const int nch = (q == 0 && !a.odd) ? 2 : 4;
            if (++ch == nch) {
                ch = 0;
                ++q;
            }
        }
    }
    for (int o = t; o < THTW; o += kFwdThreads) {
        const int oi = o / TW, oj = o - oi * TW;
        const int gi = i0 + oi, gj = j0 + oj;
        if (gi < a.H && gj < a.W) {
            const float den = acc[o];
            const float num = acc[CSP + o];
            a.out[(size_t)gi * a.W + gj] = (float)((double)a.center + (double)num / (double)den);
            if (a.eta) a.eta[(size_t)gi * a.W + gj] = den;
        }
    }
}

bf_status plan_fwd_tiles(int64_t H, int64_t W, const SpatialParams& sp, int req_h, int req_w,
                         TileGeom* g) {
    const int R = sp.R;
    for (int k = 0; k < sp.nb; ++k) {
        if (sp.r[k] > kBoxMaxRadius) {
            set_error("box radius %d exceeds %d, the largest the register-line kernel handles",
                      sp.r[k], kBoxMaxRadius);
            return BF_EUNSUPPORTED;
        }
    }
    auto lds_of = [&](int th, int tw) {
        return fwd_lds_floats(th, tw, th + 2 * R, tw + 2 * R) * sizeof(float);
    };
    auto fits = [&](int th, int tw) {
        const int eh = th + 2 * R, ew = tw + 2 * R;
        return th >= 1 && tw >= 1 && (int64_t)eh * ew <= kFwdExtMax && eh <= kFwdLine &&
               ew <= kFwdLine && tw <= kColLaneEnd - kColLane0 && lds_of(th, tw) <= 160 * 1024;
    };
    int th = req_h, tw = req_w;
    if (th <= 0 || tw <= 0) {
        // odd tile sides keep the extended pitches odd, so lanes striding by a
        // row or column of LDS hit distinct banks
        int side = 0;
        for (int s = 1; s <= kFwdLine; s += 2)
            if (fits(s, s)) side = s;
        if (side == 0) {
            set_error("spatial radius R=%d too large for the fused forward tile", R);
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
    a.nb = sp.nb;
    for (int k = 0; k < BF_MAX_BOXES; ++k) a.r[k] = sp.r[k];
    a.npairs = rp.npairs;
    a.odd = rp.odd;
    a.nsteps = 4 * rp.npairs - (rp.odd ? 0 : 2);
    a.alpha = rp.alpha;
    a.two_alpha = (float)(2.0 * rp.alpha);
    a.center = rp.center;
    for (int q = 0; q < kMaxPairs; ++q) a.chat[q] = q < rp.npairs ? rp.chat[q] : 0.0f;
    const dim3 grid((unsigned)(g.tiles_x * g.tiles_y)), block(kFwdThreads);
    const size_t lds = g.lds_bytes;
    (void)hipFuncSetAttribute((const void*)bf_fwd_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    hipLaunchKernelGGL(bf_fwd_kernel, grid, block, lds, stream, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("forward launch failed: %s", hipGetErrorString(e));
        return BF_EDEVICE;
    }
    return BF_OK;
}

}  // namespace bf
