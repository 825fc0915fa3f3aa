// Fused O(1) forward and adjoint kernels of the trigonometric bilateral
// filter (gfx950).
//
// One workgroup owns an output tile of TH x TW pixels and the extended tile
// (TH + 2R) x (TW + 2R) around it.  With g = f - T/2 (zero outside the image),
// C_m = cos(m a g), S_m = sin(m a g) and F the separable iterated-box filter
// with zero extension, the raised cosine's pair expansion (Sec. 2.3) turns
// eq. (BF)/(normalization) into eq. (final-form):
//     den = sum_m c_m (C F[C] + S F[S]),   num = sum_m c_m (C F[gC] + S F[gS]),
//     out = T/2 + num/den,  eta = den.
// The adjoint, for G = dL/dout, A = G/den and B = A (out - T/2), is
//     dL/df = sum_m c_m { (C - ma g S) F[A C] + (S + ma g C) F[A S]
//                         + ma S F[B C] - ma C F[B S]
//                         - ma A S F[gC] + ma A C F[gS]
//                         + ma B S F[C] - ma B C F[S] },       ma = m a,
// obtained by differentiating both the local factors C, S and the filtered
// auxiliary images (F is self-adjoint: symmetric w, zero extension).
// Either way every cosine pair is a list of channels, each an auxiliary image
// built on the extended tile, filtered, multiplied by a per-pixel
// coefficient and accumulated at the output pixels.  The auxiliary images
// exist only in LDS and registers; nothing per term reaches HBM.
//
// Phase: each thread keeps z = exp(j m a g) for its extended-tile pixels in
// registers and advances it once per pair by a complex multiply,
// z <- z * exp(j 2 a g), from the centre term (m = 0, z = 1) or from m = 1
// (z = exp(j a g), evaluated in FP64) for odd N.  The step factor is
// re-evaluated per pair from g by its Taylor series (|2 a g| <= pi/2 when f
// lies in [0, T] and N meets the degree bound) rather than stored.
//
// Filtering: lanes hold one whole line in registers (bf_box.h): a row of the
// extended tile for the horizontal pass, then a column of the row-filtered
// tile for the vertical pass, every box stage a running sum
// s += (x_enter - x_leave) with compile-time indices.  LDS carries only the
// bulk hand-offs: the phase owners write the channel's auxiliary image
// (plane) and its coefficients at the output pixels (coef), row lanes write
// their results transposed (T), column lanes accumulate.  Rows of channel s
// and columns of channel s-1 run at the same time on different waves; T and
// coef are double-buffered for that.
#pragma once

#include "bf_box.h"
#include "bf_internal.h"

namespace bf {

enum TileMode { kForward = 0, kBackward = 1 };

constexpr int kTileThreads = 256;
constexpr int kLine = 128;             // register line length (rows and columns)
constexpr int kColLane0 = 128;         // threads [0,128) are row lanes, [128,256) column lanes
constexpr int kPad = kLine;            // LDS slack after each line buffer
constexpr int kChunk = 8;              // outputs stored per uniform guard

template <int MODE>
struct ModeTraits;
template <>
struct ModeTraits<kForward> {
    static constexpr int kKMax = 48;   // extended pixels per thread
    static constexpr int kAcc = 2;     // den, num
};
template <>
struct ModeTraits<kBackward> {
    static constexpr int kKMax = 40;
    static constexpr int kAcc = 1;     // dL/df
};

struct TileArgs {
    const float* f;
    float* out;          // forward: filtered image; backward: dL/df
    float* eta;          // forward: optional eta
    const float* fout;   // backward: forward output
    const float* feta;   // backward: forward eta
    const float* gout;   // backward: dL/dout (NULL in a batch: 2 (fout - target))
    const float* target; // batch: SSD target (forward: per-tile loss partial)
    float* loss_part;    // batch forward: one partial SSD per tile
    int H, W;
    int TH, TW, EH, EW, tiles_x;
    int R, nb;
    int r[BF_MAX_BOXES];
    int npairs, odd, nsteps;
    float two_alpha;     // 2a: per-pair phase step per unit intensity
    float alpha_f;       // a in float (m a factors of the adjoint)
    double alpha;
    float center;
    float chat[kMaxPairs];
};

// LDS layout (floats): plane[EH*EW + kPad] | T0 | T1 | coef0 | coef1 | acc...
// T holds (TW + kChunk) columns of EH plus kPad; coef and each accumulator
// plane hold (TH + kChunk) rows of TW.  The pads let every lane load a whole
// kLine-long line and store whole chunks unconditionally; values past a
// line's end only reach outputs that are discarded.
__host__ __device__ inline size_t tile_t_stride(int TW, int EH) {
    return (size_t)(TW + kChunk) * EH + kPad;
}
__host__ __device__ inline size_t tile_o_plane(int TH, int TW) {
    return (size_t)(TH + kChunk) * TW;
}
__host__ __device__ inline size_t tile_lds_floats(int TH, int TW, int EH, int EW, int nacc) {
    return (size_t)EH * EW + kPad + 2 * tile_t_stride(TW, EH) + (2 + nacc) * tile_o_plane(TH, TW);
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

// Channels of one cosine pair.  Forward: C, gC, S, gS (centre pair: C, gC).
// Backward: AC, AS, BC, BS, gC, gS, C, S (centre pair: AC).
template <int MODE>
__device__ __forceinline__ int pair_channels(bool centre) {
    if (MODE == kForward) return centre ? 2 : 4;
    return centre ? 1 : 8;
}

// Auxiliary-image value of channel ch at a pixel: phase component times a
// per-pixel factor.
template <int MODE>
__device__ __forceinline__ float channel_input(int ch, float zr, float zi, float g, float A,
                                               float B) {
    if (MODE == kForward) {
        const float base = (ch >= 2) ? zi : zr;
        return (ch & 1) ? base * g : base;
    }
    const float base = (ch & 1) ? zi : zr;
    const int kind = ch >> 1;   // 0: A, 1: B, 2: g, 3: 1
    const float mul = kind == 0 ? A : kind == 1 ? B : kind == 2 ? g : 1.0f;
    return base * mul;
}

// Coefficient multiplying F[channel ch] at an output pixel (c = c_m, ma = m a).
template <int MODE>
__device__ __forceinline__ float channel_coef(int ch, float c, float ma, float C, float S,
                                              float g, float A, float B) {
    if (MODE == kForward) return c * ((ch >= 2) ? S : C);
    switch (ch) {
        case 0: return c * (C - ma * g * S);
        case 1: return c * (S + ma * g * C);
        case 2: return c * ma * S;
        case 3: return -c * ma * C;
        case 4: return -c * ma * A * S;
        case 5: return c * ma * A * C;
        case 6: return c * ma * B * S;
        default: return -c * ma * B * C;
    }
}

// Accumulator plane receiving channel ch (forward: den for C/S, num for gC/gS).
template <int MODE>
__device__ __forceinline__ int channel_acc(int ch) {
    return MODE == kForward ? (ch & 1) : 0;
}

// One output tile of one image (tile index tile_id) for descriptor a; all
// threads of the workgroup call it together.
template <int MODE>
__device__ void tile_body(const TileArgs& a, int tile_id, float* smem) {
    constexpr int KMAX = ModeTraits<MODE>::kKMax;
    constexpr int NACC = ModeTraits<MODE>::kAcc;
    const int EH = a.EH, EW = a.EW, TH = a.TH, TW = a.TW, R = a.R;
    const int E = EH * EW;
    const int THTW = TH * TW;
    const size_t tstride = tile_t_stride(TW, EH);
    const int OP = (int)tile_o_plane(TH, TW);
    float* plane = smem;
    float* Tbuf = plane + (size_t)E + kPad;
    float* coef = Tbuf + 2 * tstride;
    float* acc = coef + 2 * (size_t)OP;

    const int t = threadIdx.x;
    const int ty = tile_id / a.tiles_x, tx = tile_id - ty * a.tiles_x;
    const int i0 = ty * TH, j0 = tx * TW;             // output tile origin (image coords)
    const int ei0 = i0 - R, ej0 = j0 - R;             // extended tile origin
    const uint32_t magic = (uint32_t)((0x100000000ull + EW - 1) / EW);

    // ---- per-pixel state of the extended tile -----------------------------------
    float zr[KMAX], zi[KMAX], gv[KMAX], av[KMAX], bv[KMAX];
    uint64_t inimg = 0, inout = 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int p = t + kTileThreads * k;
        zr[k] = 0.0f;
        zi[k] = 0.0f;
        gv[k] = 0.0f;
        av[k] = 0.0f;
        bv[k] = 0.0f;
        if (p < E) {
            const int ei = EW == 1 ? p : (int)__umulhi((uint32_t)p, magic);
            const int ej = p - ei * EW;
            const int gi = ei0 + ei, gj = ej0 + ej;
            if (ei >= R && ei < R + TH && ej >= R && ej < R + TW) inout |= (1ull << k);
            if (gi >= 0 && gi < a.H && gj >= 0 && gj < a.W) {
                inimg |= (1ull << k);
                const size_t gidx = (size_t)gi * a.W + gj;
                const float g = a.f[gidx] - a.center;
                gv[k] = g;
                if (a.odd) {
                    double sn, cn;
                    sincos(a.alpha * (double)g, &sn, &cn);
                    zr[k] = (float)cn;
                    zi[k] = (float)sn;
                } else {
                    zr[k] = 1.0f;
                }
                if (MODE == kBackward) {
                    const float fo = a.fout[gidx];
                    const float G = a.gout ? a.gout[gidx] : 2.0f * (fo - a.target[gidx]);
                    const float A = G / a.feta[gidx];
                    av[k] = A;
                    bv[k] = A * (fo - a.center);
                }
            }
        }
    }
    for (int o = t; o < NACC * OP; o += kTileThreads) acc[o] = 0.0f;

    // Channel steps s = 0 .. nsteps-1 run over all pairs; at step s the row
    // lanes filter channel s into T[s & 1] while the column lanes filter
    // channel s-1 out of T[(s-1) & 1] and accumulate with coef[(s-1) & 1].
    int q = 0, ch = 0;           // pair and channel of step s
    int pch = -1;                // channel of step s-1 (column lanes); -1: none
    for (int s = 0; s <= a.nsteps; ++s) {
        const bool have_row = s < a.nsteps;
        if (have_row) {
            const bool centre = (q == 0) && !a.odd;
            if (ch == 0 && q > 0) {
#pragma unroll
                for (int k = 0; k < KMAX; ++k) {
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
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const int p = t + kTileThreads * k;
                if (p < E) plane[p] = channel_input<MODE>(ch, zr[k], zi[k], gv[k], av[k], bv[k]);
            }
            const float c = a.chat[q];
            const float ma = (float)(a.odd + 2 * q) * a.alpha_f;
            float* cdst = coef + (size_t)(s & 1) * OP;
            int tt = t;
            asm volatile("" : "+v"(tt));   // recompute indices per step, not per kernel
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                if (inout & (1ull << k)) {
                    const int p = tt + kTileThreads * k;
                    const int ei = EW == 1 ? p : (int)__umulhi((uint32_t)p, magic);
                    const int o = (ei - R) * TW + (p - ei * EW - R);
                    cdst[o] = channel_coef<MODE>(ch, c, ma, zr[k], zi[k], gv[k], av[k], bv[k]);
                }
            }
            (void)centre;
        }
        __syncthreads();
        const bool is_row = t < kColLane0;
        const bool active = is_row ? (have_row && t < EH) : (pch >= 0 && t - kColLane0 < TW);
        if (active) {
            const int lane = is_row ? t : t - kColLane0;
            const float* src = is_row ? plane + (size_t)lane * EW
                                      : Tbuf + (size_t)((s - 1) & 1) * tstride + (size_t)lane * EH;
            float v[kLine];
#pragma unroll
            for (int x = 0; x < kLine; ++x) v[x] = src[x];
            for (int b = 0; b < a.nb; ++b) box_dispatch<kLine>(v, a.r[b]);
            if (is_row) {
                float* dst = Tbuf + (size_t)(s & 1) * tstride + lane;
#pragma unroll
                for (int j0c = 0; j0c < kLine; j0c += kChunk) {
                    if (j0c < TW) {   // uniform; a chunk may spill into the pad
#pragma unroll
                        for (int jj = 0; jj < kChunk; ++jj)
                            dst[(size_t)(j0c + jj) * EH] = v[j0c + jj];
                    }
                }
            } else {
                const float* cw = coef + (size_t)((s - 1) & 1) * OP + lane;
                float* dst = acc + (size_t)channel_acc<MODE>(pch) * OP + lane;
#pragma unroll
                for (int i0c = 0; i0c < kLine; i0c += kChunk) {
                    if (i0c < TH) {   // uniform; rows past TH land in the pad
#pragma unroll
                        for (int ii = 0; ii < kChunk; ++ii)
                            dst[(i0c + ii) * TW] += cw[(i0c + ii) * TW] * v[i0c + ii];
                    }
                }
            }
        }
        __syncthreads();
        pch = have_row ? ch : -1;
        if (have_row) {
            if (++ch == pair_channels<MODE>((q == 0) && !a.odd)) {
                ch = 0;
                ++q;
            }
        }
    }
    double sq = 0.0;   // batch forward: this thread's share of the tile's SSD
    for (int o = t; o < THTW; o += kTileThreads) {
        const int oi = o / TW, oj = o - oi * TW;
        const int gi = i0 + oi, gj = j0 + oj;
        if (gi < a.H && gj < a.W) {
            const size_t gidx = (size_t)gi * a.W + gj;
            if (MODE == kForward) {
                const float den = acc[o];
                const float num = acc[OP + o];
                const float y = (float)((double)a.center + (double)num / (double)den);
                a.out[gidx] = y;
                if (a.eta) a.eta[gidx] = den;
                if (a.loss_part) {
                    const double d = (double)y - (double)a.target[gidx];
                    sq += d * d;
                }
            } else {
                a.out[gidx] = acc[o];
            }
        }
    }
    if (MODE == kForward && a.loss_part) {
        // fixed-order tree reduction: the same partial on every run
        __syncthreads();
        double* red = reinterpret_cast<double*>(smem);
        red[t] = sq;
        __syncthreads();
        for (int w = kTileThreads / 2; w > 0; w >>= 1) {
            if (t < w) red[t] += red[t + w];
            __syncthreads();
        }
        if (t == 0) a.loss_part[tile_id] = (float)red[0];
    }
    __syncthreads();   // LDS is reused by the next tile of a persistent workgroup
}

template <int MODE>
__global__ void __launch_bounds__(kTileThreads)
bf_tile_kernel(const TileArgs a) {
    extern __shared__ float smem[];
    tile_body<MODE>(a, blockIdx.x, smem);
}

// Host helpers shared by the single-image and batched launchers (bf_tile.hip).
bf_status plan_tiles(int mode, int64_t H, int64_t W, const SpatialParams& sp, int req_h,
                     int req_w, TileGeom* g);
void fill_tile_args(TileArgs& a, int64_t H, int64_t W, const RangeParams& rp,
                    const SpatialParams& sp, const TileGeom& g, int mode);

}  // namespace bf
