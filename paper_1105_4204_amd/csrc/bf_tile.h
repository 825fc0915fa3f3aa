// Fused O(1) forward and adjoint kernels of the trigonometric bilateral
// filter (gfx950).
//
// One workgroup of four waves owns an output tile of TH x TW pixels and the
// extended tile (EH x EW = (TH + 2R) x (TW + 2R)) around it.  With g = f - T/2
// (zero outside the image), Z_m = exp(j m a g) = C_m + j S_m and F the
// separable iterated-box filter with zero extension, the raised cosine's pair
// expansion (Sec. 2.3) turns eq. (BF)/(normalization) into eq. (final-form):
//     den = sum_m c_m (C F[C] + S F[S]),   num = sum_m c_m (C F[gC] + S F[gS]),
//     out = T/2 + num/den,  eta = den.
// Differentiating eq. (BF)/(normalization) for G = dL/dout, A = G/den,
// h = out - T/2, B = A h gives (F is self-adjoint: symmetric w, zero
// extension)
//     dL/df = sum_m c_m { (C - ma g S) F[A C] + (S + ma g C) F[A S]
//                         + ma S F[B C] - ma C F[B S] }  + a (A P - B Q),
//     P = sum_m c_m m (C F[gS] - S F[gC]),   Q = sum_m c_m m (C F[S] - S F[C]),
// with ma = m a.  P and Q are built from the forward's own filtered channels,
// so the forward accumulates them when asked (AUX) and the adjoint filters
// only the four channels A C, A S, B C, B S per pair.
//
// Work split.  Waves 0-1 are row lanes: lane i owns row i of the extended
// tile and keeps the phase Z (forward) or Y = A Z (adjoint) of all its pixels
// in registers, advancing it once per pair by Z <- Z exp(j 2 a g) (from m = 0,
// or m = 1 evaluated directly for odd N).  Waves 2-3 are column lanes: lane j
// owns output column j, keeps Z at its output pixels and its accumulators in
// registers.  Per channel step the row lanes build the channel's auxiliary
// row from their phase (times g or h read from LDS), run the box stages along
// it (bf_box.h) and store the result transposed into T[s & 1]; at the same
// time the column lanes load the previous channel's transposed rows from
// T[(s - 1) & 1], run the box stages down the column and accumulate.  Wave 2
// takes the C-type channels (C, S; A C, A S) and wave 3 the others (gC, gS;
// B C, B S), so each column wave filters two channels per pair.  The
// auxiliary images exist only in registers and one transposed LDS buffer;
// nothing per term reaches HBM.
#pragma once

#include "bf_box.h"
#include "bf_internal.h"

namespace bf {

enum TileMode { kForward = 0, kBackward = 1 };

constexpr int kTileThreads = 256;   // waves 0-1: row lanes, waves 2-3: column lanes
constexpr int kLine = 128;          // register line length (extended rows and columns)
constexpr int kLineShort = 120;     // the shorter line, for extended tiles of at most 120
constexpr int kOutMax = 64;         // output tile side limit (column-lane state)
constexpr int kColState = 2 * kOutMax;   // column lane: Z at the outputs, then the sums
constexpr int kPad = kLine;         // LDS slack after each buffer
constexpr int kChunk = 8;           // outputs stored per uniform guard

struct TileArgs {
    const float* f;
    float* out;          // forward: filtered image; adjoint: dL/df
    float* eta;          // forward: optional eta
    float* aux;          // forward: optional P and Q planes (2 H W)
    const float* paux;   // adjoint: P and Q from the forward
    const float* fout;   // adjoint: forward output
    const float* feta;   // adjoint: forward eta
    const float* gout;   // adjoint: dL/dout (NULL in a batch: 2 (fout - target))
    const float* target; // batch: SSD target
    float* loss_part;    // batch forward: one partial SSD per tile
    int H, W;
    int TH, TW, EH, EW, EWp, EHp, tiles_x;
    int R, nb;
    int r[BF_MAX_BOXES];
    int npairs, odd, nsteps;
    float alpha_f;       // a
    float two_alpha;     // 2a: per-pair phase step per unit intensity
    float center;        // T/2
    float chat[kMaxPairs];
};

// LDS pitch of a line of n floats: the smallest p >= n with p = 4 (mod 8), so
// that lanes reading consecutive lines with 16-byte loads hit distinct banks.
__host__ __device__ constexpr int tile_pitch(int n) { return ((n + 3) / 8) * 8 + 4; }
__host__ __device__ inline int tile_round(int n) { return (n + kChunk - 1) / kChunk * kChunk; }
__host__ __device__ inline int tile_plane_floats(int EH, int EWp) { return EH * EWp + kPad; }
__host__ __device__ inline int tile_t_floats(int TW, int EHp) { return tile_round(TW) * EHp + kPad; }
// Forward and GG adjoint: g at the output pixels, transposed (column j at j * kGtPitch).
constexpr int kGtPitch = tile_pitch(kOutMax);
constexpr int kGtFloats = kOutMax * kGtPitch;
// LDS layout (floats): forward gplane | T0 | T1 | gT; adjoint gplane | hplane
// | T0 | T1, or with GG (g read from global memory, where the tile's rows stay
// in L2) hplane | T0 | T1 | gT, so that a 64 x 64 adjoint tile fits.
__host__ __device__ inline size_t tile_lds_floats(int mode, int TH, int TW, int R,
                                                  bool gg = false) {
    const int EH = TH + 2 * R, EW = TW + 2 * R;
    const int planes = (mode == kBackward && !gg) ? 2 : 1;
    return (size_t)planes * tile_plane_floats(EH, tile_pitch(EW)) +
           2 * (size_t)tile_t_floats(TW, tile_pitch(EH)) +
           ((mode == kForward || gg) ? kGtFloats : 0);
}

// exp(j x) for |x| <= pi/2: cos x = 1 + x^2 P(x^2), sin x = x + x^3 Q(x^2)
// with P of degree 4 and Q of degree 3, near-minimax on that interval
// (coefficients from gen_cis_coeffs.py); truncation error below 5e-9, so the
// float32 rounding of the evaluation dominates.
template <typename T>
__device__ __forceinline__ void cis_small_t(T x, T& c, T& s) {
    const T x2 = x * x;
    T pc = (T)-2.607594922e-07f;
    pc = fma(pc, x2, (T)2.476181544e-05f);
    pc = fma(pc, x2, (T)-1.388840145e-03f);
    pc = fma(pc, x2, (T)4.166664183e-02f);
    pc = fma(pc, x2, (T)-5.000000000e-01f);
    c = fma(pc, x2, (T)1.0f);
    T ps = (T)2.599969775e-06f;
    ps = fma(ps, x2, (T)-1.980657107e-04f);
    ps = fma(ps, x2, (T)8.333016187e-03f);
    ps = fma(ps, x2, (T)-1.666665673e-01f);
    s = fma(ps * x2, x, x);
}

// The float32 evaluation (the FP64 one, cis_small_t<double>, uses the same
// float coefficients: its error is their truncation error alone).
__device__ __forceinline__ void cis_small(float x, float& c, float& s) {
    cis_small_t<float>(x, c, s);
}

// exp(j m a g) for any phase: quadrant from the FP64 phase, remainder
// |x| <= pi/4 through cis_small.  Used where a pass starts the phase of a
// pair from scratch instead of carrying it from the previous pair.
__device__ __forceinline__ void cis_direct(double malpha, float g, float& c, float& s) {
    const double th = malpha * (double)g;
    const double n = rint(th * 0.63661977236758134308);        // 2/pi
    const float x = (float)fma(-n, 1.57079632679489661923, th);  // pi/2
    float cx, sx;
    cis_small(x, cx, sx);
    const int q = ((int)n) & 3;   // |n| stays far below 2^31 for any phase used here
    c = q == 0 ? cx : q == 1 ? -sx : q == 2 ? -cx : sx;
    s = q == 0 ? sx : q == 1 ? cx : q == 2 ? -sx : -cx;
}

// v[0..L) <- src[0..L) with 16-byte LDS loads (src 16-byte aligned).
template <int L>
__device__ __forceinline__ void load_line(float (&v)[L], const float* src) {
    static_assert(L % 4 == 0, "line of whole 16-byte chunks");
    const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
    for (int k = 0; k < L / 4; ++k) {
        const float4 q = s4[k];
        v[4 * k] = q.x;
        v[4 * k + 1] = q.y;
        v[4 * k + 2] = q.z;
        v[4 * k + 3] = q.w;
    }
}

// Adjoint with GG: g = f - T/2 along extended row i of the tile, from global
// memory (the rows are L2-resident while the tile runs), in 16-byte buffer
// loads: the lane's row start is the vector offset and the chunk's column the
// scalar offset, so the 32 loads need no per-chunk address registers.  GG
// requires W, the tile width and R to be multiples of 4, f 16-byte aligned and
// 4 H W < 2^31, so that every 4-sample chunk of the extended row lies wholly
// inside or wholly outside the image; chunks outside read a clamped in-image
// chunk, whose values are never used because the phase there is zero.
constexpr int kBufferWord3 = 0x00020000;   // raw buffer resource, gfx9 family
template <int L>
__device__ __forceinline__ void load_g_row(const TileArgs& a, int ei0, int ej0, int i,
                                           float (&v)[L]) {
    const int W = __builtin_amdgcn_readfirstlane(a.W);
    const int e0 = __builtin_amdgcn_readfirstlane(ej0);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(a.f), 0, a.H * W * (int)sizeof(float), kBufferWord3);
    const int voff = min(max(ei0 + i, 0), a.H - 1) * W * (int)sizeof(float);
#pragma unroll
    for (int k = 0; k < L / 4; ++k) {
        const int soff = min(max(e0 + 4 * k, 0), W - 4) * (int)sizeof(float);   // uniform
        const auto q = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0);
        v[4 * k] = __uint_as_float(q[0]) - a.center;
        v[4 * k + 1] = __uint_as_float(q[1]) - a.center;
        v[4 * k + 2] = __uint_as_float(q[2]) - a.center;
        v[4 * k + 3] = __uint_as_float(q[3]) - a.center;
    }
}

// (zr + j zi)[x] *= exp(j step g[goff + x]) for x0 <= x < x1.
template <int x0, int x1, int L, int LG>
__device__ __forceinline__ void phase_step(float (&zr)[L], float (&zi)[L], const float (&g)[LG],
                                           int goff, float step) {
#pragma unroll
    for (int x = x0; x < x1; ++x) {
        float cu, su;
        cis_small(step * g[goff + x], cu, su);
        const float nr = zr[x] * cu - zi[x] * su;
        const float ni = zr[x] * su + zi[x] * cu;
        zr[x] = nr;
        zi[x] = ni;
    }
}

// Channels per pair: forward C, gC, S, gS (centre pair: 1, g); adjoint A C,
// B C, A S, B S (centre pair: A).  Channel ch goes to column wave 2 + (ch & 1).
template <int MODE>
__device__ __forceinline__ int pair_channels(bool centre) {
    if (MODE == kForward) return centre ? 2 : 4;
    return centre ? 1 : 4;
}

// Geometry and LDS pointers of one tile, shared by the two roles.
struct TileCtx {
    int EH, EW, TH, TW, R, EWp, EHp, tfl;
    int i0, j0, ei0, ej0;     // output and extended tile origins (image coordinates)
    int t, wave, lane;
    float* gpl;               // forward: g = f - T/2 on the extended tile
    float* hpl;               // adjoint: A, then h = out - T/2
    float* Tb;                // T0 | T1: row results, transposed
    float* gT;                // forward, GG adjoint: g at the output pixels, column-major
};

// Cooperative fill of an extended-tile plane (pitch gaps and pad zero):
// value(k) for in-image pixels at flat image index k, 0 elsewhere.  Each
// thread takes kFillBatch elements per round and evaluates value() at a
// clamped (always in-image) index without branching, so that the round's
// global loads are all in flight before the first result is used; the
// selection against the real position happens afterwards.
constexpr int kFillBatch = 8;
template <typename F>
__device__ __forceinline__ void fill_plane(const TileArgs& a, const TileCtx& c, float* dst,
                                           F value) {
    const int n = tile_plane_floats(c.EH, c.EWp);
    const uint32_t magic = (uint32_t)((0x100000000ull + c.EWp - 1) / c.EWp);
    for (int p0 = c.t; p0 < n; p0 += kFillBatch * kTileThreads) {
        float x[kFillBatch];
        bool in[kFillBatch];
#pragma unroll
        for (int u = 0; u < kFillBatch; ++u) {
            const int p = p0 + u * kTileThreads;
            const int ei = (int)__umulhi((uint32_t)p, magic);
            const int ej = p - ei * c.EWp;
            const int gi = c.ei0 + ei, gj = c.ej0 + ej;
            in[u] = p < n && ei < c.EH && ej < c.EW && gi >= 0 && gi < a.H && gj >= 0 && gj < a.W;
            const int ci = min(max(gi, 0), a.H - 1), cj = min(max(gj, 0), a.W - 1);
            x[u] = value((size_t)ci * a.W + cj);
        }
#pragma unroll
        for (int u = 0; u < kFillBatch; ++u) {
            const int p = p0 + u * kTileThreads;
            if (p < n) dst[p] = in[u] ? x[u] : 0.0f;
        }
    }
}

// Barriers of the output phase, matched by both roles: hand-over of wave 3's
// sums, then (batch forward) the loss partials, then the end of the tile.
__device__ __forceinline__ int tile_out_barriers(const TileArgs& a, int mode) {
    return (mode == kForward && a.loss_part) ? 3 : 2;
}

// Row role (waves 0-1): lane i owns extended row i.  State: A0 + j A1 = Z
// (forward) or Y = A Z (adjoint) at the row's pixels; zero outside the image.
template <int MODE, bool GG, int L>
__device__ __forceinline__ void row_role(const TileArgs& a, const TileCtx& c) {
    const int i = c.t;
    const bool act = i < c.EH;
    float A0[L], A1[L], v[L];
    if (act) {
        if (GG)
            load_g_row(a, c.ei0, c.ej0, i, v);
        else
            load_line(v, c.gpl + i * c.EWp);
        const int gi = c.ei0 + i;
        const bool rin = gi >= 0 && gi < a.H;
        const int xlo = c.ej0 < 0 ? -c.ej0 : 0;
        const int xhi = min(c.EW, a.W - c.ej0);
        if (a.odd) {
#pragma unroll
            for (int x = 0; x < L; ++x) {
                float cc, ss;
                cis_small(a.alpha_f * v[x], cc, ss);
                const bool in = rin && x >= xlo && x < xhi;
                A0[x] = in ? cc : 0.0f;
                A1[x] = in ? ss : 0.0f;
            }
        } else {
#pragma unroll
            for (int x = 0; x < L; ++x) {
                const bool in = rin && x >= xlo && x < xhi;
                A0[x] = in ? 1.0f : 0.0f;
                A1[x] = 0.0f;
            }
        }
        if (MODE == kBackward) {
            load_line(v, c.hpl + i * c.EWp);   // A
#pragma unroll
            for (int x = 0; x < L; ++x) {
                A0[x] *= v[x];
                A1[x] *= v[x];
            }
        }
    }
    if (MODE == kBackward) {
        __syncthreads();   // every row lane has read A
        fill_plane(a, c, c.hpl, [&](size_t k) { return a.fout[k] - a.center; });
        __syncthreads();
    }
    const float* mulpl = (MODE == kForward) ? c.gpl : c.hpl;
    int q = 0, ch = 0;    // pair and channel of step s
    for (int s = 0; s <= a.nsteps; ++s) {
        if (s < a.nsteps && act) {
            // The blocks that a step may or may not run are marked unlikely
            // and separated by opaque copies of ch, so each is laid out out of
            // line and a step that skips it pays a branch not taken (as in
            // the radius dispatch, bf_box.h).
            int cs = ch;
            // second half of the phase step: the previous step (the last
            // channel of pair q - 1) left g in v, below
            if (__builtin_expect(cs == 0 && q > 0, 0))
                phase_step<L / 2, L>(A0, A1, v, 0, a.two_alpha);
            asm volatile("" : "+s"(cs));
            if (__builtin_expect(cs == 0, 0)) {
#pragma unroll
                for (int x = 0; x < L; ++x) v[x] = A0[x];
            }
            asm volatile("" : "+s"(cs));
            if (__builtin_expect(cs == 1, 0)) {
                load_line(v, mulpl + i * c.EWp);
#pragma unroll
                for (int x = 0; x < L; ++x) v[x] *= A0[x];
            }
            asm volatile("" : "+s"(cs));
            if (__builtin_expect(cs == 2, 0)) {
#pragma unroll
                for (int x = 0; x < L; ++x) v[x] = A1[x];
            }
            asm volatile("" : "+s"(cs));
            if (__builtin_expect(cs == 3, 0)) {
                load_line(v, mulpl + i * c.EWp);
#pragma unroll
                for (int x = 0; x < L; ++x) v[x] *= A1[x];
            }
            for (int b = 0; b < a.nb; ++b) box_dispatch<L>(v, a.r[b]);
            float* dst = c.Tb + (s & 1) * c.tfl + i;
#pragma unroll
            for (int j0c = 0; j0c < kOutMax; j0c += kChunk) {
                if (j0c < c.TW) {   // uniform; a chunk may run into the next row's slack
#pragma unroll
                    for (int jj = 0; jj < kChunk; ++jj) dst[(j0c + jj) * c.EHp] = v[j0c + jj];
                }
            }
            // After the last channel of a pair Z is free: the first half of
            // the next pair's phase step goes here, the second half into the
            // next step, so that no single step carries all of it; g stays in
            // v for that second half.
            asm volatile("" : "+s"(cs));
            if (__builtin_expect(cs == pair_channels<MODE>(q == 0 && !a.odd) - 1 &&
                                     q + 1 < a.npairs,
                                 0)) {
                if (GG)
                    load_g_row(a, c.ei0, c.ej0, i, v);
                else
                    load_line(v, c.gpl + i * c.EWp);
                phase_step<0, L / 2>(A0, A1, v, 0, a.two_alpha);
            }
        }
        __syncthreads();
        if (s < a.nsteps && ++ch == pair_channels<MODE>(q == 0 && !a.odd)) {
            ch = 0;
            ++q;
        }
    }
    for (int k = tile_out_barriers(a, MODE); k > 0; --k) __syncthreads();
}

// Column role (waves 2-3): lane j owns output column j.  State: A0[0..64) +
// j A1[0..64) = Z at the column's outputs; tails: forward den|num (A0) and
// Q|P (A1) on wave 2|3; adjoint the partial sum (A1).  g at the outputs is
// read from LDS where it is needed.  Wave 2 filters the channels with even
// index, wave 3 the odd ones.
template <int MODE, bool AUX, bool GG, int L>
__device__ __forceinline__ void col_role(const TileArgs& a, const TileCtx& c, int tile_id) {
    static_assert(L >= kOutMax, "the line holds the column's outputs");
    const int j = c.lane;
    const bool act = j < c.TW;
    const int TH = c.TH;
    float A0[kColState], A1[kColState], v[L];
    // dst[0..kOutMax) <- g at the output pixels of column j (rows past TH: 0 or a repeat)
    auto load_gcol = [&](auto& dst) {
        if (MODE == kForward || GG) {
            const float4* s4 = reinterpret_cast<const float4*>(c.gT + j * kGtPitch);
#pragma unroll
            for (int k = 0; k < kOutMax / 4; ++k) {
                const float4 q4 = s4[k];
                dst[4 * k] = q4.x;
                dst[4 * k + 1] = q4.y;
                dst[4 * k + 2] = q4.z;
                dst[4 * k + 3] = q4.w;
            }
        } else {
            const float* gcol = c.gpl + c.R * c.EWp + c.R + j;
#pragma unroll
            for (int k = 0; k < kOutMax; ++k) dst[k] = gcol[min(k, TH - 1) * c.EWp];
        }
    };
    if (act) {
        load_gcol(v);
        if (a.odd) {
#pragma unroll
            for (int k = 0; k < kOutMax; ++k) cis_small(a.alpha_f * v[k], A0[k], A1[k]);
        } else {
#pragma unroll
            for (int k = 0; k < kOutMax; ++k) {
                A0[k] = 1.0f;
                A1[k] = 0.0f;
            }
        }
#pragma unroll
        for (int k = 0; k < kOutMax; ++k) {
            A0[kOutMax + k] = 0.0f;
            A1[kOutMax + k] = 0.0f;
        }
    }
    if (MODE == kBackward) {
        __syncthreads();
        fill_plane(a, c, c.hpl, [&](size_t k) { return a.fout[k] - a.center; });
        __syncthreads();
    }
    int q = 0, ch = 0;    // pair and channel of step s - 1
    for (int s = 0; s <= a.nsteps; ++s) {
        // The phase step of a column wave falls into a step in which the
        // other wave filters: wave 3 advances to pair q during channel 0 of
        // pair q, wave 2 to pair q + 1 at the end of the last channel of
        // pair q (an idle step for it, except in the one-channel centre pair
        // of the adjoint, where it follows the wave's own accumulation).
        auto col_phase = [&]() {
            load_gcol(v);
            phase_step<0, kOutMax>(A0, A1, v, 0, a.two_alpha);
        };
        if (s > 0 && (ch & 1) == (c.wave - 2) && act) {
            load_line(v, c.Tb + ((s - 1) & 1) * c.tfl + j * c.EHp);
            for (int b = 0; b < a.nb; ++b) box_dispatch<L>(v, a.r[b]);
            const float cq = a.chat[q];
            const float m = (float)(a.odd + 2 * q);
            // accumulate over the output rows k < TH; the channel picks the
            // coefficient (uniform), every index is a compile-time constant
            auto accumulate = [&](auto coef_of, float (&acc)[kColState]) {
#pragma unroll
                for (int i0c = 0; i0c < kOutMax; i0c += kChunk) {
                    if (i0c < TH) {
#pragma unroll
                        for (int ii = 0; ii < kChunk; ++ii) {
                            const int k = i0c + ii;
                            acc[kOutMax + k] = fmaf(coef_of(k), v[k], acc[kOutMax + k]);
                        }
                    }
                }
            };
            // one out-of-line block per channel, as in the row role
            int cs = ch;
            if (MODE == kForward) {
                const float cm = cq * m;
                if (__builtin_expect(cs < 2, 0)) {   // C F[.] into den|num; -m S F[.] into Q|P
                    accumulate([&](int k) { return cq * A0[k]; }, A0);
                    if (AUX) accumulate([&](int k) { return -cm * A1[k]; }, A1);
                }
                asm volatile("" : "+s"(cs));
                if (__builtin_expect(cs >= 2, 0)) {  // S F[.] into den|num; m C F[.] into Q|P
                    accumulate([&](int k) { return cq * A1[k]; }, A0);
                    if (AUX) accumulate([&](int k) { return cm * A0[k]; }, A1);
                }
            } else {
                const float cma = cq * m * a.alpha_f;
                float gk[kOutMax];
                if (__builtin_expect(cs == 0, 0)) {   // A C: c (C - ma g S)
                    load_gcol(gk);
                    accumulate([&](int k) { return fmaf(-cma * gk[k], A1[k], cq * A0[k]); }, A1);
                }
                asm volatile("" : "+s"(cs));
                if (__builtin_expect(cs == 2, 0)) {   // A S: c (S + ma g C)
                    load_gcol(gk);
                    accumulate([&](int k) { return fmaf(cma * gk[k], A0[k], cq * A1[k]); }, A1);
                }
                asm volatile("" : "+s"(cs));
                if (__builtin_expect(cs == 1, 0))   // B C: c ma S
                    accumulate([&](int k) { return cma * A1[k]; }, A1);
                asm volatile("" : "+s"(cs));
                if (__builtin_expect(cs == 3, 0))   // B S: -c ma C
                    accumulate([&](int k) { return -cma * A0[k]; }, A1);
            }
        }
        // one call site for both waves (wave 3 is idle in this step either way)
        const bool adv3 = c.wave == 3 && ch == 0 && q > 0;
        const bool adv2 = c.wave == 2 && q + 1 < a.npairs &&
                          ch == pair_channels<MODE>(q == 0 && !a.odd) - 1;
        if (__builtin_expect(s > 0 && act && (adv2 || adv3), 0)) col_phase();
        __syncthreads();
        if (s > 0 && ++ch == pair_channels<MODE>(q == 0 && !a.odd)) {
            ch = 0;
            ++q;
        }
    }

    // ---- outputs: wave 3 hands its sums to wave 2, which finishes the pixels ----
    float* xch = c.Tb;
    const size_t HW = (size_t)a.H * a.W;
    if (c.wave == 3 && act) {
#pragma unroll
        for (int i0c = 0; i0c < kOutMax; i0c += kChunk) {
            if (i0c < TH) {
#pragma unroll
                for (int ii = 0; ii < kChunk; ++ii) {
                    const int k = i0c + ii;
                    if (k < TH) {
                        xch[k * c.TW + j] = (MODE == kForward) ? A0[kOutMax + k] : A1[kOutMax + k];
                        const int gi = c.i0 + k, gj = c.j0 + j;
                        if (MODE == kForward && AUX && a.aux && gi < a.H && gj < a.W)
                            a.aux[(size_t)gi * a.W + gj] = A1[kOutMax + k];          // P
                    }
                }
            }
        }
    }
    __syncthreads();
    double sq = 0.0;   // batch forward: this lane's share of the tile's SSD
    if (c.wave == 2 && act) {
#pragma unroll
        for (int i0c = 0; i0c < kOutMax; i0c += kChunk) {
            if (i0c < TH) {
                // adjoint: the chunk's inputs, loaded at clamped positions
                // without branches so that they are all in flight together
                float fo8[kChunk], G8[kChunk], et8[kChunk], P8[kChunk], Q8[kChunk];
                if (MODE == kForward && a.loss_part) {   // batch forward: SSD targets
#pragma unroll
                    for (int ii = 0; ii < kChunk; ++ii) {
                        const int gi = min(c.i0 + i0c + ii, a.H - 1), gj = min(c.j0 + j, a.W - 1);
                        G8[ii] = a.target[(size_t)gi * a.W + gj];
                    }
                }
                if (MODE == kBackward) {
#pragma unroll
                    for (int ii = 0; ii < kChunk; ++ii) {
                        const int gi = min(c.i0 + i0c + ii, a.H - 1), gj = min(c.j0 + j, a.W - 1);
                        const size_t gidx = (size_t)gi * a.W + gj;
                        fo8[ii] = a.fout[gidx];
                        G8[ii] = a.gout ? a.gout[gidx] : a.target[gidx];
                        et8[ii] = a.feta[gidx];
                        P8[ii] = a.paux[gidx];
                        Q8[ii] = a.paux[HW + gidx];
                    }
                }
#pragma unroll
                for (int ii = 0; ii < kChunk; ++ii) {
                    const int k = i0c + ii;
                    const int gi = c.i0 + k, gj = c.j0 + j;
                    if (k < TH && gi < a.H && gj < a.W) {
                        const size_t gidx = (size_t)gi * a.W + gj;
                        const float other = xch[k * c.TW + j];
                        if (MODE == kForward) {
                            const float den = A0[kOutMax + k];
                            const float y =
                                (float)((double)a.center + (double)other / (double)den);
                            a.out[gidx] = y;
                            if (a.eta) a.eta[gidx] = den;
                            if (AUX && a.aux) a.aux[HW + gidx] = A1[kOutMax + k];  // Q
                            if (a.loss_part) {
                                const double d = (double)y - (double)G8[ii];
                                sq += d * d;
                            }
                        } else {
                            const float fo = fo8[ii];
                            const float G = a.gout ? G8[ii] : 2.0f * (fo - G8[ii]);
                            const float Ak = G / et8[ii];
                            const float Bk = Ak * (fo - a.center);
                            a.out[gidx] = (A1[kOutMax + k] + other) +
                                          a.alpha_f * (Ak * P8[ii] - Bk * Q8[ii]);
                        }
                    }
                }
            }
        }
    }
    if (MODE == kForward && a.loss_part) {
        // fixed-order reduction over the 64 column lanes: the same partial on every run
        double* red = reinterpret_cast<double*>(c.gpl);
        if (c.wave == 2) red[c.lane] = sq;
        __syncthreads();
        if (c.t == 2 * 64) {
            double acc = 0.0;
            for (int k = 0; k < 64; ++k) acc += red[k];
            a.loss_part[tile_id] = (float)acc;
        }
    }
    __syncthreads();   // LDS is reused by the next tile of a persistent workgroup
}

// One output tile of one image (tile index tile_id) for descriptor a; all
// 256 threads of the workgroup call it together.
template <int MODE, bool AUX, bool GG = false, int L = kLine>
__device__ __forceinline__ void tile_body(const TileArgs& a, int tile_id, float* smem) {
    TileCtx c;
    c.EH = a.EH;
    c.EW = a.EW;
    c.TH = a.TH;
    c.TW = a.TW;
    c.R = a.R;
    c.EWp = a.EWp;
    c.EHp = a.EHp;
    c.tfl = tile_t_floats(a.TW, a.EHp);
    const int pfl = tile_plane_floats(a.EH, a.EWp);
    c.gpl = GG ? nullptr : smem;
    c.hpl = (MODE == kBackward) ? (GG ? smem : smem + pfl) : nullptr;
    c.Tb = (MODE == kBackward && !GG) ? smem + 2 * pfl : smem + pfl;
    c.gT = c.Tb + 2 * c.tfl;
    c.t = threadIdx.x;
    c.wave = __builtin_amdgcn_readfirstlane(c.t >> 6);
    c.lane = c.t & 63;
    const int ty = tile_id / a.tiles_x, tx = tile_id - ty * a.tiles_x;
    c.i0 = ty * a.TH;
    c.j0 = tx * a.TW;
    c.ei0 = c.i0 - a.R;
    c.ej0 = c.j0 - a.R;

    if (!GG) fill_plane(a, c, c.gpl, [&](size_t k) { return a.f[k] - a.center; });
    if (MODE == kBackward) {
        // A = G / eta, staged where h goes once the row lanes have taken it
        fill_plane(a, c, c.hpl, [&](size_t k) {
            const float G = a.gout ? a.gout[k] : 2.0f * (a.fout[k] - a.target[k]);
            return G / a.feta[k];
        });
    }
    __syncthreads();
    if (MODE == kForward || GG) {
        // output columns, contiguous, for the column lanes' 16-byte loads
        for (int p = c.t; p < kGtFloats; p += kTileThreads) {
            const int jj = p / kGtPitch, k = p - jj * kGtPitch;
            const bool in = jj < a.TW && k < a.TH;
            if (GG) {   // from global memory: clamped load, zero outside the image
                const int gi = c.i0 + k, gj = c.j0 + jj;
                const float fv = a.f[(size_t)min(gi, a.H - 1) * a.W + min(gj, a.W - 1)];
                c.gT[p] = (in && gi < a.H && gj < a.W) ? fv - a.center : 0.0f;
            } else {
                c.gT[p] = in ? c.gpl[(k + a.R) * a.EWp + a.R + jj] : 0.0f;
            }
        }
        __syncthreads();
    }
    if (c.wave < 2)
        row_role<MODE, GG, L>(a, c);
    else
        col_role<MODE, AUX, GG, L>(a, c, tile_id);
}

template <int MODE, bool AUX, bool GG = false, int L = kLine>
__global__ void __launch_bounds__(kTileThreads)
bf_tile_kernel(const TileArgs a) {
    extern __shared__ __align__(16) float smem[];
    tile_body<MODE, AUX, GG, L>(a, blockIdx.x, smem);
}

// Host helpers shared by the single-image and batched launchers (bf_tile.hip).
bf_status plan_tiles(int mode, int64_t H, int64_t W, const SpatialParams& sp, int req_h,
                     int req_w, TileGeom* g, bool gg = false);
void fill_tile_args(TileArgs& a, int64_t H, int64_t W, const RangeParams& rp,
                    const SpatialParams& sp, const TileGeom& g, int mode);

}  // namespace bf
