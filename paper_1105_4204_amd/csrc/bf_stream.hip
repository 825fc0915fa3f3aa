// Streamed forward for wide spatial kernels: eq. (final-form) with the
// separable iterated-box averaging of Sec. 2.1 split into a column pass and a
// row pass over whole image lines, so that the work per pixel and cosine pair
// does not depend on the box radii.
//
// Column pass (bf_strm_v).  A box of width L is (1 - z^-L) / (1 - z^-1), so
// the causal composite of nb boxes is
//     b * x = S^nb d,   d[t] = sum_{A subset of boxes} (-1)^|A| x[t - sum_{k in A} L_k],
// with S the running sum (integrator).  A lane owns one image column and G
// consecutive cosine pairs and walks down the column: at each row it
// recomputes the channels at the 2^nb tap rows from f (phase, channel), forms
// d from the float samples in FP64 and runs the nb integrators in FP64.  No
// history of the filtered signal is kept, and nothing depends on the radii
// but the tap offsets.  Integrators never damp their rounding errors; in FP64
// the drift stays below 1e-5 of one sample after thousands of rows, far below
// the float32 resolution of the outputs (a fixed-point grid instead would be
// exact but, at a usable width, coarser than float32 on smooth regions, where
// its error adds up coherently over the whole window).  A lane may start
// part-way down the image: the integrator state there is a weighted sum of
// the 2R + nb rows above (closed-form binomial weights of the taps), so the
// start costs about a quarter of that many steps.  Outputs (the
// column-filtered channels C, gC, S, gS of each pair; 1, g for m = 0) go to
// row-major planes in the workspace.
//
// Row pass (bf_strm_h).  One workgroup per image row; wave w filters channel
// w of each pair along the whole row with exact int32 box sums: the samples
// are quantised, and each box stage is a wave prefix scan written to LDS and
// differenced at +-(r+1) (the prefix wraps modulo 2^32; the window sums do
// not, by the choice of scales).  Between stages the sums are shifted right
// so that the next window sum fits again.  The four filtered channels then
// meet in LDS and every thread demodulates its pixels with C and S from the
// phase recurrence Z <- Z exp(j 2 a g), accumulating den and num across the
// pairs; the last pair chunk divides in FP64.
//
// Unlike the fused tile kernel, the column-filtered channels of a chunk of
// pairs pass through device memory (16 bytes per pixel and pair, written
// once and read once); in exchange there is no halo work, and the cost is
// the same for any kernel width.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "bf_tile.h"

namespace bf {

constexpr int kSmThreads = 256;
constexpr int kSmMaxTaps = 16;        // 2^BF_MAX_BOXES
constexpr int kSmMaxGroups = 64;      // pair groups per chunk
constexpr int kSmMaxChunk = 256;      // pairs per chunk
constexpr int kSmLineMax = 81;        // row pass: samples per lane at most (odd)

// Cody-Waite split of pi/2: two 12-bit parts (exact products with |k| < 2^12)
// and a float remainder.
constexpr float kPio2A = 1.57080078125f;
constexpr float kPio2B = -4.453584551811218e-06f;
constexpr float kPio2C = -8.705516e-10f;

// exp(j theta) with theta = (mh + ml) g for |theta| up to about 1000: the
// product is carried as an unevaluated sum p + e (the exact rounding error of
// mh g through an fma), reduced by k pi/2 with the split above, and the
// remainder (|r| <= pi/4) goes through cis_small.  All float32.
__device__ __forceinline__ void cis_wide(float mh, float ml, float g, float& c, float& s) {
    const float p = mh * g;
    const float e = fmaf(mh, g, -p) + ml * g;
    const float k = rintf(p * 0.636619772f);
    float r = fmaf(-k, kPio2A, p);
    r = fmaf(-k, kPio2B, r);
    r += fmaf(-k, kPio2C, e);
    float cx, sx;
    cis_small(r, cx, sx);
    const int q = ((int)k) & 3;
    c = q == 0 ? cx : q == 1 ? -sx : q == 2 ? -cx : sx;
    s = q == 0 ? sx : q == 1 ? cx : q == 2 ? -sx : -cx;
}

struct StrmVArgs {
    const float* f;
    float* vp;              // planes [pair][4][H][Wp]
    int H, W, Wp;
    int ntaps;
    int toff[kSmMaxTaps];   // tap offsets (rows back from the current step)
    int tcoef[kSmMaxTaps];  // tap coefficients (+-1; binomial counts where offsets merge)
    int kinit;              // rows of the segment-start sums: 2R + nb
    int R;
    int npairs;             // pairs of this chunk
    int ngroups, ncolg, seg, nseg;
    float center, two_alpha;
    float mh[kSmMaxGroups], ml[kSmMaxGroups];   // m a of each group's first pair, hi + lo
};

template <int NB, int G>
__global__ void __launch_bounds__(kSmThreads) bf_strm_v(const StrmVArgs a) {
    constexpr int NT = 1 << NB;
    extern __shared__ double wtab[];   // [k][s]: integrator weights of the segment start
    const int lane = threadIdx.x & 63;
    const int H = a.H;
    // I_s[t] = sum_k w_s[k] x[t - k] with sum_k w_s[k] z^-k = D(z) / (1 - z^-1)^s,
    // D the taps' polynomial: w_s[k] = sum_j c_j C(k - o_j + s - 1, s - 1) over
    // o_j <= k (integers, exact in FP64); zero past k = 2R + nb - s.
    for (int k = threadIdx.x; k < a.kinit; k += kSmThreads) {
        double w[NB];
#pragma unroll
        for (int s = 0; s < NB; ++s) w[s] = 0.0;
        for (int j = 0; j < a.ntaps; ++j) {
            const double n = (double)(k - a.toff[j]);
            if (n >= 0.0) {
                const double c = (double)a.tcoef[j];
                double b = 1.0;   // C(n + s, s) for s = 0, 1, ...
#pragma unroll
                for (int s = 0; s < NB; ++s) {
                    w[s] += c * b;
                    b = b * (n + (double)(s + 1)) / (double)(s + 1);
                }
            }
        }
#pragma unroll
        for (int s = 0; s < NB; ++s) wtab[k * NB + s] = w[s];
    }
    __syncthreads();
    const int gw = blockIdx.x * (kSmThreads / 64) + (threadIdx.x >> 6);
    const int pg = gw % a.ngroups;
    const int rest = gw / a.ngroups;
    const int cg = rest % a.ncolg;
    const int sg = rest / a.ncolg;
    if (sg >= a.nseg) return;   // after the only barrier
    const int x = cg * 64 + lane;
    if (x >= a.W) return;
    const int n0 = sg * a.seg, n1 = min(H, n0 + a.seg);
    const int t0 = n0 + a.R;            // first step that emits a row (row n0)
    const int te = n1 + a.R;
    const float mh = a.mh[pg], ml = a.ml[pg];
    const int q0 = pg * G;
    const int nq = min(G, a.npairs - q0);
    double I[G][4][NB];
#pragma unroll
    for (int q = 0; q < G; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int s = 0; s < NB; ++s) I[q][k][s] = 0.0;

    // the state before step t0 from the rows above it: y = t0 - 1 - k in [0, H)
    {
        const int kb = max(0, t0 - H), ke = min(a.kinit - 1, t0 - 1);
        float gpre = (a.f + (size_t)min(max(t0 - 1 - kb, 0), H - 1) * a.W)[x];
        for (int k = kb; k <= ke; ++k) {
            const float g = gpre - a.center;
            gpre = (a.f + (size_t)max(t0 - 2 - k, 0) * a.W)[x];
            float ur, ui, zr, zi;
            cis_small(a.two_alpha * g, ur, ui);
            cis_wide(mh, ml, g, zr, zi);
            double w[NB];
#pragma unroll
            for (int s = 0; s < NB; ++s) w[s] = wtab[k * NB + s];
#pragma unroll
            for (int q = 0; q < G; ++q) {
                const double c0 = (double)zr, c1 = (double)(g * zr);
                const double c2 = (double)zi, c3 = (double)(g * zi);
#pragma unroll
                for (int s = 0; s < NB; ++s) {
                    I[q][0][s] = fma(w[s], c0, I[q][0][s]);
                    I[q][1][s] = fma(w[s], c1, I[q][1][s]);
                    I[q][2][s] = fma(w[s], c2, I[q][2][s]);
                    I[q][3][s] = fma(w[s], c3, I[q][3][s]);
                }
                if (q + 1 < G) {
                    const float nr = zr * ur - zi * ui;
                    zi = zr * ui + zi * ur;
                    zr = nr;
                }
            }
        }
    }

    // tap rows are wave-uniform: row base in SGPRs, the lane's column as offset
    float gnext[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int y = min(max(t0 - a.toff[j], 0), H - 1);
        gnext[j] = (a.f + (size_t)y * a.W)[x];
    }
    for (int t = t0; t < te; ++t) {
        float gcur[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) gcur[j] = gnext[j];
        // next step's taps: clamped unconditional loads, in flight during this step
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int y = min(max(t + 1 - a.toff[j], 0), H - 1);
            gnext[j] = (a.f + (size_t)y * a.W)[x];
        }
        // d = sum_j c_j x[t - o_j], the float samples summed in FP64
        double d[G][4];
#pragma unroll
        for (int q = 0; q < G; ++q)
#pragma unroll
            for (int k = 0; k < 4; ++k) d[q][k] = 0.0;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            if (j < a.ntaps) {   // uniform
                const int y = t - a.toff[j];
                const bool in = y >= 0 && y < H;
                const float g = in ? gcur[j] - a.center : 0.0f;
                float ur, ui, zr, zi;
                cis_small(a.two_alpha * g, ur, ui);
                cis_wide(mh, ml, g, zr, zi);
                zr = in ? zr : 0.0f;
                zi = in ? zi : 0.0f;
                const double c = (double)a.tcoef[j];
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    d[q][0] = fma(c, (double)zr, d[q][0]);
                    d[q][1] = fma(c, (double)(g * zr), d[q][1]);
                    d[q][2] = fma(c, (double)zi, d[q][2]);
                    d[q][3] = fma(c, (double)(g * zi), d[q][3]);
                    if (q + 1 < G) {
                        const float nr = zr * ur - zi * ui;
                        zi = zr * ui + zi * ur;
                        zr = nr;
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < G; ++q)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                I[q][k][0] += d[q][k];
#pragma unroll
                for (int s = 1; s < NB; ++s) I[q][k][s] += I[q][k][s - 1];
            }
        float* dst = a.vp + (size_t)(t - a.R) * a.Wp + x;
        const size_t plane = (size_t)H * a.Wp;
#pragma unroll
        for (int q = 0; q < G; ++q) {
            if (q < nq) {   // uniform
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    dst[((size_t)(q0 + q) * 4 + k) * plane] = (float)I[q][k][NB - 1];
            }
        }
    }
}

struct StrmHArgs {
    const float* f;
    const float* vp;
    float* out;
    float* eta;
    float* part;            // den, num partial planes (2 H W) between chunks, or NULL
    int H, W, Wp;
    int R, nb;
    int r[BF_MAX_BOXES];
    int padl, bufsz;        // LDS: per wave padl zeros, then 64 E + rmax samples
    int npairs;             // pairs of this chunk
    int centre0;            // the chunk's first pair is m = 0
    int first, last;        // first / last chunk
    float center;
    float hsc[2];           // stage-1 quantisation scale: C, S / gC, gS
    int sh[BF_MAX_BOXES][2];   // right shift after each stage
    float hout[2];          // value of one unit of the last stage's sums
    float chat[kSmMaxChunk];          // coefficients of the chunk's pairs
    float mh[kSmMaxChunk], ml[kSmMaxChunk];   // m a of each pair, hi + lo
};

// Exclusive prefix sum of v over the 64 lanes of a wave (modulo 2^32).
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, int lane) {
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t n = (uint32_t)__shfl_up((int)incl, o, 64);
        incl += lane >= o ? n : 0u;
    }
    return incl - v;
}

// E: samples per lane (odd, so lanes E words apart hit distinct LDS banks);
// the line covers 64 E >= W + 2R positions.
template <int E>
__global__ void __launch_bounds__(kSmThreads) bf_strm_h(const StrmHArgs a) {
    constexpr int NX = (64 * E + kSmThreads - 1) / kSmThreads;   // pixels per thread at most
    extern __shared__ __align__(16) uint32_t slds[];
    const int t = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int lane = t & 63;
    const int y = blockIdx.x;
    const int W = a.W, R = a.R;
    uint32_t* buf = slds + wave * a.bufsz;
    for (int i = lane; i < a.padl; i += 64) buf[i] = 0u;   // prefix before the line: 0
    uint32_t* line = buf + a.padl;
    const int nx = (W + kSmThreads - 1) / kSmThreads;

    // demodulation state of pixels x = t + 256 i: g and the two sums (the
    // phase of each pair is evaluated directly, so none is carried)
    float gx[NX], den[NX], num[NX];
    const float* frow = a.f + (size_t)y * W;
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        const int x = min(t + i * kSmThreads, W - 1);
        gx[i] = frow[x] - a.center;
        den[i] = a.first ? 0.0f : a.part[(size_t)y * W + x];
        num[i] = a.first ? 0.0f : a.part[(size_t)(a.H + y) * W + x];
    }
    __syncthreads();

    const size_t plane = (size_t)a.H * a.Wp;
    const int p0 = lane * E;
    for (int qq = 0; qq < a.npairs; ++qq) {
        const bool centre = a.centre0 && qq == 0;
        const int nch = centre ? 2 : 4;
        if (wave < nch) {
            const int cls = wave & 1;
            const float* src = a.vp + ((size_t)qq * 4 + wave) * plane + (size_t)y * a.Wp;
            const float hs = a.hsc[cls];
            // the quantised row into the line at position R + x, in 16-byte
            // buffer loads (lane offset in a register, the chunk in the
            // instruction; the buffer ends at W rounded up to 4, so chunks past
            // it read zero) and aligned 16-byte LDS stores; then the zero
            // margins [0, R) and [R + W, end of the line)
            const int W4 = (W + 3) & ~3;
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<float*>(src), 0, W4 * (int)sizeof(float), kBufferWord3);
            uint32_t* dst4 = line + R + 4 * lane;
            constexpr int NH = (NX + 1) / 2;   // two batches: half the staging registers
#pragma unroll
            for (int b = 0; b < NX; b += NH) {
                float4 ld[NH];
#pragma unroll
                for (int i = 0; i < NH; ++i) {
                    const auto q = __builtin_amdgcn_raw_buffer_load_b128(
                        rs, 16 * lane, 1024 * (b + i), 0);
                    ld[i] = make_float4(__uint_as_float(q[0]), __uint_as_float(q[1]),
                                        __uint_as_float(q[2]), __uint_as_float(q[3]));
                }
#pragma unroll
                for (int i = 0; i < NH; ++i) {
                    if (b + i < NX) {
                        uint4 o;
                        o.x = (uint32_t)__float2int_rn(ld[i].x * hs);
                        o.y = (uint32_t)__float2int_rn(ld[i].y * hs);
                        o.z = (uint32_t)__float2int_rn(ld[i].z * hs);
                        o.w = (uint32_t)__float2int_rn(ld[i].w * hs);
                        *reinterpret_cast<uint4*>(dst4 + 256 * (b + i)) = o;
                    }
                }
            }
            for (int p = lane; p < R; p += 64) line[p] = 0u;
            for (int p = R + W + lane; p < 64 * E; p += 64) line[p] = 0u;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            uint32_t v[E];
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = line[p0 + e];
            for (int k = 0; k < a.nb; ++k) {
                const int r = a.r[k];
                // inclusive prefix along the line: lane-local, then across lanes
                uint32_t tot = 0u;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    tot += v[e];
                    v[e] = tot;
                }
                const uint32_t off = wave_excl_scan(tot, lane);
#pragma unroll
                for (int e = 0; e < E; ++e) line[p0 + e] = v[e] + off;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                // window sums: prefix at p + r minus prefix at p - r - 1, in
                // blocks of 8 (a scheduling fence keeps the compiler from
                // hoisting all 2 E reads, which would hold 2 E registers)
                const uint32_t* hi = line + p0 + r;
                const uint32_t* lo = line + p0 - r - 1;
#pragma unroll
                for (int e0 = 0; e0 < E; e0 += 8) {
#pragma unroll
                    for (int e = e0; e < (e0 + 8 < E ? e0 + 8 : E); ++e) v[e] = hi[e] - lo[e];
                    __builtin_amdgcn_sched_barrier(0);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const int sh = a.sh[k][cls];
                if (k + 1 < a.nb && sh > 0) {   // uniform
                    const int rnd = 1 << (sh - 1);
#pragma unroll
                    for (int e = 0; e < E; ++e) v[e] = (uint32_t)(((int32_t)v[e] + rnd) >> sh);
                }
            }
            // the filtered channel in place of the line, for the demodulation
#pragma unroll
            for (int e = 0; e < E; ++e) line[p0 + e] = v[e];
        }
        __syncthreads();
        const float c = a.chat[qq];
        const float cc = c * a.hout[0], cg = c * a.hout[1];
        const float mh = a.mh[qq], ml = a.ml[qq];
        const uint32_t* l0 = slds + a.padl + R;
        const uint32_t* l1 = l0 + a.bufsz;
        const uint32_t* l2 = l1 + a.bufsz;
        const uint32_t* l3 = l2 + a.bufsz;
        // every pixel slot (slots past W read inside the lines and are never stored)
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            {
                const int x = t + i * kSmThreads;
                const float D0 = (float)(int32_t)l0[x];
                const float D1 = (float)(int32_t)l1[x];
                if (centre) {   // m = 0: channels 1 and g, C = 1, S = 0
                    den[i] = fmaf(cc, D0, den[i]);
                    num[i] = fmaf(cg, D1, num[i]);
                } else {
                    const float D2 = (float)(int32_t)l2[x];
                    const float D3 = (float)(int32_t)l3[x];
                    float zr, zi;
                    cis_wide(mh, ml, gx[i], zr, zi);
                    den[i] = fmaf(cc * zr, D0, fmaf(cc * zi, D2, den[i]));
                    num[i] = fmaf(cg * zr, D1, fmaf(cg * zi, D3, num[i]));
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        const int x = t + i * kSmThreads;
        if (i < nx && x < W) {
            const size_t o = (size_t)y * W + x;
            if (a.last) {
                a.out[o] = (float)((double)a.center + (double)num[i] / (double)den[i]);
                if (a.eta) a.eta[o] = den[i];
            } else {
                a.part[o] = den[i];
                a.part[(size_t)a.H * W + o] = num[i];
            }
        }
    }
}

// ---- host side -----------------------------------------------------------

namespace {

// pairs per lane in the column pass: the integrator state (4 channels x nb
// doubles per pair) must leave room for two waves per SIMD
constexpr int sm_group(int nb) { return nb <= 2 ? 6 : (nb == 3 ? 4 : 3); }

// Row-pass instantiations: samples per lane (odd).
constexpr int kSmLines[] = {9, 17, 25, 33, 37, 41, 45, 49, 57, 65, 69, 73, 81};

int line_lanes(int64_t W, int R) {
    // the row lands at R + x in 16-byte pieces, so the line spans W rounded
    // up to 4, plus R zeros on each side
    const int64_t need = (((W + 3) & ~(int64_t)3) + 2 * R + 63) / 64;
    for (int e : kSmLines)
        if (e >= need) return e;
    return 0;
}

// Sparse difference taps of the column pass: offsets sum_{k in A} L_k with
// sign (-1)^|A|, equal offsets merged.
int make_taps(const SpatialParams& sp, int* off, int* coef) {
    int n = 0;
    for (int mask = 0; mask < (1 << sp.nb); ++mask) {
        int o = 0, s = 1;
        for (int k = 0; k < sp.nb; ++k)
            if (mask & (1 << k)) {
                o += 2 * sp.r[k] + 1;
                s = -s;
            }
        int i = 0;
        while (i < n && off[i] != o) ++i;
        if (i == n) {
            off[n] = o;
            coef[n] = 0;
            ++n;
        }
        coef[i] += s;
    }
    int m = 0;
    for (int i = 0; i < n; ++i)
        if (coef[i] != 0) {
            off[m] = off[i];
            coef[m] = coef[i];
            ++m;
        }
    return m;
}

double mass_1d(const SpatialParams& sp) {
    double m = 1.0;
    for (int k = 0; k < sp.nb; ++k) m *= 2.0 * sp.r[k] + 1.0;
    return m;
}

int floor_log2(double v) { return (int)std::floor(std::log2(v)); }

}  // namespace

static size_t stream_plane_pitch(int64_t W) { return (size_t)((W + 63) / 64 * 64); }

bool stream_supported(int64_t W, const SpatialParams& sp) {
    if (sp.nb < 1 || sp.nb > BF_MAX_BOXES) return false;
    if (line_lanes(W, sp.R) == 0) return false;   // W + 2R up to 64 x 81 samples
    // FP64 integrators exact: mass * 2^22 < 2^53; row pass: a window of one
    // stage must hold at least 2^8 quantisation levels of its input
    if (mass_1d(sp) >= 2147483648.0) return false;
    for (int k = 0; k < sp.nb; ++k)
        if (2 * sp.r[k] + 1 > (1 << 22)) return false;
    return true;
}

size_t stream_workspace_bytes(int64_t H, int64_t W, int pairs) {
    return (size_t)16 * (size_t)pairs * (size_t)H * stream_plane_pitch(W) +
           (size_t)8 * (size_t)H * (size_t)W;
}

int stream_chunk_pairs(int64_t H, int64_t W, size_t ws_bytes, int npairs) {
    const size_t part = (size_t)8 * H * W;
    const size_t per = (size_t)16 * H * stream_plane_pitch(W);
    if (ws_bytes < part + per) return 0;
    size_t g = (ws_bytes - part) / per;
    g = std::min<size_t>(g, (size_t)kSmMaxChunk);
    return (int)std::min<size_t>(g, (size_t)npairs);
}

namespace {

template <int NB>
void launch_v(const StrmVArgs& a, hipStream_t s, unsigned blocks, size_t lds) {
    (void)hipFuncSetAttribute((const void*)bf_strm_v<NB, sm_group(NB)>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((bf_strm_v<NB, sm_group(NB)>), dim3(blocks), dim3(kSmThreads), lds, s, a);
}

template <int I = 0>
void launch_h(const StrmHArgs& a, int E, hipStream_t s, unsigned blocks, size_t lds) {
    if constexpr (I < (int)(sizeof(kSmLines) / sizeof(kSmLines[0]))) {
        if (E == kSmLines[I]) {
            (void)hipFuncSetAttribute((const void*)bf_strm_h<kSmLines[I]>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            hipLaunchKernelGGL(bf_strm_h<kSmLines[I]>, dim3(blocks), dim3(kSmThreads), lds, s, a);
            return;
        }
        launch_h<I + 1>(a, E, s, blocks, lds);
    }
}

}  // namespace

// Cost model per cosine pair, calibrated on MI355X: a round of fused tiles
// (one workgroup per CU) against the streamed passes' time per pixel.  The
// fused tiles shrink as R grows (the extended line is at most 128 samples);
// the streamed passes cost the same for any R.
constexpr double kFusedRoundUs = 16.0;        // per pair and round of fused tiles
constexpr double kStreamPixUs = 2.0e-5;       // per pair and pixel, both passes
constexpr double kStreamPairUs = 10.0;        // per pair: two launches, row-pass rounds

bool prefer_stream(int64_t H, int64_t W, const SpatialParams& sp, bf_status fused_status,
                   const TileGeom& g) {
    if (!stream_supported(W, sp)) return false;
    if (fused_status != BF_OK) return true;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        cus = 256;
    const double fused_us = std::ceil((double)g.tiles_x * g.tiles_y / cus) * kFusedRoundUs;
    const double stream_us = (double)H * (double)W * kStreamPixUs + kStreamPairUs;
    return stream_us < fused_us;
}

bf_status launch_stream(const float* f, float* out, float* eta, int64_t H, int64_t W,
                        const RangeParams& rp, const SpatialParams& sp, void* workspace,
                        size_t ws_bytes, hipStream_t stream) {
    if (!stream_supported(W, sp)) {
        set_error("streamed path: W + 2R = %lld exceeds %d samples, or the kernel's mass is "
                  "too large", (long long)(W + 2 * sp.R), 64 * kSmLineMax);
        return BF_EUNSUPPORTED;
    }
    const int chunk = stream_chunk_pairs(H, W, ws_bytes, rp.npairs);
    if (chunk <= 0) {
        set_error("streamed path: workspace of %zu bytes is below the %zu bytes one pair needs",
                  ws_bytes, stream_workspace_bytes(H, W, 1));
        return BF_EINVAL;
    }
    const int Wp = (int)stream_plane_pitch(W);
    float* vp = static_cast<float*>(workspace);
    float* part = vp + (size_t)4 * chunk * H * Wp;
    const double Tg = (double)rp.center;                  // |g| <= T/2
    const double mass = mass_1d(sp);

    // column pass: taps and the segment-start weights' extent
    StrmVArgs va = {};
    va.f = f;
    va.vp = vp;
    va.H = (int)H;
    va.W = (int)W;
    va.Wp = Wp;
    va.ntaps = make_taps(sp, va.toff, va.tcoef);
    va.R = sp.R;
    va.center = rp.center;
    va.two_alpha = (float)(2.0 * rp.alpha);
    va.kinit = 2 * sp.R + sp.nb;
    const size_t lds_v = (size_t)va.kinit * sp.nb * sizeof(double);
    // row pass scales: stage-1 samples |V| <= mass xmax; each stage's window
    // sum must stay below 2^30
    StrmHArgs ha = {};
    ha.f = f;
    ha.vp = vp;
    ha.out = out;
    ha.eta = eta;
    ha.part = part;
    ha.H = (int)H;
    ha.W = (int)W;
    ha.Wp = Wp;
    ha.R = sp.R;
    ha.nb = sp.nb;
    int rmax = 0;
    for (int k = 0; k < sp.nb; ++k) {
        ha.r[k] = sp.r[k];
        rmax = std::max(rmax, sp.r[k]);
    }
    const int E = line_lanes(W, sp.R);
    ha.padl = ((rmax + 1 + sp.R + 3) & ~3) - sp.R;   // line + R is 16-byte aligned
    // after the line: rmax + 1 for the window reads of unused outputs, and
    // room for the row's 16-byte stores and the demodulation's pixel slots,
    // which run to R + 256 ceil(64 E / 256)
    const int nxs = (64 * E + kSmThreads - 1) / kSmThreads;
    const int tail = std::max(rmax + 1, sp.R + kSmThreads * nxs - 64 * E);
    ha.bufsz = (ha.padl + 64 * E + tail + 3) & ~3;
    ha.center = rp.center;
    const double xmax[2] = {1.0, Tg};
    for (int c = 0; c < 2; ++c) {
        // V samples are bounded by mass * xmax (plus the quantisation slack)
        const double vmax = mass * xmax[c] * (1.0 + 1e-6) + 1.0;
        const int e1 = floor_log2(1073741824.0 / ((2.0 * sp.r[0] + 1.0) * vmax));
        ha.hsc[c] = std::ldexp(1.0f, e1);
        double qmax = vmax * std::ldexp(1.0, e1) + 1.0;
        int total = 0;
        for (int k = 0; k < sp.nb; ++k) {
            const double smax = (2.0 * sp.r[k] + 1.0) * qmax;   // window sum of stage k
            int sh = 0;
            if (k + 1 < sp.nb) {
                const double lim = 1073741824.0 / (2.0 * sp.r[k + 1] + 1.0);
                while (smax / std::ldexp(1.0, sh) + 1.0 > lim) ++sh;
                qmax = smax / std::ldexp(1.0, sh) + 1.0;
                total += sh;
            }
            ha.sh[k][c] = sh;
        }
        ha.hout[c] = (float)std::ldexp(1.0, total - e1);
    }
    const size_t lds_h = (size_t)4 * ha.bufsz * sizeof(uint32_t);
    if (lds_h > 160 * 1024) {
        set_error("streamed path: row pass needs %zu bytes of LDS", lds_h);
        return BF_EUNSUPPORTED;
    }

    // the column pass's parallelism: 64-column groups x pair groups x row
    // segments, with 2R warm-up rows per segment; pick the segment count
    // with the least modelled time (waves in flight: 8 per CU)
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int ncolg = (int)((W + 63) / 64);
    const double slots = 8.0 * cus;

    const int nchunks = (rp.npairs + chunk - 1) / chunk;
    for (int ci = 0; ci < nchunks; ++ci) {
        const int qb = ci * chunk;
        const int np = std::min(chunk, rp.npairs - qb);
        const int G = sm_group(sp.nb);
        const int ngroups = (np + G - 1) / G;
        va.npairs = np;
        va.ngroups = ngroups;
        va.ncolg = ncolg;
        for (int g = 0; g < ngroups; ++g) {
            const double ma = (double)(rp.odd + 2 * (qb + g * G)) * rp.alpha;
            va.mh[g] = (float)ma;
            va.ml[g] = (float)(ma - (double)va.mh[g]);
        }
        int best = 1;
        double best_cost = 1e300;
        for (int ns = 1; ns <= 64; ++ns) {
            const int seg = (int)((H + ns - 1) / ns);
            if (ns > 1 && seg < 16) break;
            const double waves = (double)ncolg * ngroups * ns;
            const double start = ns > 1 ? 0.25 * (2.0 * sp.R + sp.nb) : 0.25 * sp.R;
            const double cost = std::ceil(waves / slots) * (seg + start) +
                                0.05 * waves / slots * (seg + start);
            if (cost < best_cost) {
                best_cost = cost;
                best = ns;
            }
        }
        va.nseg = best;
        va.seg = (int)((H + best - 1) / best);
        const long long waves = (long long)ncolg * ngroups * va.nseg;
        const unsigned vblocks = (unsigned)((waves + 3) / 4);
        switch (sp.nb) {
            case 1: launch_v<1>(va, stream, vblocks, lds_v); break;
            case 2: launch_v<2>(va, stream, vblocks, lds_v); break;
            case 3: launch_v<3>(va, stream, vblocks, lds_v); break;
            default: launch_v<4>(va, stream, vblocks, lds_v); break;
        }
        ha.npairs = np;
        ha.centre0 = (qb == 0 && rp.odd == 0) ? 1 : 0;
        ha.first = ci == 0;
        ha.last = ci == nchunks - 1;
        for (int q = 0; q < np; ++q) {
            ha.chat[q] = rp.chat[qb + q];
            const double ma = (double)(rp.odd + 2 * (qb + q)) * rp.alpha;
            ha.mh[q] = (float)ma;
            ha.ml[q] = (float)(ma - (double)ha.mh[q]);
        }
        launch_h(ha, E, stream, (unsigned)H, lds_h);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("streamed path launch: %s", hipGetErrorString(e));
        return BF_EDEVICE;
    }
    return BF_OK;
}

}  // namespace bf
