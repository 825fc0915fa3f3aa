// Streamed forward for wide spatial kernels: eq. (final-form) with the
// separable iterated-box averaging of Sec. 2.1 split into a column pass and a
// row pass over whole image lines, so that the work per pixel and cosine pair
// does not depend on the box radii.
//
// Column pass (bf_strm_v).  A box of width L is (1 - z^-L) / (1 - z^-1), so
// the causal composite of nb boxes is
//     b * x = S^nb d,   d[t] = sum_{A subset of boxes} (-1)^|A| x[t - sum_{k in A} L_k],
// with S the running sum (integrator).  On integer samples every step is an
// exact integer operation: the channels are quantised once (a fixed-point
// grid close to float32 resolution), the sparse difference d takes 2^nb taps
// of them, and the nb integrators run in FP64, which is exact for integers
// below 2^53 (the composite's mass times the largest sample stays below that).
// A lane owns one image column and G consecutive cosine pairs and walks down
// the column; the taps are recomputed from f at their rows (phase, channel,
// quantisation), so no history of the filtered signal is kept and nothing
// depends on the radii except the tap offsets.  A lane may start part-way
// down the image: it then treats the rows above its segment's halo as zero
// and runs 2R warm-up rows, which reproduces the true integrator state
// exactly.  Outputs (the column-filtered channels C, gC, S, gS of each pair;
// 1, g for m = 0) go to row-major planes in the workspace.
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
constexpr int kSmLineMax = 81;        // row pass: samples per lane at most (odd)
constexpr float kSmMagic = 12582912.0f;   // 1.5 * 2^23: fma(x, s, M) rounds x s to an integer

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
    int toff[kSmMaxTaps];       // tap offsets (rows back from the current step)
    float tsc[kSmMaxTaps][2];   // sign of the tap's coefficient times the scale (C, S / gC, gS)
    int tmul[kSmMaxTaps];       // |coefficient|: 1, or a binomial count where offsets merge
    uint32_t dbias;             // minus the magic constant's bits times sum |c_j|
    int R;
    int npairs;             // pairs of this chunk
    int ngroups, ncolg, seg, nseg;
    float center, two_alpha;
    float vinv[2];          // inverse quantisation scale: C, S / gC, gS
    float mh[kSmMaxGroups], ml[kSmMaxGroups];   // m a of each group's first pair, hi + lo
};

template <int NB, int G>
__global__ void __launch_bounds__(kSmThreads) bf_strm_v(const StrmVArgs a) {
    constexpr int NT = 1 << NB;
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * (kSmThreads / 64) + (threadIdx.x >> 6);
    const int pg = gw % a.ngroups;
    const int rest = gw / a.ngroups;
    const int cg = rest % a.ncolg;
    const int sg = rest / a.ncolg;
    if (sg >= a.nseg) return;
    const int x = cg * 64 + lane;
    if (x >= a.W) return;   // no barriers or LDS in this kernel
    const int H = a.H;
    const int n0 = sg * a.seg, n1 = min(H, n0 + a.seg);
    const int ylo = max(n0 - a.R, 0);   // rows above read as zero (warm-up from zero state)
    const int tb = ylo, te = n1 + a.R, tout = n0 + a.R;
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
    // tap rows are wave-uniform: row base in SGPRs, the lane's column as offset
    float gnext[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int y = min(max(tb - a.toff[j], 0), H - 1);
        gnext[j] = (a.f + (size_t)y * a.W)[x];
    }
    for (int t = tb; t < te; ++t) {
        float gcur[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) gcur[j] = gnext[j];
        // next step's taps: clamped unconditional loads, in flight during this step
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int y = min(max(t + 1 - a.toff[j], 0), H - 1);
            gnext[j] = (a.f + (size_t)y * a.W)[x];
        }
        // d = sum_j c_j q_j: the sign of c_j rides on the quantisation scale
        // (round to nearest even is odd-symmetric), |c_j| multiplies, and the
        // magic constant's bits, added once per unit of |c_j|, are removed
        // by the starting value
        uint32_t d[G][4];
#pragma unroll
        for (int q = 0; q < G; ++q)
#pragma unroll
            for (int k = 0; k < 4; ++k) d[q][k] = a.dbias;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            if (j < a.ntaps) {   // uniform
                const int y = t - a.toff[j];
                const bool in = y >= ylo && y < H;
                const float g = in ? gcur[j] - a.center : 0.0f;
                float ur, ui, zr, zi;
                cis_small(a.two_alpha * g, ur, ui);
                cis_wide(mh, ml, g, zr, zi);
                zr = in ? zr : 0.0f;
                zi = in ? zi : 0.0f;
                const float sc = a.tsc[j][0], sg2 = a.tsc[j][1];
                const uint32_t mul = (uint32_t)a.tmul[j];
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    const uint32_t b0 = __float_as_uint(fmaf(zr, sc, kSmMagic));
                    const uint32_t b1 = __float_as_uint(fmaf(g * zr, sg2, kSmMagic));
                    const uint32_t b2 = __float_as_uint(fmaf(zi, sc, kSmMagic));
                    const uint32_t b3 = __float_as_uint(fmaf(g * zi, sg2, kSmMagic));
                    if (mul == 1u) {   // uniform
                        d[q][0] += b0;
                        d[q][1] += b1;
                        d[q][2] += b2;
                        d[q][3] += b3;
                    } else {
                        d[q][0] += mul * b0;
                        d[q][1] += mul * b1;
                        d[q][2] += mul * b2;
                        d[q][3] += mul * b3;
                    }
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
                I[q][k][0] += (double)(int32_t)d[q][k];
#pragma unroll
                for (int s = 1; s < NB; ++s) I[q][k][s] += I[q][k][s - 1];
            }
        if (t >= tout) {   // uniform
            float* dst = a.vp + (size_t)(t - a.R) * a.Wp + x;
            const size_t plane = (size_t)H * a.Wp;
#pragma unroll
            for (int q = 0; q < G; ++q) {
                if (q < nq) {   // uniform
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        dst[((size_t)(q0 + q) * 4 + k) * plane] =
                            (float)(I[q][k][NB - 1] * (double)a.vinv[k & 1]);
                }
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
    float center, two_alpha;
    float mh, ml;           // m a of the chunk's first pair, hi + lo
    float hsc[2];           // stage-1 quantisation scale: C, S / gC, gS
    int sh[BF_MAX_BOXES][2];   // right shift after each stage
    float hout[2];          // value of one unit of the last stage's sums
    float chat[kMaxPairs];  // coefficients of the chunk's pairs
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

    // demodulation state of pixels x = t + 256 i
    float zr[NX], zi[NX], ur[NX], ui[NX], den[NX], num[NX];
    const float* frow = a.f + (size_t)y * W;
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        if (i < nx) {   // uniform
            const int x = min(t + i * kSmThreads, W - 1);
            const float g = frow[x] - a.center;
            cis_small(a.two_alpha * g, ur[i], ui[i]);
            cis_wide(a.mh, a.ml, g, zr[i], zi[i]);
            den[i] = a.first ? 0.0f : a.part[(size_t)y * W + x];
            num[i] = a.first ? 0.0f : a.part[(size_t)(a.H + y) * W + x];
        }
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
            // the quantised row into the line at position R + x, in coalesced
            // 16-byte loads (plane rows are 256-byte aligned, Wp >= W rounded
            // up to 4); the margins [0, R) and [R + W4, 64 E) are zero
            const int W4 = (W + 3) & ~3;
            for (int x = 4 * lane; x < W4; x += 256) {
                const float4 q = *reinterpret_cast<const float4*>(src + x);
                uint4 o;
                o.x = (uint32_t)__float2int_rn(q.x * hs);
                o.y = (uint32_t)__float2int_rn((x + 1 < W ? q.y : 0.0f) * hs);
                o.z = (uint32_t)__float2int_rn((x + 2 < W ? q.z : 0.0f) * hs);
                o.w = (uint32_t)__float2int_rn((x + 3 < W ? q.w : 0.0f) * hs);
                *reinterpret_cast<uint4*>(line + R + x) = o;
            }
            for (int p = lane; p < R; p += 64) line[p] = 0u;
            for (int p = R + W4 + lane; p < 64 * E; p += 64) line[p] = 0u;
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
                // window sums: prefix at p + r minus prefix at p - r - 1
                const uint32_t* hi = line + p0 + r;
                const uint32_t* lo = line + p0 - r - 1;
#pragma unroll
                for (int e = 0; e < E; ++e) v[e] = hi[e] - lo[e];
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
        const uint32_t* l0 = slds + a.padl + R;
        const uint32_t* l1 = l0 + a.bufsz;
        const uint32_t* l2 = l1 + a.bufsz;
        const uint32_t* l3 = l2 + a.bufsz;
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            if (i < nx) {   // uniform
                const int x = min(t + i * kSmThreads, W - 1);
                const float D0 = (float)(int32_t)l0[x];
                const float D1 = (float)(int32_t)l1[x];
                if (centre) {   // m = 0: channels 1 and g, C = 1, S = 0
                    den[i] = fmaf(cc, D0, den[i]);
                    num[i] = fmaf(cg, D1, num[i]);
                } else {
                    const float D2 = (float)(int32_t)l2[x];
                    const float D3 = (float)(int32_t)l3[x];
                    den[i] = fmaf(cc * zr[i], D0, fmaf(cc * zi[i], D2, den[i]));
                    num[i] = fmaf(cg * zr[i], D1, fmaf(cg * zi[i], D3, num[i]));
                }
                const float nr = zr[i] * ur[i] - zi[i] * ui[i];
                zi[i] = zr[i] * ui[i] + zi[i] * ur[i];
                zr[i] = nr;
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
constexpr int sm_group(int nb) { return nb <= 2 ? 8 : (nb == 3 ? 6 : 4); }

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
    g = std::min<size_t>(g, (size_t)kSmMaxGroups * 4);
    return (int)std::min<size_t>(g, (size_t)npairs);
}

namespace {

template <int NB>
void launch_v(const StrmVArgs& a, hipStream_t s, unsigned blocks) {
    hipLaunchKernelGGL((bf_strm_v<NB, sm_group(NB)>), dim3(blocks), dim3(kSmThreads), 0, s, a);
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
    const double stream_us = (double)H * (double)W * kStreamPixUs;
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

    // column pass: |x s| < 2^21 keeps the magic-constant rounding exact
    StrmVArgs va = {};
    va.f = f;
    va.vp = vp;
    va.H = (int)H;
    va.W = (int)W;
    va.Wp = Wp;
    int tcoef[kSmMaxTaps];
    va.ntaps = make_taps(sp, va.toff, tcoef);
    va.R = sp.R;
    va.center = rp.center;
    va.two_alpha = (float)(2.0 * rp.alpha);
    const int ev[2] = {21, floor_log2(2097152.0 / Tg)};
    for (int c = 0; c < 2; ++c) va.vinv[c] = std::ldexp(1.0f, -ev[c]);
    uint32_t units = 0;
    for (int j = 0; j < va.ntaps; ++j) {
        const int s = tcoef[j] > 0 ? 1 : -1;
        for (int c = 0; c < 2; ++c) va.tsc[j][c] = (float)s * std::ldexp(1.0f, ev[c]);
        va.tmul[j] = tcoef[j] > 0 ? tcoef[j] : -tcoef[j];
        units += (uint32_t)va.tmul[j];
    }
    uint32_t mbits;
    std::memcpy(&mbits, &kSmMagic, sizeof mbits);
    va.dbias = 0u - mbits * units;
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
    ha.bufsz = (ha.padl + 64 * E + rmax + 1 + 3) & ~3;
    ha.center = rp.center;
    ha.two_alpha = va.two_alpha;
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
            const double cost = std::ceil(waves / slots) * (seg + 2.0 * sp.R) +
                                0.05 * waves / slots * (seg + 2.0 * sp.R);
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
            case 1: launch_v<1>(va, stream, vblocks); break;
            case 2: launch_v<2>(va, stream, vblocks); break;
            case 3: launch_v<3>(va, stream, vblocks); break;
            default: launch_v<4>(va, stream, vblocks); break;
        }
        ha.npairs = np;
        ha.centre0 = (qb == 0 && rp.odd == 0) ? 1 : 0;
        ha.first = ci == 0;
        ha.last = ci == nchunks - 1;
        const double ma = (double)(rp.odd + 2 * qb) * rp.alpha;
        ha.mh = (float)ma;
        ha.ml = (float)(ma - (double)ha.mh);
        for (int q = 0; q < np; ++q) ha.chat[q] = rp.chat[qb + q];
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
