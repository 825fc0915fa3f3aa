// Staged forward for spatial kernels too wide for the fused tile kernel
// (sum of radii R > 63): the same eq. (final-form) evaluation, pair by pair,
// with the separable iterated-box averaging of Sec. 2.1 split into two
// passes over the whole image.
//
// Per cosine pair m (coefficient c_m), with g = f - T/2 and
// C + j S = exp(j m a g) evaluated directly (range reduction in FP64, then
// the |x| <= pi/4 polynomial):
//   vertical pass   (bf_stage_v): lane = image column; a 256-sample register
//     line down the column holds a channel (C, gC, S, gS; 1, g for m = 0)
//     on the extended rows, the box stages run along it, and the up to 176
//     outputs are written to a row-major plane V_ch (consecutive lanes,
//     consecutive columns);
//   horizontal pass (bf_stage_h): lane = image row; a 256-sample line along
//     the row is read from V_ch in 16-byte loads, the box stages run along
//     it, and the up to 64 outputs are demodulated and accumulated into den
//     and num (column-major, read-modify-write).
// A V_ch row carries at least 128 zero columns on each side (the zero
// extension of the horizontal pass, R <= 124); the left margin is
// 128 + (R mod 4) columns and the pitch a multiple of 4, so that every
// horizontal line starts on a 16-byte boundary.  A final pass divides in FP64 and writes out (and eta)
// row-major.  The planes live in a caller-provided workspace: unlike the
// fused kernel, this path keeps the filtered channels of one pair in device
// memory between its two passes.  Wide kernels have a large mass
// (the sum of w) against w(0), so where a pixel has few similar neighbours
// the pair terms cancel heavily; both passes use compensated running sums.
#include <algorithm>
#include <cmath>

#include "bf_tile.h"

namespace bf {

constexpr int kStLine = 256;      // register line of the staged passes
constexpr int kStThreads = 256;   // four waves: one per channel of a pair
constexpr int kStCols = 64;       // vertical pass: columns per workgroup
constexpr int kStOutV = 176;      // vertical pass: outputs per line, at most (written
                                  // straight from registers, so only the line bounds it)
constexpr int kStRows = 64;       // horizontal pass: rows per workgroup
constexpr int kStOutH = 128;      // horizontal pass: outputs per line, at most
constexpr int kStHalf = 64;       // horizontal pass: outputs per hand-over round
constexpr int kStMargin = 128;    // zero columns at least on each side of a V row (>= R)
static_assert(kStHalf % 4 == 0 && kStOutH == 2 * kStHalf,
              "the four waves share the output columns of a round; two rounds at most");
static_assert(kStThreads == 256 && kStCols == 64 && kStLine % 64 == 0,
              "the phase hand-over: four waves, 16 rows each per block of 64");

struct StageArgs {
    const float* f;
    float* vp;          // 4 row-major planes of H rows: V_ch[y * Wp + margin + x]
    float* den_t;       // column-major accumulators
    float* num_t;
    float* out;
    float* eta;
    int H, W, R, nb;
    int r[BF_MAX_BOXES];
    int Wp;             // V row pitch: W + 260 rounded up to a multiple of 64
    int margin;         // left margin: kStMargin + R mod 4, so margin - R is a multiple of 4
    int nout_v;         // outputs per vertical line: min(256 - 2R, kStOutV)
    int nout_h;         // outputs per horizontal line: min(256 - 2R, kStOutH), multiple of 4
    int centre;         // this pair is m = 0 (channels 1, g)
    float c;            // c_m
    double malpha;      // m a
    float center;       // T/2
};

// Vertical pass.  Workgroup: 64 columns x one segment of nout_v output rows;
// the 256 extended rows of g are staged in LDS once, then wave w builds
// channel w (C, gC, S, gS; 1, g for m = 0) down its 64 columns, filters it
// and writes its outputs row by row into V_ch.
// One wave per SIMD: the 256-sample line needs the whole register file.
__global__ void __launch_bounds__(kStThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
bf_stage_v(const StageArgs a) {
    extern __shared__ __align__(16) float lds[];
    float* gtile = lds;                                   // [256][kStCols]
    float* stg = lds + kStLine * kStCols;                 // [4][64][kStCols]
    const int t = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int lane = t & 63;
    const int x0 = blockIdx.x * kStCols;
    const int y0 = blockIdx.y * a.nout_v;
    const int ey0 = y0 - a.R;
    // clamped, unconditional loads in batches of 8 per thread, then the
    // selection against the real position (a guarded load would wait alone)
    for (int p0 = t; p0 < kStLine * kStCols; p0 += 8 * kStThreads) {
        float v8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int p = p0 + u * kStThreads;
            const int yy = p / kStCols, xx = p - yy * kStCols;
            const int gy = min(max(ey0 + yy, 0), a.H - 1), gx = min(x0 + xx, a.W - 1);
            v8[u] = a.f[(size_t)gy * a.W + gx];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int p = p0 + u * kStThreads;
            const int yy = p / kStCols, xx = p - yy * kStCols;
            const int gy = ey0 + yy, gx = x0 + xx;
            if (p < kStLine * kStCols)
                gtile[p] = (gy >= 0 && gy < a.H && gx < a.W) ? v8[u] - a.center : 0.0f;
        }
    }
    __syncthreads();
    const int nch = a.centre ? 2 : 4;
    const int ch = wave;
    const int x = x0 + lane;
    float v[kStLine];
    if (a.centre) {   // channels 1 and g: no phase
        if (ch < nch) {
#pragma unroll
            for (int y = 0; y < kStLine; ++y) {
                const int gy = ey0 + y;
                const bool in = x < a.W && gy >= 0 && gy < a.H;
                const float g = gtile[y * kStCols + lane];
                v[y] = in ? ((ch == 0) ? 1.0f : g) : 0.0f;
            }
        }
    } else {
        // Every channel needs the phase of every sample: per block of 64
        // rows each wave evaluates it for 16 of them and hands the four
        // channel values (C, gC, S, gS; zero outside the image) over
        // through LDS.  The flag is uniform, so all four waves pass the
        // barriers.
#pragma unroll
        for (int blk = 0; blk < kStLine / 64; ++blk) {
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int yl = wave * 16 + u;
                const int y = blk * 64 + yl;
                const int gy = ey0 + y;
                const bool in = x < a.W && gy >= 0 && gy < a.H;
                const float g = gtile[y * kStCols + lane];
                float cc, ss;
                cis_direct(a.malpha, g, cc, ss);
                cc = in ? cc : 0.0f;
                ss = in ? ss : 0.0f;
                stg[(0 * 64 + yl) * kStCols + lane] = cc;
                stg[(1 * 64 + yl) * kStCols + lane] = g * cc;
                stg[(2 * 64 + yl) * kStCols + lane] = ss;
                stg[(3 * 64 + yl) * kStCols + lane] = g * ss;
            }
            __syncthreads();
#pragma unroll
            for (int yl = 0; yl < 64; ++yl) v[blk * 64 + yl] = stg[(ch * 64 + yl) * kStCols + lane];
            __syncthreads();
        }
    }
    if (ch < nch && x < a.W) {   // columns past W stay zero: they are the margin
        for (int b = 0; b < a.nb; ++b) box_dispatch<kStLine, true>(v, a.r[b]);
        float* dst = a.vp + (size_t)ch * a.H * a.Wp + a.margin + x;
#pragma unroll
        for (int y0c = 0; y0c < kStOutV; y0c += kChunk) {
            if (y0c < a.nout_v) {   // uniform
#pragma unroll
                for (int yy = 0; yy < kChunk; ++yy) {
                    const int Y = y0 + y0c + yy;
                    if (y0c + yy < a.nout_v && Y < a.H) dst[(size_t)Y * a.Wp] = v[y0c + yy];
                }
            }
        }
    }
}

// Horizontal pass.  Workgroup: 64 rows x nout_h output columns; wave w
// filters channel w along its rows, demodulates with C or S at the outputs,
// and the four contributions are summed in a fixed order into den and num.
// ROUNDS: hand-over rounds of kStHalf outputs (1 when nout_h <= kStHalf).
template <int ROUNDS>
__global__ void __launch_bounds__(kStThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
bf_stage_h(const StageArgs a) {
    constexpr int kOut = ROUNDS * kStHalf;   // outputs per line at most
    __shared__ float gt[kStRows][kStOutH + 1];
    __shared__ float red[4][kStHalf][kStRows + 1];
    __shared__ float csm[2][kStHalf][kStRows + 1];   // C and S at a round's outputs
    const int t = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int lane = t & 63;
    const int yb = blockIdx.y * kStRows;
    const int y = yb + lane;
    const int x0 = blockIdx.x * a.nout_h;
    const int ex0 = x0 - a.R;   // margin + ex0 is a multiple of 4
    const int yc = min(y, a.H - 1);
    for (int p0 = t; p0 < kStRows * kOut; p0 += 8 * kStThreads) {
        float v8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int p = p0 + u * kStThreads;
            const int yy = p / kOut, k = p - yy * kOut;
            const int Y = min(yb + yy, a.H - 1), X = min(max(x0 + k, 0), a.W - 1);
            v8[u] = a.f[(size_t)Y * a.W + X];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int p = p0 + u * kStThreads;
            const int yy = p / kOut, k = p - yy * kOut;
            const int Y = yb + yy, X = x0 + k;
            if (p < kStRows * kOut)
                gt[yy][k] = (Y < a.H && X >= 0 && X < a.W && k < a.nout_h) ? v8[u] - a.center
                                                                            : 0.0f;
        }
    }
    __syncthreads();
    const int nch = a.centre ? 2 : 4;
    const int ch = wave;
    float v[kStLine];
    if (ch < nch) {
        // 16-byte buffer loads along the lane's row of V_ch: the row (from
        // the workgroup's first) is the vector offset, the wave-uniform
        // column the scalar offset; the resource spans the workgroup's rows.
        // The line starts on a 16-byte boundary and at column ex0 >= -R,
        // inside the left margin; samples past the row's end belong to
        // positions no kept output reads (or come back as zero past the
        // resource).  Rows past H read row H - 1 and are never stored.
        const int ms = __builtin_amdgcn_readfirstlane(a.margin);
        const int Hs = __builtin_amdgcn_readfirstlane(a.H);
        const int Wps = __builtin_amdgcn_readfirstlane(a.Wp);
        const int e0 = __builtin_amdgcn_readfirstlane(ex0);
        const int ybs = __builtin_amdgcn_readfirstlane(yb);
        const int nrows = min(Hs - ybs, kStRows);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            a.vp + (size_t)ch * Hs * Wps + (size_t)ybs * Wps, 0,
            nrows * Wps * (int)sizeof(float), kBufferWord3);
        const int voff = (yc - yb) * Wps * (int)sizeof(float);
#pragma unroll
        for (int k = 0; k < kStLine / 4; ++k) {
            const int soff = (ms + e0 + 4 * k) * (int)sizeof(float);   // uniform
            const auto q = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0);
            v[4 * k] = __uint_as_float(q[0]);
            v[4 * k + 1] = __uint_as_float(q[1]);
            v[4 * k + 2] = __uint_as_float(q[2]);
            v[4 * k + 3] = __uint_as_float(q[3]);
        }
        for (int b = 0; b < a.nb; ++b) box_dispatch<kStLine, true>(v, a.r[b]);
    }
    // The outputs are handed over in rounds of kStHalf columns (the LDS
    // arrays hold one round); every test below is uniform, so all four
    // waves pass the barriers.
#pragma unroll
    for (int h = 0; h < ROUNDS; ++h) {
        const int k0 = h * kStHalf;
        if (k0 >= a.nout_h) break;
        if (!a.centre) {
            // the phase at the round's outputs, once per pixel: wave w
            // evaluates columns k0 + 16 w .. k0 + 16 w + 15 of every row
#pragma unroll
            for (int u = 0; u < kStHalf / 4; ++u) {
                const int kk = wave * (kStHalf / 4) + u;
                float cc, ss;
                cis_direct(a.malpha, gt[lane][k0 + kk], cc, ss);
                csm[0][kk][lane] = cc;
                csm[1][kk][lane] = ss;
            }
            __syncthreads();
        }
        if (ch < nch) {
            if (a.centre) {
#pragma unroll
                for (int kk = 0; kk < kStHalf; ++kk) red[ch][kk][lane] = a.c * v[k0 + kk];
            } else {
                const int cs = ch >= 2 ? 1 : 0;
#pragma unroll
                for (int kk = 0; kk < kStHalf; ++kk)
                    red[ch][kk][lane] = a.c * v[k0 + kk] * csm[cs][kk][lane];
            }
        }
        __syncthreads();
        // fixed-order sums: den = (C F[C] + S F[S]), num = (C F[gC] + S F[gS]);
        // wave w updates the round's columns 16 w .. 16 w + 15 of its rows,
        // the loads of all 16 first (clamped, unconditional), then the stores
        if (y < a.H) {
            constexpr int kPer = kStHalf / 4;
            float d16[kPer], n16[kPer];
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int k = k0 + wave * kPer + u;
                const size_t idx = (size_t)min(max(x0 + k, 0), a.W - 1) * a.H + y;
                d16[u] = a.den_t[idx];
                n16[u] = a.num_t[idx];
            }
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int kk = wave * kPer + u, k = k0 + kk;
                const int X = x0 + k;
                if (k < a.nout_h && X >= 0 && X < a.W) {
                    const float d =
                        a.centre ? red[0][kk][lane] : red[0][kk][lane] + red[2][kk][lane];
                    const float n =
                        a.centre ? red[1][kk][lane] : red[1][kk][lane] + red[3][kk][lane];
                    a.den_t[(size_t)X * a.H + y] = d16[u] + d;
                    a.num_t[(size_t)X * a.H + y] = n16[u] + n;
                }
            }
        }
        __syncthreads();   // the next round rewrites csm and red
    }
}

__global__ void bf_stage_zero(float* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

// Zeroes the columns of the V planes that the vertical pass never writes:
// [0, margin) and [margin + W, Wp) of every row (Wp - W per row, 4 H rows).
__global__ void bf_stage_margins(float* vp, int H, int W, int Wp, int margin) {
    const size_t per_row = (size_t)(Wp - W);
    const size_t n = (size_t)4 * H * per_row;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t row = i / per_row;
        const int j = (int)(i - row * per_row);
        const int col = j < margin ? j : W + j;
        vp[row * Wp + col] = 0.0f;
    }
}

// out = T/2 + num/den (FP64), eta = den; column-major in, row-major out
// through a 32 x 32 LDS transpose.
__global__ void __launch_bounds__(256)
bf_stage_final(const StageArgs a) {
    __shared__ double tn[32][33];
    __shared__ float td[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    for (int j = ty; j < 32; j += 8) {
        const int X = bx + j, Y = by + tx;   // read column X, rows by..by+31
        if (X < a.W && Y < a.H) {
            const size_t k = (size_t)X * a.H + Y;
            const float d = a.den_t[k];
            td[j][tx] = d;
            tn[j][tx] = (double)a.num_t[k] / (double)d;
        }
    }
    __syncthreads();
    for (int i = ty; i < 32; i += 8) {
        const int Y = by + i, X = bx + tx;
        if (X < a.W && Y < a.H) {
            const size_t k = (size_t)Y * a.W + X;
            a.out[k] = (float)((double)a.center + tn[tx][i]);
            if (a.eta) a.eta[k] = td[tx][i];
        }
    }
}

// margin <= kStMargin + 3 columns on the left, at least kStMargin on the
// right, rows starting on 256-byte boundaries (a pitch off those boundaries
// measured 14 % slower on the 4096^2 workload)
static int staged_pitch(int64_t W) { return (int)((W + 2 * kStMargin + 4 + 63) / 64 * 64); }

// nout_h for the sum of radii R: at most 256 - 2R (every kept output sees its
// whole box in the line), a multiple of 4 (16-byte aligned lines), and one
// or two whole hand-over rounds where the line allows: a partial second
// round costs as much as a full one (sigma_s 30 at 2048^2: 80 outputs per
// line measured 7.8 ms, 64 outputs 7.2 ms).
static int staged_nout_h(int R) {
    const int room = kStLine - 2 * R;
    if (room >= kStOutH) return kStOutH;
    return std::min(room, kStHalf) / 4 * 4;
}

size_t staged_workspace_bytes(int64_t H, int64_t W) {
    return ((size_t)4 * (size_t)H * (size_t)staged_pitch(W) + (size_t)2 * H * W) * sizeof(float);
}

bool staged_supported(const SpatialParams& sp) {
    for (int k = 0; k < sp.nb; ++k)
        if (sp.r[k] > kBoxMaxRadius) return false;
    return sp.R <= kStMargin && staged_nout_h(sp.R) >= 4;
}

// Cost model, per cosine pair, calibrated on MI355X (2048^2, N = 66): a round
// of fused tiles (one workgroup per CU) takes about 16 us whatever the tile
// size, a round of staged workgroups about 33 us in either pass.  The fused
// tiles shrink as R grows (the extended line is at most 128 samples), so
// past R of about 42 (2048^2) the staged passes are faster.
bool prefer_staged(int64_t H, int64_t W, const SpatialParams& sp, bf_status fused_status,
                   const TileGeom& g) {
    if (!staged_supported(sp)) return false;
    if (fused_status != BF_OK) return true;
    // compute units of the current device (queried per call: no shared state
    // between threads or devices)
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        cus = 256;
    auto rounds = [&](double blocks) { return std::ceil(blocks / cus); };
    const int nout_v = std::min(kStLine - 2 * sp.R, kStOutV);
    const int nout_h = staged_nout_h(sp.R);
    const double bv = std::ceil((double)W / kStCols) * std::ceil((double)H / nout_v);
    const double bh = std::ceil((double)W / nout_h) * std::ceil((double)H / kStRows);
    const double fused_us = rounds((double)g.tiles_x * g.tiles_y) * 16.0;
    const double staged_us = (rounds(bv) + rounds(bh)) * 33.0;
    return staged_us < fused_us;
}

bf_status launch_staged(const float* f, float* out, float* eta, int64_t H, int64_t W,
                        const RangeParams& rp, const SpatialParams& sp, void* workspace,
                        hipStream_t stream) {
    StageArgs a = {};
    const size_t HW = (size_t)H * (size_t)W;
    float* ws = static_cast<float*>(workspace);
    a.Wp = staged_pitch(W);
    const size_t vplanes = (size_t)4 * (size_t)H * (size_t)a.Wp;
    a.f = f;
    a.vp = ws;
    a.den_t = ws + vplanes;
    a.num_t = ws + vplanes + HW;
    a.out = out;
    a.eta = eta;
    a.H = (int)H;
    a.W = (int)W;
    a.R = sp.R;
    a.nb = sp.nb;
    for (int k = 0; k < BF_MAX_BOXES; ++k) a.r[k] = sp.r[k];
    a.nout_v = std::min(kStLine - 2 * sp.R, kStOutV);
    a.nout_h = staged_nout_h(sp.R);
    a.margin = kStMargin + sp.R % 4;   // margin + x0 - R is a multiple of 4 for x0 = b nout_h
    a.center = rp.center;
    // g tile, then the phase hand-over
    const size_t lds_v = ((size_t)kStLine * kStCols + (size_t)4 * 64 * kStCols) * sizeof(float);
    (void)hipFuncSetAttribute((const void*)bf_stage_v, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_v);
    hipLaunchKernelGGL(bf_stage_zero, dim3(1024), dim3(256), 0, stream, a.den_t, 2 * HW);
    hipLaunchKernelGGL(bf_stage_margins, dim3(1024), dim3(256), 0, stream, a.vp, a.H, a.W, a.Wp,
                       a.margin);
    const dim3 gv((unsigned)((W + kStCols - 1) / kStCols),
                  (unsigned)((H + a.nout_v - 1) / a.nout_v));
    const dim3 gh((unsigned)((W + a.nout_h - 1) / a.nout_h),
                  (unsigned)((H + kStRows - 1) / kStRows));
    for (int q = 0; q < rp.npairs; ++q) {
        const int m = rp.odd + 2 * q;
        a.centre = (m == 0);
        a.c = rp.chat[q];
        a.malpha = (double)m * rp.alpha;
        hipLaunchKernelGGL(bf_stage_v, gv, dim3(kStThreads), lds_v, stream, a);
        if (a.nout_h > kStHalf)
            hipLaunchKernelGGL(bf_stage_h<2>, gh, dim3(kStThreads), 0, stream, a);
        else
            hipLaunchKernelGGL(bf_stage_h<1>, gh, dim3(kStThreads), 0, stream, a);
    }
    hipLaunchKernelGGL(bf_stage_final, dim3((unsigned)((W + 31) / 32), (unsigned)((H + 31) / 32)),
                       dim3(256), 0, stream, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("staged forward launch failed: %s", hipGetErrorString(e));
        return BF_EDEVICE;
    }
    return BF_OK;
}

}  // namespace bf
