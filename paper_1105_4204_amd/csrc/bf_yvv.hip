// Forward filter with the recursive Gaussian spatial kernel of Young and van
// Vliet (the O(1) spatial filter the paper's experiments use, Sec. 3),
// evaluated through eq. (final-form) pair by pair.
//
// The recursive filter has infinite support, so it cannot be cut into tiles
// with a finite halo without changing the result; each pass instead runs
// along whole image lines.  With zero-extended data the causal pass starts
// from zero state at the first sample, and the anticausal pass starts, past
// the last sample, from the state the causal output's ringing leaves there
// (the matrix M of make_yvv), so every line is filtered exactly as on an
// infinite zero-padded line.
//
// Pairs go in groups of kYvPairs: a thread starts the phase of the group's
// first pair from the FP64-reduced angle (cis_direct) and reaches the others
// by the recurrence Z <- Z exp(j 2 a g).  Waves 0..3 of a workgroup take the
// channels C, gC, S, gS (g = f - T/2; C + j S = Z; for m = 0 the channels are
// 1 and g, and the S pair is zero).  A launch chunk covers up to
// kYvChunkGroups groups; its filtered channels live in the workspace:
//   vertical pass   (bf_yvv_v): lane = image column, walking down the rows:
//     builds the channel, runs the causal pass (results stored), then the
//     anticausal pass back up (in place);
//   horizontal pass (bf_yvv_h): lane = image row; 64 x 16 blocks go through
//     LDS so that global accesses stay coalesced; causal pass left to right
//     (in place), then the anticausal pass right to left, demodulated on the
//     fly: each thread sums c_m (C or S) F[channel] over its group's pairs,
//     and the C and S waves' sums (gC and gS for num) are added through LDS
//     into the group's den and num partial planes;
//   bf_yvv_reduce adds a chunk's partial planes into den and num in a fixed
//   order; bf_yvv_final divides in FP64 and writes out and eta.
// The pairs are split into launch chunks of equal size (at most 40 pairs, so
// the 66-degree workload runs as one chunk), so that no chunk is a small tail
// with few workgroups.
// Unlike the fused box kernel, the filtered channels of a chunk pass through
// device memory: this path is bound by HBM traffic, about 108 bytes per pixel
// and pair (24 bytes per pixel, channel and pair, plus the per-group and
// per-chunk terms).
#include <algorithm>

#include "bf_tile.h"

namespace bf {

constexpr int kYvThreads = 256;      // four waves, one per channel
constexpr int kYvPairs = 2;          // pairs per thread (one direct phase, one recurrence step)
constexpr int kYvChunkGroups = 20;   // groups per launch chunk, at most (40 pairs)
constexpr int kYvBlk = 16;           // horizontal pass: columns per LDS block
constexpr int kYvBlkP = kYvBlk + 1;
constexpr int kYvRowsPer = 64 / kYvBlk;   // rows one block transfer instruction covers
constexpr int kYvRows = 16;          // vertical pass: rows whose loads are issued together

struct YvArgs {
    const float* f;
    float* ws;           // channel planes: plane ((g * kYvPairs + p) * 4 + ch), H*W each
    float* part;         // partial planes: den and num of group g at (2 g) and (2 g + 1)
    float* den;
    float* num;
    float* out;
    float* eta;
    int H, W;
    int q0;              // first pair of the chunk
    int npairs, odd;
    double B, a1, a2, a3;   // recursion in FP64: its state amplifies rounding by ~1/B
    double M[9];
    float two_alpha, center;
    double alpha;
    float chat[kMaxPairs];
};

// Channel ch of phase (zr, zi) and g: C, gC, S, gS.
__device__ __forceinline__ float yv_channel(int ch, float zr, float zi, float g) {
    const float base = (ch < 2) ? zr : zi;
    return (ch & 1) ? g * base : base;
}

// Phases of the kYvPairs pairs q0 + p at intensity g.
__device__ __forceinline__ void yv_phases(const YvArgs& a, int qg, float g, float (&zr)[kYvPairs],
                                          float (&zi)[kYvPairs]) {
    const int m0 = a.odd + 2 * qg;
    cis_direct((double)m0 * a.alpha, g, zr[0], zi[0]);
    float cu, su;
    cis_small(a.two_alpha * g, cu, su);
#pragma unroll
    for (int p = 1; p < kYvPairs; ++p) {
        zr[p] = zr[p - 1] * cu - zi[p - 1] * su;
        zi[p] = zr[p - 1] * su + zi[p - 1] * cu;
    }
}

// Vertical pass: one wave per channel, one lane per image column.
__global__ void __launch_bounds__(kYvThreads) bf_yvv_v(const YvArgs a) {
    const int lane = threadIdx.x & 63;
    const int ch = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int grp = blockIdx.y;
    const int qg = a.q0 + grp * kYvPairs;                  // first pair of the group
    const int x = blockIdx.x * 64 + lane;
    const bool col = x < a.W;
    const size_t HW = (size_t)a.H * a.W;
    float* planes = a.ws + (size_t)grp * kYvPairs * 4 * HW + (size_t)ch * HW;
    const int np = min(kYvPairs, a.npairs - qg);           // valid pairs of the group (>= 1)
    double s1[kYvPairs], s2[kYvPairs], s3[kYvPairs];
#pragma unroll
    for (int p = 0; p < kYvPairs; ++p) s1[p] = s2[p] = s3[p] = 0.0;
    const int xc = col ? x : 0;
    // rows in blocks of kYvRows: the block's loads are all issued before its
    // dependent recursion steps
    for (int yb = 0; yb < a.H; yb += kYvRows) {
        // clamped, unconditional loads: all of a block's loads are in flight
        // before the first is used (a guarded load would wait on its own)
        float gb[kYvRows];
#pragma unroll
        for (int j = 0; j < kYvRows; ++j) {
            const int y = min(yb + j, a.H - 1);
            gb[j] = a.f[(size_t)y * a.W + xc];
        }
#pragma unroll
        for (int j = 0; j < kYvRows; ++j) gb[j] = (col && yb + j < a.H) ? gb[j] - a.center : 0.0f;
#pragma unroll
        for (int j = 0; j < kYvRows; ++j) {
            if (yb + j < a.H) {
                const size_t k = (size_t)(yb + j) * a.W + xc;
                float zr[kYvPairs], zi[kYvPairs];
                yv_phases(a, qg, gb[j], zr, zi);
#pragma unroll
                for (int p = 0; p < kYvPairs; ++p) {
                    const float u = col ? yv_channel(ch, zr[p], zi[p], gb[j]) : 0.0f;
                    const double w = a.B * (double)u + a.a1 * s1[p] + a.a2 * s2[p] + a.a3 * s3[p];
                    s3[p] = s2[p];
                    s2[p] = s1[p];
                    s1[p] = w;
                    if (col && p < np) planes[(size_t)p * 4 * HW + k] = (float)w;
                }
            }
        }
    }
    double v1[kYvPairs], v2[kYvPairs], v3[kYvPairs];
#pragma unroll
    for (int p = 0; p < kYvPairs; ++p) {
        v1[p] = a.M[0] * s1[p] + a.M[1] * s2[p] + a.M[2] * s3[p];
        v2[p] = a.M[3] * s1[p] + a.M[4] * s2[p] + a.M[5] * s3[p];
        v3[p] = a.M[6] * s1[p] + a.M[7] * s2[p] + a.M[8] * s3[p];
    }
    if (!col) return;
    for (int yt = a.H - 1; yt >= 0; yt -= kYvRows) {
        float wb[kYvRows][kYvPairs];
#pragma unroll
        for (int j = 0; j < kYvRows; ++j) {
            const int y = max(yt - j, 0);
#pragma unroll
            for (int p = 0; p < kYvPairs; ++p) {
                const int pc = min(p, np - 1);
                wb[j][p] = planes[(size_t)pc * 4 * HW + (size_t)y * a.W + x];
            }
        }
#pragma unroll
        for (int j = 0; j < kYvRows; ++j) {
            const int y = yt - j;
            if (y >= 0) {
#pragma unroll
                for (int p = 0; p < kYvPairs; ++p) {
                    if (p < np) {
                        const double v = a.B * (double)wb[j][p] + a.a1 * v1[p] + a.a2 * v2[p] +
                                         a.a3 * v3[p];
                        v3[p] = v2[p];
                        v2[p] = v1[p];
                        v1[p] = v;
                        planes[(size_t)p * 4 * HW + (size_t)y * a.W + x] = (float)v;
                    }
                }
            }
        }
    }
}

// Horizontal pass: one wave per channel, one lane per image row; 64 x 16
// blocks of each plane are moved through LDS with coalesced accesses.  Three
// workgroups share a CU (39 KB of LDS and at most 168 registers a lane each),
// which hides part of the FP64 recursion's latency and lets the 544
// workgroups of a 2048^2, N = 66 forward run in one round (two workgroups of
// 64 x 32 blocks per CU: 6.0 -> 5.1 ms per forward; three of 64 x 16: 4.9).
__global__ void __launch_bounds__(kYvThreads, 3) bf_yvv_h(const YvArgs a) {
    __shared__ float blk[4][kYvPairs][64][kYvBlkP];
    __shared__ float gblk[64][kYvBlkP];
    const int lane = threadIdx.x & 63;
    const int ch = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int grp = blockIdx.y;
    const int qg = a.q0 + grp * kYvPairs;
    const int y0 = blockIdx.x * 64;
    const size_t HW = (size_t)a.H * a.W;
    float* planes = a.ws + (size_t)grp * kYvPairs * 4 * HW + (size_t)ch * HW;
    float* part = a.part + (size_t)grp * 2 * HW;
    const int np = min(kYvPairs, a.npairs - qg);
    float cq[kYvPairs];
#pragma unroll
    for (int p = 0; p < kYvPairs; ++p) cq[p] = p < np ? a.chat[qg + p] : 0.0f;
    // block transfers: lane l moves column l % kYvBlk of rows
    // kYvRowsPer r + l / kYvBlk.  Double buffering: while a block is filtered
    // from LDS, the next block's values are already on their way into
    // registers (t, tg), from clamped positions without branches; they are
    // masked when written to LDS.  Blocks of 16 columns keep the workgroup's
    // LDS within a quarter of the CU's, so four workgroups fit on a CU.
    const int bc = lane % kYvBlk, br = lane / kYvBlk;
    float t[kYvPairs][kYvBlk];
    float tg[kYvBlk / 4];
    auto fetch_blk = [&](int x0) {
        const int x = min(x0 + bc, a.W - 1);
#pragma unroll
        for (int p = 0; p < kYvPairs; ++p) {
            const int pc = min(p, np - 1);
#pragma unroll
            for (int r = 0; r < kYvBlk; ++r) {
                const int y = min(y0 + kYvRowsPer * r + br, a.H - 1);
                t[p][r] = planes[(size_t)pc * 4 * HW + (size_t)y * a.W + x];
            }
        }
    };
    auto put_blk = [&](int x0) {
#pragma unroll
        for (int p = 0; p < kYvPairs; ++p) {
#pragma unroll
            for (int r = 0; r < kYvBlk; ++r) {
                const int row = kYvRowsPer * r + br;
                blk[ch][p][row][bc] = (y0 + row < a.H && x0 + bc < a.W) ? t[p][r] : 0.0f;
            }
        }
    };
    // g of a block: wave w moves the rows kYvRowsPer r + l / kYvBlk for r in
    // [w kYvBlk / 4, (w + 1) kYvBlk / 4)
    constexpr int NG = kYvBlk / 4;
    auto fetch_g = [&](int x0) {
        const int x = min(x0 + bc, a.W - 1);
#pragma unroll
        for (int r = 0; r < NG; ++r) {
            const int y = min(y0 + kYvRowsPer * (NG * ch + r) + br, a.H - 1);
            tg[r] = a.f[(size_t)y * a.W + x];
        }
    };
    auto put_g = [&](int x0) {
#pragma unroll
        for (int r = 0; r < NG; ++r) {
            const int row = kYvRowsPer * (NG * ch + r) + br;
            gblk[row][bc] = (y0 + row < a.H && x0 + bc < a.W) ? tg[r] - a.center : 0.0f;
        }
    };
    auto store_blk = [&](int x0) {
        for (int p = 0; p < np; ++p) {
#pragma unroll 8
            for (int r = 0; r < kYvBlk; ++r) {
                const int row = kYvRowsPer * r + br, y = y0 + row, x = x0 + bc;
                if (y < a.H && x < a.W)
                    planes[(size_t)p * 4 * HW + (size_t)y * a.W + x] = blk[ch][p][row][bc];
            }
        }
    };
    double s1[kYvPairs], s2[kYvPairs], s3[kYvPairs];
#pragma unroll
    for (int p = 0; p < kYvPairs; ++p) s1[p] = s2[p] = s3[p] = 0.0;
    const int nblk = (a.W + kYvBlk - 1) / kYvBlk;
    // causal, left to right
    fetch_blk(0);
    for (int b = 0; b < nblk; ++b) {
        const int x0 = b * kYvBlk;
        put_blk(x0);
        if (b + 1 < nblk) fetch_blk(x0 + kYvBlk);
        __syncthreads();
        const int ncol = min(kYvBlk, a.W - x0);
        for (int c = 0; c < ncol; ++c) {
#pragma unroll
            for (int p = 0; p < kYvPairs; ++p) {
                if (p < np) {
                    const double w = a.B * (double)blk[ch][p][lane][c] + a.a1 * s1[p] +
                                     a.a2 * s2[p] + a.a3 * s3[p];
                    s3[p] = s2[p];
                    s2[p] = s1[p];
                    s1[p] = w;
                    blk[ch][p][lane][c] = (float)w;
                }
            }
        }
        __syncthreads();
        store_blk(x0);
        __syncthreads();
    }
    double v1[kYvPairs], v2[kYvPairs], v3[kYvPairs];
#pragma unroll
    for (int p = 0; p < kYvPairs; ++p) {
        v1[p] = a.M[0] * s1[p] + a.M[1] * s2[p] + a.M[2] * s3[p];
        v2[p] = a.M[3] * s1[p] + a.M[4] * s2[p] + a.M[5] * s3[p];
        v3[p] = a.M[6] * s1[p] + a.M[7] * s2[p] + a.M[8] * s3[p];
    }
    // anticausal, right to left, demodulated into the partial plane (the
    // causal stores above are complete: the loads below are issued after the
    // last barrier, and each lane's loads follow its own stores)
    fetch_blk((nblk - 1) * kYvBlk);
    fetch_g((nblk - 1) * kYvBlk);
    for (int b = nblk - 1; b >= 0; --b) {
        const int x0 = b * kYvBlk;
        put_blk(x0);
        put_g(x0);
        if (b > 0) {
            fetch_blk(x0 - kYvBlk);
            fetch_g(x0 - kYvBlk);
        }
        __syncthreads();
        const int ncol = min(kYvBlk, a.W - x0);
        for (int c = ncol - 1; c >= 0; --c) {
            const float g = gblk[lane][c];
            float zr[kYvPairs], zi[kYvPairs];
            yv_phases(a, qg, g, zr, zi);
            float acc = 0.0f;
#pragma unroll
            for (int p = 0; p < kYvPairs; ++p) {
                if (p < np) {
                    const double v = a.B * (double)blk[ch][p][lane][c] + a.a1 * v1[p] +
                                     a.a2 * v2[p] + a.a3 * v3[p];
                    v3[p] = v2[p];
                    v2[p] = v1[p];
                    v1[p] = v;
                    acc = fmaf(cq[p] * ((ch < 2) ? zr[p] : zi[p]), (float)v, acc);
                }
            }
            blk[ch][0][lane][c] = acc;
        }
        __syncthreads();
        // den partial = C + S waves, num partial = gC + gS waves
        if (ch < 2) {
            for (int r = 0; r < kYvBlk; ++r) {
                const int row = kYvRowsPer * r + br, y = y0 + row, x = x0 + bc;
                if (y < a.H && x < a.W)
                    part[(size_t)ch * HW + (size_t)y * a.W + x] =
                        blk[ch][0][row][bc] + blk[ch + 2][0][row][bc];
            }
        }
        __syncthreads();
    }
}

// den (+)= sum over the chunk's groups of the C and S partials, num likewise,
// in a fixed order.
__global__ void bf_yvv_reduce(const YvArgs a, int ngroups, int first) {
    const size_t HW = (size_t)a.H * a.W;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < HW;
         i += (size_t)gridDim.x * blockDim.x) {
        float d = first ? 0.0f : a.den[i];
        float n = first ? 0.0f : a.num[i];
        for (int g = 0; g < ngroups; ++g) {
            const float* p = a.part + (size_t)g * 2 * HW + i;
            d += p[0];
            n += p[HW];
        }
        a.den[i] = d;
        a.num[i] = n;
    }
}

__global__ void bf_yvv_final(const YvArgs a) {
    const size_t HW = (size_t)a.H * a.W;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < HW;
         i += (size_t)gridDim.x * blockDim.x) {
        const float d = a.den[i];
        a.out[i] = (float)((double)a.center + (double)a.num[i] / (double)d);
        if (a.eta) a.eta[i] = d;
    }
}

// Groups per launch chunk: the pairs split into the fewest chunks of at most
// kYvChunkGroups groups, all of (nearly) the same size.
static int yvv_chunk_groups(int npairs) {
    const int groups = (npairs + kYvPairs - 1) / kYvPairs;
    const int chunks = (groups + kYvChunkGroups - 1) / kYvChunkGroups;
    return (groups + chunks - 1) / chunks;
}

// Sized for the largest chunk any pair count up to npairs can produce (term
// truncation may lower the count, and a balanced split of fewer groups can
// have larger chunks).
size_t yvv_workspace_bytes(int64_t H, int64_t W, int npairs) {
    const int G = std::min(kYvChunkGroups, (npairs + kYvPairs - 1) / kYvPairs);
    const size_t planes = (size_t)G * kYvPairs * 4 + (size_t)G * 2 + 2;
    return planes * (size_t)H * (size_t)W * sizeof(float);
}

bf_status launch_yvv(const float* f, float* out, float* eta, int64_t H, int64_t W,
                     const RangeParams& rp, const YvvParams& yp, void* workspace,
                     size_t workspace_bytes, hipStream_t stream) {
    if (workspace_bytes < yvv_workspace_bytes(H, W, rp.npairs)) {
        set_error("workspace of %zu bytes is smaller than the %zu bytes needed", workspace_bytes,
                  yvv_workspace_bytes(H, W, rp.npairs));
        return BF_EINVAL;
    }
    YvArgs a = {};
    const size_t HW = (size_t)H * (size_t)W;
    const int G = yvv_chunk_groups(rp.npairs);
    float* ws = static_cast<float*>(workspace);
    a.f = f;
    a.ws = ws;
    a.part = ws + (size_t)G * kYvPairs * 4 * HW;
    a.den = a.part + (size_t)G * 2 * HW;
    a.num = a.den + HW;
    a.out = out;
    a.eta = eta;
    a.H = (int)H;
    a.W = (int)W;
    a.npairs = rp.npairs;
    a.odd = rp.odd;
    a.B = yp.B;
    a.a1 = yp.a1;
    a.a2 = yp.a2;
    a.a3 = yp.a3;
    for (int k = 0; k < 9; ++k) a.M[k] = yp.M[k];
    a.two_alpha = (float)(2.0 * rp.alpha);
    a.alpha = rp.alpha;
    a.center = rp.center;
    for (int q = 0; q < rp.npairs; ++q) a.chat[q] = rp.chat[q];
    const unsigned cols = (unsigned)((W + 63) / 64), rows = (unsigned)((H + 63) / 64);
    const unsigned flat = (unsigned)std::min<size_t>((HW + 255) / 256, 4096);
    int first = 1;
    for (int q0 = 0; q0 < rp.npairs; q0 += G * kYvPairs) {
        a.q0 = q0;
        const int ng = std::min(G, (rp.npairs - q0 + kYvPairs - 1) / kYvPairs);
        hipLaunchKernelGGL(bf_yvv_v, dim3(cols, (unsigned)ng), dim3(kYvThreads), 0, stream, a);
        hipLaunchKernelGGL(bf_yvv_h, dim3(rows, (unsigned)ng), dim3(kYvThreads), 0, stream, a);
        hipLaunchKernelGGL(bf_yvv_reduce, dim3(flat), dim3(256), 0, stream, a, ng, first);
        first = 0;
    }
    hipLaunchKernelGGL(bf_yvv_final, dim3(flat), dim3(256), 0, stream, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("recursive-Gaussian forward launch failed: %s", hipGetErrorString(e));
        return BF_EDEVICE;
    }
    return BF_OK;
}

}  // namespace bf
