// Space-variant spatial kernel (Sec. 4, space-variant extension): the unit
// box around pixel x has its own half-width r(x) <= Rm, the range kernel is
// the fixed raised cosine, and eq. (final-form) still holds pixel by pixel
// because each auxiliary image is averaged with the kernel of the pixel
// being filtered:
//     den(x) = sum_m c_m (C F_x[C] + S F_x[S]),
//     num(x) = sum_m c_m (C F_x[gC] + S F_x[gS]),   out = T/2 + num/den,
// with F_x[u] the sum of u over the box of half-width r(x), zero outside the
// image.  A box sum of any size costs four reads of a summed-area table, so
// the work per pixel and term does not depend on the radii.
//
// One workgroup of 256 threads owns a 32 x 32 output tile and the extended
// tile of side E = 32 + 2 Rh around it (Rh = Rm rounded up to a multiple of
// 4, so rows are 16-byte aligned and E is a multiple of 8).  Thread t keeps,
// in registers, g = f - T/2 and the phase Z = exp(j m a g) of the extended
// pixels t, t + 256, ... (zero outside the image), plus the phase, radius and
// FP64 accumulators of the output pixels t, t + 256, t + 512, t + 768.  Per
// channel of a pair:
//   1. every thread writes the channel (C, gC, S, gS; 1, g for m = 0) of its
//      extended pixels to an FP32 staging plane in LDS;
//   2. one thread per extended row forms the running row sums in FP64 into
//      the summed-area table (row 0 and column 0 stay zero);
//   3. one thread per extended column accumulates the table down the column;
//   4. each output pixel reads the four corners of its box and accumulates
//      c_m times its own C or S times the box sum into den or num.
// The table is kept in FP64: its entries grow with the tile area (up to
// about 1e6 for the g-weighted channels), and FP32 corners would lose about
// 1e-4 of a small box's sum.  The phase advances by the recurrence
// Z <- Z exp(j 2 a g) once per pair; nothing per term reaches HBM.
#include <algorithm>

#include "bf_tile.h"

namespace bf {

constexpr int kSvThreads = 256;
constexpr int kSvTile = 32;                    // output tile side
constexpr int kSvMaxR = 31;                    // largest half-width
constexpr int kSvMaxE = kSvTile + 2 * 32;      // extended side with Rm rounded up to 32
constexpr int kSvOwn = (kSvMaxE * kSvMaxE + kSvThreads - 1) / kSvThreads;   // 36
constexpr int kSvOut = kSvTile * kSvTile / kSvThreads;                      // 4
constexpr size_t kSvLdsPerCu = 160 * 1024;   // LDS of one CU

struct SvArgs {
    const float* f;
    const int32_t* rmap;
    float* out;
    float* eta;
    int H, W;
    int Rm;          // largest radius accepted (radii are clamped to it)
    int Rh;          // halo: Rm rounded up to a multiple of 4
    int E;           // extended side: kSvTile + 2 Rh
    int tiles_x;
    int npairs, odd;
    float alpha_f, two_alpha, center;
    float chat[kMaxPairs];
};

__host__ __device__ inline size_t sv_lds_bytes(int E) {
    return (size_t)E * E * sizeof(float) + (size_t)(E + 1) * (E + 1) * sizeof(double);
}

// MINW waves per SIMD: 2 when two workgroups' tables fit the CU's LDS
// (at most 256 registers a lane, a few spilled), else 1.
template <int MINW>
__global__ void __launch_bounds__(kSvThreads, MINW) bf_sv_kernel(const SvArgs a) {
    extern __shared__ __align__(16) float smem[];
    const int E = a.E, Sp = a.E + 1, EE = a.E * a.E;
    float* stg = smem;                                          // E x E, pitch E
    double* sat = reinterpret_cast<double*>(smem + EE);         // (E+1) x (E+1)
    const int t = threadIdx.x;
    const int ty = blockIdx.x / a.tiles_x, tx = blockIdx.x - ty * a.tiles_x;
    const int i0 = ty * kSvTile, j0 = tx * kSvTile;
    const int ei0 = i0 - a.Rh, ej0 = j0 - a.Rh;

    // extended pixels owned by this thread: g and Z (zero outside the image)
    float g[kSvOwn], zr[kSvOwn], zi[kSvOwn];
#pragma unroll
    for (int k = 0; k < kSvOwn; ++k) {
        const int p = t + kSvThreads * k;
        const int ei = p / E, ej = p - ei * E;
        const int gi = ei0 + ei, gj = ej0 + ej;
        const bool in = p < EE && gi >= 0 && gi < a.H && gj >= 0 && gj < a.W;
        // clamped, unconditional load: the loads of all k are in flight together
        const int ci = min(max(gi, 0), a.H - 1), cj = min(max(gj, 0), a.W - 1);
        const float fv = a.f[(size_t)ci * a.W + cj];
        const float gv = in ? fv - a.center : 0.0f;
        g[k] = gv;
        float c = 1.0f, s = 0.0f;
        if (a.odd) cis_small(a.alpha_f * gv, c, s);
        zr[k] = in ? c : 0.0f;
        zi[k] = in ? s : 0.0f;
    }
    // output pixels owned by this thread
    float go[kSvOut], zor[kSvOut], zoi[kSvOut];
    int ro[kSvOut];
    double den[kSvOut], num[kSvOut];
#pragma unroll
    for (int k = 0; k < kSvOut; ++k) {
        const int p = t + kSvThreads * k;
        const int oi = p / kSvTile, oj = p - oi * kSvTile;
        const int gi = min(i0 + oi, a.H - 1), gj = min(j0 + oj, a.W - 1);
        const size_t gidx = (size_t)gi * a.W + gj;
        go[k] = a.f[gidx] - a.center;
        ro[k] = min(max(a.rmap[gidx], 0), a.Rm);
        float c = 1.0f, s = 0.0f;
        if (a.odd) cis_small(a.alpha_f * go[k], c, s);
        zor[k] = c;
        zoi[k] = s;
        den[k] = 0.0;
        num[k] = 0.0;
    }
    // row 0 and column 0 of the table are zero for the whole tile
    for (int p = t; p < Sp; p += kSvThreads) {
        sat[p] = 0.0;
        sat[(size_t)p * Sp] = 0.0;
    }

    for (int q = 0; q < a.npairs; ++q) {
        if (q > 0) {
#pragma unroll
            for (int k = 0; k < kSvOwn; ++k) {
                float cu, su;
                cis_small(a.two_alpha * g[k], cu, su);
                const float nr = zr[k] * cu - zi[k] * su;
                const float ni = zr[k] * su + zi[k] * cu;
                zr[k] = nr;
                zi[k] = ni;
            }
#pragma unroll
            for (int k = 0; k < kSvOut; ++k) {
                float cu, su;
                cis_small(a.two_alpha * go[k], cu, su);
                const float nr = zor[k] * cu - zoi[k] * su;
                const float ni = zor[k] * su + zoi[k] * cu;
                zor[k] = nr;
                zoi[k] = ni;
            }
        }
        const int nch = (q == 0 && !a.odd) ? 2 : 4;
        const double cq = (double)a.chat[q];
        for (int ch = 0; ch < nch; ++ch) {
            // 1. channel of the extended pixels into the staging plane
#pragma unroll
            for (int k = 0; k < kSvOwn; ++k) {
                const int p = t + kSvThreads * k;
                if (p < EE) {
                    const float base = (ch < 2) ? zr[k] : zi[k];
                    stg[p] = (ch & 1) ? g[k] * base : base;
                }
            }
            __syncthreads();
            // 2. running row sums (FP64) into rows 1..E of the table; E is a
            // multiple of 8 and every block of 8 samples is loaded before it
            // is summed, so LDS latency is paid once per block
            if (t < E) {
                const float4* row = reinterpret_cast<const float4*>(stg + t * E);
                double* dst = sat + (size_t)(t + 1) * Sp + 1;
                double s = 0.0;
                for (int x8 = 0; x8 < E / 8; ++x8) {
                    const float4 u0 = row[2 * x8], u1 = row[2 * x8 + 1];
                    const float u[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        s += (double)u[k];
                        dst[8 * x8 + k] = s;
                    }
                }
            }
            __syncthreads();
            // 3. running column sums, in place, 8 rows loaded at a time
            if (t < E) {
                double* col = sat + Sp + 1 + t;
                double s = 0.0;
                for (int y8 = 0; y8 < E; y8 += 8) {
                    double c8[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) c8[k] = col[(size_t)(y8 + k) * Sp];
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        s += c8[k];
                        col[(size_t)(y8 + k) * Sp] = s;
                    }
                }
            }
            __syncthreads();
            // 4. box sums at the output pixels; demodulate and accumulate
#pragma unroll
            for (int k = 0; k < kSvOut; ++k) {
                const int p = t + kSvThreads * k;
                const int oi = p / kSvTile, oj = p - oi * kSvTile;
                const int r = ro[k];
                const int a0 = a.Rh + oi - r, a1 = a.Rh + oi + r + 1;
                const int b0 = a.Rh + oj - r, b1 = a.Rh + oj + r + 1;
                const double box = sat[(size_t)a1 * Sp + b1] - sat[(size_t)a0 * Sp + b1] -
                                   sat[(size_t)a1 * Sp + b0] + sat[(size_t)a0 * Sp + b0];
                const double w = cq * (double)((ch < 2) ? zor[k] : zoi[k]) * box;
                if (ch & 1)
                    num[k] += w;
                else
                    den[k] += w;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kSvOut; ++k) {
        const int p = t + kSvThreads * k;
        const int oi = p / kSvTile, oj = p - oi * kSvTile;
        const int gi = i0 + oi, gj = j0 + oj;
        if (gi < a.H && gj < a.W) {
            const size_t gidx = (size_t)gi * a.W + gj;
            a.out[gidx] = (float)((double)a.center + num[k] / den[k]);
            if (a.eta) a.eta[gidx] = (float)den[k];
        }
    }
}

bf_status launch_sv(const float* f, const int32_t* rmap, float* out, float* eta, int64_t H,
                    int64_t W, int32_t rmax, const RangeParams& rp, hipStream_t stream) {
    if (rmax < 0 || rmax > kSvMaxR) {
        set_error("space-variant radius bound %d outside [0, %d]", rmax, kSvMaxR);
        return rmax < 0 ? BF_EINVAL : BF_EUNSUPPORTED;
    }
    if (H > (int64_t)1 << 30 || W > (int64_t)1 << 30) {
        set_error("image too large");
        return BF_ERANGE;
    }
    SvArgs a = {};
    a.f = f;
    a.rmap = rmap;
    a.out = out;
    a.eta = eta;
    a.H = (int)H;
    a.W = (int)W;
    a.Rm = rmax;
    a.Rh = (rmax + 3) / 4 * 4;   // E = 32 + 2 Rh is then a multiple of 8
    a.E = kSvTile + 2 * a.Rh;
    a.tiles_x = (int)((W + kSvTile - 1) / kSvTile);
    const int64_t tiles_y = (H + kSvTile - 1) / kSvTile;
    if ((int64_t)a.tiles_x * tiles_y > INT32_MAX) {
        set_error("too many tiles");
        return BF_ERANGE;
    }
    a.npairs = rp.npairs;
    a.odd = rp.odd;
    a.alpha_f = (float)rp.alpha;
    a.two_alpha = (float)(2.0 * rp.alpha);
    a.center = rp.center;
    for (int q = 0; q < rp.npairs; ++q) a.chat[q] = rp.chat[q];
    const size_t lds = sv_lds_bytes(a.E);
    const dim3 grid((unsigned)(a.tiles_x * tiles_y));
    if (2 * lds <= kSvLdsPerCu) {   // two workgroups per CU (rmax up to 24)
        (void)hipFuncSetAttribute((const void*)bf_sv_kernel<2>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(bf_sv_kernel<2>, grid, dim3(kSvThreads), lds, stream, a);
    } else {
        (void)hipFuncSetAttribute((const void*)bf_sv_kernel<1>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(bf_sv_kernel<1>, grid, dim3(kSvThreads), lds, stream, a);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("space-variant forward launch failed: %s", hipGetErrorString(e));
        return BF_EDEVICE;
    }
    return BF_OK;
}

}  // namespace bf
