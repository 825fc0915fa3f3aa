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
//     on the extended rows, the box stages run along it, and the 256 - 2R
//     outputs are written, transposed, to a column-major plane V_ch;
//   horizontal pass (bf_stage_h): lane = image row; a 256-sample line along
//     the row is read from V_ch (coalesced thanks to the transposed layout),
//     the box stages run along it, and the 64 outputs are demodulated and
//     accumulated into den and num (column-major, read-modify-write).
// A final pass divides in FP64 and writes out (and eta) row-major.  The
// planes live in a caller-provided workspace of 24 bytes per pixel: unlike
// the fused kernel, this path keeps the filtered channels of one pair in
// device memory between its two passes.  Wide kernels have a large mass
// (the sum of w) against w(0), so where a pixel has few similar neighbours
// the pair terms cancel heavily; both passes use compensated running sums.
#include <algorithm>

#include "bf_tile.h"

namespace bf {

constexpr int kStLine = 256;      // register line of the staged passes
constexpr int kStOutH = 64;       // outputs per horizontal line
constexpr int kStVThreads = 256;  // columns per vertical workgroup
constexpr int kStHRows = 64;      // rows per horizontal workgroup (one wave)
constexpr int kStTrPitch = kStVThreads + 1;

struct StageArgs {
    const float* f;
    float* vt;          // 4 column-major H x W planes: V_ch[x * H + y]
    float* den_t;       // column-major accumulators
    float* num_t;
    float* out;
    float* eta;
    int H, W, R, nb;
    int r[BF_MAX_BOXES];
    int nout_v;         // outputs per vertical line: 256 - 2R, at most 128
    int nout_h;         // outputs per horizontal line: min(64, 256 - 2R)
    int centre;         // this pair is m = 0 (channels 1, g)
    float c;            // c_m
    double malpha;      // m a
    float center;       // T/2
};

// exp(j m a g) for any phase: quadrant from the FP64 phase, remainder
// |x| <= pi/4 through cis_small.
__device__ __forceinline__ void cis_direct(double malpha, float g, float& c, float& s) {
    const double th = malpha * (double)g;
    const double n = rint(th * 0.63661977236758134308);        // 2/pi
    const float x = (float)fma(-n, 1.57079632679489661923, th);  // pi/2
    float cx, sx;
    cis_small(x, cx, sx);
    const int q = ((int)(long long)n) & 3;
    c = q == 0 ? cx : q == 1 ? -sx : q == 2 ? -cx : sx;
    s = q == 0 ? sx : q == 1 ? cx : q == 2 ? -sx : -cx;
}

// One wave per SIMD: the 256-sample line needs the whole register file.
__global__ void __launch_bounds__(kStVThreads) __attribute__((amdgpu_waves_per_eu(1, 1)))
bf_stage_v(const StageArgs a) {
    extern __shared__ __align__(16) float tr[];   // nout_v x kStTrPitch
    const int t = threadIdx.x;
    const int x = blockIdx.x * kStVThreads + t;
    const int y0 = blockIdx.y * a.nout_v;
    const int ey0 = y0 - a.R;
    const int xc = min(x, a.W - 1);
    const size_t HW = (size_t)a.H * a.W;
    const int nch = a.centre ? 2 : 4;
    for (int ch = 0; ch < nch; ++ch) {
        // opaque per channel: keeps the 256 row masks and addresses from being
        // hoisted out of the channel loop (and spilled)
        int eyo = ey0;
        asm volatile("" : "+s"(eyo));
        float v[kStLine];
#pragma unroll
        for (int y0c = 0; y0c < kStLine; y0c += kChunk) {
            // a chunk of loads at a time: the barrier keeps the compiler from
            // issuing all 256 loads (and holding their addresses) up front
            asm volatile("" ::: "memory");
#pragma unroll
            for (int y = y0c; y < y0c + kChunk; ++y) {
                const int gy = eyo + y;
                const bool in = x < a.W && gy >= 0 && gy < a.H;
                const int gyc = min(max(gy, 0), a.H - 1);
                const float g = in ? a.f[(unsigned)(gyc * a.W + xc)] - a.center : 0.0f;
                float val;
                if (a.centre) {
                    val = (ch == 0) ? 1.0f : g;
                } else {
                    float cc, ss;
                    cis_direct(a.malpha, g, cc, ss);
                    const float base = (ch >= 2) ? ss : cc;
                    val = (ch & 1) ? g * base : base;
                }
                v[y] = in ? val : 0.0f;
            }
        }
        for (int b = 0; b < a.nb; ++b) box_dispatch<kStLine, false, true>(v, a.r[b]);
#pragma unroll
        for (int y0c = 0; y0c < 2 * kStOutH; y0c += kChunk) {
            if (y0c < a.nout_v) {
#pragma unroll
                for (int yy = 0; yy < kChunk; ++yy)
                    if (y0c + yy < a.nout_v) tr[(y0c + yy) * kStTrPitch + t] = v[y0c + yy];
            }
        }
        __syncthreads();
        // transposed, coalesced write: consecutive threads, consecutive rows of one column
        float* dst = a.vt + (size_t)ch * HW;
        for (int p = t; p < kStVThreads * a.nout_v; p += kStVThreads) {
            const int xl = p / a.nout_v, yl = p - xl * a.nout_v;
            const int X = blockIdx.x * kStVThreads + xl, Y = y0 + yl;
            if (X < a.W && Y < a.H) dst[(size_t)X * a.H + Y] = tr[yl * kStTrPitch + xl];
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kStHRows) __attribute__((amdgpu_waves_per_eu(1, 1)))
bf_stage_h(const StageArgs a) {
    __shared__ float gt[kStHRows][kStOutH + 1];
    const int t = threadIdx.x;
    const int y = blockIdx.y * kStHRows + t;
    const int x0 = blockIdx.x * a.nout_h;
    const int ex0 = x0 - a.R;
    const int yc = min(y, a.H - 1);
    const size_t HW = (size_t)a.H * a.W;
    for (int p = t; p < kStHRows * kStOutH; p += kStHRows) {
        const int yy = p / kStOutH, k = p - yy * kStOutH;
        const int Y = blockIdx.y * kStHRows + yy, X = x0 + k;
        gt[yy][k] = (Y < a.H && X < a.W && k < a.nout_h) ? a.f[(size_t)Y * a.W + X] - a.center
                                                         : 0.0f;
    }
    __syncthreads();
    float den[kStOutH], num[kStOutH], trig[kStOutH];
#pragma unroll
    for (int k = 0; k < kStOutH; ++k) {
        den[k] = 0.0f;
        num[k] = 0.0f;
    }
    const int nch = a.centre ? 2 : 4;
    for (int ch = 0; ch < nch; ++ch) {
        if (!a.centre && (ch == 0 || ch == 2)) {   // C for channels 0, 1; S for 2, 3
#pragma unroll
            for (int k = 0; k < kStOutH; ++k) {
                float cc, ss;
                cis_direct(a.malpha, gt[t][k], cc, ss);
                trig[k] = (ch == 0) ? cc : ss;
            }
        }
        float v[kStLine];
        const float* src = a.vt + (size_t)ch * HW;
        int exo = ex0;
        asm volatile("" : "+s"(exo));
#pragma unroll
        for (int x0c = 0; x0c < kStLine; x0c += 4 * kChunk) {
            asm volatile("" ::: "memory");
#pragma unroll
            for (int x = x0c; x < x0c + 4 * kChunk; ++x) {
                const int gx = exo + x;
                const bool in = y < a.H && gx >= 0 && gx < a.W;
                const int gxc = min(max(gx, 0), a.W - 1);
                const float val = src[(unsigned)(gxc * a.H + yc)];
                v[x] = in ? val : 0.0f;
            }
        }
        for (int b = 0; b < a.nb; ++b) box_dispatch<kStLine, false, true>(v, a.r[b]);
        const bool to_num = ch & 1;   // gC, gS (g for the centre pair)
#pragma unroll
        for (int k = 0; k < kStOutH; ++k) {
            const float w = a.c * (a.centre ? 1.0f : trig[k]) * v[k];
            if (to_num)
                num[k] += w;
            else
                den[k] += w;
        }
    }
    if (y < a.H) {
#pragma unroll
        for (int k = 0; k < kStOutH; ++k) {
            const int X = x0 + k;
            if (k < a.nout_h && X < a.W) {
                a.den_t[(size_t)X * a.H + y] += den[k];
                a.num_t[(size_t)X * a.H + y] += num[k];
            }
        }
    }
}

__global__ void bf_stage_zero(float* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
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

size_t staged_workspace_bytes(int64_t H, int64_t W) {
    return (size_t)6 * (size_t)H * (size_t)W * sizeof(float);
}

bool staged_supported(const SpatialParams& sp) {
    for (int k = 0; k < sp.nb; ++k)
        if (sp.r[k] > kBoxMaxRadius) return false;
    return 2 * sp.R < kStLine;
}

bf_status launch_staged(const float* f, float* out, float* eta, int64_t H, int64_t W,
                        const RangeParams& rp, const SpatialParams& sp, void* workspace,
                        hipStream_t stream) {
    StageArgs a = {};
    const size_t HW = (size_t)H * (size_t)W;
    float* ws = static_cast<float*>(workspace);
    a.f = f;
    a.vt = ws;
    a.den_t = ws + 4 * HW;
    a.num_t = ws + 5 * HW;
    a.out = out;
    a.eta = eta;
    a.H = (int)H;
    a.W = (int)W;
    a.R = sp.R;
    a.nb = sp.nb;
    for (int k = 0; k < BF_MAX_BOXES; ++k) a.r[k] = sp.r[k];
    a.nout_v = std::min(kStLine - 2 * sp.R, 2 * kStOutH);
    a.nout_h = std::min(kStLine - 2 * sp.R, kStOutH);
    a.center = rp.center;
    const size_t lds_v = (size_t)a.nout_v * kStTrPitch * sizeof(float);
    (void)hipFuncSetAttribute((const void*)bf_stage_v, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_v);
    hipLaunchKernelGGL(bf_stage_zero, dim3(1024), dim3(256), 0, stream, a.den_t, 2 * HW);
    const dim3 gv((unsigned)((W + kStVThreads - 1) / kStVThreads),
                  (unsigned)((H + a.nout_v - 1) / a.nout_v));
    const dim3 gh((unsigned)((W + a.nout_h - 1) / a.nout_h),
                  (unsigned)((H + kStHRows - 1) / kStHRows));
    for (int q = 0; q < rp.npairs; ++q) {
        const int m = rp.odd + 2 * q;
        a.centre = (m == 0);
        a.c = rp.chat[q];
        a.malpha = (double)m * rp.alpha;
        hipLaunchKernelGGL(bf_stage_v, gv, dim3(kStVThreads), lds_v, stream, a);
        hipLaunchKernelGGL(bf_stage_h, gh, dim3(kStHRows), 0, stream, a);
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
