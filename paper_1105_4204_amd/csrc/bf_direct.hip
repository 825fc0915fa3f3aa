// Direct-window bilateral filter (gfx950): eq. (BF)/(normalization) summed
// pixel by pixel over the (2R+1)^2 window with the exact raised cosine
// cos(a (f_y - f_x))^N and the iterated-box weights.  O((2R+1)^2) per pixel:
// the reference cost the paper's O(1) method removes, used as the speed
// baseline and as an independent GPU cross-check of the fused kernel.
#include "bf_internal.h"

namespace bf {

constexpr int kDirTile = 16;            // 16 x 16 output pixels per workgroup
constexpr int kDirKMax = 2 * BF_MAX_BOXES * BF_MAX_RADIUS + 1;
constexpr int kDirLdsTileMax = 32 * 1024;   // floats of f staged in LDS when it fits

struct DirArgs {
    const float* f;
    float* out;
    float* eta;
    int H, W, R, nb, N;
    int r[BF_MAX_BOXES];
    float alpha;
    int tiles_x;
    int staged;        // 1: the (16+2R)^2 input window is staged in LDS
};

// x^N by binary powering (N uniform across the wave).
__device__ __forceinline__ float pow_n(float x, int N) {
    float r = 1.0f, b = x;
    while (N) {
        if (N & 1) r *= b;
        b *= b;
        N >>= 1;
    }
    return r;
}

__global__ void __launch_bounds__(kDirTile * kDirTile)
bf_direct_kernel(const DirArgs a) {
    __shared__ double kd[kDirKMax];
    __shared__ double kt[kDirKMax];
    __shared__ float kf[kDirKMax];
    extern __shared__ float tile[];
    const int t = threadIdx.x;
    const int nt = kDirTile * kDirTile;
    const int L = 2 * a.R + 1;
    // ---- composite 1-D kernel: unit impulse convolved with each box, exact
    // integers in double, then scaled by its peak into float ------------------
    for (int i = t; i < L; i += nt) kd[i] = (i == a.R) ? 1.0 : 0.0;
    __syncthreads();
    for (int b = 0; b < a.nb; ++b) {
        const int r = a.r[b];
        for (int i = t; i < L; i += nt) {
            double s = 0.0;
            for (int d = -r; d <= r; ++d) {
                const int u = i - d;
                if (u >= 0 && u < L) s += kd[u];
            }
            kt[i] = s;
        }
        __syncthreads();
        for (int i = t; i < L; i += nt) kd[i] = kt[i];
        __syncthreads();
    }
    const double kmax = kd[a.R];
    for (int i = t; i < L; i += nt) kf[i] = (float)(kd[i] / kmax);

    const int by = blockIdx.x / a.tiles_x, bx = blockIdx.x - by * a.tiles_x;
    const int i0 = by * kDirTile, j0 = bx * kDirTile;
    const int S = kDirTile + 2 * a.R;
    if (a.staged) {
        // clamped, unconditional loads in batches of 8, then the selection
        for (int p0 = t; p0 < S * S; p0 += 8 * nt) {
            float v8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int p = p0 + u * nt;
                const int si = p / S, sj = p - si * S;
                const int gi = min(max(i0 - a.R + si, 0), a.H - 1);
                const int gj = min(max(j0 - a.R + sj, 0), a.W - 1);
                v8[u] = a.f[(size_t)gi * a.W + gj];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int p = p0 + u * nt;
                const int si = p / S, sj = p - si * S;
                const int gi = i0 - a.R + si, gj = j0 - a.R + sj;
                if (p < S * S)
                    tile[p] = (gi >= 0 && gi < a.H && gj >= 0 && gj < a.W) ? v8[u] : 0.0f;
            }
        }
    }
    __syncthreads();
    const int li = t / kDirTile, lj = t - li * kDirTile;
    const int gi = i0 + li, gj = j0 + lj;
    if (gi >= a.H || gj >= a.W) return;
    const float fx = a.f[(size_t)gi * a.W + gj];
    const int y0 = max(gi - a.R, 0), y1 = min(gi + a.R, a.H - 1);
    const int x0 = max(gj - a.R, 0), x1 = min(gj + a.R, a.W - 1);
    float num = 0.0f, den = 0.0f;
    for (int y = y0; y <= y1; ++y) {
        const float ky = kf[y - gi + a.R];
        for (int x = x0; x <= x1; ++x) {
            const float fy = a.staged ? tile[(y - i0 + a.R) * S + (x - j0 + a.R)]
                                      : a.f[(size_t)y * a.W + x];
            const float w = ky * kf[x - gj + a.R];
            const float ph = w * pow_n(cosf(a.alpha * (fy - fx)), a.N);
            num += ph * fy;
            den += ph;
        }
    }
    a.out[(size_t)gi * a.W + gj] = num / den;
    if (a.eta) a.eta[(size_t)gi * a.W + gj] = (float)((double)den * kmax * kmax);
}

bf_status launch_direct(const float* f, float* out, float* eta, int64_t H, int64_t W,
                        const RangeParams& rp, const SpatialParams& sp, hipStream_t stream) {
    DirArgs a;
    a.f = f;
    a.out = out;
    a.eta = eta;
    a.H = (int)H;
    a.W = (int)W;
    a.R = sp.R;
    a.nb = sp.nb;
    a.N = rp.N;
    for (int k = 0; k < BF_MAX_BOXES; ++k) a.r[k] = sp.r[k];
    a.alpha = (float)rp.alpha;
    a.tiles_x = (int)((W + kDirTile - 1) / kDirTile);
    const int tiles_y = (int)((H + kDirTile - 1) / kDirTile);
    const int S = kDirTile + 2 * sp.R;
    a.staged = (S * S <= kDirLdsTileMax) ? 1 : 0;
    const size_t lds = a.staged ? (size_t)S * S * sizeof(float) : 0;
    (void)hipFuncSetAttribute((const void*)bf_direct_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(bf_direct_kernel, dim3((unsigned)(a.tiles_x * tiles_y)),
                       dim3(kDirTile * kDirTile), lds, stream, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("direct launch failed: %s", hipGetErrorString(e));
        return BF_EDEVICE;
    }
    return BF_OK;
}

}  // namespace bf
