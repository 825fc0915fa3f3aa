// Debug helper for the input precondition of Sec. 2.1: every intensity lies
// in [0, T], which keeps the raised-cosine kernel non-negative.  The filter
// itself does not test it on the hot path; this pass counts the pixels that
// break it (NaN included) into a caller-provided device counter.
#include <algorithm>

#include "bf_internal.h"

namespace bf {

__global__ void bf_check_clear(unsigned* count) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = 0u;
}

__global__ void __launch_bounds__(256) bf_check_kernel(const float* f, size_t n, float T,
                                                       unsigned* count) {
    unsigned bad = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const float x = f[i];
        bad += !(x >= 0.0f && x <= T);   // false for NaN too
    }
    if (bad) atomicAdd(count, bad);
}

bf_status launch_check_range(const float* f, int64_t H, int64_t W, float T, unsigned* count,
                             hipStream_t stream) {
    const size_t n = (size_t)H * (size_t)W;
    const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(bf_check_clear, dim3(1), dim3(64), 0, stream, count);
    hipLaunchKernelGGL(bf_check_kernel, dim3(blocks), dim3(256), 0, stream, f, n, T, count);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("range check launch failed: %s", hipGetErrorString(e));
        return BF_EDEVICE;
    }
    return BF_OK;
}

}  // namespace bf
