// Register-resident running box sums over a line held in a static array.
//
// A lane keeps one line (a row or a column of a tile) in registers and
// applies the box stages of the separable spatial kernel in place.  The box
// radius is a template parameter, so every index is a compile-time constant
// and the line stays in VGPRs; box_dispatch() selects the instantiation for a
// run-time radius with a chain of wave-uniform tests.
#pragma once

#include <hip/hip_runtime.h>

namespace bf {

constexpr int kBoxMaxRadius = 31;   // radii handled by the register-line kernels

// v[i] <- sum_{d=0}^{2R} v[i+d] for i in [0, L-2R): the box of width 2R+1
// whose output at i is centred at i + R.  Running sum s += (enter - leave);
// the difference for the next output is taken before the current output
// overwrites its slot, so each new sum lands in place without register moves.
// COMP adds Kahan compensation to the running sum (four adds per output
// instead of one), which keeps its rounding from drifting along long lines of
// large values; the fused kernel does not need it, the wide-kernel passes do.
template <int L, int R, bool COMP = false>
__device__ __forceinline__ void box_stage(float (&v)[L]) {
    static_assert(2 * R < L, "line shorter than the box");
    constexpr int W = 2 * R + 1;
    float s = 0.0f, comp = 0.0f;
#pragma unroll
    for (int d = 0; d < W; ++d) {
        if (COMP) {
            const float y = v[d] - comp;
            const float u = s + y;
            comp = (u - s) - y;
            s = u;
        } else {
            s += v[d];
        }
    }
    float t = (W < L) ? v[W] - v[0] : 0.0f;
    v[0] = s;
#pragma unroll
    for (int i = 1; i < L - 2 * R; ++i) {
        const float tn = (i + W < L) ? v[i + W] - v[i] : 0.0f;
        if (COMP) {
            const float y = t - comp;
            const float u = s + y;
            comp = (u - s) - y;
            s = u;
        } else {
            s += t;
        }
        v[i] = s;
        t = tn;
    }
}

// Applies box_stage<L, r> for a wave-uniform run-time r (held in an SGPR):
// uniform tests one after another, each guarding its stage in its own block.
// The empty asm makes r opaque between blocks, so the compiler cannot fold
// the tests into one multi-way branch (whose join would merge the line from
// many paths, with register copies and spills where the caller keeps much
// other state live), and every join is two-way with the line in place.  Each
// stage body is marked unlikely, so it is laid out away from the tests: a
// candidate that does not match costs a test and a branch not taken, not a
// jump over a whole stage.  The radii are split first into four buckets of
// eight by tests of the same kind, so a dispatch runs 4 + 8 tests.
//
// Measured in the tile kernels (2048^2, boxes 9, 9, 10, N = 66): stage bodies
// in line with 32 tests, adjoint 3.95 ms; bodies out of line, 3.22 ms; with
// the buckets, 3.10 ms (forward 3.60, 3.18, 2.98 ms).  A binary search and an
// early exit after the matching stage add joins: the former spilled heavily,
// the latter slowed the forward.
template <int L, int R, int RE, bool COMP>
__device__ __forceinline__ void box_chain(float (&v)[L], int r) {
    if constexpr (R <= RE && 2 * R < L) {
        if (__builtin_expect(r == R, 0)) box_stage<L, R, COMP>(v);
        asm volatile("" : "+s"(r));
        box_chain<L, R + 1, RE, COMP>(v, r);
    }
}

template <int L, bool COMP = false>
__device__ __forceinline__ void box_dispatch(float (&v)[L], int r) {
    r = __builtin_amdgcn_readfirstlane(r);
    const int q = r >> 3;
    if (q == 0) box_chain<L, 0, 7, COMP>(v, r);
    asm volatile("" : "+s"(r));
    if (q == 1) box_chain<L, 8, 15, COMP>(v, r);
    asm volatile("" : "+s"(r));
    if (q == 2) box_chain<L, 16, 23, COMP>(v, r);
    asm volatile("" : "+s"(r));
    if (q == 3) box_chain<L, 24, kBoxMaxRadius, COMP>(v, r);
}

}  // namespace bf
