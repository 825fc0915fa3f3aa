// Streamed forward and adjoint: eq. (final-form) with the separable
// iterated-box averaging of Sec. 2.1 split into a column pass and a row pass
// over whole image lines, so that the work per pixel and cosine pair does
// not depend on the box radii.
//
// Column pass (bf_strm_v).  A box of width L is (1 - z^-L) / (1 - z^-1), so
// the causal composite of nb boxes is
//     b * x = S^nb d,   d[t] = sum_{A subset of boxes} (-1)^|A| x[t - sum_{k in A} L_k],
// with S the running sum (integrator).  A lane owns one image column and G
// consecutive cosine pairs and walks down the column: at each row it
// recomputes the channels at the 2^nb tap rows from f (the first pair's phase
// directly, the others by an FP64 rotation), forms d with FP64 fused
// multiply-adds (tap coefficient times g, A or B exact) and runs the nb
// integrators in FP64.  No
// history of the filtered signal is kept, and nothing depends on the radii
// but the tap offsets.  Integrators never damp their rounding errors; in FP64
// the drift stays far below the float32 resolution of the outputs over
// segments of at most 2048 rows (a fixed-point grid instead would be
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
// are quantised on a grid scaled to the row's largest magnitude (so a window
// sum of the first stage stays below 2^30), and each box stage is a wave
// prefix scan written to LDS and differenced at +-(r+1) (the prefix wraps
// modulo 2^32; the window sums do not).  Between stages the sums are shifted
// right so that the next window sum fits again.  The four filtered channels
// then meet in LDS and every thread demodulates its pixels with C and S
// (evaluated directly every kSmPhaseSync pairs and rotated in between where
// the line is short enough to keep the phases in registers, else directly for
// each pair), accumulating den and num (and, for the adjoint's sake, P and Q)
// across the pairs; the last pair chunk divides in FP64.
//
// The adjoint (see the fused kernel's header for its formula) runs the same
// two passes on the channels A C, B C, A S, B S (A = G / eta, B = A (out -
// T/2), precomputed planes), demodulates with its own coefficients and adds
// the closing term a (A P - B Q).
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
constexpr int kSmMaxChunk = 256;      // pairs per chunk
constexpr int kSmMaxGroups = (kSmMaxChunk + 2) / 3;   // pair groups per chunk (groups of 3 or more)
constexpr int kSmLineMax = 81;        // row pass: samples per lane at most (odd)
constexpr int kSmSegMax = 2048;       // column pass: rows per segment at most
constexpr int kSmPhaseSync = 8;       // row pass: pairs between direct phase evaluations
constexpr int kSmAhead = 1;           // column pass: rows of tap loads in flight
enum SmMode { kSmFwd = 0, kSmBwd = 1 };

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

// Image pointers read from device memory (the batch kernels' per-image
// arguments) are generic to the compiler, which then emits flat accesses that
// it can only wait for all at once; these casts make them global.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gload_ptr(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gstore_ptr(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

// The adjoint's per-pixel weights A = G / eta and B = A (out - T/2), stored
// interleaved so that one 8-byte load brings both.
struct __attribute__((aligned(8))) AbPair {
    float a, b;
};

struct StrmVArgs {
    const float* f;
    const float* ab;        // adjoint: A and B, interleaved per pixel (2 H W)
    float* vp;              // planes [pair][4][H][Wp]
    int H, W, Wp;
    int ntaps;
    int toff[kSmMaxTaps];   // tap offsets (rows back from the current step)
    int tcoef[kSmMaxTaps];  // tap coefficients (+-1; binomial counts where offsets merge)
    int kinit;              // rows of the segment-start sums: 2R + nb
    int R;
    int npairs;             // pairs of this chunk
    int ngroups, ncolg, seg, nseg;
    int gsize;              // pairs per group (three boxes: 4 to 8 forward, 4 to 7 adjoint)
    float center;
    double two_alpha;       // 2 a
    double ma[kSmMaxGroups];   // m a of each group's first pair
};

// Z <- Z U, complex, in FP64 (the next pair's phase).
__device__ __forceinline__ void rotate(double& zr, double& zi, double ur, double ui) {
    const double nr = fma(zr, ur, -zi * ui);
    zi = fma(zr, ui, zi * ur);
    zr = nr;
}

constexpr double kPiD = 3.14159265358979323846;
constexpr double kInvPiD = 0.31830988618379067154;

// The phase of a sample for a group's first pair, in FP64: theta = m0 a g
// splits as k pi + r with |r| <= pi/2, exp(j theta) = (-1)^k exp(j r), and
// the step to the next pair u = exp(j 2 a g).  Returns whether k is odd:
// the caller folds that sign into its weights instead of into Z.
__device__ __forceinline__ bool group_phase(double ma, double two_alpha, double g, double& zr,
                                            double& zi, double& ur, double& ui) {
    const double th = ma * g;
    const double k = rint(th * kInvPiD);
    cis_small_t<double>(fma(-k, kPiD, th), zr, zi);
    cis_small_t<double>(two_alpha * g, ur, ui);
    return ((int)k) & 1;
}

// The phases of a group's G pairs, Z_0, Z_1 = Z_0 U, then the three-term
// recurrence Z_{q+1} = 2 Re(U) Z_q - Z_{q-1} (two FP64 operations a pair
// instead of a complex product's four).
template <int G>
struct PairSteps {
    double zr, zi, pr, pi, ur, ui;
    __device__ __forceinline__ PairSteps(double zr0, double zi0, double ur0, double ui0)
        : zr(zr0), zi(zi0), pr(0.0), pi(0.0), ur(ur0), ui(ui0) {}
    __device__ __forceinline__ void next(int q) {
        if (q + 1 >= G) return;
        const double cr = zr, ci = zi;
        if (q == 0) {
            rotate(zr, zi, ur, ui);
        } else {
            zr = fma(2.0 * ur, zr, -pr);
            zi = fma(2.0 * ur, zi, -pi);
        }
        pr = cr;
        pi = ci;
    }
};

// The integrator weights of a segment start, wtab[k][s] for k < kinit:
// I_s[t] = sum_k w_s[k] x[t - k] with sum_k w_s[k] z^-k = D(z) / (1 - z^-1)^s,
// D the taps' polynomial: w_s[k] = sum_j c_j C(k - o_j + s - 1, s - 1) over
// o_j <= k (integers, exact in FP64); zero past k = 2R + nb - s.  Threads
// tid, tid + nthr, ... fill the table.
template <int NB>
__device__ __forceinline__ void strm_weights(const StrmVArgs& a, double* wtab, int tid,
                                             int nthr) {
    for (int k = tid; k < a.kinit; k += nthr) {
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
}

// One wave of the column pass: wave gw of the image's (pair group, column
// group, segment) space walks its segment down its 64 columns.
template <int NB, int G, int MODE>
__device__ __forceinline__ void strm_v_body(const StrmVArgs& a, int gw, const double* wtab) {
    constexpr int NT = 1 << NB;
    constexpr bool BWD = MODE == kSmBwd;
    const int lane = threadIdx.x & 63;
    const int H = a.H;
    const int pg = gw % a.ngroups;
    const int rest = gw / a.ngroups;
    const int cg = rest % a.ncolg;
    const int sg = rest / a.ncolg;
    if (sg >= a.nseg) return;
    const int x = cg * 64 + lane;
    if (x >= a.W) return;
    const int n0 = sg * a.seg, n1 = min(H, n0 + a.seg);
    const int t0 = n0 + a.R;            // first step that emits a row (row n0)
    const int te = n1 + a.R;
    const double ma = a.ma[pg];
    const int q0 = pg * G;
    const int nq = min(G, a.npairs - q0);
    const auto* F = gload_ptr(a.f);
    const auto* AB = gload_ptr(reinterpret_cast<const AbPair*>(a.ab));
    auto* VP = gstore_ptr(a.vp);
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
        size_t o = (size_t)min(max(t0 - 1 - kb, 0), H - 1) * a.W + x;
        float gpre = F[o], apre = BWD ? AB[o].a : 0.0f, bpre = BWD ? AB[o].b : 0.0f;
        for (int k = kb; k <= ke; ++k) {
            const float g = gpre - a.center, av = apre, bv = bpre;
            o = (size_t)max(t0 - 2 - k, 0) * a.W + x;
            gpre = F[o];
            if (BWD) {
                apre = AB[o].a;
                bpre = AB[o].b;
            }
            double Zr, Zi, Ur, Ui;
            const double sg = group_phase(ma, a.two_alpha, (double)g, Zr, Zi, Ur, Ui) ? -1.0 : 1.0;
            double w[NB];
#pragma unroll
            for (int s = 0; s < NB; ++s) w[s] = wtab[k * NB + s];
            const double v0 = BWD ? sg * (double)av : sg;
            const double v1 = BWD ? sg * (double)bv : sg * (double)g;
            PairSteps<G> ps(Zr, Zi, Ur, Ui);
#pragma unroll
            for (int q = 0; q < G; ++q) {
                const double c[4] = {v0 * ps.zr, v1 * ps.zr, v0 * ps.zi, v1 * ps.zi};
#pragma unroll
                for (int ch = 0; ch < 4; ++ch)
#pragma unroll
                    for (int s = 0; s < NB; ++s) I[q][ch][s] = fma(w[s], c[ch], I[q][ch][s]);
                ps.next(q);
            }
        }
    }

    // tap rows are wave-uniform: row base in SGPRs, the lane's column as
    // offset; the taps of the next PF rows are in flight (clamped,
    // unconditional loads) while a row is computed: kSmAhead where the
    // integrators fill the registers (three and four boxes), four rows for
    // one box and two for two, whose few waves on small images would
    // otherwise wait on every row's loads (within the registers that keep
    // their waves per SIMD)
    constexpr int PF = NB == 1 ? 4 : NB == 2 ? 2 : kSmAhead;
    float gq[PF][NT], aq[PF][NT], bq[PF][NT];
#pragma unroll
    for (int p = 0; p < PF; ++p)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const size_t o = (size_t)min(max(t0 + p - a.toff[j], 0), H - 1) * a.W;
            gq[p][j] = (F + o)[x];
            if (BWD) {
                aq[p][j] = (AB + o)[x].a;
                bq[p][j] = (AB + o)[x].b;
            }
        }
    for (int t = t0; t < te; ++t) {
        float gcur[NT], acur[NT], bcur[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            gcur[j] = gq[0][j];
            if (BWD) {
                acur[j] = aq[0][j];
                bcur[j] = bq[0][j];
            }
        }
#pragma unroll
        for (int p = 0; p + 1 < PF; ++p)
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                gq[p][j] = gq[p + 1][j];
                if (BWD) {
                    aq[p][j] = aq[p + 1][j];
                    bq[p][j] = bq[p + 1][j];
                }
            }
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const size_t o = (size_t)min(max(t + PF - a.toff[j], 0), H - 1) * a.W;
            gq[PF - 1][j] = (F + o)[x];
            if (BWD) {
                aq[PF - 1][j] = (AB + o)[x].a;
                bq[PF - 1][j] = (AB + o)[x].b;
            }
        }
        // d = sum_j c_j x[t - o_j] in FP64, added tap by tap into the first
        // integrator (no separate sum: its 4 G doubles would cost the
        // registers of a wave): the channels of a sample are v0 Z and v1 Z
        // (forward v = (1, g), adjoint v = (A, B)) with Z the pair's phase
        // carried in FP64 from the group's first pair; c_j v is exact
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            if (j < a.ntaps) {   // uniform
                const int y = t - a.toff[j];
                const bool in = y >= 0 && y < H;
                const double g = in ? (double)(gcur[j] - a.center) : 0.0;
                double Zr, Zi, Ur, Ui;
                const bool neg = group_phase(ma, a.two_alpha, g, Zr, Zi, Ur, Ui);
                const double c0 = in ? (double)a.tcoef[j] : 0.0;
                const double cj = neg ? -c0 : c0;   // (-1)^k of the phase folded in
                const double w0 = BWD ? cj * (double)acur[j] : cj;
                const double w1 = BWD ? cj * (double)bcur[j] : cj * g;
                PairSteps<G> ps(Zr, Zi, Ur, Ui);
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    I[q][0][0] = fma(w0, ps.zr, I[q][0][0]);
                    I[q][1][0] = fma(w1, ps.zr, I[q][1][0]);
                    I[q][2][0] = fma(w0, ps.zi, I[q][2][0]);
                    I[q][3][0] = fma(w1, ps.zi, I[q][3][0]);
                    ps.next(q);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < G; ++q)
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int s = 1; s < NB; ++s) I[q][k][s] += I[q][k][s - 1];
        auto* dst = VP + (size_t)(t - a.R) * a.Wp + x;
        const size_t plane = (size_t)H * a.Wp;
#pragma unroll
        for (int q = 0; q < G; ++q) {
            if (q < nq) {   // uniform
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    __builtin_nontemporal_store((float)I[q][k][NB - 1],
                                                &dst[((size_t)(q0 + q) * 4 + k) * plane]);
            }
        }
    }
}

// Workgroups are dealt to the eight XCDs in turn (workgroup b on XCD b mod
// 8).  Consecutive column-pass tasks are the pair groups of one column group
// and segment, which read the same tap rows: this mapping puts four
// consecutive logical workgroups (sixteen waves) on one XCD, so that they
// share its L2, and keeps the order of the task list window by window (the
// last, incomplete window maps to itself).
__device__ __forceinline__ unsigned xcd_local_block(unsigned b, unsigned nblk) {
    const unsigned full = nblk & ~31u;
    if (b >= full) return b;
    const unsigned w = b & ~31u;
    return w + 4u * (b & 7u) + ((b - w) >> 3);
}

template <int NB, int G, int MODE>
__global__ void __launch_bounds__(kSmThreads) bf_strm_v(const StrmVArgs a) {
    extern __shared__ double wtab[];   // [k][s]: integrator weights of the segment start
    strm_weights<NB>(a, wtab, threadIdx.x, kSmThreads);
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int blk = (int)xcd_local_block(blockIdx.x, gridDim.x);
    strm_v_body<NB, G, MODE>(a, blk * (kSmThreads / 64) + wave, wtab);
}

// A = G / eta and B = A (out - T/2), the adjoint's per-pixel weights.
__global__ void __launch_bounds__(kSmThreads) bf_strm_ab(const float* gout, const float* feta,
                                                          const float* fout, float* ab,
                                                          size_t n, float center) {
    for (size_t i = (size_t)blockIdx.x * kSmThreads + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kSmThreads) {
        const float A = gout[i] / feta[i];
        ab[2 * i] = A;
        ab[2 * i + 1] = A * (fout[i] - center);
    }
}

struct StrmHArgs {
    const float* f;
    const float* vp;
    float* out;             // forward: filtered image; adjoint: dL/df
    float* eta;             // forward: optional eta
    float* aux;             // forward: optional P and Q planes (2 H W)
    const float* faux;      // adjoint: P and Q of the forward
    const float* ab;        // adjoint: A and B, interleaved per pixel (2 H W)
    float* part;            // partial sums between chunks (den, num, P, Q; adjoint: one)
    int H, W, Wp;
    int R, nb;
    int r[BF_MAX_BOXES];
    int padl, bufsz;        // LDS: per wave padl zeros, then the line and its tail
    int npairs;             // pairs of this chunk
    int m0;                 // m of the chunk's first pair
    int first, last;        // first / last chunk
    float center, alpha;
    int sh[BF_MAX_BOXES];   // right shift after each stage
    int shtot;              // their sum
    float L1;               // width of the first box
    float chat[kSmMaxChunk];                  // coefficients of the chunk's pairs
    float mh[kSmMaxChunk], ml[kSmMaxChunk];   // m a of each pair, hi + lo
};

// Lane moves within the wave through DPP (no LDS round trip): row_shr:n
// (0x110 + n) takes the value n lanes below within each row of 16 lanes,
// row_bcast:15 (0x142) the last lane of the row below, row_bcast:31 (0x143)
// lane 31; lanes without a source, and rows outside ROWS, read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_move(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}

// Inclusive prefix over the 64 lanes of a wave of the values combined by op
// (addition modulo 2^32, or the maximum of non-negative floats' bits): a
// scan within each row of 16 lanes, then row 0's total into row 1 and row
// 2's into row 3, then rows 0-1's total into rows 2 and 3.
template <typename Op>
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, Op op) {
    v = op(v, dpp_move<0x111, 0xf>(v));
    v = op(v, dpp_move<0x112, 0xf>(v));
    v = op(v, dpp_move<0x114, 0xf>(v));
    v = op(v, dpp_move<0x118, 0xf>(v));
    v = op(v, dpp_move<0x142, 0xa>(v));
    v = op(v, dpp_move<0x143, 0xc>(v));
    return v;
}

// Exclusive prefix sum of v over the 64 lanes of a wave (modulo 2^32).
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, int lane) {
    (void)lane;
    return wave_incl_scan(v, [](uint32_t a, uint32_t b) { return a + b; }) - v;
}

// The largest of v >= 0 over the wave (non-negative floats order as their bits).
__device__ __forceinline__ float wave_max(float v) {
    const uint32_t m = wave_incl_scan(__float_as_uint(v),
                                      [](uint32_t a, uint32_t b) { return a > b ? a : b; });
    return __uint_as_float((uint32_t)__builtin_amdgcn_readlane((int)m, 63));
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// E: samples per lane (odd, so lanes E words apart hit distinct LDS banks);
// the line covers 64 E >= W + 2R positions.  MODE: forward (AUX: also the
// adjoint's sums P and Q) or adjoint.
template <int E, int MODE, bool AUX>
__device__ __forceinline__ void strm_h_body(const StrmHArgs& a, int y) {
    constexpr int NX = (64 * E + kSmThreads - 1) / kSmThreads;   // pixels per thread at most
    constexpr bool BWD = MODE == kSmBwd;
    constexpr int NACC = BWD ? 1 : (AUX ? 4 : 2);   // sums per pixel
    extern __shared__ __align__(16) uint32_t slds[];
    const int t = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int lane = t & 63;
    const int W = a.W, R = a.R;
    const size_t HW = (size_t)a.H * W;
    uint32_t* buf = slds + wave * a.bufsz;
    for (int i = lane; i < a.padl; i += 64) buf[i] = 0u;   // prefix before the line: 0
    uint32_t* line = buf + a.padl;
    float* linef = reinterpret_cast<float*>(line);
    const int nx = (W + kSmThreads - 1) / kSmThreads;

    // demodulation state of pixels x = t + 256 i: g and the sums; on short
    // lines also the phase of the current pair and the step to the next
    // (exp(j 2 a g)), evaluated directly every kSmPhaseSync pairs and
    // rotated in between; on long lines (registers) every pair directly
    constexpr bool CARRY = NX <= 9;
    constexpr int NP = CARRY ? NX : 1;
    float gx[NX], acc[NACC][NX];
    float pc[NP], ps[NP], ur[NP], ui[NP];
    const auto* frow = gload_ptr(a.f) + (size_t)y * W;
    const auto* PART = gload_ptr(a.part);
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        const int x = min(t + i * kSmThreads, W - 1);
        gx[i] = frow[x] - a.center;
        if (CARRY) cis_small(2.0f * a.alpha * gx[i], ur[i % NP], ui[i % NP]);
#pragma unroll
        for (int c = 0; c < NACC; ++c)
            acc[c][i] = a.first ? 0.0f : PART[c * HW + (size_t)y * W + x];
    }
    __syncthreads();

    const size_t plane = (size_t)a.H * a.Wp;
    const int p0 = lane * E;
    // piece i (256 samples) of this wave's channel of pair q: 16-byte buffer
    // loads (lane offset in a register, the piece in the instruction; the
    // buffer ends at W rounded up to 4, so pieces past it read zero)
    const int W4 = (W + 3) & ~3;
    auto piece = [&](int q, int i) {
        const float* src = a.vp + ((size_t)q * 4 + wave) * plane + (size_t)y * a.Wp;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float*>(src), 0, W4 * (int)sizeof(float), kBufferWord3);
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, 16 * lane, 1024 * i, 0);
        return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]),
                           __uint_as_float(v[3]));
    };
    // short lines (two pieces at most): the next pair's row is loaded while
    // this pair is filtered (the few registers it takes are there; a row with
    // many pairs on one workgroup otherwise waits on every pair's loads)
    constexpr bool PREF = NX <= 2;
    float4 nxt[NX];
    if (PREF && a.npairs > 0) {
#pragma unroll
        for (int i = 0; i < NX; ++i) nxt[i] = piece(0, i);
    }
    for (int qq = 0; qq < a.npairs; ++qq) {
        const int m = a.m0 + 2 * qq;
        const bool centre = m == 0;
        const int nch = centre ? (BWD ? 1 : 2) : 4;
        float4 cur[NX];
        if (PREF) {
#pragma unroll
            for (int i = 0; i < NX; ++i) cur[i] = nxt[i];
            if (qq + 1 < a.npairs) {   // uniform
#pragma unroll
                for (int i = 0; i < NX; ++i) nxt[i] = piece(qq + 1, i);
            }
        }
        if (wave < nch) {
            // the row into the line at position R + x, raw, with aligned
            // 16-byte LDS stores; then the zero margins [0, R) and [R + W,
            // end of the line)
            float* dst4 = linef + R + 4 * lane;
            if (PREF) {
#pragma unroll
                for (int i = 0; i < NX; ++i) *reinterpret_cast<float4*>(dst4 + 256 * i) = cur[i];
            } else {
                constexpr int NH = (NX + 1) / 2;   // two batches: half the staging registers
#pragma unroll
                for (int b = 0; b < NX; b += NH) {
                    float4 ld[NH];
#pragma unroll
                    for (int i = 0; i < NH; ++i)
                        if (b + i < NX) ld[i] = piece(qq, b + i);
#pragma unroll
                    for (int i = 0; i < NH; ++i)
                        if (b + i < NX) *reinterpret_cast<float4*>(dst4 + 256 * (b + i)) = ld[i];
                }
            }
            // zero margins (over the row padding past W as well): one store
            // per lane, and a loop only where a margin is wider than the wave
            const int rm = R + W;
            if (lane < R) line[lane] = 0u;
            if (R > 64)   // uniform
                for (int p = lane + 64; p < R; p += 64) line[p] = 0u;
            if (rm + lane < 64 * E) line[rm + lane] = 0u;
            if (64 * E - rm > 64)   // uniform
                for (int p = rm + lane + 64; p < 64 * E; p += 64) line[p] = 0u;
            wave_sync_lds();
            // the lane's samples and the row's largest magnitude
            float xs[E];
            float vmax = 0.0f;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                xs[e] = linef[p0 + e];
                vmax = fmaxf(vmax, fabsf(xs[e]));
            }
            // the grid: |q| L1 < 2^30 for the row's largest sample; each
            // sample rounded to the nearest grid point (in float: an FP64
            // rounding here held the lane's samples as doubles, and the
            // registers cost more occupancy than the instruction saved)
            vmax = wave_max(vmax);
            const int e1 = vmax > 0.0f ? 30 - __builtin_amdgcn_frexp_expf(a.L1 * vmax) : 0;
            uint32_t v[E];
#pragma unroll
            for (int e = 0; e < E; ++e)
                v[e] = (uint32_t)__float2int_rn(ldexpf(xs[e], e1));
            for (int k = 0; k < a.nb; ++k) {
                const int r = a.r[k];
                // inclusive prefix along the line: the lane's total (three-input
                // adds), its offset from the lanes below, then the running sum
                // from that offset
                uint32_t tot = v[0];
#pragma unroll
                for (int e = 1; e < E; ++e) tot += v[e];
                uint32_t run = wave_excl_scan(tot, lane);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    run += v[e];
                    line[p0 + e] = run;
                }
                wave_sync_lds();
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
                wave_sync_lds();
                // onto the next stage's grid, rounded to nearest (truncation's
                // bias would add up coherently over the later windows)
                const int sh = a.sh[k];
                if (k + 1 < a.nb && sh > 0) {   // uniform
                    const int rnd = 1 << (sh - 1);
#pragma unroll
                    for (int e = 0; e < E; ++e) v[e] = (uint32_t)(((int32_t)v[e] + rnd) >> sh);
                }
            }
            // the filtered channel times the pair's coefficient, as float, in
            // place of the line
            const float cs = ldexpf(a.chat[qq], a.shtot - e1);
#pragma unroll
            for (int e = 0; e < E; ++e) linef[p0 + e] = (float)(int32_t)v[e] * cs;
        }
        __syncthreads();
        const float mh = a.mh[qq], ml = a.ml[qq];
        const float fm = (float)m;
        const float* l0 = reinterpret_cast<const float*>(slds) + a.padl + R;
        const float* l1 = l0 + a.bufsz;
        const float* l2 = l1 + a.bufsz;
        const float* l3 = l2 + a.bufsz;
        const bool direct = !CARRY || qq % kSmPhaseSync == 0;   // uniform
        // every pixel slot (slots past W read inside the lines and are never
        // stored); the lines already carry the pair's coefficient
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            const int x = t + i * kSmThreads;
            const float D0 = l0[x];
            if (centre) {   // m = 0: C = 1, S = 0
                acc[0][i] += D0;
                if (!BWD) acc[1][i] += l1[x];
                if (CARRY) {
                    pc[i % NP] = 1.0f;
                    ps[i % NP] = 0.0f;
                }
            } else {
                const float D1 = l1[x], D2 = l2[x], D3 = l3[x];
                float C, S;
                if (direct) {
                    cis_wide(mh, ml, gx[i], C, S);
                } else {
                    const int k = i % NP;
                    C = pc[k] * ur[k] - ps[k] * ui[k];
                    S = pc[k] * ui[k] + ps[k] * ur[k];
                }
                if (CARRY) {
                    pc[i % NP] = C;
                    ps[i % NP] = S;
                }
                if (!BWD) {
                    acc[0][i] = fmaf(C, D0, fmaf(S, D2, acc[0][i]));
                    acc[1][i] = fmaf(C, D1, fmaf(S, D3, acc[1][i]));
                    if (AUX) {
                        const float mC = fm * C, mS = fm * S;
                        acc[2][i] = fmaf(mC, D3, fmaf(-mS, D1, acc[2][i]));
                        acc[3][i] = fmaf(mC, D2, fmaf(-mS, D0, acc[3][i]));
                    }
                } else {
                    // c {(C - ma g S) F[AC] + (S + ma g C) F[AS] + ma (S F[BC] - C F[BS])}
                    const float u = mh * gx[i];
                    float t2 = fmaf(fmaf(-u, S, C), D0, acc[0][i]);
                    t2 = fmaf(fmaf(u, C, S), D2, t2);
                    t2 = fmaf(mh * S, D1, t2);
                    acc[0][i] = fmaf(-mh * C, D3, t2);
                }
            }
        }
        __syncthreads();
    }
    auto* part = gstore_ptr(a.part);
    auto* out = gstore_ptr(a.out);
    auto* eta = gstore_ptr(a.eta);
    auto* aux = gstore_ptr(a.aux);
    const auto* ab = gload_ptr(reinterpret_cast<const AbPair*>(a.ab));
    const auto* faux = gload_ptr(a.faux);
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        const int x = t + i * kSmThreads;
        if (i < nx && x < W) {
            const size_t o = (size_t)y * W + x;
            if (!a.last) {
#pragma unroll
                for (int c = 0; c < NACC; ++c) part[c * HW + o] = acc[c][i];
            } else if (!BWD) {
                out[o] = (float)((double)a.center + (double)acc[1][i] / (double)acc[0][i]);
                if (a.eta) eta[o] = acc[0][i];
                if (AUX) {
                    aux[o] = acc[2][i];
                    aux[HW + o] = acc[3][i];
                }
            } else {
                const float A = ab[o].a, B = ab[o].b;
                const float P = faux[o], Q = faux[HW + o];
                out[o] = fmaf(a.alpha, A * P - B * Q, acc[0][i]);
            }
        }
    }
}

template <int E, int MODE, bool AUX>
__global__ void __launch_bounds__(kSmThreads) bf_strm_h(const StrmHArgs a) {
    strm_h_body<E, MODE, AUX>(a, blockIdx.x);
}

// ---- batches: the same passes over many images, one launch per pass ---------

struct SbTask {
    int img;     // image of the batch
    int unit;    // column pass: wave in the image's space; row pass: image row
};

// Column pass over a batch: wave gw takes task gw (its image's arguments are
// read from device memory; the segment-start weights go to a wave-private
// slice of LDS of kinit_max * NB doubles).
// Three boxes: each image's own group size (4 .. G), so that one launch
// serves every image of the batch.
template <int NB, int G, int MODE>
__device__ __forceinline__ void sb_v_dispatch(const StrmVArgs& a, int unit, const double* wtab) {
    if constexpr (NB == 3 && G > 4) {
        if (a.gsize < G) {
            sb_v_dispatch<NB, G - 1, MODE>(a, unit, wtab);
            return;
        }
    }
    strm_v_body<NB, G, MODE>(a, unit, wtab);
}

template <int NB, int G, int MODE>
__global__ void __launch_bounds__(kSmThreads) bf_sb_v(const StrmVArgs* __restrict__ args,
                                                      const SbTask* __restrict__ tasks,
                                                      int ntasks, int wslice) {
    extern __shared__ double wt[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gw = (int)xcd_local_block(blockIdx.x, gridDim.x) * (kSmThreads / 64) + wave;
    if (gw >= ntasks) return;   // no block barriers in this kernel
    const int img = __builtin_amdgcn_readfirstlane(tasks[gw].img);
    const int unit = __builtin_amdgcn_readfirstlane(tasks[gw].unit);
    const StrmVArgs& a = args[img];
    double* wtab = wt + (size_t)wave * wslice;
    strm_weights<NB>(a, wtab, threadIdx.x & 63, 64);
    wave_sync_lds();
    sb_v_dispatch<NB, G, MODE>(a, unit, wtab);
}

// Row pass over a batch: workgroup b filters row tasks[b].unit of image
// tasks[b].img (all images of one launch share the line length E).
template <int E, int MODE, bool AUX>
__global__ void __launch_bounds__(kSmThreads) bf_sb_h(const StrmHArgs* __restrict__ args,
                                                      const SbTask* __restrict__ tasks) {
    const int img = __builtin_amdgcn_readfirstlane(tasks[blockIdx.x].img);
    const int y = __builtin_amdgcn_readfirstlane(tasks[blockIdx.x].unit);
    strm_h_body<E, MODE, AUX>(args[img], y);
}

struct SbLossImg {
    const float* out;
    const float* eta;
    const float* target;
    float* ab;          // A, B of the image, interleaved per pixel
    int H, W;
    float center;
};

// Per row of every image: the SSD loss gradient G = 2 (out - target), the
// adjoint's weights A = G / eta and B = A (out - T/2), and the row's partial
// sum of squared differences (a fixed-order block reduction).
__global__ void __launch_bounds__(kSmThreads) bf_sb_lossab(const SbLossImg* __restrict__ imgs,
                                                           const SbTask* __restrict__ tasks,
                                                           float* row_part) {
    __shared__ float red[kSmThreads];
    const SbTask tk = tasks[blockIdx.x];
    const SbLossImg& m = imgs[tk.img];
    const auto* out = gload_ptr(m.out);
    const auto* target = gload_ptr(m.target);
    const auto* eta = gload_ptr(m.eta);
    auto* ab = gstore_ptr(reinterpret_cast<AbPair*>(m.ab));
    const int W = m.W;
    const float center = m.center;
    float acc = 0.0f;
    for (int x = threadIdx.x; x < W; x += kSmThreads) {
        const size_t o = (size_t)tk.unit * W + x;
        const float ov = out[o];
        const float d = ov - target[o];
        const float A = 2.0f * d / eta[o];
        ab[o].a = A;
        ab[o].b = A * (ov - center);
        acc = fmaf(d, d, acc);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kSmThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) row_part[blockIdx.x] = red[0];
}

// loss[i] = the sum of image i's row partials (rows row_first[i] ..
// row_first[i] + H_i - 1 of the row task list), in a fixed order.
__global__ void __launch_bounds__(kSmThreads) bf_sb_lossred(const float* row_part,
                                                            const int* row_first,
                                                            const int* row_count, float* loss) {
    __shared__ float red[kSmThreads];
    const int i = blockIdx.x;
    float acc = 0.0f;
    for (int r = threadIdx.x; r < row_count[i]; r += kSmThreads) acc += row_part[row_first[i] + r];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kSmThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[i] = red[0];
}

// ---- host side -----------------------------------------------------------

namespace {

// Pairs per lane in the column pass: the integrator state (4 channels x nb
// doubles per pair) must leave room for two waves per SIMD.  Three boxes run
// groups of 4 to 8 (forward) or 4 to 7 (adjoint, whose taps also carry A and
// B): per tap a group pays one phase evaluation (about 38 instructions) and
// about 8 per pair, so the largest group wins unless it leaves empty slots
// in the last group (34 pairs: 5 groups of 7, against 6 of 6 or 5 of 8; 16
// pairs: 2 groups of 8 forward, 3 of 6 adjoint).
int group_pairs(int nb, int np, int mode) {
    if (nb <= 2) return 6;
    if (nb >= 4) return 3;
    const int gmax = mode == kSmBwd ? 7 : 8;
    int best = 4;
    for (int g = 5; g <= gmax; ++g)
        if ((np + g - 1) / g * (38 + 8 * g) < (np + best - 1) / best * (38 + 8 * best)) best = g;
    return best;
}
// the column-pass variant: box count and group size
constexpr int vkey(int nb, int G) { return nb * 8 + G; }

// Row-pass instantiations: samples per lane (odd).
constexpr int kSmLines[] = {3,  5,  7,  9,  11, 13, 15, 17, 19, 21, 23, 25, 27, 29,
                            31, 33, 37, 41, 45, 49, 57, 65, 69, 73, 81};

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

// Plane rows start on 256-byte boundaries; narrow images keep 16-byte rows
// (a 1-pixel-wide image would otherwise pad every row 64-fold).
size_t plane_pitch(int64_t W) {
    return W < 64 ? (size_t)((W + 3) / 4 * 4) : (size_t)((W + 63) / 64 * 64);
}

template <int NB, int G, int MODE>
void launch_v(const StrmVArgs& a, hipStream_t s, unsigned blocks, size_t lds) {
    auto k = bf_strm_v<NB, G, MODE>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(kSmThreads), lds, s, a);
}

template <int MODE, bool AUX, int I = 0>
void launch_h(const StrmHArgs& a, int E, hipStream_t s, unsigned blocks, size_t lds) {
    if constexpr (I < (int)(sizeof(kSmLines) / sizeof(kSmLines[0]))) {
        if (E == kSmLines[I]) {
            auto k = bf_strm_h<kSmLines[I], MODE, AUX>;
            (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds);
            hipLaunchKernelGGL(k, dim3(blocks), dim3(kSmThreads), lds, s, a);
            return;
        }
        launch_h<MODE, AUX, I + 1>(a, E, s, blocks, lds);
    }
}

}  // namespace

bool stream_supported(int64_t W, const SpatialParams& sp) {
    if (sp.nb < 1 || sp.nb > BF_MAX_BOXES) return false;
    if (line_lanes(W, sp.R) == 0) return false;   // W + 2R up to 64 x 81 samples
    // row pass: a window of one stage must hold 2^8 levels of its input
    // within 2^30; column pass: the segment-start weights stay exact
    if (mass_1d(sp) >= 2147483648.0) return false;
    for (int k = 0; k < sp.nb; ++k)
        if (2 * sp.r[k] + 1 > (1 << 22)) return false;
    return true;
}

size_t stream_workspace_bytes(int64_t H, int64_t W, int pairs) {
    return (size_t)16 * (size_t)pairs * (size_t)H * plane_pitch(W) +
           (size_t)24 * (size_t)H * (size_t)W;
}

size_t stream_default_workspace(int64_t H, int64_t W, int npairs) {
    const size_t per = (size_t)16 * H * plane_pitch(W);
    const size_t budget = std::max<size_t>(kStreamBudget / per, kStreamChunkPairs);
    const size_t pairs = std::min<size_t>(std::min<size_t>(budget, (size_t)npairs), kSmMaxChunk);
    return stream_workspace_bytes(H, W, (int)pairs);
}

int stream_chunk_pairs(int64_t H, int64_t W, size_t ws_bytes, int npairs) {
    const size_t fixed = (size_t)24 * H * W;
    const size_t per = (size_t)16 * H * plane_pitch(W);
    if (ws_bytes < fixed + per) return 0;
    size_t g = (ws_bytes - fixed) / per;
    g = std::min<size_t>(g, (size_t)kSmMaxChunk);
    return (int)std::min<size_t>(g, (size_t)npairs);
}

// Which evaluation runs by default.  Measured on MI355X, the streamed passes
// beat the fused tiles at every size tried, forward and adjoint: 64^2 to
// 2048^2, radii 1 to 16 per box (2048^2, N = 66, boxes 9, 9, 10: forward with
// the adjoint's sums 2.20 -> 1.67 ms, adjoint 2.27 -> 1.73 ms; 256^2, box
// r = 5: 0.20 -> 0.067 ms).  The fused tiles pay a whole round per tile for
// every pair and their halo work grows with R; the streamed passes pay
// 32 bytes of device memory per pixel and pair, the same for any R.  So the
// streamed passes run wherever they apply (W + 2R within their line), the
// fused tiles elsewhere.
bool prefer_stream(int64_t H, int64_t W, const SpatialParams& sp, bf_status fused_status,
                   const TileGeom& g) {
    (void)H;
    (void)fused_status;
    (void)g;
    return stream_supported(W, sp);
}

namespace {

// Everything of one image's two passes but the pair chunk.
struct StreamSetup {
    int mode;         // forward or adjoint
    StrmVArgs va;
    StrmHArgs ha;
    int E;            // row-pass samples per lane
    size_t lds_v;     // column pass: the segment-start weights
    size_t lds_h;     // row pass: four line buffers
};

// row pass: the first stage's grid comes from each row's largest sample
// (|q| L1 < 2^30); the shifts after each stage keep the next window sum below
// 2^30 for that worst case
bf_status stream_setup(int mode, const StreamIO& io, int64_t H, int64_t W,
                       const RangeParams& rp, const SpatialParams& sp, float* vp, float* part,
                       float* ab, StreamSetup* o) {
    const bool bwd = mode == kSmBwd;
    const int Wp = (int)plane_pitch(W);
    o->mode = mode;
    StrmVArgs& va = o->va;
    va = StrmVArgs{};
    va.f = io.f;
    va.ab = ab;
    va.vp = vp;
    va.H = (int)H;
    va.W = (int)W;
    va.Wp = Wp;
    va.ntaps = make_taps(sp, va.toff, va.tcoef);
    va.R = sp.R;
    va.center = rp.center;
    va.two_alpha = 2.0 * rp.alpha;
    va.kinit = 2 * sp.R + sp.nb;
    o->lds_v = (size_t)va.kinit * sp.nb * sizeof(double);

    StrmHArgs& ha = o->ha;
    ha = StrmHArgs{};
    ha.f = io.f;
    ha.vp = vp;
    ha.out = bwd ? io.gf : io.out;
    ha.eta = io.eta;
    ha.aux = io.aux;
    ha.faux = io.faux;
    ha.ab = ab;
    ha.part = part;
    ha.H = (int)H;
    ha.W = (int)W;
    ha.Wp = Wp;
    ha.R = sp.R;
    ha.nb = sp.nb;
    ha.center = rp.center;
    ha.alpha = (float)rp.alpha;
    ha.L1 = (float)(2 * sp.r[0] + 1);
    int rmax = 0;
    for (int k = 0; k < sp.nb; ++k) {
        ha.r[k] = sp.r[k];
        rmax = std::max(rmax, sp.r[k]);
    }
    double qmax = 1073741824.0 / (2.0 * sp.r[0] + 1.0) + 1.0;
    ha.shtot = 0;
    for (int k = 0; k < sp.nb; ++k) {
        const double smax = (2.0 * sp.r[k] + 1.0) * qmax;   // window sum of stage k
        int sh = 0;
        if (k + 1 < sp.nb) {
            const double lim = 1073741824.0 / (2.0 * sp.r[k + 1] + 1.0);
            while (smax / std::ldexp(1.0, sh) + 1.0 > lim) ++sh;
            qmax = smax / std::ldexp(1.0, sh) + 1.0;
            ha.shtot += sh;
        }
        ha.sh[k] = sh;
    }
    o->E = line_lanes(W, sp.R);
    ha.padl = ((rmax + 1 + sp.R + 3) & ~3) - sp.R;   // line + R is 16-byte aligned
    // after the line: rmax + 1 for the window reads of unused outputs, and
    // room for the row's 16-byte stores and the demodulation's pixel slots,
    // which run to R + 256 ceil(64 E / 256)
    const int nxs = (64 * o->E + kSmThreads - 1) / kSmThreads;
    const int tail = std::max(rmax + 1, sp.R + kSmThreads * nxs - 64 * o->E);
    ha.bufsz = (ha.padl + 64 * o->E + tail + 3) & ~3;
    o->lds_h = (size_t)4 * ha.bufsz * sizeof(uint32_t);
    if (o->lds_h > 160 * 1024) {
        set_error("streamed path: row pass needs %zu bytes of LDS", o->lds_h);
        return BF_EUNSUPPORTED;
    }
    return BF_OK;
}

// The pair chunk qb .. qb + np - 1 (chunk ci of nchunks) and nseg column
// segments.
void stream_chunk(StreamSetup& s, const RangeParams& rp, const SpatialParams& sp, int qb, int np,
                  int ci, int nchunks, int nseg) {
    const int G = group_pairs(sp.nb, np, s.mode);
    const int ngroups = (np + G - 1) / G;
    StrmVArgs& va = s.va;
    va.gsize = G;
    va.npairs = np;
    va.ngroups = ngroups;
    va.ncolg = (va.W + 63) / 64;
    for (int g = 0; g < ngroups; ++g) {
        const double ma = (double)(rp.odd + 2 * (qb + g * G)) * rp.alpha;
        va.ma[g] = ma;
    }
    va.nseg = nseg;
    va.seg = (va.H + nseg - 1) / nseg;
    StrmHArgs& ha = s.ha;
    ha.npairs = np;
    ha.m0 = rp.odd + 2 * qb;
    ha.first = ci == 0;
    ha.last = ci == nchunks - 1;
    for (int q = 0; q < np; ++q) {
        ha.chat[q] = rp.chat[qb + q];
        const double ma = (double)(rp.odd + 2 * (qb + q)) * rp.alpha;
        ha.mh[q] = (float)ma;
        ha.ml[q] = (float)(ma - (double)ha.mh[q]);
    }
}

// The fewest segments of at most kSmSegMax rows (the FP64 integrators'
// rounding drifts roughly as the cube of the rows run: a 16384-row column
// reached 3e-2 gray; each segment starts from the exact state).
int min_segments(int64_t H) { return (int)((H + kSmSegMax - 1) / kSmSegMax); }

// Segment count of a single image's column pass: the least modelled time with
// `slots` waves in flight, a segment start costing about a quarter of a step
// per row above it.
int image_segments(int64_t H, int64_t W, const SpatialParams& sp, int ngroups, double slots) {
    const int ncolg = (int)((W + 63) / 64);
    const int ns0 = min_segments(H);
    int best = ns0;
    double best_cost = 1e300;
    for (int ns = ns0; ns <= ns0 + 64; ++ns) {
        const int seg = (int)((H + ns - 1) / ns);
        if (ns > ns0 && seg < 16) break;
        const double waves = (double)ncolg * ngroups * ns;
        const double start = ns > 1 ? 0.25 * (2.0 * sp.R + sp.nb) : 0.25 * sp.R;
        const double cost = std::ceil(waves / slots) * (seg + start) +
                            0.05 * waves / slots * (seg + start);
        if (cost < best_cost) {
            best_cost = cost;
            best = ns;
        }
    }
    return best;
}

double device_slots() {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return 8.0 * std::max(cus, 1);   // two waves per SIMD
}

template <int MODE>
void launch_v_key(int key, const StrmVArgs& va, hipStream_t stream, unsigned blocks,
                  size_t lds) {
    switch (key) {
        case vkey(1, 6): launch_v<1, 6, MODE>(va, stream, blocks, lds); break;
        case vkey(2, 6): launch_v<2, 6, MODE>(va, stream, blocks, lds); break;
        case vkey(3, 4): launch_v<3, 4, MODE>(va, stream, blocks, lds); break;
        case vkey(3, 5): launch_v<3, 5, MODE>(va, stream, blocks, lds); break;
        case vkey(3, 6): launch_v<3, 6, MODE>(va, stream, blocks, lds); break;
        case vkey(3, 7): launch_v<3, 7, MODE>(va, stream, blocks, lds); break;
        case vkey(3, 8):   // forward only
            if constexpr (MODE == kSmFwd) launch_v<3, 8, MODE>(va, stream, blocks, lds);
            break;
        default: launch_v<4, 3, MODE>(va, stream, blocks, lds); break;
    }
}

void launch_v_mode(int mode, int key, const StrmVArgs& va, hipStream_t stream, unsigned blocks,
                   size_t lds) {
    if (mode == kSmBwd)
        launch_v_key<kSmBwd>(key, va, stream, blocks, lds);
    else
        launch_v_key<kSmFwd>(key, va, stream, blocks, lds);
}

void launch_h_mode(int mode, bool aux, const StrmHArgs& ha, int E, hipStream_t stream,
                   unsigned blocks, size_t lds) {
    if (mode == kSmBwd)
        launch_h<kSmBwd, false>(ha, E, stream, blocks, lds);
    else if (aux)
        launch_h<kSmFwd, true>(ha, E, stream, blocks, lds);
    else
        launch_h<kSmFwd, false>(ha, E, stream, blocks, lds);
}

}  // namespace

bf_status launch_stream(int mode, const StreamIO& io, int64_t H, int64_t W,
                        const RangeParams& rp, const SpatialParams& sp, void* workspace,
                        size_t ws_bytes, hipStream_t stream) {
    if (!stream_supported(W, sp)) {
        set_error("streamed path: W + 2R = %lld exceeds %d samples, or the kernel's mass is "
                  "too large", (long long)(W + 2 * sp.R), 64 * kSmLineMax);
        return BF_EUNSUPPORTED;
    }
    int chunk = stream_chunk_pairs(H, W, ws_bytes, rp.npairs);
    if (chunk <= 0) {
        set_error("streamed path: workspace of %zu bytes is below the %zu bytes one pair needs",
                  ws_bytes, stream_workspace_bytes(H, W, 1));
        return BF_EINVAL;
    }
    if (rp.npairs > 0) {   // as many chunks as the workspace needs, of equal size
        const int n = (rp.npairs + chunk - 1) / chunk;
        chunk = (rp.npairs + n - 1) / n;
    }
    const bool bwd = mode == kSmBwd;
    const bool aux = !bwd && io.aux != nullptr;
    const int Wp = (int)plane_pitch(W);
    const size_t HW = (size_t)H * (size_t)W;
    float* vp = static_cast<float*>(workspace);
    float* part = vp + (size_t)4 * chunk * H * Wp;
    float* ab = part + 4 * HW;
    StreamSetup su;
    bf_status st = stream_setup(mode, io, H, W, rp, sp, vp, part, ab, &su);
    if (st != BF_OK) return st;
    if (bwd) {
        const unsigned nb = (unsigned)std::min<size_t>((HW + kSmThreads - 1) / kSmThreads, 4096);
        hipLaunchKernelGGL(bf_strm_ab, dim3(nb), dim3(kSmThreads), 0, stream, io.gout, io.feta,
                           io.fout, ab, HW, rp.center);
    }
    const double slots = device_slots();
    const int nchunks = (rp.npairs + chunk - 1) / chunk;
    for (int ci = 0; ci < nchunks; ++ci) {
        const int qb = ci * chunk;
        const int np = std::min(chunk, rp.npairs - qb);
        const int G = group_pairs(sp.nb, np, mode);
        const int nseg = image_segments(H, W, sp, (np + G - 1) / G, slots);
        stream_chunk(su, rp, sp, qb, np, ci, nchunks, nseg);
        const long long waves = (long long)su.va.ncolg * su.va.ngroups * nseg;
        launch_v_mode(mode, vkey(sp.nb, G), su.va, stream, (unsigned)((waves + 3) / 4),
                      su.lds_v);
        launch_h_mode(mode, aux, su.ha, su.E, stream, (unsigned)H, su.lds_h);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("streamed path launch: %s", hipGetErrorString(e));
        return BF_EDEVICE;
    }
    return BF_OK;
}

// ---- batches ----------------------------------------------------------------

struct StreamBatch {
    int n = 0;
    bool bwd = false;               // bound with targets: loss and adjoint too
    std::vector<RangeParams> rp;
    std::vector<SpatialParams> sp;
    std::vector<StreamSetup> fw, bw;   // per image: forward and adjoint arguments
    std::vector<int64_t> H, W;
    std::vector<size_t> vp_off, hw_off;   // per image: plane and pixel-plane offsets
    std::vector<int> nseg;                 // per image: column segments
    std::vector<SbLossImg> li;
    struct Group {
        int key;        // column pass: nb; row pass: E
        int off, count; // slice of the task list
        size_t lds;
    };
    std::vector<Group> vgroups[2], hgroups;   // column launches per direction; row launches
    int nrows = 0;
    float* loss = nullptr;
    // device memory (owned)
    float* planes = nullptr;        // column-filtered channels of every image, all pairs
    float* aux = nullptr;           // forward -> adjoint sums P, Q
    float* ab = nullptr;            // adjoint weights A, B
    StrmVArgs* va_f = nullptr;
    StrmVArgs* va_b = nullptr;
    StrmHArgs* ha_f = nullptr;
    StrmHArgs* ha_b = nullptr;
    SbLossImg* li_d = nullptr;
    SbTask* vtasks[2] = {nullptr, nullptr};   // column tasks: forward, adjoint (group sizes differ)
    SbTask* htasks = nullptr;
    SbTask* rows = nullptr;         // every row of every image, image by image
    float* row_part = nullptr;
    int* row_first = nullptr;
    int* row_count = nullptr;
    int nhtasks = 0;
};

namespace {

template <typename T>
bf_status sb_alloc(T** p, size_t count) {
    if (hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        set_error("hipMalloc of %zu bytes for the streamed batch failed", count * sizeof(T));
        return BF_ENOMEM;
    }
    return BF_OK;
}

template <typename T>
bf_status sb_upload(T* d, const std::vector<T>& h) {
    if (h.empty()) return BF_OK;
    if (hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
        set_error("upload of the streamed batch tables failed");
        return BF_EDEVICE;
    }
    return BF_OK;
}

}  // namespace

bool stream_batch_supported(int64_t H, int64_t W, const SpatialParams& sp, int npairs) {
    (void)H;
    // the batch's column pass keeps a segment-start weight table per wave
    // (2R + nb rows of nb doubles), four waves to a workgroup, in LDS
    const size_t lds = (size_t)(kSmThreads / 64) * (2 * sp.R + sp.nb) * sp.nb * sizeof(double);
    return stream_supported(W, sp) && npairs <= kSmMaxGroups * group_pairs(sp.nb, npairs, kSmBwd) &&
           npairs <= kSmMaxChunk && lds <= (size_t)160 * 1024;
}

void stream_batch_destroy(StreamBatch* b) {
    if (!b) return;
    (void)hipFree(b->planes);
    (void)hipFree(b->aux);
    (void)hipFree(b->ab);
    (void)hipFree(b->va_f);
    (void)hipFree(b->va_b);
    (void)hipFree(b->ha_f);
    (void)hipFree(b->ha_b);
    (void)hipFree(b->li_d);
    (void)hipFree(b->vtasks[0]);
    (void)hipFree(b->vtasks[1]);
    (void)hipFree(b->htasks);
    (void)hipFree(b->rows);
    (void)hipFree(b->row_part);
    (void)hipFree(b->row_first);
    (void)hipFree(b->row_count);
    delete b;
}

bf_status stream_batch_create(int n, const int64_t* H, const int64_t* W, const RangeParams* rp,
                              const SpatialParams* sp, StreamBatch** out) {
    StreamBatch* b = new StreamBatch();
    b->n = n;
    b->rp.assign(rp, rp + n);
    b->sp.assign(sp, sp + n);
    b->H.assign(H, H + n);
    b->W.assign(W, W + n);
    b->fw.resize(n);
    b->bw.resize(n);
    b->vp_off.resize(n);
    b->hw_off.resize(n);
    size_t planes = 0, pix = 0;
    for (int i = 0; i < n; ++i) {
        if (!stream_batch_supported(H[i], W[i], sp[i], rp[i].npairs)) {
            set_error("image %d: outside the streamed passes' limits", i);
            stream_batch_destroy(b);
            return BF_EUNSUPPORTED;
        }
        b->vp_off[i] = planes;
        planes += (size_t)4 * rp[i].npairs * H[i] * plane_pitch(W[i]);
        b->hw_off[i] = pix;
        pix += (size_t)H[i] * W[i];
        b->nrows += (int)H[i];
    }
    bf_status st;
    if ((st = sb_alloc(&b->planes, planes)) != BF_OK || (st = sb_alloc(&b->aux, 2 * pix)) != BF_OK ||
        (st = sb_alloc(&b->ab, 2 * pix)) != BF_OK || (st = sb_alloc(&b->va_f, n)) != BF_OK ||
        (st = sb_alloc(&b->va_b, n)) != BF_OK || (st = sb_alloc(&b->ha_f, n)) != BF_OK ||
        (st = sb_alloc(&b->ha_b, n)) != BF_OK || (st = sb_alloc(&b->li_d, n)) != BF_OK ||
        (st = sb_alloc(&b->rows, b->nrows)) != BF_OK ||
        (st = sb_alloc(&b->row_part, b->nrows)) != BF_OK ||
        (st = sb_alloc(&b->row_first, n)) != BF_OK || (st = sb_alloc(&b->row_count, n)) != BF_OK) {
        stream_batch_destroy(b);
        return st;
    }
    // column segments: the fewest (at most kSmSegMax rows each), then more
    // for every image while the batch has fewer than two waves per device
    // slot (a small batch would leave most of the device idle), as long as
    // a segment keeps at least 64 rows and twice its warm-up
    b->nseg.resize(n);
    {
        const double slots = device_slots();
        auto waves = [&](int f) {
            double w = 0.0;
            for (int i = 0; i < n; ++i) {
                const int G = group_pairs(sp[i].nb, rp[i].npairs, kSmFwd);
                const int ns0 = min_segments(H[i]);
                const int64_t lim = std::max<int64_t>(64, 2 * (2 * sp[i].R + sp[i].nb));
                int ns = ns0 * f;
                while (ns > ns0 && (H[i] + ns - 1) / ns < lim) --ns;
                b->nseg[i] = ns;
                w += (double)((W[i] + 63) / 64) * ((rp[i].npairs + G - 1) / G) * ns;
            }
            return w;
        };
        for (int f = 1; f <= 8; ++f)
            if (waves(f) >= 2.0 * slots) break;
    }
    // task lists: column waves grouped by box count, longest first (cost:
    // rows times taps times the group's size-dependent work); rows grouped
    // by line length, image by image
    struct VT {
        double cost;
        int key;
        SbTask t;
    };
    std::vector<SbTask> vtasks[2];
    for (int mode = 0; mode < 2; ++mode) {
        std::vector<VT> vt;
        for (int i = 0; i < n; ++i) {
            const int G = group_pairs(sp[i].nb, rp[i].npairs, mode);
            const int ngroups = (rp[i].npairs + G - 1) / G;
            const int nseg = b->nseg[i];
            const int ncolg = (int)((W[i] + 63) / 64);
            const int seg = (int)((H[i] + nseg - 1) / nseg);
            const double cost = (seg + 0.25 * (2.0 * sp[i].R + sp[i].nb)) * (1 << sp[i].nb) *
                                (38.0 + 8.0 * G);
            const int key = sp[i].nb;   // one launch per box count
            for (int u = 0; u < ncolg * ngroups * nseg; ++u) vt.push_back({cost, key, {i, u}});
        }
        std::stable_sort(vt.begin(), vt.end(), [](const VT& a, const VT& c) {
            return a.key < c.key || (a.key == c.key && a.cost > c.cost);
        });
        auto& vg = b->vgroups[mode];
        for (size_t k = 0; k < vt.size(); ++k) {
            if (vg.empty() || vg.back().key != vt[k].key) vg.push_back({vt[k].key, (int)k, 0, 0});
            vg.back().count++;
            vtasks[mode].push_back(vt[k].t);
        }
    }
    std::vector<SbTask> rows;
    std::vector<int> row_first(n), row_count(n);
    for (int i = 0; i < n; ++i) {
        row_first[i] = (int)rows.size();
        row_count[i] = (int)H[i];
        for (int y = 0; y < (int)H[i]; ++y) rows.push_back({i, y});
    }
    std::vector<int> E(n);
    for (int i = 0; i < n; ++i) E[i] = line_lanes(W[i], sp[i].R);
    std::vector<SbTask> htasks;
    std::vector<int> keys(E.begin(), E.end());
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    // within a line length, the images with the most pairs first: a row's
    // work grows with its pair count, and the longest rows should not be the
    // last to start
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int u, int v) { return rp[u].npairs > rp[v].npairs; });
    for (int e : keys) {
        b->hgroups.push_back({e, (int)htasks.size(), 0, 0});
        for (int i : order)
            if (E[i] == e)
                for (int y = 0; y < (int)H[i]; ++y) htasks.push_back({i, y});
        b->hgroups.back().count = (int)htasks.size() - b->hgroups.back().off;
    }
    b->nhtasks = (int)htasks.size();
    if ((st = sb_alloc(&b->vtasks[0], vtasks[0].size())) != BF_OK ||
        (st = sb_alloc(&b->vtasks[1], vtasks[1].size())) != BF_OK ||
        (st = sb_alloc(&b->htasks, htasks.size())) != BF_OK ||
        (st = sb_upload(b->vtasks[0], vtasks[0])) != BF_OK ||
        (st = sb_upload(b->vtasks[1], vtasks[1])) != BF_OK ||
        (st = sb_upload(b->htasks, htasks)) != BF_OK ||
        (st = sb_upload(b->rows, rows)) != BF_OK || (st = sb_upload(b->row_first, row_first)) != BF_OK ||
        (st = sb_upload(b->row_count, row_count)) != BF_OK) {
        stream_batch_destroy(b);
        return st;
    }
    *out = b;
    return BF_OK;
}

bf_status stream_batch_bind(StreamBatch* b, const float* const* f, const float* const* target,
                            float* const* out, float* const* eta, float* const* gf, float* loss) {
    const int n = b->n;
    b->bwd = gf != nullptr;
    std::vector<StrmVArgs> vaf(n), vab(n);
    std::vector<StrmHArgs> haf(n), hab(n);
    b->li.assign(n, SbLossImg{});
    for (auto& vg : b->vgroups)
        for (auto& g : vg) g.lds = 0;
    for (auto& g : b->hgroups) g.lds = 0;
    for (int i = 0; i < n; ++i) {
        const int64_t H = b->H[i], W = b->W[i];
        float* vp = b->planes + b->vp_off[i];
        float* aux = b->aux + 2 * b->hw_off[i];
        float* ab = b->ab + 2 * b->hw_off[i];
        StreamIO io = {};
        io.f = f[i];
        io.out = out[i];
        io.eta = eta ? eta[i] : nullptr;
        io.aux = b->bwd ? aux : nullptr;
        bf_status st = stream_setup(kSmFwd, io, H, W, b->rp[i], b->sp[i], vp, nullptr, ab,
                                    &b->fw[i]);
        if (st != BF_OK) return st;
        const int nseg = b->nseg[i];
        stream_chunk(b->fw[i], b->rp[i], b->sp[i], 0, b->rp[i].npairs, 0, 1, nseg);
        vaf[i] = b->fw[i].va;
        haf[i] = b->fw[i].ha;
        if (b->bwd) {
            StreamIO jo = {};
            jo.f = f[i];
            jo.fout = out[i];
            jo.feta = eta[i];
            jo.faux = aux;
            jo.gf = gf[i];
            st = stream_setup(kSmBwd, jo, H, W, b->rp[i], b->sp[i], vp, nullptr, ab, &b->bw[i]);
            if (st != BF_OK) return st;
            stream_chunk(b->bw[i], b->rp[i], b->sp[i], 0, b->rp[i].npairs, 0, 1, nseg);
            vab[i] = b->bw[i].va;
            hab[i] = b->bw[i].ha;
            b->li[i] = SbLossImg{out[i], eta[i], target[i], ab, (int)H, (int)W, b->rp[i].center};
        }
        for (auto& vg : b->vgroups)
            for (auto& g : vg)
                if (g.key == b->sp[i].nb)
                    g.lds = std::max(g.lds, (size_t)(kSmThreads / 64) * b->fw[i].lds_v);
        for (auto& g : b->hgroups)
            if (g.key == b->fw[i].E) g.lds = std::max(g.lds, b->fw[i].lds_h);
    }
    bf_status st;
    if ((st = sb_upload(b->va_f, vaf)) != BF_OK || (st = sb_upload(b->ha_f, haf)) != BF_OK)
        return st;
    if (b->bwd && ((st = sb_upload(b->va_b, vab)) != BF_OK ||
                   (st = sb_upload(b->ha_b, hab)) != BF_OK || (st = sb_upload(b->li_d, b->li)) != BF_OK))
        return st;
    for (const auto& vg : b->vgroups)
        for (const auto& g : vg)
            if (g.lds > 160 * 1024) {
                set_error("streamed batch: the segment-start weights need %zu bytes of LDS",
                          g.lds);
                return BF_EUNSUPPORTED;
            }
    b->loss = loss;
    return BF_OK;
}

namespace {

template <int NB, int G, int MODE>
void launch_sb_v(const StrmVArgs* args, const SbTask* tasks, int count, size_t lds,
                 hipStream_t s) {
    auto k = bf_sb_v<NB, G, MODE>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    const int wslice = (int)(lds / sizeof(double) / (kSmThreads / 64));
    hipLaunchKernelGGL(k, dim3((unsigned)((count + 3) / 4)), dim3(kSmThreads), lds, s, args,
                       tasks, count, wslice);
}

template <int MODE>
void launch_sb_v_key(int key, const StrmVArgs* args, const SbTask* tasks, int count, size_t lds,
                     hipStream_t s) {
    switch (key) {   // the box count; three boxes take every group size in one kernel
        case 1: launch_sb_v<1, 6, MODE>(args, tasks, count, lds, s); break;
        case 2: launch_sb_v<2, 6, MODE>(args, tasks, count, lds, s); break;
        case 3: launch_sb_v<3, MODE == kSmBwd ? 7 : 8, MODE>(args, tasks, count, lds, s); break;
        default: launch_sb_v<4, 3, MODE>(args, tasks, count, lds, s); break;
    }
}

template <int MODE, bool AUX, int I = 0>
void launch_sb_h(const StrmHArgs* args, const SbTask* tasks, int count, int E, size_t lds,
                 hipStream_t s) {
    if constexpr (I < (int)(sizeof(kSmLines) / sizeof(kSmLines[0]))) {
        if (E == kSmLines[I]) {
            auto k = bf_sb_h<kSmLines[I], MODE, AUX>;
            (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds);
            hipLaunchKernelGGL(k, dim3((unsigned)count), dim3(kSmThreads), lds, s, args, tasks);
            return;
        }
        launch_sb_h<MODE, AUX, I + 1>(args, tasks, count, E, lds, s);
    }
}

void sb_passes(const StreamBatch* b, int mode, bool aux, hipStream_t s, bool col, bool row) {
    const StrmVArgs* va = mode == kSmBwd ? b->va_b : b->va_f;
    const StrmHArgs* ha = mode == kSmBwd ? b->ha_b : b->ha_f;
    for (const auto& g : b->vgroups[mode == kSmBwd ? 1 : 0]) {
        if (!col) break;
        const SbTask* t = b->vtasks[mode == kSmBwd ? 1 : 0] + g.off;
        if (mode == kSmBwd)
            launch_sb_v_key<kSmBwd>(g.key, va, t, g.count, g.lds, s);
        else
            launch_sb_v_key<kSmFwd>(g.key, va, t, g.count, g.lds, s);
    }
    for (const auto& g : b->hgroups) {
        if (!row) break;
        const SbTask* t = b->htasks + g.off;
        if (mode == kSmBwd)
            launch_sb_h<kSmBwd, false>(ha, t, g.count, g.key, g.lds, s);
        else if (aux)
            launch_sb_h<kSmFwd, true>(ha, t, g.count, g.key, g.lds, s);
        else
            launch_sb_h<kSmFwd, false>(ha, t, g.count, g.key, g.lds, s);
    }
}

}  // namespace

bf_status stream_batch_stage(const StreamBatch* b, int stage, hipStream_t s) {
    switch (stage) {
        case 0: sb_passes(b, kSmFwd, b->bwd, s, true, false); break;
        case 1: sb_passes(b, kSmFwd, b->bwd, s, false, true); break;
        case 2:
            if (b->bwd) {
                hipLaunchKernelGGL(bf_sb_lossab, dim3((unsigned)b->nrows), dim3(kSmThreads), 0, s,
                                   b->li_d, b->rows, b->row_part);
                if (b->loss)
                    hipLaunchKernelGGL(bf_sb_lossred, dim3((unsigned)b->n), dim3(kSmThreads), 0,
                                       s, b->row_part, b->row_first, b->row_count, b->loss);
            }
            break;
        case 3:
            if (b->bwd) sb_passes(b, kSmBwd, false, s, true, false);
            break;
        case 4:
            if (b->bwd) sb_passes(b, kSmBwd, false, s, false, true);
            break;
        default:
            set_error("stage %d is not one of 0..4", stage);
            return BF_EINVAL;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("streamed batch launch: %s", hipGetErrorString(e));
        return BF_EDEVICE;
    }
    return BF_OK;
}

bf_status stream_batch_launch(const StreamBatch* b, hipStream_t s) {
    for (int stage = 0; stage < 5; ++stage) {
        const bf_status st = stream_batch_stage(b, stage, s);
        if (st != BF_OK) return st;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("streamed batch launch: %s", hipGetErrorString(e));
        return BF_EDEVICE;
    }
    return BF_OK;
}

}  // namespace bf
