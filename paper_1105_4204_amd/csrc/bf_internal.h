// Internal declarations shared by the host code and the HIP kernels of the
// trigonometric bilateral filter library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bf_trig.h"

namespace bf {

// Largest number of cosine pairs: floor(BF_MAX_DEGREE / 2) + 1.
constexpr int kMaxPairs = BF_MAX_DEGREE / 2 + 1;

// Host-side description of one filter evaluation: everything derived from
// (T, sigma_r, N, radii) before a launch.
struct RangeParams {
    int32_t N;        // degree of the raised cosine
    int32_t npairs;   // cosine pairs actually evaluated (trailing zero coefficients dropped)
    int32_t odd;      // N mod 2: the first pair has m = 1 instead of m = 0
    double alpha;     // 1 / (sigma_r sqrt N): phase per unit of intensity and unit of m
    float center;     // T/2: intensities are re-centred before modulation
    float chat[kMaxPairs];
};

struct SpatialParams {
    int32_t nb;       // boxes per axis
    int32_t r[BF_MAX_BOXES];
    int32_t R;        // sum of radii: half-width of the composite kernel
};

// Recursive Gaussian spatial filter (Young and van Vliet): line-pass
// coefficients and the map from the causal end state to the anticausal
// start state (row-major 3 x 3).
constexpr double kYvvMinSigma = 0.5;
constexpr double kYvvMaxSigma = 64.0;
struct YvvParams {
    double B, a1, a2, a3;
    double M[9];
    double k0;       // centre tap of the two-pass impulse response (mass 1)
};

// Host helpers (bf_host.cpp).
void set_error(const char* fmt, ...);
bf_status make_range(double T, double sigma_r, int32_t N_req, RangeParams* rp);
bf_status make_spatial(const bf_spatial_spec* spec, SpatialParams* sp);
bf_status truncate_pairs(RangeParams* rp, const SpatialParams& sp, double T, double tol,
                         double* bound_out);
bf_status truncate_pairs_km(RangeParams* rp, double k0, double mass, double T, double tol,
                            double* bound_out);
bf_status check_image(const void* p, int64_t H, int64_t W, const char* name);
bf_status make_yvv(double sigma_s, YvvParams* yp);
bool overlaps(const void* a, const void* b, int64_t bytes);   // two ranges of `bytes` each
bool overlaps(const void* a, int64_t abytes, const void* b, int64_t bbytes);

// Tile geometry of the fused forward/backward kernels.
struct TileGeom {
    int TH, TW;       // output tile
    int EH, EW;       // extended tile (output + halo of R on every side)
    int EWp, EHp;     // LDS pitches of extended rows and of transposed rows
    int tiles_x, tiles_y;
    size_t lds_bytes;
    bool gg;          // adjoint: g read from global memory (one LDS plane)
    int line;         // register line length of the single-image kernels (120 or 128)
};

bf_status plan_fwd_tiles(int64_t H, int64_t W, const SpatialParams& sp, int req_h, int req_w,
                         TileGeom* g);
bf_status launch_fwd(const float* f, float* out, float* eta, float* aux, int64_t H, int64_t W,
                     const RangeParams& rp, const SpatialParams& sp, const TileGeom& g,
                     hipStream_t stream);
// Count of pixels outside [0, T] (NaN included) into a device counter (bf_check.hip).
bf_status launch_check_range(const float* f, int64_t H, int64_t W, float T, unsigned* count,
                             hipStream_t stream);
bf_status launch_direct(const float* f, float* out, float* eta, int64_t H, int64_t W,
                        const RangeParams& rp, const SpatialParams& sp, hipStream_t stream);
bf_status plan_bwd_tiles(int64_t H, int64_t W, const SpatialParams& sp, int req_h, int req_w,
                         TileGeom* g, const float* f);
// Streamed forward and adjoint (bf_stream.hip): whole-line column and row
// passes whose cost does not depend on the radii; the column-filtered
// channels of a chunk of pairs pass through a workspace.
struct StreamIO {
    const float* f;
    float* out;           // forward
    float* eta;           // forward, optional
    float* aux;           // forward, optional (P, Q)
    const float* fout;    // adjoint: the forward's out, eta and P, Q
    const float* feta;
    const float* faux;
    const float* gout;    // adjoint: dL/dout
    float* gf;            // adjoint: dL/df
};
constexpr int kStreamFwd = 0, kStreamBwd = 1;
bool stream_supported(int64_t W, const SpatialParams& sp);
size_t stream_workspace_bytes(int64_t H, int64_t W, int pairs);   // planes + partials + A, B
int stream_chunk_pairs(int64_t H, int64_t W, size_t ws_bytes, int npairs);
bool prefer_stream(int64_t H, int64_t W, const SpatialParams& sp, bf_status fused_status,
                   const TileGeom& g);
bf_status launch_stream(int mode, const StreamIO& io, int64_t H, int64_t W,
                        const RangeParams& rp, const SpatialParams& sp, void* workspace,
                        size_t ws_bytes, hipStream_t stream);
// A batch through the streamed passes: every pass over every image in one
// launch per box count or line length (plan-owned planes for all pairs of
// all images, the adjoint's sums and weights, task tables).
struct StreamBatch;
bool stream_batch_supported(int64_t H, int64_t W, const SpatialParams& sp, int npairs);
bf_status stream_batch_create(int n, const int64_t* H, const int64_t* W, const RangeParams* rp,
                              const SpatialParams* sp, StreamBatch** out);
bf_status stream_batch_bind(StreamBatch* b, const float* const* f, const float* const* target,
                            float* const* out, float* const* eta, float* const* gf, float* loss);
bf_status stream_batch_launch(const StreamBatch* b, hipStream_t s);
bf_status stream_batch_stage(const StreamBatch* b, int stage, hipStream_t s);
void stream_batch_destroy(StreamBatch* b);
// Pairs per chunk of the workspace bf_trig_workspace_bytes recommends; the
// library's own workspace and bf_trig_workspace_bytes_ex hold every pair up
// to a budget of 16 GiB of planes (but at least this many pairs): a few per
// cent of the device's memory, 64 pairs at 4096^2.
constexpr int kStreamChunkPairs = 16;
constexpr size_t kStreamBudget = (size_t)16 << 30;
size_t stream_default_workspace(int64_t H, int64_t W, int npairs);
// The library's own streamed-path workspace for the current device (bf_api.cpp):
// library_workspace takes a lock and orders `stream` after the previous user;
// library_workspace_done records that use and releases the lock.
bf_status library_workspace(size_t need, hipStream_t stream, void** out);
bf_status library_workspace_done(hipStream_t stream);
// Space-variant box kernel through tile-local summed-area tables (bf_sv.hip).
bf_status launch_sv(const float* f, const int32_t* rmap, float* out, float* eta, int64_t H,
                    int64_t W, int32_t rmax, const RangeParams& rp, hipStream_t stream);
// Recursive Gaussian forward over whole image lines (bf_yvv.hip).
size_t yvv_workspace_bytes(int64_t H, int64_t W, int npairs);
bf_status launch_yvv(const float* f, float* out, float* eta, int64_t H, int64_t W,
                     const RangeParams& rp, const YvvParams& yp, void* workspace,
                     size_t workspace_bytes, hipStream_t stream);
bf_status launch_bwd(const float* f, const float* out, const float* eta, const float* aux,
                     const float* gout, float* gf, int64_t H, int64_t W, const RangeParams& rp,
                     const SpatialParams& sp, const TileGeom& g, hipStream_t stream);

}  // namespace bf
