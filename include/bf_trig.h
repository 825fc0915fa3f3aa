/*
 * bf_trig.h -- C ABI of the constant-time trigonometric bilateral filter for
 * AMD MI355X (gfx950).
 *
 * The filter is the unbiased bilateral filter of Chaudhury, Sage and Unser,
 * "Fast O(1) bilateral filtering using trigonometric range kernels":
 *
 *     out(x) = sum_y w(y) phi(f(x-y) - f(x)) f(x-y) / eta(x)         eq. (BF)
 *     eta(x) = sum_y w(y) phi(f(x-y) - f(x))                 eq. (normalization)
 *
 * with the raised-cosine range kernel phi(s) = cos(alpha s)^N of Sec. 2.3,
 * scaled as in Sec. 2.5 / Algorithm 1 (gamma = pi/2T, rho = gamma sigma_r,
 * alpha = gamma/(rho sqrt N) = 1/(sigma_r sqrt N)), and a separable spatial
 * kernel w(dy,dx) = k(dy) k(dx) where k is the convolution of n_boxes
 * unit-height boxes of widths 2 radius[i] + 1 (the O(1) box / iterated-box
 * averaging of Sec. 2.1).  The sums run over pixels inside the image (the
 * auxiliary images are zero-extended).  The library evaluates it in O(1) per
 * pixel per term through the binomial expansion of Sec. 2.3 and eq.
 * (final-form): pairs of auxiliary images exp(+-j m alpha f), f exp(+-j m
 * alpha f) are filtered by running box sums and demodulated per pixel.
 *
 * Conventions shared by every entry point:
 *  - Images are row-major H x W float32 arrays in DEVICE memory owned by the
 *    caller (e.g. torch tensors); the library never frees them.
 *  - Input intensities are expected in [0, T] (Sec. 2.1); this precondition
 *    keeps the kernel non-negative and is not checked on the hot path.
 *  - eta uses the unnormalised integer box weights (the mass of w cancels in
 *    the ratio).
 *  - Calls are asynchronous on opts->stream (a hipStream_t; NULL = the null
 *    stream).  Argument errors are reported synchronously, before anything is
 *    enqueued; launch errors as BF_EDEVICE.  No function throws.
 *  - bf_last_error() returns a thread-local description of the last failure.
 */
#ifndef BF_TRIG_H
#define BF_TRIG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BF_OK = 0,
    BF_EINVAL = 1,       /* null pointer, non-positive size, bad spec, aliasing */
    BF_ERANGE = 2,       /* degree below the bound of Sec. 2.5, N or radius too large */
    BF_ENOMEM = 3,       /* device or host allocation failed */
    BF_EDEVICE = 4,      /* HIP runtime / launch error */
    BF_ECAPTURE = 5,     /* call not allowed while the stream is being captured */
    BF_EUNSUPPORTED = 6  /* valid request outside what the library implements */
} bf_status;

#define BF_MAX_BOXES 4      /* iterated boxes per axis */
#define BF_MAX_RADIUS 256   /* per box (BF_ERANGE above).  The fused kernel takes
                               radii <= 31 with R = sum of radii <= 63; the
                               streamed passes take any radii up to this with
                               W + 2R <= 5184 and prod(2 radius + 1) < 2^31 */
#define BF_MAX_DEGREE 1024  /* largest raised-cosine degree N */

/* bf_opts.path: which forward evaluation runs. */
#define BF_PATH_AUTO 0      /* the library's choice (cost model) */
#define BF_PATH_FUSED 1     /* fused tile kernel (radii <= 31, R <= 63) */
#define BF_PATH_STREAMED 2  /* streamed whole-line passes (any R the limits allow) */

/* Spatial kernel: n_boxes boxes per axis (1 = plain box; 3 approximates a
 * Gaussian, Sec. 2.1 and Algorithm 1 step 4).  radius[i] >= 0; box i has
 * 2 radius[i] + 1 taps, the same in x and y. */
typedef struct {
    int32_t n_boxes;
    int32_t radius[BF_MAX_BOXES];
} bf_spatial_spec;

/* Optional per-call settings; a NULL bf_opts* means all defaults. */
typedef struct {
    void* stream;        /* hipStream_t; NULL = null stream */
    int32_t N;           /* 0 = ceil((2T/(pi sigma_r))^2) (Algorithm 1 step 2);
                            else the degree, which must be >= that bound */
    float* eta_out;      /* optional H*W device buffer for eta (the backward
                            needs it); NULL = not written */
    int32_t tile_h;      /* 0 = library choice; else output tile rows */
    int32_t tile_w;      /* 0 = library choice; else output tile columns */
    float* aux_out;      /* forward only: optional 2*H*W device buffer for the
                            two auxiliary sums the backward needs (see
                            bf_trig_backward); NULL = not computed */
    void* workspace;     /* device scratch of the streamed passes (forward and
                            backward; see bf_trig_workspace_bytes), 256-byte
                            aligned, not overlapping the images; NULL = the
                            library's own */
    int64_t workspace_bytes;
    float trunc_tol;     /* 0 = every cosine pair; > 0 = drop the outer pairs
                            while the bound of bf_range_truncate stays <= this
                            many gray levels (forward and backward must agree) */
    int32_t path;        /* forward and backward: BF_PATH_AUTO (0),
                            BF_PATH_FUSED or BF_PATH_STREAMED */
} bf_opts;

/* Algorithm 1 steps 1-2: N = ceil((gamma sigma_r)^-2), gamma = pi/(2T).
 * T > 0, sigma_r > 0.  BF_ERANGE if N would exceed BF_MAX_DEGREE. */
bf_status bf_range_degree(double T, double sigma_r, int32_t* N_out);

/* Sec. 2.3 binomial expansion folded into cosine pairs:
 *   cos^N(t) = sum_q c[q] cos(m_q t),  m_q = (N mod 2) + 2q,
 *   c[q] = 2^-N C(N, N/2) for m_q = 0, else 2^(1-N) C(N, (N-m_q)/2),
 * computed in extended precision and rounded to float.  Writes
 * n = floor(N/2)+1 values to c_out (capacity cap); *n_out = n. */
bf_status bf_range_coeffs(int32_t N, float* c_out, int32_t cap, int32_t* n_out);

/* Term truncation with an error bound (the acceleration for small sigma_r
 * the paper leaves open in Sec. 3).  Removing the pairs q >= Q drops the
 * binomial mass delta = sum_{q>=Q} c[q] from the kernel, |phi - phi_Q| <= delta,
 * and since the normaliser of eq. (normalization) is at least w(0) (phi >= 0
 * when N meets the degree bound, phi(0) = 1):
 *     |out_Q - out| <= T delta sum(w) / (w(0) - delta sum(w)).
 * Writes the fewest pairs Q whose bound is <= tol (gray levels) and the bound
 * itself (0 when nothing is dropped).  Pairs whose float coefficient is zero
 * are never counted. */
bf_status bf_range_truncate(int32_t N, double T, const bf_spatial_spec* spatial_spec,
                            double tol, int32_t* npairs_out, double* bound_out);

/* Radii of n_boxes iterated boxes whose combined variance approximates
 * sigma_s^2 (a Gaussian spatial filter of Algorithm 1 step 4): ideal width
 * sqrt(12 sigma_s^2 / n + 1), mixing the nearest odd widths below and above,
 * the narrower ones first, ties to the narrower. */
bf_status bf_spatial_gaussian(double sigma_s, int32_t n_boxes, bf_spatial_spec* out);

/* Device workspace of the streamed passes for image size H x W and this
 * spatial kernel: 0 when the library evaluates this geometry with the fused
 * tile kernel (no workspace), otherwise the recommended size,
 * 16 P H Wp + 24 H W bytes for P = 16 cosine pairs, Wp = W rounded up to a
 * multiple of 64 (of 4 for W < 64).  The streamed passes (Sec. 2.1, eq. (final-form)) filter
 * the four channels of each pair along whole columns and then whole rows;
 * the column-filtered channels of a chunk of pairs wait in the workspace
 * between the two passes, the partial sums between chunks (and the adjoint's
 * per-pixel weights).  Any size from one pair's (P = 1) up works: smaller
 * workspaces only mean more chunks.
 * The library's choice (BF_PATH_AUTO) is the streamed passes wherever they
 * apply (W + 2R <= 5184 and a kernel mass prod(2 radius + 1) below 2^31):
 * they are faster than the fused tiles at every size measured and their cost
 * does not grow with the radii.  The fused kernel takes the other images its
 * limits allow.  BF_EUNSUPPORTED when neither evaluation handles the kernel. */
bf_status bf_trig_workspace_bytes(int64_t H, int64_t W, const bf_spatial_spec* spatial_spec,
                                  int64_t* bytes_out);

/* The same for a given degree (T, sigma_r and N as for the forward): the
 * recommended size holds every cosine pair of that degree in one chunk, up to
 * 16 GiB of planes (at least 16 pairs; 64 pairs at 4096^2), which is the size
 * of the library's own workspace.  A smaller workspace runs the pairs in
 * chunks of equal size.  0 where the fused kernel is used. */
bf_status bf_trig_workspace_bytes_ex(int64_t H, int64_t W, float T, float sigma_r, int32_t N,
                                     const bf_spatial_spec* spatial_spec, int64_t* bytes_out);

/* Forward filter, eq. (BF)/(normalization) with the raised-cosine kernel.
 * f: H*W input; out: H*W output (must not overlap f).  sigma_r > 0, T > 0.
 * Equivalent to bf_trig_forward_ex with opts == NULL: every kernel width the
 * limits above allow runs; where the streamed passes run, the library uses a
 * workspace of its own (the size bf_trig_workspace_bytes_ex recommends: every
 * pair in one chunk up to 16 GiB of planes), allocated on first need per
 * device and kept until the process ends, so such a call may not be captured
 * (BF_ECAPTURE) and may return BF_ENOMEM.  Calls that share it are ordered on
 * the device, whatever their streams.
 *
 * bf_trig_forward_ex: opts->path forces either evaluation, and a tile
 * override forces the fused kernel; opts->eta_out and opts->aux_out (the
 * adjoint's sums) work on both; a caller workspace smaller than one pair's
 * returns BF_EINVAL. */
bf_status bf_trig_forward(const float* f, int64_t H, int64_t W, float T, float sigma_r,
                          const bf_spatial_spec* spatial_spec, float* out);

bf_status bf_trig_forward_ex(const float* f, int64_t H, int64_t W, float T, float sigma_r,
                             const bf_spatial_spec* spatial_spec, float* out,
                             const bf_opts* opts);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): bf_trig_forward_ex
 * with the streamed passes' workspace taken from a static device array of
 * 64 MiB that the library holds on each device it runs on (from its first
 * use until the process ends); nothing is allocated or freed.  opts->workspace
 * must be NULL (BF_EINVAL otherwise); the other options are as for
 * bf_trig_forward_ex.  Path choice: the streamed passes where they apply
 * (W + 2R <= 5184) and one cosine pair fits the array, 16 H Wp + 24 H W <=
 * 64 MiB (chunks of as many pairs as fit); otherwise the fused kernel where
 * it holds the spatial kernel (it needs no workspace); otherwise BF_ERANGE,
 * as for BF_PATH_STREAMED forced on an image whose pair does not fit.  Every
 * call on one device shares that device's array: calls that overlap on one
 * device (different streams, or host threads) race and must be serialised
 * by the caller.  Nothing in the array needs to start at zero. */
bf_status bf_trig_forward_noalloc(const float* f, int64_t H, int64_t W, float T,
                                  float sigma_r, const bf_spatial_spec* spatial_spec,
                                  float* out, const bf_opts* opts);

/* Adjoint: grad_f = (d out / d f)^T grad_out, the exact derivative of eq.
 * (BF)/(normalization) for the raised-cosine kernel, evaluated term by term
 * on the expansion of eq. (final-form).  out, eta and aux are the forward's
 * outputs for the same f and parameters (opts->N must match): aux holds the
 * planes P = sum_m c_m m (C_m F[g S_m] - S_m F[g C_m]) and
 * Q = sum_m c_m m (C_m F[S_m] - S_m F[C_m]) (g = f - T/2, C_m + j S_m =
 * exp(j m alpha g)), which the forward writes to opts->aux_out.  aux may be
 * NULL: the library then recomputes P and Q with a forward of its own (one
 * forward more, written into the library's workspace, allocated on first
 * need and kept; not allowed during stream capture: BF_ECAPTURE).  f, out,
 * eta, grad_out and grad_f are H*W, aux 2*H*W; grad_f must not overlap the
 * inputs.  opts->aux_out is ignored.  When W and the kernel half-width R are
 * multiples of 4, f is 16-byte aligned and 4 H W < 2^31, the adjoint reads g
 * from global memory and fits tiles up to 64 x 64 (widths a multiple of 4);
 * otherwise it stages g in LDS and fits smaller tiles.  An explicit
 * opts->tile_h x tile_w that fits neither returns BF_EINVAL.  Path choice,
 * opts->path and the workspace are as for the forward: by default the
 * streamed passes wherever they apply, which filter the four channels A C,
 * B C, A S, B S of each pair (A = grad_out / eta, B = A (out - T/2)) and
 * demodulate with the adjoint's coefficients. */
bf_status bf_trig_backward(const float* f, const float* out, const float* eta,
                           const float* aux, const float* grad_out, int64_t H, int64_t W,
                           float T, float sigma_r, const bf_spatial_spec* spatial_spec,
                           float* grad_f, const bf_opts* opts);

/* Space-variant spatial kernel (Sec. 4, space-variant extension): the unit
 * box around pixel (i, j) has half-width radius[i*W + j], clamped to
 * [0, rmax], in both directions; the range kernel is the fixed raised
 * cosine.  out(x) = sum_{|y-x|_inf <= r(x)} phi(f(y)-f(x)) f(y) / eta(x) over
 * in-image y, eta(x) the same sum without f(y), evaluated through eq.
 * (final-form) with box sums read from summed-area tables, so the cost per
 * pixel does not depend on the radii.  radius: device int32 H*W (caller-owned,
 * not modified).  0 <= rmax <= 31 (BF_EUNSUPPORTED above).  opts: stream, N,
 * eta_out and trunc_tol as for the forward (the truncation bound is taken for
 * the rmax box); tiles, aux_out and workspace are ignored.  out must not
 * overlap f, radius or eta_out.  Asynchronous on opts->stream. */
bf_status bf_sv_forward(const float* f, const int32_t* radius, int64_t H, int64_t W, float T,
                        float sigma_r, int32_t rmax, float* out, const bf_opts* opts);

/* Recursive Gaussian spatial kernel: the filter of Young and van Vliet
 * (Signal Processing 44(2), 1995), which the paper's experiments use for the
 * spatial averaging (Sec. 3), in place of the iterated boxes.  Each axis is
 * filtered by a third-order causal pass and an anticausal pass with the
 * published coefficients for standard deviation sigma_s in [0.5, 64]
 * (BF_ERANGE outside), over whole image lines with zero extension at both
 * ends, so the spatial kernel is the exact two-sided impulse response of the
 * passes (infinite support).  Evaluated through eq. (final-form) like the
 * forward; the filtered channels of up to 40 cosine pairs at a time pass
 * through opts->workspace (required; at least bf_yvv_workspace_bytes bytes,
 * device memory, not overlapping the images).  opts: stream, N, eta_out and
 * trunc_tol (the bound of bf_range_truncate with this kernel's centre tap and
 * mass); tiles and aux_out are ignored.  out must not overlap f or eta_out.
 * Asynchronous on opts->stream; no adjoint.
 * bf_yvv_coeffs writes the line-pass coefficients for sigma_s to coeffs_out[0..4):
 * the gain B and a1, a2, a3 of the recursions above (host only; BF_ERANGE for
 * sigma_s outside [0.5, 64]). */
bf_status bf_yvv_coeffs(double sigma_s, double* coeffs_out);
bf_status bf_yvv_workspace_bytes(int64_t H, int64_t W, float T, float sigma_r, int32_t N,
                                 int64_t* bytes_out);
bf_status bf_yvv_forward(const float* f, int64_t H, int64_t W, float T, float sigma_r,
                         float sigma_s, float* out, const bf_opts* opts);

/* Direct-window filter: the same eq. (BF)/(normalization) summed pixel by
 * pixel over the whole window, O((2R+1)^2) per pixel (the baseline the paper
 * compares its O(1) method with).  Same arguments as the forward. */
bf_status bf_direct_forward(const float* f, int64_t H, int64_t W, float T, float sigma_r,
                            const bf_spatial_spec* spatial_spec, float* out,
                            const bf_opts* opts);

/* Debug helper for the precondition of Sec. 2.1 (intensities in [0, T], which
 * keeps the raised-cosine kernel non-negative; the filters do not test it).
 * Writes to *count_dev (device memory, one uint32, caller-owned) the number
 * of pixels of the H x W device image f that lie outside [0, T] or are NaN.
 * Asynchronous on stream (a hipStream_t; NULL = the null stream): the count
 * is valid once the stream has reached this call.  BF_EINVAL for a NULL
 * pointer, a non-positive size or T not positive and finite. */
bf_status bf_check_range(const float* f, int64_t H, int64_t W, float T, uint32_t* count_dev,
                         void* stream);

/* ---- batches of images of different sizes and parameters ------------------
 * For callers that filter many images (e.g. the colour channels of Fig. 4 or
 * a training batch) in one launch.  A plan fixes the images' sizes and
 * parameters and owns every device table and workspace it needs.
 * bf_batch_bind attaches the caller's device buffers (host arrays of n device
 * pointers each; it uploads them synchronously and may not be called during
 * stream capture).  With target and grad_f non-NULL the batch computes, per
 * image, out = BF(f), the SSD loss sum((out - target)^2) (into loss[i] if loss
 * is non-NULL) and grad_f = d loss / d f; eta must then be non-NULL.  With
 * grad_f NULL only the forward runs.  bf_batch_launch enqueues the whole batch
 * on stream, in one of two evaluations (bf_batch_plan_create_ex): the
 * streamed passes over all images (a short fixed sequence of kernels), or one
 * persistent work-queue kernel of fused tiles (plus a tiny counter-reset
 * kernel): forward tiles first, longest first, then the per-image loss
 * reductions, then the adjoint tiles, each of which waits (bounded) until all
 * forward tiles of its image are done.  It allocates and synchronises
 * nothing, so it may be captured into a hipGraph and replayed.
 * bf_batch_check synchronises the device and reports BF_EDEVICE if a wait in
 * the last launch hit its bound (the results are then invalid).  Tile shapes
 * of the fused evaluation come from the descriptors; the timing-based tile
 * tuner that fills them (with a per-device cache file) is part of the Python
 * layer only, not of this ABI. */
typedef struct {
    int64_t H, W;
    float T, sigma_r;
    int32_t N;                   /* 0 = automatic degree */
    bf_spatial_spec spatial;
    int32_t tile_h, tile_w;      /* forward tile; 0 = library choice */
    int32_t bwd_tile_h, bwd_tile_w; /* adjoint tile; 0 = library choice */
    float trunc_tol;             /* as bf_opts.trunc_tol; 0 = every pair */
} bf_image_desc;

typedef struct bf_batch_plan bf_batch_plan;

bf_status bf_batch_plan_create(const bf_image_desc* descs, int32_t n, bf_batch_plan** plan);
/* path: BF_PATH_AUTO (bf_batch_plan_create) runs the batch through the
 * streamed passes when every image is within their limits (W + 2R <= 5184,
 * at most 256 cosine pairs, 32 (2R + nb) nb bytes <= 160 KiB for the column
 * pass's weight tables: R <= 638 with four boxes), else through the
 * persistent fused-tile kernel;
 * BF_PATH_FUSED and BF_PATH_STREAMED force one (BF_EUNSUPPORTED if an image
 * is outside the streamed passes' limits).  The streamed batch enqueues a
 * short sequence of kernels instead of one persistent kernel: the column
 * pass and then the row pass over all images (one launch per box count and
 * per line length), the loss and the adjoint's weights, then the adjoint's
 * two passes; it owns the column-filtered planes of every pair of every
 * image (16 bytes per pixel and pair) and ignores the tile fields. */
bf_status bf_batch_plan_create_ex(const bf_image_desc* descs, int32_t n, int32_t path,
                                  bf_batch_plan** plan);
bf_status bf_batch_bind(bf_batch_plan* plan, const float* const* f, const float* const* target,
                        float* const* out, float* const* eta, float* const* grad_f,
                        float* loss /* device, n floats, or NULL */);
bf_status bf_batch_launch(bf_batch_plan* plan, void* stream);
/* One stage of bf_batch_launch, for timing each of them on its own: on the
 * streamed passes 0 = forward column pass, 1 = forward row pass, 2 = loss and
 * the adjoint's weights, 3 = adjoint column pass, 4 = adjoint row pass
 * (stages without work for this binding enqueue nothing); the persistent
 * fused kernel has the single stage 0.  The stages of one step must be
 * enqueued in this order on one stream. */
bf_status bf_batch_launch_stage(bf_batch_plan* plan, int32_t stage, void* stream);
/* The evaluation the plan chose: BF_PATH_FUSED or BF_PATH_STREAMED (-1 for a
 * NULL plan). */
int32_t bf_batch_plan_path(const bf_batch_plan* plan);
bf_status bf_batch_check(bf_batch_plan* plan);
void bf_batch_plan_destroy(bf_batch_plan* plan);

const char* bf_status_string(bf_status s);
const char* bf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BF_TRIG_H */
