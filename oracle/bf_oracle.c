/*
 * FP64 reference oracle for the constant-time trigonometric bilateral filter
 * (Chaudhury, Sage, Unser: "Fast O(1) bilateral filtering using trigonometric
 * range kernels").
 *
 * THIS IS TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or helper with the HIP library: it is the plain
 * definition of the filter written out as a brute-force window sum, in double
 * precision, so that a reader can check it against the paper by eye.
 *
 * Definitions followed (paper section / equation):
 *  - Unbiased bilateral filter, eq. (BF) and eq. (normalization), Sec. 1:
 *        out(x) = sum_y w(y) phi(f(x-y) - f(x)) f(x-y)  /  eta(x)
 *        eta(x) = sum_y w(y) phi(f(x-y) - f(x))
 *    discretised on the pixel grid; the sums run over the support of w
 *    restricted to pixels inside the image (the auxiliary images are
 *    zero-extended outside the image, which is the same thing).
 *  - Range kernel: the raised cosine of Sec. 2.3, with the width control of
 *    Sec. 2.5 (eq. (convergence1)) and Algorithm 1 step 3:
 *        phi(s) = cos(alpha s)^N,   alpha = gamma / (rho sqrt(N)),
 *        gamma = pi / (2T), rho = gamma sigma_r   =>  alpha = 1/(sigma_r sqrt N).
 *    N = 0 is the degenerate kernel phi == 1 (pure spatial averaging).
 *  - Degree rule, Algorithm 1 step 2 / Sec. 2.5 (N >= (gamma sigma)^-2),
 *    read as the ceiling of (gamma sigma_r)^-2.
 *  - Spatial kernel w(dy,dx) = k(dy) k(dx) where k is the explicit discrete
 *    convolution of n unit-height boxes of widths 2 r_i + 1 (the O(1) box /
 *    iterated-box averaging of Sec. 2.1, eq. (averaging)).  The mass of w
 *    cancels in the ratio, so the unnormalised integer weights are used.
 *  - Gradient: exact derivative of out with respect to f for an upstream
 *    gradient G = dL/dout, using phi'(s) = -N alpha cos^(N-1)(alpha s)
 *    sin(alpha s):
 *      dL/df(z) = sum_x w(x-z) A(x) [phi'(f_z - f_x)(f_z - out_x) + phi(f_z - f_x)]
 *               - A(z) sum_y w(z-y) phi'(f_y - f_z)(f_y - out_z),   A = G/eta.
 *    (Differentiating eq. (BF)/(normalization) once; the neighbour term and
 *    the centre term are the two ways f(z) enters out(x).)
 *
 * Image layout: row-major H x W doubles, pixel (i, j) at f[i*W + j].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAX_BOXES 8

/* Number of OpenMP threads a parallel region of the oracle uses. */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Algorithm 1 steps 1-2: gamma = pi/2T, rho = gamma sigma_r,
 * N = ceil(rho^-2) = ceil((2T / (pi sigma_r))^2).  Returns -1 on bad input. */
int64_t oracle_range_degree(double T, double sigma_r)
{
    if (!(T > 0.0) || !(sigma_r > 0.0)) return -1;
    double gamma = M_PI / (2.0 * T);
    double rho = gamma * sigma_r;
    double n = ceil(1.0 / (rho * rho));
    if (n < 1.0) n = 1.0;
    return (int64_t)n;
}

/* The raised-cosine range kernel phi(s) = cos(alpha s)^N (Sec. 2.3, 2.5). */
double oracle_phi(double s, int64_t N, double sigma_r)
{
    if (N == 0) return 1.0;
    double alpha = 1.0 / (sigma_r * sqrt((double)N));
    return pow(cos(alpha * s), (double)N);
}

/* phi'(s) = -N alpha cos(alpha s)^(N-1) sin(alpha s). */
static double oracle_dphi(double s, int64_t N, double sigma_r)
{
    if (N == 0) return 0.0;
    double alpha = 1.0 / (sigma_r * sqrt((double)N));
    double c = cos(alpha * s);
    double cm = (N == 1) ? 1.0 : pow(c, (double)(N - 1));
    return -(double)N * alpha * cm * sin(alpha * s);
}

/* 1-D composite spatial kernel: explicit convolution of boxes of widths
 * 2 r_i + 1, all taps 1.  Writes 2R+1 weights, R = sum r_i.  Returns R, or -1. */
int64_t oracle_spatial_kernel(const int32_t* radii, int32_t n_boxes, double* k_out)
{
    if (n_boxes < 1 || n_boxes > ORACLE_MAX_BOXES) return -1;
    int64_t R = 0;
    for (int i = 0; i < n_boxes; ++i) {
        if (radii[i] < 0) return -1;
        R += radii[i];
    }
    int64_t len = 2 * R + 1;
    double* cur = (double*)calloc((size_t)len, sizeof(double));
    double* nxt = (double*)calloc((size_t)len, sizeof(double));
    /* start from a unit impulse at the centre and convolve with each box */
    cur[R] = 1.0;
    for (int b = 0; b < n_boxes; ++b) {
        int64_t r = radii[b];
        for (int64_t t = 0; t < len; ++t) {
            double s = 0.0;
            for (int64_t d = -r; d <= r; ++d) {
                int64_t u = t - d;
                if (u >= 0 && u < len) s += cur[u];
            }
            nxt[t] = s;
        }
        double* tmp = cur; cur = nxt; nxt = tmp;
    }
    memcpy(k_out, cur, (size_t)len * sizeof(double));
    free(cur);
    free(nxt);
    return R;
}

/* Direct window sum at one pixel (i, j): writes numerator and eta. */
static void pixel_sums(const double* f, int64_t H, int64_t W, int64_t i, int64_t j,
                       const double* k, int64_t R, int64_t N, double sigma_r,
                       double* num_out, double* eta_out)
{
    double fx = f[i * W + j];
    double num = 0.0, eta = 0.0;
    int64_t i0 = i - R < 0 ? 0 : i - R, i1 = i + R > H - 1 ? H - 1 : i + R;
    int64_t j0 = j - R < 0 ? 0 : j - R, j1 = j + R > W - 1 ? W - 1 : j + R;
    for (int64_t y = i0; y <= i1; ++y) {
        double ky = k[y - i + R];
        const double* row = f + y * W;
        for (int64_t x = j0; x <= j1; ++x) {
            double wgt = ky * k[x - j + R];
            double fy = row[x];
            double ph = oracle_phi(fy - fx, N, sigma_r);
            num += wgt * ph * fy;
            eta += wgt * ph;
        }
    }
    *num_out = num;
    *eta_out = eta;
}

static int check_args(const double* f, int64_t H, int64_t W, double sigma_r, int64_t N,
                      const int32_t* radii, int32_t n_boxes)
{
    if (!f || H <= 0 || W <= 0 || N < 0 || !radii) return -1;
    if (N > 0 && !(sigma_r > 0.0)) return -1;
    if (n_boxes < 1 || n_boxes > ORACLE_MAX_BOXES) return -1;
    for (int b = 0; b < n_boxes; ++b) if (radii[b] < 0) return -1;
    return 0;
}

/* Forward filter over the whole image (eq. (BF), (normalization)).
 * out and eta_out (optional) are H*W.  Returns 0, or -1 on bad arguments. */
int oracle_forward(const double* f, int64_t H, int64_t W, double sigma_r, int64_t N,
                   const int32_t* radii, int32_t n_boxes, double* out, double* eta_out)
{
    if (check_args(f, H, W, sigma_r, N, radii, n_boxes) || !out) return -1;
    int64_t R = 0;
    for (int b = 0; b < n_boxes; ++b) R += radii[b];
    double* k = (double*)malloc((size_t)(2 * R + 1) * sizeof(double));
    oracle_spatial_kernel(radii, n_boxes, k);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < H; ++i) {
        for (int64_t j = 0; j < W; ++j) {
            double num, eta;
            pixel_sums(f, H, W, i, j, k, R, N, sigma_r, &num, &eta);
            out[i * W + j] = num / eta;
            if (eta_out) eta_out[i * W + j] = eta;
        }
    }
    free(k);
    return 0;
}

/* Forward filter at a list of flat pixel indices idx[0..n): out[t], eta[t]. */
int oracle_forward_at(const double* f, int64_t H, int64_t W, double sigma_r, int64_t N,
                      const int32_t* radii, int32_t n_boxes, const int64_t* idx, int64_t n,
                      double* out, double* eta_out)
{
    if (check_args(f, H, W, sigma_r, N, radii, n_boxes) || !out || (n > 0 && !idx)) return -1;
    for (int64_t t = 0; t < n; ++t) if (idx[t] < 0 || idx[t] >= H * W) return -1;
    int64_t R = 0;
    for (int b = 0; b < n_boxes; ++b) R += radii[b];
    double* k = (double*)malloc((size_t)(2 * R + 1) * sizeof(double));
    oracle_spatial_kernel(radii, n_boxes, k);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < n; ++t) {
        double num, eta;
        pixel_sums(f, H, W, idx[t] / W, idx[t] % W, k, R, N, sigma_r, &num, &eta);
        out[t] = num / eta;
        if (eta_out) eta_out[t] = eta;
    }
    free(k);
    return 0;
}

/* Gradient dL/df at a list of pixels z = idx[t], for an upstream gradient G
 * given as a full H*W image.  out/eta of the pixels around each z are
 * recomputed here from f (never taken from a caller).  grad[t] receives
 * dL/df(z).  Returns 0, or -1. */
int oracle_grad_at(const double* f, int64_t H, int64_t W, double sigma_r, int64_t N,
                   const int32_t* radii, int32_t n_boxes, const double* G,
                   const int64_t* idx, int64_t n, double* grad)
{
    if (check_args(f, H, W, sigma_r, N, radii, n_boxes) || !G || !grad || (n > 0 && !idx))
        return -1;
    for (int64_t t = 0; t < n; ++t) if (idx[t] < 0 || idx[t] >= H * W) return -1;
    int64_t R = 0;
    for (int b = 0; b < n_boxes; ++b) R += radii[b];
    double* k = (double*)malloc((size_t)(2 * R + 1) * sizeof(double));
    oracle_spatial_kernel(radii, n_boxes, k);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < n; ++t) {
        int64_t zi = idx[t] / W, zj = idx[t] % W;
        double fz = f[idx[t]];
        int64_t i0 = zi - R < 0 ? 0 : zi - R, i1 = zi + R > H - 1 ? H - 1 : zi + R;
        int64_t j0 = zj - R < 0 ? 0 : zj - R, j1 = zj + R > W - 1 ? W - 1 : zj + R;
        double acc = 0.0;
        /* neighbour term: every centre x whose window holds z */
        for (int64_t xi = i0; xi <= i1; ++xi) {
            for (int64_t xj = j0; xj <= j1; ++xj) {
                double num_x, eta_x;
                pixel_sums(f, H, W, xi, xj, k, R, N, sigma_r, &num_x, &eta_x);
                double out_x = num_x / eta_x;
                double A = G[xi * W + xj] / eta_x;
                double fx = f[xi * W + xj];
                double wgt = k[zi - xi + R] * k[zj - xj + R];
                double s = fz - fx;
                acc += wgt * A * (oracle_dphi(s, N, sigma_r) * (fz - out_x)
                                  + oracle_phi(s, N, sigma_r));
            }
        }
        /* centre term: z as the pixel of interest */
        double num_z, eta_z;
        pixel_sums(f, H, W, zi, zj, k, R, N, sigma_r, &num_z, &eta_z);
        double out_z = num_z / eta_z;
        double Az = G[idx[t]] / eta_z;
        double c = 0.0;
        for (int64_t yi = i0; yi <= i1; ++yi) {
            for (int64_t yj = j0; yj <= j1; ++yj) {
                double fy = f[yi * W + yj];
                double wgt = k[yi - zi + R] * k[yj - zj + R];
                c += wgt * oracle_dphi(fy - fz, N, sigma_r) * (fy - out_z);
            }
        }
        grad[t] = acc - Az * c;
    }
    free(k);
    return 0;
}

/* Space-variant extension (Sec. 4, "Space-variant extension"): the spatial
 * kernel changes from pixel to pixel while the range kernel stays fixed.
 * Here the kernel at pixel x is the unit box of half-width rmap[x] in both
 * directions, so
 *     out(x) = sum_{|y - x|_inf <= r(x)} phi(f(y) - f(x)) f(y) / eta(x),
 *     eta(x) = sum_{same y} phi(f(y) - f(x)),
 * with y restricted to the image (the zero extension of the auxiliary images
 * leaves only in-image pixels in both sums).  Written out directly, one
 * window per pixel; rmap is H*W with entries >= 0.  Returns 0, or -1. */
int oracle_forward_sv(const double* f, int64_t H, int64_t W, double sigma_r, int64_t N,
                      const int32_t* rmap, double* out, double* eta_out)
{
    if (!f || !rmap || !out || H <= 0 || W <= 0 || N < 0) return -1;
    if (N > 0 && !(sigma_r > 0.0)) return -1;
    for (int64_t p = 0; p < H * W; ++p) if (rmap[p] < 0) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < H; ++i) {
        for (int64_t j = 0; j < W; ++j) {
            int64_t r = rmap[i * W + j];
            double fx = f[i * W + j];
            int64_t i0 = i - r < 0 ? 0 : i - r, i1 = i + r > H - 1 ? H - 1 : i + r;
            int64_t j0 = j - r < 0 ? 0 : j - r, j1 = j + r > W - 1 ? W - 1 : j + r;
            double num = 0.0, eta = 0.0;
            for (int64_t y = i0; y <= i1; ++y) {
                for (int64_t x = j0; x <= j1; ++x) {
                    double fy = f[y * W + x];
                    double ph = oracle_phi(fy - fx, N, sigma_r);
                    num += ph * fy;
                    eta += ph;
                }
            }
            out[i * W + j] = num / eta;
            if (eta_out) eta_out[i * W + j] = eta;
        }
    }
    return 0;
}

/* ---- Recursive Gaussian spatial kernel (Sec. 3: the paper's own code averages
 * in space with the recursive O(1) Gaussian of its image-processing reference,
 * i.e. the filter of Young and van Vliet, Signal Processing 44(2), 1995).
 *
 * Published recipe, for a target standard deviation s >= 0.5:
 *   q  = 0.98711 s - 0.96330                      (s >= 2.5)
 *   q  = 3.97156 - 4.14554 sqrt(1 - 0.26891 s)     (0.5 <= s < 2.5)
 *   b0 = 1.57825 + 2.44413 q + 1.4281 q^2 + 0.422205 q^3
 *   b1 = 2.44413 q + 2.85619 q^2 + 1.26661 q^3
 *   b2 = -(1.4281 q^2 + 1.26661 q^3)
 *   b3 = 0.422205 q^3
 *   B  = 1 - (b1 + b2 + b3) / b0
 * causal pass      w[n] = B u[n] + (b1 w[n-1] + b2 w[n-2] + b3 w[n-3]) / b0,
 * anticausal pass  v[n] = B w[n] + (b1 v[n+1] + b2 v[n+2] + b3 v[n+3]) / b0.
 * On an infinite line of zero-extended data the two passes are a linear,
 * shift-invariant, symmetric filter; the spatial kernel of the bilateral
 * filter is its impulse response in x times the same in y. */

/* Writes B, b1/b0, b2/b0, b3/b0.  Returns 0, or -1 for s < 0.5. */
int oracle_yvv_coeffs(double s, double* c_out)
{
    if (!(s >= 0.5) || !c_out) return -1;
    double q = (s >= 2.5) ? 0.98711 * s - 0.96330 : 3.97156 - 4.14554 * sqrt(1.0 - 0.26891 * s);
    double b0 = 1.57825 + 2.44413 * q + 1.4281 * q * q + 0.422205 * q * q * q;
    double b1 = 2.44413 * q + 2.85619 * q * q + 1.26661 * q * q * q;
    double b2 = -(1.4281 * q * q + 1.26661 * q * q * q);
    double b3 = 0.422205 * q * q * q;
    c_out[0] = 1.0 - (b1 + b2 + b3) / b0;
    c_out[1] = b1 / b0;
    c_out[2] = b2 / b0;
    c_out[3] = b3 / b0;
    return 0;
}

/* The two passes over a finite line u[0..n) with zero state before the
 * first sample (causal) and after the last (anticausal).  out may equal u. */
int oracle_yvv_line(const double* u, int64_t n, double s, double* out)
{
    double c[4];
    if (!u || !out || n <= 0 || oracle_yvv_coeffs(s, c)) return -1;
    double* w = (double*)malloc((size_t)n * sizeof(double));
    double w1 = 0.0, w2 = 0.0, w3 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double x = c[0] * u[i] + c[1] * w1 + c[2] * w2 + c[3] * w3;
        w[i] = x;
        w3 = w2; w2 = w1; w1 = x;
    }
    double v1 = 0.0, v2 = 0.0, v3 = 0.0;
    for (int64_t i = n - 1; i >= 0; --i) {
        double x = c[0] * w[i] + c[1] * v1 + c[2] * v2 + c[3] * v3;
        out[i] = x;
        v3 = v2; v2 = v1; v1 = x;
    }
    free(w);
    return 0;
}

/* Impulse response k[d + D], |d| <= D, of the two passes on an infinite
 * line: the impulse sits in the middle of a zero line long enough (pad on
 * both sides) that the response has decayed below double precision at its
 * ends.  Returns 0, or -1. */
int oracle_yvv_kernel(double s, int64_t D, double* k_out)
{
    double c[4];
    if (D < 0 || !k_out || oracle_yvv_coeffs(s, c)) return -1;
    int64_t pad = (int64_t)(60.0 * s) + 200;
    int64_t n = 2 * (D + pad) + 1;
    double* line = (double*)calloc((size_t)n, sizeof(double));
    line[D + pad] = 1.0;
    oracle_yvv_line(line, n, s, line);
    memcpy(k_out, line + pad, (size_t)(2 * D + 1) * sizeof(double));
    free(line);
    return 0;
}

/* Bilateral filter with an explicit separable spatial kernel
 * w(dy, dx) = k[dy + D] k[dx + D], |dy|, |dx| <= D: the same direct window
 * sums as oracle_forward, at the flat pixel indices idx[0..n) (all pixels when
 * idx is NULL, n = H W). */
int oracle_forward_kernel(const double* f, int64_t H, int64_t W, double sigma_r, int64_t N,
                          const double* k, int64_t D, const int64_t* idx, int64_t n,
                          double* out, double* eta_out)
{
    if (!f || !k || !out || H <= 0 || W <= 0 || N < 0 || D < 0) return -1;
    if (N > 0 && !(sigma_r > 0.0)) return -1;
    if (!idx && n != H * W) return -1;
    for (int64_t t = 0; idx && t < n; ++t) if (idx[t] < 0 || idx[t] >= H * W) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < n; ++t) {
        int64_t p = idx ? idx[t] : t;
        double num, eta;
        pixel_sums(f, H, W, p / W, p % W, k, D, N, sigma_r, &num, &eta);
        out[t] = num / eta;
        if (eta_out) eta_out[t] = eta;
    }
    return 0;
}
