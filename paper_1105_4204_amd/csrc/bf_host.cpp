// Host-side parameter derivation and argument checking for the trigonometric
// bilateral filter: degree rule (Algorithm 1 steps 1-2), binomial cosine-pair
// coefficients (Sec. 2.3), iterated-box radii for a Gaussian spatial filter,
// validation and the thread-local error text.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "bf_internal.h"

namespace bf {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

// ceil((2T / (pi sigma_r))^2), i.e. ceil(rho^-2) with rho = gamma sigma_r and
// gamma = pi / 2T (Algorithm 1 steps 1-2, Sec. 2.5); at least 1.
static bf_status degree_rule(double T, double sigma_r, int32_t* N) {
    if (!(T > 0.0) || !(sigma_r > 0.0) || !isfinite(T) || !isfinite(sigma_r)) {
        set_error("T and sigma_r must be positive and finite (T=%g, sigma_r=%g)", T, sigma_r);
        return BF_EINVAL;
    }
    const double rho = (M_PI / (2.0 * T)) * sigma_r;
    const double n = ceil(1.0 / (rho * rho));
    if (n > (double)BF_MAX_DEGREE) {
        set_error("degree %.0f needed for sigma_r=%g, T=%g exceeds BF_MAX_DEGREE=%d", n, sigma_r,
                  T, BF_MAX_DEGREE);
        return BF_ERANGE;
    }
    *N = n < 1.0 ? 1 : (int32_t)n;
    return BF_OK;
}

// c[q] for the pair m_q = (N mod 2) + 2q of cos^N = sum_n 2^-N C(N,n) e^{j(2n-N)t}:
// the terms n and N-n share frequency |2n-N| and fold to 2 * 2^-N C(N,n) cos(m t).
// log C(N,n) - N log 2 in long double, then exp and one rounding to float.
static void pair_coeffs(int32_t N, float* c, int32_t* n_out) {
    const int32_t np = N / 2 + 1;
    const long double lN = lgammal((long double)N + 1.0L) - (long double)N * logl(2.0L);
    for (int32_t q = 0; q < np; ++q) {
        const int32_t m = (N & 1) + 2 * q;
        const int32_t n = (N - m) / 2;
        const long double lc =
            lN - lgammal((long double)n + 1.0L) - lgammal((long double)(N - n) + 1.0L);
        long double v = expl(lc);
        if (m > 0) v *= 2.0L;
        c[q] = (float)v;
    }
    *n_out = np;
}

bf_status make_range(double T, double sigma_r, int32_t N_req, RangeParams* rp) {
    int32_t Nmin = 0;
    bf_status st = degree_rule(T, sigma_r, &Nmin);
    if (st != BF_OK) return st;
    int32_t N = Nmin;
    if (N_req != 0) {
        if (N_req < 0 || N_req > BF_MAX_DEGREE) {
            set_error("degree N=%d outside [1, %d]", N_req, BF_MAX_DEGREE);
            return BF_ERANGE;
        }
        if (N_req < Nmin) {
            set_error("degree N=%d below the bound ceil((2T/(pi sigma_r))^2)=%d: the raised "
                      "cosine would turn negative inside [-T, T]", N_req, Nmin);
            return BF_ERANGE;
        }
        N = N_req;
    }
    rp->N = N;
    rp->odd = N & 1;
    rp->alpha = 1.0 / (sigma_r * sqrt((double)N));
    rp->center = (float)(0.5 * T);
    int32_t np = 0;
    pair_coeffs(N, rp->chat, &np);
    // Coefficients that round to exactly zero in float contribute exactly zero.
    while (np > 1 && rp->chat[np - 1] == 0.0f) --np;
    rp->npairs = np;
    return BF_OK;
}

// Composite 1-D kernel of the boxes (integer weights): its centre value k0 and
// its mass.  w(0) = k0^2 and sum w = mass^2 for the separable 2-D kernel.
static void kernel_centre_and_mass(const SpatialParams& sp, double* k0, double* mass) {
    const int L = 2 * sp.R + 1;
    double k[2 * BF_MAX_BOXES * BF_MAX_RADIUS + 1] = {0.0};
    double t[2 * BF_MAX_BOXES * BF_MAX_RADIUS + 1];
    k[sp.R] = 1.0;
    for (int b = 0; b < sp.nb; ++b) {
        for (int i = 0; i < L; ++i) {
            double acc = 0.0;
            for (int d = -sp.r[b]; d <= sp.r[b]; ++d)
                if (i - d >= 0 && i - d < L) acc += k[i - d];
            t[i] = acc;
        }
        for (int i = 0; i < L; ++i) k[i] = t[i];
    }
    double m = 1.0;
    for (int b = 0; b < sp.nb; ++b) m *= (double)(2 * sp.r[b] + 1);
    *k0 = k[sp.R];
    *mass = m;
}

// Term truncation with an error bound.  Dropping the pairs q >= Q removes the
// binomial mass delta = sum_{q >= Q} c_q, and |phi - phi_Q| <= delta on the
// whole range.  With num and den the centred sums (|g| <= T/2, so |num/den|
// <= T/2) and den >= w(0) (the centre pixel always counts with phi(0) = 1,
// and phi >= 0 when N meets the degree bound):
//     |out_Q - out| <= T delta sum(w) / (w(0) - delta sum(w)).
// Keeps the fewest pairs whose bound is <= tol (tol in the units of f).
bf_status truncate_pairs(RangeParams* rp, const SpatialParams& sp, double T, double tol,
                         double* bound_out) {
    double k0 = 0.0, mass = 0.0;
    kernel_centre_and_mass(sp, &k0, &mass);
    return truncate_pairs_km(rp, k0, mass, T, tol, bound_out);
}

// The same for any separable kernel given by its 1-D centre tap k0 and mass.
bf_status truncate_pairs_km(RangeParams* rp, double k0, double mass, double T, double tol,
                            double* bound_out) {
    if (!(tol > 0.0) || !isfinite(tol)) {
        set_error("truncation tolerance must be positive and finite (%g)", tol);
        return BF_EINVAL;
    }
    const double w0 = k0 * k0, sw = mass * mass;
    // exact tail masses in long double, from the same log-binomials as the
    // coefficients
    const int32_t N = rp->N, np = N / 2 + 1;
    long double tail[kMaxPairs + 1];
    tail[np] = 0.0L;
    const long double lN = lgammal((long double)N + 1.0L) - (long double)N * logl(2.0L);
    for (int32_t q = np - 1; q >= 0; --q) {
        const int32_t m = (N & 1) + 2 * q;
        const int32_t n = (N - m) / 2;
        long double v = expl(lN - lgammal((long double)n + 1.0L) -
                             lgammal((long double)(N - n) + 1.0L));
        if (m > 0) v *= 2.0L;
        tail[q] = tail[q + 1] + v;
    }
    auto bound = [&](int32_t Q) {
        const double d = (double)tail[Q];
        const double den = w0 - d * sw;
        return den > 0.0 ? T * d * sw / den : INFINITY;
    };
    int32_t Q = 1;
    while (Q < rp->npairs && !(bound(Q) <= tol)) ++Q;
    if (Q < rp->npairs) rp->npairs = Q;
    if (bound_out) *bound_out = Q < np ? bound(Q) : 0.0;
    return BF_OK;
}

bf_status make_spatial(const bf_spatial_spec* spec, SpatialParams* sp) {
    if (!spec) {
        set_error("spatial_spec is NULL");
        return BF_EINVAL;
    }
    if (spec->n_boxes < 1 || spec->n_boxes > BF_MAX_BOXES) {
        set_error("n_boxes=%d outside [1, %d]", spec->n_boxes, BF_MAX_BOXES);
        return BF_EINVAL;
    }
    sp->nb = spec->n_boxes;
    sp->R = 0;
    for (int i = 0; i < BF_MAX_BOXES; ++i) sp->r[i] = 0;
    for (int i = 0; i < spec->n_boxes; ++i) {
        if (spec->radius[i] < 0) {
            set_error("radius[%d]=%d is negative", i, spec->radius[i]);
            return BF_EINVAL;
        }
        if (spec->radius[i] > BF_MAX_RADIUS) {
            set_error("radius[%d]=%d exceeds BF_MAX_RADIUS=%d", i, spec->radius[i], BF_MAX_RADIUS);
            return BF_ERANGE;
        }
        sp->r[i] = spec->radius[i];
        sp->R += spec->radius[i];
    }
    return BF_OK;
}

bf_status check_image(const void* p, int64_t H, int64_t W, const char* name) {
    if (!p) {
        set_error("%s is NULL", name);
        return BF_EINVAL;
    }
    if (H <= 0 || W <= 0) {
        set_error("image size %lld x %lld must be positive", (long long)H, (long long)W);
        return BF_EINVAL;
    }
    if (H > (1 << 20) || W > (1 << 20) || H * W > (int64_t)1 << 31) {
        set_error("image size %lld x %lld too large", (long long)H, (long long)W);
        return BF_ERANGE;
    }
    return BF_OK;
}

bool overlaps(const void* a, const void* b, int64_t bytes) {
    return overlaps(a, bytes, b, bytes);
}

bool overlaps(const void* a, int64_t abytes, const void* b, int64_t bbytes) {
    if (!a || !b) return false;
    const char* pa = (const char*)a;
    const char* pb = (const char*)b;
    return pa < pb + bbytes && pb < pa + abytes;
}

// Recursive Gaussian of Young and van Vliet (Signal Processing 44(2), 1995),
// the spatial filter of the paper's own experiments (Sec. 3).  From the
// requested standard deviation s: q by their fit, then the third-order
// denominator b0..b3 and the gain B that makes the DC response one; each
// line is filtered by
//   causal      w[n] = B u[n] + a1 w[n-1] + a2 w[n-2] + a3 w[n-3]
//   anticausal  v[n] = B w[n] + a1 v[n+1] + a2 v[n+2] + a3 v[n+3]
// with a_i = b_i / b0.  Zero-extended data before the first sample leave the
// causal pass with zero state.  Past the last sample the data are zero too,
// but the causal output is not: it rings on as w[n] = sum a_i w[n-i], and the
// anticausal pass must start from where that ringing leaves it.  M maps the
// causal state at the end of a line, (w[n-1], w[n-2], w[n-3]), to the
// anticausal start (v[n], v[n+1], v[n+2]); it is found here in FP64 by running
// the ringing of each unit state until it has died out and filtering it back.
bf_status make_yvv(double s, YvvParams* yp) {
    if (!(s >= kYvvMinSigma) || !(s <= kYvvMaxSigma)) {
        set_error("sigma_s=%g outside [%g, %g]", s, kYvvMinSigma, kYvvMaxSigma);
        return BF_ERANGE;
    }
    const double q = (s >= 2.5) ? 0.98711 * s - 0.96330 : 3.97156 - 4.14554 * sqrt(1.0 - 0.26891 * s);
    const double b0 = 1.57825 + 2.44413 * q + 1.4281 * q * q + 0.422205 * q * q * q;
    const double b1 = 2.44413 * q + 2.85619 * q * q + 1.26661 * q * q * q;
    const double b2 = -(1.4281 * q * q + 1.26661 * q * q * q);
    const double b3 = 0.422205 * q * q * q;
    const double a[3] = {b1 / b0, b2 / b0, b3 / b0};
    const double B = 1.0 - (b1 + b2 + b3) / b0;
    const int K = 200 * (int)ceil(q) + 2000;   // the ringing decays by e per ~q samples at worst
    double* w = (double*)malloc((size_t)K * sizeof(double));
    if (!w) {
        set_error("host allocation failed");
        return BF_ENOMEM;
    }
    for (int k = 0; k < 3; ++k) {
        double w1 = k == 0, w2 = k == 1, w3 = k == 2;   // w[n-1], w[n-2], w[n-3]
        for (int i = 0; i < K; ++i) {
            const double x = a[0] * w1 + a[1] * w2 + a[2] * w3;
            w[i] = x;
            w3 = w2;
            w2 = w1;
            w1 = x;
        }
        double v1 = 0.0, v2 = 0.0, v3 = 0.0;
        for (int i = K - 1; i >= 0; --i) {
            const double x = B * w[i] + a[0] * v1 + a[1] * v2 + a[2] * v3;
            v3 = v2;
            v2 = v1;
            v1 = x;
            if (i <= 2) yp->M[3 * i + k] = x;   // row i: v[n+i]
        }
    }
    // centre tap of the two-pass impulse response (its mass is one)
    {
        const int L = K / 2;
        double* line = (double*)calloc((size_t)(2 * L + 1), sizeof(double));
        if (!line) {
            free(w);
            set_error("host allocation failed");
            return BF_ENOMEM;
        }
        line[L] = 1.0;
        double w1 = 0.0, w2 = 0.0, w3 = 0.0;
        for (int i = 0; i <= 2 * L; ++i) {
            const double x = B * line[i] + a[0] * w1 + a[1] * w2 + a[2] * w3;
            line[i] = x;
            w3 = w2;
            w2 = w1;
            w1 = x;
        }
        double v1 = 0.0, v2 = 0.0, v3 = 0.0;
        for (int i = 2 * L; i >= L; --i) {
            const double x = B * line[i] + a[0] * v1 + a[1] * v2 + a[2] * v3;
            v3 = v2;
            v2 = v1;
            v1 = x;
        }
        yp->k0 = v1;
        free(line);
    }
    free(w);
    yp->B = B;
    yp->a1 = a[0];
    yp->a2 = a[1];
    yp->a3 = a[2];
    return BF_OK;
}

}  // namespace bf

using namespace bf;

extern "C" {

bf_status bf_range_truncate(int32_t N, double T, const bf_spatial_spec* spatial_spec,
                            double tol, int32_t* npairs_out, double* bound_out) {
    if (!npairs_out) {
        set_error("npairs_out is NULL");
        return BF_EINVAL;
    }
    if (N < 1 || N > BF_MAX_DEGREE || !(T > 0.0)) {
        set_error("need 1 <= N <= %d and T > 0 (N=%d, T=%g)", BF_MAX_DEGREE, N, T);
        return BF_ERANGE;
    }
    SpatialParams sp;
    bf_status st = make_spatial(spatial_spec, &sp);
    if (st != BF_OK) return st;
    RangeParams rp;
    rp.N = N;
    rp.odd = N & 1;
    int32_t np = 0;
    pair_coeffs(N, rp.chat, &np);
    while (np > 1 && rp.chat[np - 1] == 0.0f) --np;
    rp.npairs = np;
    st = truncate_pairs(&rp, sp, T, tol, bound_out);
    if (st != BF_OK) return st;
    *npairs_out = rp.npairs;
    return BF_OK;
}

bf_status bf_yvv_coeffs(double sigma_s, double* coeffs_out) {
    if (!coeffs_out) {
        set_error("coeffs_out is NULL");
        return BF_EINVAL;
    }
    YvvParams yp;
    const bf_status st = make_yvv(sigma_s, &yp);
    if (st != BF_OK) return st;
    coeffs_out[0] = yp.B;
    coeffs_out[1] = yp.a1;
    coeffs_out[2] = yp.a2;
    coeffs_out[3] = yp.a3;
    return BF_OK;
}

bf_status bf_range_degree(double T, double sigma_r, int32_t* N_out) {
    if (!N_out) {
        set_error("N_out is NULL");
        return BF_EINVAL;
    }
    return degree_rule(T, sigma_r, N_out);
}

bf_status bf_range_coeffs(int32_t N, float* c_out, int32_t cap, int32_t* n_out) {
    if (!c_out || !n_out) {
        set_error("c_out / n_out is NULL");
        return BF_EINVAL;
    }
    if (N < 0 || N > BF_MAX_DEGREE) {
        set_error("N=%d outside [0, %d]", N, BF_MAX_DEGREE);
        return BF_ERANGE;
    }
    if (cap < N / 2 + 1) {
        set_error("capacity %d < %d coefficients", cap, N / 2 + 1);
        return BF_EINVAL;
    }
    pair_coeffs(N, c_out, n_out);
    return BF_OK;
}

bf_status bf_spatial_gaussian(double sigma_s, int32_t n_boxes, bf_spatial_spec* out) {
    if (!out) {
        set_error("out is NULL");
        return BF_EINVAL;
    }
    if (!(sigma_s >= 0.0) || !isfinite(sigma_s) || n_boxes < 1 || n_boxes > BF_MAX_BOXES) {
        set_error("sigma_s=%g must be >= 0 and n_boxes=%d in [1, %d]", sigma_s, n_boxes,
                  BF_MAX_BOXES);
        return BF_EINVAL;
    }
    // A box of odd width w has variance (w^2 - 1)/12; n boxes of ideal width
    // w* = sqrt(12 sigma^2/n + 1) reach sigma^2.  Use m boxes of the largest odd
    // width wl <= w* and n - m of wl + 2, with m the rounded solution of
    // m (wl^2-1)/12 + (n-m) ((wl+2)^2-1)/12 = sigma^2.
    const double wideal = sqrt(12.0 * sigma_s * sigma_s / n_boxes + 1.0);
    int wl = (int)floor(wideal);
    if (wl % 2 == 0) --wl;
    if (wl < 1) wl = 1;
    const int wu = wl + 2;
    const double mideal = (n_boxes * (double)wl * wl + 4.0 * n_boxes * wl + 3.0 * n_boxes -
                           12.0 * sigma_s * sigma_s) / (4.0 * wl + 4.0);
    int m = (int)floor(mideal + 0.5);
    if (m < 0) m = 0;
    if (m > n_boxes) m = n_boxes;
    out->n_boxes = n_boxes;
    for (int i = 0; i < BF_MAX_BOXES; ++i) out->radius[i] = 0;
    for (int i = 0; i < n_boxes; ++i) out->radius[i] = ((i < m ? wl : wu) - 1) / 2;
    for (int i = 0; i < n_boxes; ++i) {
        if (out->radius[i] > BF_MAX_RADIUS) {
            set_error("sigma_s=%g needs radius %d > BF_MAX_RADIUS", sigma_s, out->radius[i]);
            return BF_ERANGE;
        }
    }
    return BF_OK;
}

const char* bf_status_string(bf_status s) {
    switch (s) {
        case BF_OK: return "BF_OK";
        case BF_EINVAL: return "BF_EINVAL: invalid argument";
        case BF_ERANGE: return "BF_ERANGE: parameter out of range";
        case BF_ENOMEM: return "BF_ENOMEM: out of memory";
        case BF_EDEVICE: return "BF_EDEVICE: HIP runtime error";
        case BF_ECAPTURE: return "BF_ECAPTURE: not allowed during stream capture";
        case BF_EUNSUPPORTED: return "BF_EUNSUPPORTED: not supported by this library";
    }
    return "unknown bf_status";
}

const char* bf_last_error(void) { return g_err; }

}  // extern "C"
