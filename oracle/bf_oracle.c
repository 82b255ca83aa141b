/*
 * FP64 reference implementation of the accelerated shiftable bilateral filter
 * (K. N. Chaudhury, "Acceleration of the shiftable O(1) algorithm for
 * bilateral filtering and non-local means").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test-suite, the package smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header, table
 * or constant with the GPU library.
 *
 * Everything is plain double precision and follows the paper's steps in the
 * paper's order.  OpenMP only splits loops over independent rows/columns/
 * pixels; no sum is reordered, so results do not depend on the thread count.
 *
 * Readings of passages the paper leaves open:
 *  - Sec. 2, Prop. 2.1 and Algorithm 1 step 4 print "f(x) - max f(x-y)", which
 *    is never positive.  The proof (|t| = max(t,-t) and the symmetry of the
 *    window) gives T = max_x [max_{y} f(x-y) - f(x)]; that is what is computed.
 *  - The window Omega is the square |y1|,|y2| <= R (the separable max filter
 *    needs a square); windows are clipped at the image border.
 *  - Eq. (trunc) prints the upper summation limit as M+1; the printed Fig. 1
 *    numbers (N=263, M=111, 42 terms) come out of "the smallest M whose
 *    cumulative mass sum_{n<=M} exceeds eps/2" with eps = 0.01.  That reading
 *    is used; the mass dropped on each side is then at most eps/2.
 *  - Algorithm 2 step 3 leaves N real; it is rounded to the nearest integer
 *    (this reproduces every entry of Table 1) and is at least 1.
 *  - Eq. (Chernoff) leaves M real; it is rounded down and clamped at 0.
 *  - The sigma_r bands of Algorithm 2 step 4 are in 8-bit intensity units; for
 *    other ranges sigma_r is rescaled by 255/range before the comparison.
 *  - For non-integer T (float images) the order uses ceil(T).
 *  - Where the denominator (f2) is not positive the output is the input pixel.
 *  - The paper does not name its O(1) spatial smoother.  Three operators are
 *    provided, all separable and zero-extended outside the image:
 *      FIR: taps exp(-j^2 / (2 sigma_s^2)) for |j| <= R;
 *      IIR: the recursive Gaussian of Young and van Vliet (Signal Processing
 *           44, 1995), causal pass then anticausal pass, applied to the
 *           zero-extended signal;
 *      BOX: the constant spatial filter of Section 4 (the comparison with
 *           integral histograms), unit taps for |j| <= R, R its radius.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_MEM 2

/* ------------------------------------------------------------------------ */
/* Appendix (MAX-FILTER): running maxima with a reset every W = 2R+1 samples. */
/* Output i is the maximum of in[i-R .. i+R] clipped to [0, n).              */
/* ------------------------------------------------------------------------ */
int orc_maxfilter_1d(const double *in, long n, long R, double *out)
{
    if (n < 1 || R < 0) return ORC_ERR_ARG;
    const long W = 2 * R + 1;
    /* padded sequence g: R copies of -inf, the signal, then -inf up to a
     * multiple of W so that the partitions are all of length W. */
    long np = n + 2 * R;
    long nblk = (np + W - 1) / W;
    long len = nblk * W;
    double *g = (double *)malloc(sizeof(double) * len);
    double *l = (double *)malloc(sizeof(double) * len);
    double *r = (double *)malloc(sizeof(double) * len);
    if (!g || !l || !r) { free(g); free(l); free(r); return ORC_ERR_MEM; }
    for (long e = 0; e < len; e++) {
        long i = e - R;
        g[e] = (i >= 0 && i < n) ? in[i] : -INFINITY;
    }
    for (long k = 0; k < nblk; k++) {
        long a = k * W;
        l[a] = g[a];                                  /* left running max   */
        for (long e = a + 1; e < a + W; e++) l[e] = g[e] > l[e - 1] ? g[e] : l[e - 1];
        r[a + W - 1] = g[a + W - 1];                  /* right running max  */
        for (long e = a + W - 2; e >= a; e--) r[e] = g[e] > r[e + 1] ? g[e] : r[e + 1];
    }
    /* window of output i is g[i .. i+2R]: max(r[i], l[i+2R]) */
    for (long i = 0; i < n; i++) {
        double a = r[i], b = l[i + 2 * R];
        out[i] = a > b ? a : b;
    }
    free(g); free(l); free(r);
    return ORC_OK;
}

/* Algorithm 1: row MAX-FILTER, then column MAX-FILTER, then
 * T = max_x [Mx(x) - f(x)]  (Prop. 2.1, sign as read from its proof). */
int orc_range_T(const double *f, long H, long W, long R, double *Mx, double *T_out)
{
    if (H < 1 || W < 1 || R < 0) return ORC_ERR_ARG;
    double *m = (double *)malloc(sizeof(double) * H * W);
    double *own = NULL;
    if (!Mx) { own = (double *)malloc(sizeof(double) * H * W); Mx = own; }
    if (!m || !Mx) { free(m); free(own); return ORC_ERR_MEM; }
    int err = 0;
#pragma omp parallel for schedule(static) reduction(|:err)
    for (long y = 0; y < H; y++) err |= orc_maxfilter_1d(f + y * W, W, R, m + y * W);
#pragma omp parallel reduction(|:err)
    {
        double *col = (double *)malloc(sizeof(double) * H);
        double *res = (double *)malloc(sizeof(double) * H);
        if (!col || !res) err |= ORC_ERR_MEM;
        else {
#pragma omp for schedule(static)
            for (long x = 0; x < W; x++) {
                for (long y = 0; y < H; y++) col[y] = m[y * W + x];
                err |= orc_maxfilter_1d(col, H, R, res);
                for (long y = 0; y < H; y++) Mx[y * W + x] = res[y];
            }
        }
        free(col); free(res);
    }
    double T = 0.0;
    for (long p = 0; p < H * W; p++) {
        double d = Mx[p] - f[p];
        if (d > T) T = d;
    }
    *T_out = T;
    free(m); free(own);
    return err;
}

/* ------------------------------------------------------------------------ */
/* Section 1.3 and Section 3: order N and truncation M                       */
/* ------------------------------------------------------------------------ */

/* Algorithm 2 step 3: N = 0.405 (T / sigma_r)^2, rounded, at least 1. */
int orc_order(double T, double sigma_r)
{
    double v = 0.405 * (T / sigma_r) * (T / sigma_r);
    long n = (long)floor(v + 0.5);
    if (n < 1) n = 1;
    return (int)n;
}

/* Binomial weight 2^-N C(N, n) of eq. (expansion), through log-gamma. */
double orc_coef(int N, int n)
{
    if (n < 0 || n > N) return 0.0;
    double lg = lgamma((double)N + 1.0) - lgamma((double)n + 1.0) - lgamma((double)(N - n) + 1.0);
    return exp(lg - (double)N * log(2.0));
}

/* Eq. (trunc), read as: smallest M with sum_{n=0}^{M} 2^-N C(N,n) > eps/2. */
int orc_trunc_exact(int N, double eps)
{
    double s = 0.0;
    for (int m = 0; m <= N; m++) {
        s += orc_coef(N, m);
        if (s > 0.5 * eps) return m;
    }
    return N / 2;
}

/* Eq. (Chernoff): M = (N - sqrt(4 N log(2/eps))) / 2, rounded down, >= 0. */
int orc_trunc_chernoff(int N, double eps)
{
    double v = 0.5 * ((double)N - sqrt(4.0 * (double)N * log(2.0 / eps)));
    long m = (long)floor(v);
    if (m < 0) m = 0;
    return (int)m;
}

/* Algorithm 2 step 4: the rule depends on sigma_r (8-bit units). */
int orc_trunc_rule(int N, double sigma_r8, double eps)
{
    int M;
    if (sigma_r8 > 40.0) M = 0;
    else if (sigma_r8 > 10.0) M = orc_trunc_exact(N, eps);
    else M = orc_trunc_chernoff(N, eps);
    if (M > N / 2) M = N / 2;
    return M;
}

/* Eq. (RCconv): the raised cosine cos^N(s / (sqrt(N) sigma_r)). */
double orc_phi(double s, int N, double sigma_r)
{
    return pow(cos(s / (sqrt((double)N) * sigma_r)), (double)N);
}

/* Eq. (approx): the truncated series, terms n = M .. N-M. */
double orc_phi_eps(double s, int N, int M, double sigma_r)
{
    double acc = 0.0, scale = sqrt((double)N) * sigma_r;
    for (int n = M; n <= N - M; n++)
        acc += orc_coef(N, n) * cos((double)(2 * n - N) * s / scale);
    return acc;
}

/* ------------------------------------------------------------------------ */
/* Spatial operators (eq. (GF)), one dimension, zero extension               */
/* ------------------------------------------------------------------------ */

/* FIR: out[i] = sum_{|j|<=R, 0<=i+j<n} exp(-j^2/(2 sigma^2)) in[i+j] */
static void fir_1d(const double *in, long n, double sigma, long R, double *out)
{
    for (long i = 0; i < n; i++) {
        double acc = 0.0;
        for (long j = -R; j <= R; j++) {
            long k = i + j;
            if (k < 0 || k >= n) continue;
            acc += exp(-(double)(j * j) / (2.0 * sigma * sigma)) * in[k];
        }
        out[i] = acc;
    }
}

/* BOX: out[i] = sum_{|j|<=R, 0<=i+j<n} in[i+j] */
static void box_1d(const double *in, long n, long R, double *out)
{
    for (long i = 0; i < n; i++) {
        double acc = 0.0;
        for (long j = -R; j <= R; j++) {
            long k = i + j;
            if (k < 0 || k >= n) continue;
            acc += in[k];
        }
        out[i] = acc;
    }
}

/* Young & van Vliet (1995) coefficients, valid for sigma >= 0.5. */
void orc_yvv_coefs(double sigma, double *coef /* [4]: B, b1/b0, b2/b0, b3/b0 */)
{
    double q = sigma >= 2.5 ? 0.98711 * sigma - 0.96330
                            : 3.97156 - 4.14554 * sqrt(1.0 - 0.26891 * sigma);
    double q2 = q * q, q3 = q2 * q;
    double b0 = 1.57825 + 2.44413 * q + 1.4281 * q2 + 0.422205 * q3;
    double b1 = 2.44413 * q + 2.85619 * q2 + 1.26661 * q3;
    double b2 = -(1.4281 * q2 + 1.26661 * q3);
    double b3 = 0.422205 * q3;
    coef[0] = 1.0 - (b1 + b2 + b3) / b0;
    coef[1] = b1 / b0;
    coef[2] = b2 / b0;
    coef[3] = b3 / b0;
}

/* Number of zeros appended after the signal so that the anticausal pass of the
 * zero-extended signal starts from a state below 1e-20 of the signal level. */
static long yvv_pad(double sigma) { return (long)ceil(40.0 * sigma) + 64; }

/* IIR: causal pass w[i] = B x[i] + a1 w[i-1] + a2 w[i-2] + a3 w[i-3] from rest,
 * then anticausal pass y[i] = B w[i] + a1 y[i+1] + a2 y[i+2] + a3 y[i+3],
 * over the signal followed by zeros (the zero extension). */
static void iir_1d(const double *in, long n, const double *cf, long pad, double *buf_w,
                   double *buf_y, double *out)
{
    const double B = cf[0], a1 = cf[1], a2 = cf[2], a3 = cf[3];
    long L = n + pad;
    for (long i = 0; i < L; i++) {
        double x = i < n ? in[i] : 0.0;
        double w1 = i >= 1 ? buf_w[i - 1] : 0.0;
        double w2 = i >= 2 ? buf_w[i - 2] : 0.0;
        double w3 = i >= 3 ? buf_w[i - 3] : 0.0;
        buf_w[i] = B * x + a1 * w1 + a2 * w2 + a3 * w3;
    }
    for (long i = L - 1; i >= 0; i--) {
        double y1 = i + 1 < L ? buf_y[i + 1] : 0.0;
        double y2 = i + 2 < L ? buf_y[i + 2] : 0.0;
        double y3 = i + 3 < L ? buf_y[i + 3] : 0.0;
        buf_y[i] = B * buf_w[i] + a1 * y1 + a2 * y2 + a3 * y3;
    }
    for (long i = 0; i < n; i++) out[i] = buf_y[i];
}

#define ORC_OP_FIR 0
#define ORC_OP_IIR 1
#define ORC_OP_BOX 2

/* 1-D operator along a strided line (used for the tests of the operators). */
int orc_blur_1d(const double *in, long n, int op, double sigma, long R, double *out)
{
    if (n < 1 || sigma <= 0.0) return ORC_ERR_ARG;
    if (op == ORC_OP_FIR) { fir_1d(in, n, sigma, R, out); return ORC_OK; }
    if (op == ORC_OP_BOX) { box_1d(in, n, R, out); return ORC_OK; }
    if (op != ORC_OP_IIR || sigma < 0.5) return ORC_ERR_ARG;
    double cf[4];
    orc_yvv_coefs(sigma, cf);
    long pad = yvv_pad(sigma);
    double *bw = (double *)malloc(sizeof(double) * (n + pad));
    double *by = (double *)malloc(sizeof(double) * (n + pad));
    if (!bw || !by) { free(bw); free(by); return ORC_ERR_MEM; }
    iir_1d(in, n, cf, pad, bw, by, out);
    free(bw); free(by);
    return ORC_OK;
}

/* Separable 2-D operator, in place: every row, then every column. */
int orc_blur_2d(double *img, long H, long W, int op, double sigma, long R)
{
    if (H < 1 || W < 1 || sigma <= 0.0) return ORC_ERR_ARG;
    if (op == ORC_OP_IIR && sigma < 0.5) return ORC_ERR_ARG;
    if (op != ORC_OP_FIR && op != ORC_OP_IIR && op != ORC_OP_BOX) return ORC_ERR_ARG;
    double cf[4] = {0, 0, 0, 0};
    long pad = 0;
    if (op == ORC_OP_IIR) { orc_yvv_coefs(sigma, cf); pad = yvv_pad(sigma); }
    long nmax = (H > W ? H : W);
    int err = 0;
#pragma omp parallel reduction(|:err)
    {
        double *line = (double *)malloc(sizeof(double) * nmax);
        double *res = (double *)malloc(sizeof(double) * nmax);
        double *bw = (double *)malloc(sizeof(double) * (nmax + pad));
        double *by = (double *)malloc(sizeof(double) * (nmax + pad));
        if (!line || !res || !bw || !by) err |= ORC_ERR_MEM;
        else {
#pragma omp for schedule(static)
            for (long y = 0; y < H; y++) {
                double *row = img + y * W;
                if (op == ORC_OP_FIR) fir_1d(row, W, sigma, R, res);
                else if (op == ORC_OP_BOX) box_1d(row, W, R, res);
                else iir_1d(row, W, cf, pad, bw, by, res);
                memcpy(row, res, sizeof(double) * W);
            }
#pragma omp for schedule(static)
            for (long x = 0; x < W; x++) {
                for (long y = 0; y < H; y++) line[y] = img[y * W + x];
                if (op == ORC_OP_FIR) fir_1d(line, H, sigma, R, res);
                else if (op == ORC_OP_BOX) box_1d(line, H, R, res);
                else iir_1d(line, H, cf, pad, bw, by, res);
                for (long y = 0; y < H; y++) img[y * W + x] = res[y];
            }
        }
        free(line); free(res); free(bw); free(by);
    }
    return err;
}

/* ------------------------------------------------------------------------ */
/* SHIFTABLE-BF (Section 1.2, steps 1-4) with the truncated kernel (approx)   */
/* ------------------------------------------------------------------------ */
/*
 * For every kept term n = M..N-M, with omega_n = (2n-N)/(sqrt(N) sigma_r) and
 * weight c_n = 2^-N C(N,n), the shift identity
 *     cos(omega (f(y) - f(x))) = cos(omega f(y)) cos(omega f(x))
 *                              + sin(omega f(y)) sin(omega f(x))
 * gives the basis images f cos, f sin, cos, sin of omega f (step 2); each is
 * smoothed by the spatial operator (step 3); eqs. (f1), (f2) then assemble the
 * numerator P and the denominator Q (step 4).
 */
int orc_shiftable_bf(const double *f, long H, long W, int op, double sigma_s, long R,
                     int N, int M, double sigma_r, double *out, double *P, double *Q,
                     long *n_nonpos)
{
    if (H < 1 || W < 1 || N < 1 || M < 0 || 2 * M > N || sigma_r <= 0.0) return ORC_ERR_ARG;
    long HW = H * W;
    double *pl = (double *)malloc(sizeof(double) * HW * 4);
    double *ownP = NULL, *ownQ = NULL;
    if (!P) { ownP = (double *)malloc(sizeof(double) * HW); P = ownP; }
    if (!Q) { ownQ = (double *)malloc(sizeof(double) * HW); Q = ownQ; }
    if (!pl || !P || !Q) { free(pl); free(ownP); free(ownQ); return ORC_ERR_MEM; }
    for (long p = 0; p < HW; p++) { P[p] = 0.0; Q[p] = 0.0; }
    const double scale = sqrt((double)N) * sigma_r;
    int err = 0;
    for (int n = M; n <= N - M && !err; n++) {
        const double c = orc_coef(N, n);
        const double om = (double)(2 * n - N) / scale;
        double *Fc = pl, *Fs = pl + HW, *Gc = pl + 2 * HW, *Gs = pl + 3 * HW;
#pragma omp parallel for schedule(static)
        for (long p = 0; p < HW; p++) {
            double th = om * f[p];
            Gc[p] = cos(th);
            Gs[p] = sin(th);
            Fc[p] = f[p] * Gc[p];
            Fs[p] = f[p] * Gs[p];
        }
        for (int k = 0; k < 4 && !err; k++) err |= orc_blur_2d(pl + k * HW, H, W, op, sigma_s, R);
#pragma omp parallel for schedule(static)
        for (long p = 0; p < HW; p++) {
            double th = om * f[p];
            double co = cos(th), si = sin(th);
            P[p] += c * (co * Fc[p] + si * Fs[p]);
            Q[p] += c * (co * Gc[p] + si * Gs[p]);
        }
    }
    long bad = 0;
    for (long p = 0; p < HW; p++) {
        if (Q[p] > 0.0 && isfinite(Q[p]) && isfinite(P[p])) out[p] = P[p] / Q[p];
        else { out[p] = f[p]; bad++; }
    }
    if (n_nonpos) *n_nonpos = bad;
    free(pl); free(ownP); free(ownQ);
    return err;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2 (improved SHIFTABLE-BF)                                       */
/* ------------------------------------------------------------------------ */
int orc_algorithm2(const double *f, long H, long W, int op, double sigma_s, long R,
                   double sigma_r, double eps, double range, int t_local, double t_value,
                   double *out, double *T_out, int *N_out, int *M_out, long *n_nonpos)
{
    if (H < 1 || W < 1 || sigma_s <= 0.0 || sigma_r <= 0.0 || !(eps > 0.0 && eps < 1.0) ||
        range <= 0.0 || R < 0)
        return ORC_ERR_ARG;
    /* step 1: R is given by the caller (a factor of sigma_s) */
    /* step 2: T from Algorithm 1, or the global value */
    double T = t_value;
    if (t_local) {
        int e = orc_range_T(f, H, W, R, NULL, &T);
        if (e) return e;
    }
    double Tu = ceil(T);
    /* step 3 */
    int N = orc_order(Tu, sigma_r);
    /* step 4 */
    int M = orc_trunc_rule(N, sigma_r * 255.0 / range, eps);
    if (T_out) *T_out = T;
    if (N_out) *N_out = N;
    if (M_out) *M_out = M;
    /* steps 5-6 */
    return orc_shiftable_bf(f, H, W, op, sigma_s, R, N, M, sigma_r, out, NULL, NULL, n_nonpos);
}

/* Direct evaluation of eq. (BF) at chosen pixels with the truncated range
 * kernel phi_eps and the FIR (or BOX) spatial kernel on the clipped square
 * window:
 *   out(x) = sum_y w(y) phi_eps(f(x-y) - f(x)) f(x-y) / sum_y w(y) phi_eps(...)
 * Used for sampled parity at sizes where the full expansion is too slow. */
int orc_direct_at(const double *f, long H, long W, int op, double sigma_s, long R, int N, int M,
                  double sigma_r, const long *ys, const long *xs, long npts, double *out)
{
    if (H < 1 || W < 1 || R < 0 || N < 1 || M < 0 || 2 * M > N) return ORC_ERR_ARG;
    if (op != ORC_OP_FIR && op != ORC_OP_BOX) return ORC_ERR_ARG;
    double *w1 = (double *)malloc(sizeof(double) * (2 * R + 1));
    if (!w1) return ORC_ERR_MEM;
    for (long j = -R; j <= R; j++)
        w1[j + R] = op == ORC_OP_BOX ? 1.0 : exp(-(double)(j * j) / (2.0 * sigma_s * sigma_s));
#pragma omp parallel for schedule(dynamic)
    for (long t = 0; t < npts; t++) {
        long y0 = ys[t], x0 = xs[t];
        double fx = f[y0 * W + x0], num = 0.0, den = 0.0;
        for (long dy = -R; dy <= R; dy++) {
            long y = y0 + dy;
            if (y < 0 || y >= H) continue;
            for (long dx = -R; dx <= R; dx++) {
                long x = x0 + dx;
                if (x < 0 || x >= W) continue;
                double fy = f[y * W + x];
                double k = w1[dy + R] * w1[dx + R] * orc_phi_eps(fy - fx, N, M, sigma_r);
                num += k * fy;
                den += k;
            }
        }
        out[t] = den > 0.0 ? num / den : fx;
    }
    free(w1);
    return ORC_OK;
}

int orc_direct_fir_at(const double *f, long H, long W, double sigma_s, long R, int N, int M,
                      double sigma_r, const long *ys, const long *xs, long npts, double *out)
{
    return orc_direct_at(f, H, W, ORC_OP_FIR, sigma_s, R, N, M, sigma_r, ys, xs, npts, out);
}
