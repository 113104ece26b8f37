/*
 * tm_oracle.c -- CPU oracle for multi-receptive-field tone mapping with integral images
 * and integral histograms (Yang et al., "Mobile-end Tone Mapping based on Integral Image
 * and Integral Histogram", arXiv 2102.01289).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's CPU-baseline
 * leg may load this library.  It shares no code, header or table with the HIP library.
 *
 * Plain, slow, obviously correct loops.  Floating point is FP64; the integral images are
 * double-double (about 106 significant bits), so box sums are exact to far below any
 * tolerance used against the GPU.  Counts are uint64.  Build with -ffp-contract=off so the
 * error-free transformations below are not fused away.
 *
 * Conventions (the readings of the paper that fix them are listed with each function):
 *   images are row-major [H][W]; pixel (x, y) is column x, row y;
 *   integral tables are (H+1) x (W+1): entry [y+1][x+1] holds the sum over x' <= x,
 *   y' <= y, and row 0 / column 0 are zero (the "x = -1" / "y = -1" corners).
 *
 * Threads (orc_set_threads, default 1): the per-pixel loops of orc_forward and orc_backward
 * may run on several OpenMP threads, each pixel computed exactly as on one thread; every
 * sum across pixels is then taken serially in pixel order from per-pixel terms, so results
 * are bitwise the same for any thread count.  Used only to time the oracle on all host cores.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int g_threads = 1;

/* Number of OpenMP threads of the per-pixel loops (>= 1). */
void orc_set_threads(int n) { g_threads = n > 0 ? n : 1; }

/* ------------------------------------------------------------------ double-double */
typedef struct { double hi, lo; } dd_t;

/* Knuth's TwoSum: s + e == a + b exactly. */
static void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double bv = x - a;
    double av = x - bv;
    *s = x;
    *e = (a - av) + (b - bv);
}

/* Dekker's FastTwoSum, valid when |a| >= |b| or a == 0. */
static void fast_two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    *s = x;
    *e = b - (x - a);
}

static dd_t dd_add(dd_t a, dd_t b)
{
    double s1, s2, t1, t2;
    two_sum(a.hi, b.hi, &s1, &s2);
    two_sum(a.lo, b.lo, &t1, &t2);
    s2 += t1;
    fast_two_sum(s1, s2, &s1, &s2);
    s2 += t2;
    fast_two_sum(s1, s2, &s1, &s2);
    dd_t r = {s1, s2};
    return r;
}

static dd_t dd_neg(dd_t a)
{
    dd_t r = {-a.hi, -a.lo};
    return r;
}

static dd_t dd_from(double a)
{
    dd_t r = {a, 0.0};
    return r;
}

/* ------------------------------------------------------------------ Eq. 11 */
/* Luminance i = 0.2126 R + 0.7152 G + 0.0722 B (Section III, Eq. 11).
 * Reading: the coefficients are rounded to FP32 and the sum is evaluated left to right in
 * FP32 with fused multiply-adds: i = fma(0.0722, B, fma(0.7152, G, 0.2126 * R)).
 * rgb is planar [3][H][W]. */
void orc_luminance(const float *rgb, int64_t H, int64_t W, float *lum)
{
    const int64_t np = H * W;
    const float *R = rgb, *G = rgb + np, *B = rgb + 2 * np;
    for (int64_t p = 0; p < np; ++p) {
        float t = 0.2126f * R[p];
        t = fmaf(0.7152f, G[p], t);
        lum[p] = fmaf(0.0722f, B[p], t);
    }
}

/* ------------------------------------------------------------------ bins (Eq. 7) */
/* Equal-width bins of the log image (Section II-A, Eq. 7 and the text after Eq. 9).
 * edges[0..n-2] are the ascending FP32 bin edges in the linear domain; a pixel belongs to
 * bin b = #{k : lum >= edges[k-1]}, k = 1..n-1, so bins are half-open [e_k, e_{k+1}). */
void orc_bins(const float *lum, int64_t np, const float *edges, int n, int32_t *bins)
{
    for (int64_t p = 0; p < np; ++p) {
        int32_t b = 0;
        for (int k = 1; k < n; ++k)
            if (lum[p] >= edges[k - 1])
                b += 1;
        bins[p] = b;
    }
}

/* ------------------------------------------------------------------ Eq. 8 */
/* Integral histogram: per-bin indicator planes h_k (Eq. 7) and their integral images H_k
 * (Eq. 8), built as a row prefix then a column prefix of each indicator plane.
 * cumulative == 0: out holds n planes H_k, k = 0..n-1.
 * cumulative != 0: out holds n-1 planes G_k = sum_{j<k} H_j, k = 1..n-1 (formed by adding
 * the per-bin planes, so it follows from Eq. 8 directly).
 * Each plane is (H+1) x (W+1) uint64 with a zero row 0 and column 0. */
void orc_integral_histogram(const int32_t *bins, int64_t H, int64_t W, int n, int cumulative,
                            uint64_t *out)
{
    const int64_t ld = W + 1, ps = (H + 1) * (W + 1);
    const int planes = cumulative ? n - 1 : n;
    memset(out, 0, (size_t)planes * (size_t)ps * sizeof(uint64_t));
    uint64_t *hk = (uint64_t *)malloc((size_t)ps * sizeof(uint64_t));
    for (int k = 0; k < n; ++k) {
        memset(hk, 0, (size_t)ps * sizeof(uint64_t));
        for (int64_t y = 0; y < H; ++y) {          /* row prefix of h_k */
            uint64_t run = 0;
            for (int64_t x = 0; x < W; ++x) {
                run += (bins[y * W + x] == k) ? 1u : 0u;
                hk[(y + 1) * ld + (x + 1)] = run;
            }
        }
        for (int64_t x = 0; x < W; ++x)             /* column prefix */
            for (int64_t y = 1; y < H; ++y)
                hk[(y + 1) * ld + (x + 1)] += hk[y * ld + (x + 1)];
        if (!cumulative) {
            memcpy(out + (size_t)k * ps, hk, (size_t)ps * sizeof(uint64_t));
        } else {
            for (int kk = k + 1; kk < n; ++kk) {    /* H_k contributes to G_kk for kk > k */
                uint64_t *g = out + (size_t)(kk - 1) * ps;
                for (int64_t i = 0; i < ps; ++i)
                    g[i] += hk[i];
            }
        }
    }
    free(hk);
}

/* ------------------------------------------------------------------ Eq. 5 */
/* Integral image I(x, y) = sum_{x'<=x, y'<=y} i(x', y') (Eq. 5) of v (square == 0) or of
 * v^2 (square != 0), in double-double: a row prefix then a column prefix.  v^2 of an FP32
 * value is exact in FP64.  Output (H+1) x (W+1) hi/lo planes with zero row 0, column 0. */
void orc_integral_image(const float *v, int64_t H, int64_t W, int square, double *hi,
                        double *lo)
{
    const int64_t ld = W + 1;
    for (int64_t x = 0; x <= W; ++x) { hi[x] = 0.0; lo[x] = 0.0; }
    for (int64_t y = 0; y < H; ++y) {
        dd_t run = dd_from(0.0);
        hi[(y + 1) * ld] = 0.0;
        lo[(y + 1) * ld] = 0.0;
        for (int64_t x = 0; x < W; ++x) {
            double a = (double)v[y * W + x];
            if (square)
                a = a * a;
            run = dd_add(run, dd_from(a));
            hi[(y + 1) * ld + x + 1] = run.hi;
            lo[(y + 1) * ld + x + 1] = run.lo;
        }
    }
    for (int64_t x = 1; x <= W; ++x)
        for (int64_t y = 2; y <= H; ++y) {
            dd_t up = {hi[(y - 1) * ld + x], lo[(y - 1) * ld + x]};
            dd_t me = {hi[y * ld + x], lo[y * ld + x]};
            dd_t r = dd_add(me, up);
            hi[y * ld + x] = r.hi;
            lo[y * ld + x] = r.lo;
        }
}

/* Double-double SAT of an FP64 plane (used by the backward oracle). */
static void sat_dd_f64(const double *a, int64_t H, int64_t W, dd_t *out)
{
    const int64_t ld = W + 1;
    for (int64_t x = 0; x <= W; ++x) out[x] = dd_from(0.0);
    for (int64_t y = 0; y < H; ++y) {
        dd_t run = dd_from(0.0);
        out[(y + 1) * ld] = dd_from(0.0);
        for (int64_t x = 0; x < W; ++x) {
            run = dd_add(run, dd_from(a[y * W + x]));
            out[(y + 1) * ld + x + 1] = run;
        }
    }
    for (int64_t x = 1; x <= W; ++x)
        for (int64_t y = 2; y <= H; ++y)
            out[y * ld + x] = dd_add(out[y * ld + x], out[(y - 1) * ld + x]);
}

/* ------------------------------------------------------------------ windows */
/* Receptive field of radius (rx, ry) centred on (x, y), as Algorithm 1 indexes it:
 * x- = x - (rx + 1), x+ = x + rx, likewise in y.  Reading: the window is clamped to the
 * image (x- >= -1, x+ <= W-1, ...), and the pixel count is that of the clamped window.
 * The box is x- < x' <= x+, y- < y' <= y+ as in Eq. 6. */
typedef struct { int64_t xm, xp, ym, yp; } win_t;

static win_t window_of(int64_t x, int64_t y, int64_t W, int64_t H, int64_t rx, int64_t ry)
{
    win_t w;
    w.xm = x - (rx + 1); if (w.xm < -1) w.xm = -1;
    w.xp = x + rx;       if (w.xp > W - 1) w.xp = W - 1;
    w.ym = y - (ry + 1); if (w.ym < -1) w.ym = -1;
    w.yp = y + ry;       if (w.yp > H - 1) w.yp = H - 1;
    return w;
}

/* Eq. 6 / Eq. 9: I(A) + I(C) - I(B) - I(D) with A = (x-, y-), B = (x+, y-), C = (x+, y+),
 * D = (x-, y+), on a table with a zero row 0 / column 0 (index shift by one). */
static dd_t box_dd(const dd_t *t, int64_t ld, win_t w)
{
    dd_t A = t[(w.ym + 1) * ld + (w.xm + 1)];
    dd_t B = t[(w.ym + 1) * ld + (w.xp + 1)];
    dd_t C = t[(w.yp + 1) * ld + (w.xp + 1)];
    dd_t D = t[(w.yp + 1) * ld + (w.xm + 1)];
    return dd_add(dd_add(A, C), dd_neg(dd_add(B, D)));
}

static uint64_t box_u64(const uint64_t *t, int64_t ld, win_t w)
{
    uint64_t A = t[(w.ym + 1) * ld + (w.xm + 1)];
    uint64_t B = t[(w.ym + 1) * ld + (w.xp + 1)];
    uint64_t C = t[(w.yp + 1) * ld + (w.xp + 1)];
    uint64_t D = t[(w.yp + 1) * ld + (w.xm + 1)];
    return A + C - B - D;
}

/* ------------------------------------------------------------------ per-scale terms */
/* One receptive field's contribution at one pixel, from the window's histogram f_k and
 * its sums S1 = sum v, S2 = sum v^2:
 *   Eq. 1: P = (1/T) sum_{k < b} f_k with T = sum_k f_k and b the centre pixel's bin
 *          (strict "<", so the centre's own bin is excluded);
 *   Eq. 2: L_j = min L_d + (max L_d - min L_d) P;
 *   Eq. 10 (reading): the population variance S2/N - (S1/N)^2, clamped at zero;
 *   Eq. 4: W_j = var / (var + eps). */
typedef struct { double L, P, var, W, S1, N; int clamped; } scale_t;

static scale_t scale_terms(const uint64_t *f, int n, int b, double S1, double S2, double N,
                           double eps, double ldmin, double ldmax)
{
    scale_t r;
    uint64_t T = 0, below = 0;
    for (int k = 0; k < n; ++k) {
        T += f[k];
        if (k < b)
            below += f[k];
    }
    r.P = (double)below / (double)T;
    r.L = ldmin + (ldmax - ldmin) * r.P;
    double m = S1 / N;
    double var = S2 / N - m * m;
    r.clamped = !(var > 0.0);
    r.var = var > 0.0 ? var : 0.0;
    r.W = r.var / (r.var + eps);
    r.S1 = S1;
    r.N = N;
    return r;
}

/* Eq. 3: L = sum_j W_j L_j / sum_j W_j.  Reading: when every weight is zero (all windows
 * flat) the fused value is the plain mean of the L_j. */
static double fuse(const scale_t *sc, int s, double *D_out, double *Pbar_out)
{
    double num = 0.0, den = 0.0, pn = 0.0, lsum = 0.0, psum = 0.0;
    for (int j = 0; j < s; ++j) {
        num += sc[j].W * sc[j].L;
        pn += sc[j].W * sc[j].P;
        den += sc[j].W;
        lsum += sc[j].L;
        psum += sc[j].P;
    }
    *D_out = den;
    if (den > 0.0) {
        *Pbar_out = pn / den;
        return num / den;
    }
    *Pbar_out = psum / s;
    return lsum / s;
}

/* ------------------------------------------------------------------ tables bundle */
typedef struct {
    int64_t H, W, ld;
    int n;
    int32_t *bins;
    uint64_t *hist;   /* n per-bin planes, (H+1)(W+1) each */
    dd_t *s1, *s2;    /* integral images of v and v^2 */
} tables_t;

static void tables_free(tables_t *t)
{
    free(t->bins); free(t->hist); free(t->s1); free(t->s2);
    memset(t, 0, sizeof(*t));
}

/* The image whose window variance Eq. 10 takes: the luminance itself (linear), or, with
 * var_log set, its natural logarithm l = ln(max(v, FLT_MIN)) in FP64 (the log-domain
 * alternative of Section II-A's "integral image of i and i^2"). */
static double var_image_px(float v, int var_log)
{
    if (!var_log)
        return (double)v;
    const double m = (double)v > (double)FLT_MIN ? (double)v : (double)FLT_MIN;
    return log(m);
}

static int tables_build(const float *v, int64_t H, int64_t W, const float *edges, int n,
                        int var_log, tables_t *t)
{
    memset(t, 0, sizeof(*t));
    t->H = H; t->W = W; t->ld = W + 1; t->n = n;
    const int64_t ps = (H + 1) * (W + 1);
    t->bins = (int32_t *)malloc((size_t)(H * W) * sizeof(int32_t));
    t->hist = (uint64_t *)malloc((size_t)n * (size_t)ps * sizeof(uint64_t));
    t->s1 = (dd_t *)malloc((size_t)ps * sizeof(dd_t));
    t->s2 = (dd_t *)malloc((size_t)ps * sizeof(dd_t));
    double *hi = (double *)malloc((size_t)ps * sizeof(double));
    double *lo = (double *)malloc((size_t)ps * sizeof(double));
    if (!t->bins || !t->hist || !t->s1 || !t->s2 || !hi || !lo) {
        free(hi); free(lo); tables_free(t);
        return -1;
    }
    orc_bins(v, H * W, edges, n, t->bins);
    orc_integral_histogram(t->bins, H, W, n, 0, t->hist);
    if (!var_log) {
        orc_integral_image(v, H, W, 0, hi, lo);
        for (int64_t i = 0; i < ps; ++i) { t->s1[i].hi = hi[i]; t->s1[i].lo = lo[i]; }
        orc_integral_image(v, H, W, 1, hi, lo);
        for (int64_t i = 0; i < ps; ++i) { t->s2[i].hi = hi[i]; t->s2[i].lo = lo[i]; }
        free(hi); free(lo);
        return 0;
    }
    free(hi); free(lo);
    /* Eq. 5 of l and l^2, both in FP64, accumulated in double-double */
    double *a = (double *)malloc((size_t)(H * W) * sizeof(double));
    if (!a) { tables_free(t); return -1; }
    for (int64_t i = 0; i < H * W; ++i) a[i] = var_image_px(v[i], 1);
    sat_dd_f64(a, H, W, t->s1);
    for (int64_t i = 0; i < H * W; ++i) a[i] = a[i] * a[i];
    sat_dd_f64(a, H, W, t->s2);
    free(a);
    return 0;
}

static void pixel_scales(const tables_t *t, int64_t x, int64_t y, int s, const int32_t *rx,
                         const int32_t *ry, double eps, double ldmin, double ldmax,
                         scale_t *sc, uint64_t *f)
{
    const int64_t ps = (t->H + 1) * (t->W + 1);
    const int b = t->bins[y * t->W + x];
    for (int j = 0; j < s; ++j) {
        win_t w = window_of(x, y, t->W, t->H, rx[j], ry[j]);
        for (int k = 0; k < t->n; ++k)                          /* Eq. 9 */
            f[k] = box_u64(t->hist + (size_t)k * ps, t->ld, w);
        dd_t b1 = box_dd(t->s1, t->ld, w);                      /* Eq. 6 */
        dd_t b2 = box_dd(t->s2, t->ld, w);
        double N = (double)((w.xp - w.xm) * (w.yp - w.ym));
        sc[j] = scale_terms(f, t->n, b, b1.hi + b1.lo, b2.hi + b2.lo, N, eps, ldmin, ldmax);
    }
}

/* ------------------------------------------------------------------ forward */
/* The whole method on one luminance image v [H][W] (Sections II and II-A):
 * bins (Eq. 7), integral histogram (Eq. 8), integral images of v and v^2 (Eq. 5), then for
 * every pixel and every receptive field j: Eq. 9 histogram, Eq. 1 CDF, Eq. 2 tone value,
 * Eq. 6 sums, Eq. 10 variance, Eq. 4 weight; finally the Eq. 3 fusion.
 * var_log: take Eq. 10's variance of l = ln(max(v, FLT_MIN)) instead of v (the bins are
 * those of v either way).
 * Optional per-scale outputs (each s x H x W, nullable): Lj, Wj, varj.
 * Returns 0, or -1 if memory could not be allocated. */
int orc_forward(const float *v, int64_t H, int64_t W, const float *edges, int n, int s,
                const int32_t *rx, const int32_t *ry, double eps, double ldmin, double ldmax,
                int var_log, double *L, double *Lj, double *Wj, double *varj)
{
    tables_t t;
    if (n < 1 || n > 256 || s < 1 || s > 16)
        return -1;
    if (tables_build(v, H, W, edges, n, var_log, &t))
        return -1;
    const int64_t np = H * W;
#pragma omp parallel for num_threads(g_threads) schedule(dynamic, 16)
    for (int64_t y = 0; y < H; ++y) {
        scale_t sc[16];
        uint64_t f[256];
        for (int64_t x = 0; x < W; ++x) {
            pixel_scales(&t, x, y, s, rx, ry, eps, ldmin, ldmax, sc, f);
            double D, Pbar;
            L[y * W + x] = fuse(sc, s, &D, &Pbar);
            for (int j = 0; j < s; ++j) {
                if (Lj) Lj[j * np + y * W + x] = sc[j].L;
                if (Wj) Wj[j * np + y * W + x] = sc[j].W;
                if (varj) varj[j * np + y * W + x] = sc[j].var;
            }
        }
    }
    tables_free(&t);
    return 0;
}

/* Same method for a list of pixels, with every window histogram and window sum taken
 * directly over the window's pixels (no integral tables): the brute-force definition of
 * Eq. 1-4 and 10, used to pin orc_forward and to check sampled pixels of large images.
 * pix holds flat indices y*W + x. */
int orc_forward_direct(const float *v, int64_t H, int64_t W, const float *edges, int n, int s,
                       const int32_t *rx, const int32_t *ry, double eps, double ldmin,
                       double ldmax, int var_log, const int64_t *pix, int64_t npix, double *L)
{
    uint64_t *f = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    if (!f)
        return -1;
    scale_t sc[16];
    for (int64_t q = 0; q < npix; ++q) {
        const int64_t x = pix[q] % W, y = pix[q] / W;
        int32_t b;
        orc_bins(&v[y * W + x], 1, edges, n, &b);
        for (int j = 0; j < s; ++j) {
            win_t w = window_of(x, y, W, H, rx[j], ry[j]);
            memset(f, 0, (size_t)n * sizeof(uint64_t));
            dd_t a1 = dd_from(0.0), a2 = dd_from(0.0);
            for (int64_t yy = w.ym + 1; yy <= w.yp; ++yy)
                for (int64_t xx = w.xm + 1; xx <= w.xp; ++xx) {
                    const float vv = v[yy * W + xx];
                    int32_t bb;
                    orc_bins(&vv, 1, edges, n, &bb);
                    f[bb] += 1;
                    const double q = var_image_px(vv, var_log);
                    a1 = dd_add(a1, dd_from(q));
                    a2 = dd_add(a2, dd_from(q * q));
                }
            double N = (double)((w.xp - w.xm) * (w.yp - w.ym));
            sc[j] = scale_terms(f, n, b, a1.hi + a1.lo, a2.hi + a2.lo, N, eps, ldmin, ldmax);
        }
        double D, Pbar;
        L[q] = fuse(sc, s, &D, &Pbar);
    }
    free(f);
    return 0;
}

/* ------------------------------------------------------------------ backward */
/* Gradient of sum_p g(p) L(p) with respect to the luminance v and the scalars
 * (eps, min L_d, max L_d), derived from Eq. 1-4, 6 and 10:
 *   the histogram terms are piecewise constant in v (their derivative is zero almost
 *   everywhere) and the bin edges are held fixed, so v enters only through the variances;
 *   dL/dW_j = (L_j - L)/D with D = sum_j W_j;  dW_j/dvar_j = eps/(var_j + eps)^2;
 *   dvar_j/dS2_j = 1/N_j,  dvar_j/dS1_j = -2 S1_j/N_j^2;  dS1_j(p)/dv(q) = [q in win_j(p)],
 *   dS2_j(p)/dv(q) = 2 v(q) [q in win_j(p)].
 * With a_j(p) = g(p) (L_j - L)/D eps/(var_j + eps)^2 (zero when var_j was clamped, or when
 * D = 0), A1_j = -2 a_j S1_j / N_j^2 and A2_j = a_j / N_j:
 *   dv(q) = sum_j sum_{p : q in win_j(p)} (A1_j(p) + 2 v(q) A2_j(p)).
 * q lies in the clamped window of p exactly when p lies in the clamped window of q (both
 * are |p - q| <= r per axis inside the image), so the inner sum is the same clamped box sum
 * applied to the planes A1_j, A2_j; it is evaluated with a double-double integral image.
 * Scalars: dL/deps = sum_j (L_j - L)/D * (-var_j/(var_j + eps)^2),
 *          dL/dmin L_d = 1 - Pbar, dL/dmax L_d = Pbar, Pbar = sum_j W_j P_j / D.
 * grad_params = {d/deps, d/dmin L_d, d/dmax L_d}.
 * var_log: the log-domain variant (Eq. 10 of l = ln(max(v, FLT_MIN)); the bins stay those of
 * v).  The same derivation holds with l in place of v, which gives dL/dl(q); the chain rule
 * through the logarithm then gives dv(q) = dL/dl(q) / v(q) where v(q) > FLT_MIN, and 0 where
 * the floor is taken (the floor is a constant there).  Returns 0 or -1 (allocation). */
int orc_backward(const float *v, int64_t H, int64_t W, const float *edges, int n, int s,
                 const int32_t *rx, const int32_t *ry, double eps, double ldmin, double ldmax,
                 int var_log, const double *g, double *grad_v, double *grad_params)
{
    tables_t t;
    if (n < 1 || n > 256 || s < 1 || s > 16)
        return -1;
    if (tables_build(v, H, W, edges, n, var_log, &t))
        return -1;
    const int64_t np = H * W, ld = W + 1, ps = (H + 1) * (W + 1);
    double *A1 = (double *)malloc((size_t)s * (size_t)np * sizeof(double));
    double *A2 = (double *)malloc((size_t)s * (size_t)np * sizeof(double));
    dd_t *sat = (dd_t *)malloc((size_t)ps * sizeof(dd_t));
    /* per-pixel terms of the scalar gradients, summed below in pixel order */
    double *te = (double *)malloc((size_t)s * (size_t)np * sizeof(double));
    double *tmin = (double *)malloc((size_t)np * sizeof(double));
    double *tmax = (double *)malloc((size_t)np * sizeof(double));
    unsigned char *dpos = (unsigned char *)malloc((size_t)np);
    if (!A1 || !A2 || !sat || !te || !tmin || !tmax || !dpos) {
        free(A1); free(A2); free(sat); free(te); free(tmin); free(tmax); free(dpos);
        tables_free(&t);
        return -1;
    }
#pragma omp parallel for num_threads(g_threads) schedule(dynamic, 16)
    for (int64_t y = 0; y < H; ++y) {
        scale_t sc[16];
        uint64_t f[256];
        for (int64_t x = 0; x < W; ++x) {
            const int64_t p = y * W + x;
            pixel_scales(&t, x, y, s, rx, ry, eps, ldmin, ldmax, sc, f);
            double D, Pbar;
            double Lp = fuse(sc, s, &D, &Pbar);
            tmin[p] = g[p] * (1.0 - Pbar);
            tmax[p] = g[p] * Pbar;
            dpos[p] = D > 0.0;
            for (int j = 0; j < s; ++j) {
                double a = 0.0;
                te[j * np + p] = 0.0;
                if (D > 0.0) {
                    double dLdW = (sc[j].L - Lp) / D;
                    double den = sc[j].var + eps;
                    te[j * np + p] = g[p] * dLdW * (-sc[j].var / (den * den));
                    if (!sc[j].clamped)
                        a = g[p] * dLdW * eps / (den * den);
                }
                A1[j * np + p] = -2.0 * a * sc[j].S1 / (sc[j].N * sc[j].N);
                A2[j * np + p] = a / sc[j].N;
            }
        }
    }
    double geps = 0.0, gmin = 0.0, gmax = 0.0;
    for (int64_t p = 0; p < np; ++p) {
        gmin += tmin[p];
        gmax += tmax[p];
        if (dpos[p])
            for (int j = 0; j < s; ++j)
                geps += te[j * np + p];
    }
    for (int64_t p = 0; p < np; ++p)
        grad_v[p] = 0.0;
    for (int j = 0; j < s; ++j) {
        for (int pass = 0; pass < 2; ++pass) {
            sat_dd_f64(pass == 0 ? A1 + j * np : A2 + j * np, H, W, sat);
#pragma omp parallel for num_threads(g_threads) schedule(static)
            for (int64_t y = 0; y < H; ++y)
                for (int64_t x = 0; x < W; ++x) {
                    win_t w = window_of(x, y, W, H, rx[j], ry[j]);
                    dd_t bx = box_dd(sat, ld, w);
                    double val = bx.hi + bx.lo;
                    if (pass == 1)
                        val *= 2.0 * var_image_px(v[y * W + x], var_log);
                    grad_v[y * W + x] += val;
                }
        }
    }
    if (var_log)   /* d l / d v */
        for (int64_t p = 0; p < np; ++p)
            grad_v[p] = (double)v[p] > (double)FLT_MIN ? grad_v[p] / (double)v[p] : 0.0;
    grad_params[0] = geps;
    grad_params[1] = gmin;
    grad_params[2] = gmax;
    free(A1); free(A2); free(sat); free(te); free(tmin); free(tmax); free(dpos);
    tables_free(&t);
    return 0;
}

/* Clamped box sum of an FP64 plane at every pixel (the operator whose adjoint the backward
 * uses), exposed so the tests can check that it is self-adjoint. */
int orc_box_filter(const double *a, int64_t H, int64_t W, int32_t rx, int32_t ry, double *out)
{
    const int64_t ps = (H + 1) * (W + 1);
    dd_t *sat = (dd_t *)malloc((size_t)ps * sizeof(dd_t));
    if (!sat)
        return -1;
    sat_dd_f64(a, H, W, sat);
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            dd_t bx = box_dd(sat, W + 1, window_of(x, y, W, H, rx, ry));
            out[y * W + x] = bx.hi + bx.lo;
        }
    free(sat);
    return 0;
}

/* ------------------------------------------------------------------ colour (Eq. 12) */
/* Colour restoration (Section II-D, Eq. 12): every channel keeps its ratio to the input
 * luminance, compressed by the exponent sat, and is scaled by the tone-mapped luminance:
 *   out_c = (c / v)^sat * L,  c = R, G, B   (planar rgb, c at rgb + c*H*W).
 * Readings: channel values below 0 count as 0; where v == 0 the ratio is 1.  FP64. */
void orc_color_restore(const float *rgb, const float *v, const double *L, int64_t H,
                       int64_t W, double sat, double *out)
{
    const int64_t np = H * W;
    for (int c = 0; c < 3; ++c)
        for (int64_t p = 0; p < np; ++p) {
            double cin = (double)rgb[c * np + p];
            if (cin < 0.0)
                cin = 0.0;
            const double ratio = v[p] > 0.0f ? cin / (double)v[p] : 1.0;
            out[c * np + p] = pow(ratio, sat) * L[p];
        }
}
