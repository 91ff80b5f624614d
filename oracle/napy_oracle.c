/*
 * napy_oracle.c -- plain FP64 CPU oracle for all-pairs Pearson and Spearman
 * correlation with pairwise deletion of missing values.
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists to check the GPU library; only
 * the tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or helper with the GPU path.
 *
 * What it computes (NApy, arXiv 2505.00448):
 *   - Section 3.2: for a variable pair (g, h) the pairwise-complete set I(g,h)
 *     holds the samples where both values are present; it may be empty.
 *   - Section 3.5.2: Pearson's coefficient on I(g,h); undefined (NaN) when
 *     |I| <= 1.  Zero variance of either side on I is also undefined (reading:
 *     the paper is silent; this follows the usual definition).
 *   - Section 3.5.3: Spearman's coefficient on I(g,h) with ranks taken inside
 *     I(g,h) and tied values given the average of their ranks; undefined when
 *     |I| <= 1 or either side is all tied on I.
 *
 * The computation is written directly from those definitions: for every pair
 * the samples of I are collected, Pearson is a two-pass mean/deviation sum,
 * and Spearman sorts each side of I afresh (O(n log n) per pair) and takes the
 * Pearson coefficient of the average ranks.  No blocking, fusion or reuse
 * across pairs.  P-values are computed by the Python driver (oracle.py).
 *
 * Missing values: NaN is always missing; with use_sentinel != 0 a value equal
 * to `sentinel` is missing as well (the paper's user-chosen missing marker,
 * Section 3.3).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double v;
    int64_t k; /* index inside the pairwise-complete list */
} orc_item;

static int orc_missing(double v, int use_sentinel, double sentinel)
{
    return isnan(v) || (use_sentinel && v == sentinel);
}

static int orc_cmp(const void* a, const void* b)
{
    double x = ((const orc_item*)a)->v, y = ((const orc_item*)b)->v;
    return (x < y) ? -1 : (x > y) ? 1 : 0;
}

/* Two-pass Pearson coefficient of two length-n vectors; NaN if n <= 1 or if
 * either vector is constant (checked exactly on the values). */
static double orc_pearson_vec(const double* a, const double* b, int64_t n)
{
    if (n <= 1) return NAN;
    double amin = a[0], amax = a[0], bmin = b[0], bmax = b[0];
    double sa = 0.0, sb = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        sa += a[k];
        sb += b[k];
        if (a[k] < amin) amin = a[k];
        if (a[k] > amax) amax = a[k];
        if (b[k] < bmin) bmin = b[k];
        if (b[k] > bmax) bmax = b[k];
    }
    if (amin == amax || bmin == bmax) return NAN;
    double ma = sa / (double)n, mb = sb / (double)n;
    double sab = 0.0, saa = 0.0, sbb = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double da = a[k] - ma, db = b[k] - mb;
        sab += da * db;
        saa += da * da;
        sbb += db * db;
    }
    double r = sab / sqrt(saa * sbb);
    if (r > 1.0) r = 1.0;
    if (r < -1.0) r = -1.0;
    return r;
}

/* Collect the pairwise-complete samples of (g, h) into a, b (and their sample
 * indices into idx when non-NULL); returns |I(g,h)|. */
static int64_t orc_collect(const double* X, int64_t S, int64_t ldx, int64_t g, int64_t h,
                           int use_sentinel, double sentinel,
                           double* a, double* b, int64_t* idx)
{
    int64_t n = 0;
    for (int64_t i = 0; i < S; ++i) {
        double xg = X[i * ldx + g], xh = X[i * ldx + h];
        if (orc_missing(xg, use_sentinel, sentinel) || orc_missing(xh, use_sentinel, sentinel))
            continue;
        a[n] = xg;
        b[n] = xh;
        if (idx) idx[n] = i;
        ++n;
    }
    return n;
}

/* Average ranks (1-based) of v[0..n) written to out[0..n).  Equal values
 * (IEEE equality, so -0 ties +0) share the mean of the positions they span. */
static void orc_average_ranks(const double* v, int64_t n, orc_item* scratch, double* out)
{
    for (int64_t k = 0; k < n; ++k) {
        scratch[k].v = v[k];
        scratch[k].k = k;
    }
    qsort(scratch, (size_t)n, sizeof(orc_item), orc_cmp);
    int64_t s = 0;
    while (s < n) {
        int64_t e = s + 1;
        while (e < n && scratch[e].v == scratch[s].v) ++e;
        /* positions s+1 .. e (1-based) share the rank (s + 1 + e) / 2 */
        double rk = 0.5 * (double)(s + 1 + e);
        for (int64_t t = s; t < e; ++t) out[scratch[t].k] = rk;
        s = e;
    }
}

typedef struct {
    double *a, *b, *ra, *rb;
    orc_item* items;
} orc_buf;

static int orc_buf_init(orc_buf* w, int64_t S)
{
    size_t m = (size_t)(S > 0 ? S : 1);
    w->a = (double*)malloc(m * sizeof(double));
    w->b = (double*)malloc(m * sizeof(double));
    w->ra = (double*)malloc(m * sizeof(double));
    w->rb = (double*)malloc(m * sizeof(double));
    w->items = (orc_item*)malloc(m * sizeof(orc_item));
    return w->a && w->b && w->ra && w->rb && w->items;
}

static void orc_buf_free(orc_buf* w)
{
    free(w->a);
    free(w->b);
    free(w->ra);
    free(w->rb);
    free(w->items);
}

static void orc_pair(const double* X, int64_t S, int64_t ldx, int64_t g, int64_t h,
                     int use_sentinel, double sentinel, int spearman, orc_buf* w,
                     double* r_out, int64_t* n_out)
{
    int64_t n = orc_collect(X, S, ldx, g, h, use_sentinel, sentinel, w->a, w->b, NULL);
    *n_out = n;
    if (n <= 1) {
        *r_out = NAN;
        return;
    }
    if (!spearman) {
        *r_out = orc_pearson_vec(w->a, w->b, n);
        return;
    }
    orc_average_ranks(w->a, n, w->items, w->ra);
    orc_average_ranks(w->b, n, w->items, w->rb);
    *r_out = orc_pearson_vec(w->ra, w->rb, n);
}

static void orc_set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Full F x F matrices (both triangles and the diagonal).  r: F*F doubles,
 * n: F*F int64, row-major with leading dimension F.  Returns 0, or -1 when a
 * per-thread buffer could not be allocated. */
int orc_all_pairs(const double* X, int64_t S, int64_t F, int64_t ldx,
                  int use_sentinel, double sentinel, int spearman, int nthreads,
                  double* r, int64_t* n)
{
    int failed = 0;
    orc_set_threads(nthreads);
#pragma omp parallel
    {
        orc_buf w;
        int ok = orc_buf_init(&w, S);
        if (!ok) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t g = 0; g < F; ++g) {
            if (!ok) continue;
            for (int64_t h = g; h < F; ++h) {
                double rv;
                int64_t nv;
                orc_pair(X, S, ldx, g, h, use_sentinel, sentinel, spearman, &w, &rv, &nv);
                r[g * F + h] = rv;
                r[h * F + g] = rv;
                n[g * F + h] = nv;
                n[h * F + g] = nv;
            }
        }
        orc_buf_free(&w);
    }
    return failed ? -1 : 0;
}

/* Listed pairs (gi[k], hi[k]) for k < npairs; r, n have npairs entries. */
int orc_pairs(const double* X, int64_t S, int64_t F, int64_t ldx,
              int use_sentinel, double sentinel, int spearman, int nthreads,
              const int64_t* gi, const int64_t* hi, int64_t npairs,
              double* r, int64_t* n)
{
    int failed = 0;
    (void)F;
    orc_set_threads(nthreads);
#pragma omp parallel
    {
        orc_buf w;
        int ok = orc_buf_init(&w, S);
        if (!ok) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < npairs; ++k) {
            if (!ok) continue;
            orc_pair(X, S, ldx, gi[k], hi[k], use_sentinel, sentinel, spearman, &w, &r[k], &n[k]);
        }
        orc_buf_free(&w);
    }
    return failed ? -1 : 0;
}

/* Average ranks of both sides of one pair, scattered back to sample order:
 * rank_g[i], rank_h[i] for i in I(g,h), NaN for every other sample.
 * Returns |I(g,h)| or -1 on allocation failure. */
int64_t orc_pair_ranks(const double* X, int64_t S, int64_t ldx, int64_t g, int64_t h,
                       int use_sentinel, double sentinel, double* rank_g, double* rank_h)
{
    orc_buf w;
    int64_t* idx = (int64_t*)malloc((size_t)(S > 0 ? S : 1) * sizeof(int64_t));
    if (!idx || !orc_buf_init(&w, S)) {
        free(idx);
        return -1;
    }
    for (int64_t i = 0; i < S; ++i) {
        rank_g[i] = NAN;
        rank_h[i] = NAN;
    }
    int64_t n = orc_collect(X, S, ldx, g, h, use_sentinel, sentinel, w.a, w.b, idx);
    if (n > 0) {
        orc_average_ranks(w.a, n, w.items, w.ra);
        orc_average_ranks(w.b, n, w.items, w.rb);
        for (int64_t k = 0; k < n; ++k) {
            rank_g[idx[k]] = w.ra[k];
            rank_h[idx[k]] = w.rb[k];
        }
    }
    orc_buf_free(&w);
    free(idx);
    return n;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
