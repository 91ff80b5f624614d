/*
 * napy.h -- C ABI of libnapy: all-pairs Pearson and Spearman correlation with
 * pairwise deletion of missing values on one AMD MI355X (gfx950).
 *
 * Method: NApy, "Efficient Statistics in Python for Large-Scale Heterogeneous
 * Data with Enhanced Support for Missing Data" (arXiv 2505.00448).
 *   - Section 3.2 defines the pairwise-complete set I(g,h) of a variable pair:
 *     the samples where neither value is missing (it may be empty).
 *   - Section 3.5.2: Pearson correlation on I(g,h), two-sided p from the Beta
 *     CDF; r and p undefined (NaN) for |I| <= 1, p defined from |I| = 2 on.
 *   - Section 3.5.3: Spearman correlation on I(g,h), each variable sorted
 *     once, ranks re-derived inside I(g,h) in linear time, ties given their
 *     average rank, two-sided p from the t distribution; rho and p undefined
 *     for |I| <= 1, p undefined for |I| <= 2.
 *   - Section 3.4: outputs are F x F matrices, entry (i, j) for variables i, j.
 *
 * Conventions shared by every entry point below:
 *   - Every data pointer is a DEVICE pointer (hipMalloc'd or a PyTorch CUDA
 *     tensor's data) unless the comment says host.  The caller owns every
 *     buffer and the stream; the library never allocates device or host
 *     memory and keeps no state between calls (napy_pearson_noalloc's fixed
 *     scratch array, loaded with the library, is the one exception).
 *   - Input X is samples x variables, row-major, float32: element (i, c) at
 *     X[i * ldx + c], ldx >= F.  NaN marks a missing value; with
 *     opts->use_sentinel != 0 a value equal to opts->sentinel is missing too.
 *     +-Inf is a precondition violation (results undefined).
 *   - Outputs are full symmetric F x F row-major matrices with leading
 *     dimension ldo >= F (both triangles and the diagonal are written):
 *     r and p float64, n int32.  Any of r, p, n may be NULL (not computed).
 *     Undefined statistics are NaN, not errors.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous: they enqueue kernels and return; no device to
 *     host traffic and no synchronisation happen inside a call.  Calls on
 *     different streams with distinct buffers may run concurrently, also
 *     from different host threads (the only process-wide setting, a
 *     kernel's dynamic-LDS limit, is made once per device under an atomic
 *     flag).
 *   - `ws` is a caller-owned device workspace of at least the size returned
 *     by the matching *_workspace() query (pure host function), aligned to
 *     256 bytes.  Its contents on entry do not matter.
 *   - Return value: a napy_status.  Arguments are validated on the host
 *     before any HIP call, so a bad argument returns NAPY_E_INVALID (or
 *     NAPY_E_WORKSPACE / NAPY_E_UNSUPPORTED) without touching the device.
 *     NAPY_E_HIP reports a failed launch; napy_last_error() then describes it.
 *     On any error the outputs are undefined.
 */
#ifndef NAPY_H
#define NAPY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NAPY_OK = 0,
    NAPY_E_INVALID = 1,     /* NULL input, negative size, ld too small, bad option */
    NAPY_E_WORKSPACE = 2,   /* ws NULL or ws_bytes below the query's value */
    NAPY_E_UNSUPPORTED = 3, /* shape outside the supported range (see each call) */
    NAPY_E_HIP = 4          /* a HIP runtime call or kernel launch failed */
} napy_status;

typedef enum {
    NAPY_PREC_FP32 = 0,   /* FP32 MFMA contractions, FP64 flush and combine */
    NAPY_PREC_BF16X3 = 1, /* split-BF16 MFMA contractions, FP32 accumulate,
                             FP64 flush and combine */
    NAPY_PREC_FP64 = 2    /* FP64 MFMA contractions (validation mode) */
} napy_precision;

typedef struct {
    int32_t precision;    /* napy_precision; used by the Pearson calls */
    int32_t use_sentinel; /* 0: only NaN is missing; 1: also x == sentinel */
    float sentinel;       /* the user's missing-value marker (Section 3.3) */
    int32_t reserved;     /* must be 0 */
} napy_opts;

/* Static description of a status code (host, never NULL). */
const char* napy_strerror(int status);

/* Thread-local text describing the last NAPY_E_HIP / NAPY_E_UNSUPPORTED of
 * the calling thread (host, never NULL, "" if none). */
const char* napy_last_error(void);

/* Library version as "major.minor.patch" (host, static string). */
const char* napy_version(void);

/* ------------------------------------------------------------------------
 * Pearson (Sections 3.2, 3.5.2).  Per pair over I(g,h): n, r clamped to
 * [-1, 1], and p = I_{1-r^2}((n-2)/2, 1/2).  n <= 1 -> r = p = NaN;
 * n = 2 -> r = +-1, p = 1; zero variance of either side on I -> r = p = NaN.
 * Computed as masked dense contractions on the matrix cores after centring
 * every variable on its observed mean (r is shift invariant).  A pair whose
 * variance about its own mean is below 0.9 of its second moment about the
 * column mean on either side (complete samples far from the column mean,
 * or a side constant on I) is recomputed from the raw values in FP64 by two
 * passes about the pair's means, and its zero variance decided exactly
 * (minimum = maximum on I); such pairs cost O(S) each.
 * Supported: 1 <= F <= 65535, 1 <= S <= 2^31 - 1.
 * ------------------------------------------------------------------------ */
size_t napy_pearson_workspace(int64_t S, int64_t F, const napy_opts* opts);

int napy_pearson(const float* X, int64_t S, int64_t F, int64_t ldx,
                 double* r, double* p, int32_t* n, int64_t ldo,
                 void* ws, size_t ws_bytes, const napy_opts* opts, void* stream);

/* ------------------------------------------------------------------------
 * Allocation-free Pearson, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): napy_pearson without a workspace argument.  Its scratch
 * memory is a fixed array of 128 MiB inside the library, one per device the
 * library runs on, held until the process ends; the call allocates nothing
 * (no hipMalloc/hipFree or allocating library routine).  The caller still
 * passes X and the outputs.  Results meet the same bars as napy_pearson's
 * (the split of the samples, and so the order of the FP64 partial sums, may
 * differ when the default split needs more than the array).  Shapes whose
 * scratch need exceeds 128 MiB even unsplit return NAPY_E_UNSUPPORTED, with
 * the sizes in napy_last_error() (about F <= 2,000 variables).  Every call on
 * one device uses that device's array: calls that overlap in time on the same
 * device (different streams or host threads) race and give undefined results;
 * calls that follow each other in stream order are fine.
 * ------------------------------------------------------------------------ */
int napy_pearson_noalloc(const float* X, int64_t S, int64_t F, int64_t ldx,
                         double* r, double* p, int32_t* n, int64_t ldo,
                         const napy_opts* opts, void* stream);

/* ------------------------------------------------------------------------
 * Spearman (Sections 3.2, 3.5.3).  Each variable's observed values are sorted
 * once; for every pair the ranks inside I(g,h) are re-derived by a prefix
 * count of the partner's presence along that sorted order, with average
 * ranks for ties (IEEE equality: -0 ties +0).  rho is the Pearson
 * coefficient of those ranks, computed from exact integer sums.
 * n <= 1 -> rho = p = NaN; n = 2 -> p = NaN; all tied on I -> NaN.
 * Supported: 1 <= S <= 65535 samples (sorted orders hold 16-bit sample
 * indices; columns longer than 24576 are sorted and walked through global
 * memory), 1 <= F <= 65535.
 * ------------------------------------------------------------------------ */
size_t napy_spearman_workspace(int64_t S, int64_t F, const napy_opts* opts);

int napy_spearman(const float* X, int64_t S, int64_t F, int64_t ldx,
                  double* r, double* p, int32_t* n, int64_t ldo,
                  void* ws, size_t ws_bytes, const napy_opts* opts, void* stream);

/* ------------------------------------------------------------------------
 * Stage timing: napy_pearson / napy_spearman with `stage_events`, a host
 * array of 4 caller-created hipEvent_t handles (passed as void*; a NULL
 * entry is skipped).  Event 0 is recorded on `stream` before the first
 * kernel, events 1..3 after each stage:
 *   Pearson:  1 column statistics, 2 masked contractions, 3 combine + p;
 *   Spearman: 1 sort of every column and the partner blocks' presence
 *             planes, 2 per-pair re-ranking scan (k_spearman_pairs
 *             alone), 3 combine + p.
 * Results are those of the plain calls.
 * ------------------------------------------------------------------------ */
int napy_pearson_profiled(const float* X, int64_t S, int64_t F, int64_t ldx,
                          double* r, double* p, int32_t* n, int64_t ldo,
                          void* ws, size_t ws_bytes, const napy_opts* opts, void* stream,
                          void* const* stage_events);

int napy_spearman_profiled(const float* X, int64_t S, int64_t F, int64_t ldx,
                           double* r, double* p, int32_t* n, int64_t ldo,
                           void* ws, size_t ws_bytes, const napy_opts* opts, void* stream,
                           void* const* stage_events);

/* ------------------------------------------------------------------------
 * Differentiation of the Pearson matrix (no counterpart in the paper; the
 * derivative of the Section 3.5.2 definition).
 *
 * napy_pearson_fwd: napy_pearson plus `saved`, caller-owned float64
 * [7][F][F] (ld F): n, Sx, Sy, Sxx, Syy, Sxy per ordered pair (g, h), the
 * sums over I(g,h) of 1, x_g, x_h, x_g^2, x_h^2 and x_g x_h, where x is the
 * data centred on each variable's observed mean, then r (NaN where
 * undefined).  Workspace as napy_pearson_workspace.
 *
 * napy_pearson_backward: given dR = dL/dR (float32, F x F, row-major, ld ldr;
 * entries (g, h) and (h, g) are both read, the diagonal is ignored because
 * r_gg is constant), writes dX = dL/dX (float32, S x F, ld lddx).  Missing
 * entries get exactly 0, as do entries whose pairs have undefined r (NaN in
 * saved's r plane).  X, opts and S, F must be the forward's.
 * ------------------------------------------------------------------------ */
int napy_pearson_fwd(const float* X, int64_t S, int64_t F, int64_t ldx,
                     double* r, double* p, int32_t* n, int64_t ldo, double* saved,
                     void* ws, size_t ws_bytes, const napy_opts* opts, void* stream);

size_t napy_pearson_backward_workspace(int64_t S, int64_t F, const napy_opts* opts);

int napy_pearson_backward(const float* X, int64_t S, int64_t F, int64_t ldx,
                          const double* saved, const float* dR, int64_t ldr,
                          float* dX, int64_t lddx,
                          void* ws, size_t ws_bytes, const napy_opts* opts, void* stream);

/* ------------------------------------------------------------------------
 * Subset queries on a resident base matrix (the paper's interactive
 * explorer use case, Section 1): a query is a set of rows (samples) and a
 * list of columns (variables) of the base X (S x F).  The result is exactly
 * the full call applied to X[rows][:, cols] (Fq x Fq outputs, ld ldo >= Fq).
 *
 * rows: device int32 [Sq], distinct, ascending, each in [0, S).
 * cols: device int32 [Fq], distinct, each in [0, F).
 *
 * Spearman subsets reuse a prepared base: napy_spearman_base_prepare sorts
 * every column of X once into `base` (caller-owned device buffer of
 * napy_spearman_base_bytes(S, F) bytes, 256-byte aligned), and
 * napy_spearman_subset compacts each selected column's sorted order by the
 * row set, so no query sorts again.  The base stays valid while X is
 * unchanged; S <= 24576 (the compaction holds a base column in LDS).
 * ------------------------------------------------------------------------ */
size_t napy_pearson_subset_workspace(int64_t Sq, int64_t Fq, const napy_opts* opts);

int napy_pearson_subset(const float* X, int64_t S, int64_t F, int64_t ldx,
                        const int32_t* rows, int64_t Sq, const int32_t* cols, int64_t Fq,
                        double* r, double* p, int32_t* n, int64_t ldo,
                        void* ws, size_t ws_bytes, const napy_opts* opts, void* stream);

size_t napy_spearman_base_bytes(int64_t S, int64_t F);

int napy_spearman_base_prepare(const float* X, int64_t S, int64_t F, int64_t ldx,
                               void* base, size_t base_bytes,
                               const napy_opts* opts, void* stream);

size_t napy_spearman_subset_workspace(int64_t S, int64_t Sq, int64_t Fq, const napy_opts* opts);

int napy_spearman_subset(const void* base, int64_t S, int64_t F,
                         const int32_t* rows, int64_t Sq, const int32_t* cols, int64_t Fq,
                         double* r, double* p, int32_t* n, int64_t ldo,
                         void* ws, size_t ws_bytes, const napy_opts* opts, void* stream);

/* ------------------------------------------------------------------------
 * Multiple-testing correction of an all-pairs p matrix (Section 3.4).
 *
 * The tests are the unordered pairs {i, j}, i != j, whose p-value is defined:
 * the upper triangle (i < j) of p is read, NaN entries are not tests, and m
 * is the number of the others.  With those m values in ascending order
 * p_(1) <= ... <= p_(m):
 *   NAPY_ADJ_BONFERRONI  min(1, m p)                    (Dunn 1961)
 *   NAPY_ADJ_BH          min(1, min_{l >= k} m p_(l) / l) for p = p_(k)
 *                        (Benjamini-Hochberg step-up)
 *   NAPY_ADJ_BY          as BH with m replaced by m c(m),
 *                        c(m) = sum_{i=1..m} 1/i (Benjamini-Yekutieli)
 * The result is written to both triangles of out (F x F float64, ld ldo >= F);
 * the diagonal (self-tests, not counted) and undefined pairs are NaN.  p holds
 * values in [0, 1] or NaN (anything else is a precondition violation) and is
 * read only: out may equal p (then ldo == ldp), any other overlap is not
 * allowed.  1 <= F <= 65535.  napy_adjust_workspace(F) bytes of workspace
 * (pure host function; about 12 B per pair rounded up to a power of two).
 * ------------------------------------------------------------------------ */
typedef enum {
    NAPY_ADJ_BONFERRONI = 0,
    NAPY_ADJ_BH = 1,
    NAPY_ADJ_BY = 2
} napy_adjust_method;

size_t napy_adjust_workspace(int64_t F);

int napy_adjust_pvalues(const double* p, int64_t F, int64_t ldp, double* out, int64_t ldo,
                        int32_t method, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Categorical x continuous tests with pairwise deletion (Section 3.5):
 * two-sample t-test (Student or Welch) and one-way ANOVA.
 *
 * L is S x FC float32 (leading dimension ldl >= FC) holding label-encoded
 * categorical features (Section 3.3: integers from 0); X is S x FQ float32
 * (ldx >= FQ) holding continuous features; missing values as for napy_pearson
 * (NaN, or opts->sentinel with use_sentinel).  Each pair (g, h) uses the
 * samples where both L[., g] and X[., h] are present.  Outputs are FC x FQ
 * row-major with leading dimension ldo >= FQ, entry (g, h) for categorical
 * feature g and continuous feature h (Section 3.4): the statistic (t or F,
 * float64), its two-sided p-value (float64) and n = |I(g, h)| (int32).  All
 * three output pointers are required.
 *
 * napy_ttest: groups are label 0 and label 1, t = (mean_0 - mean_1) / se;
 *   welch = 0 Student (pooled variance, df = n0 + n1 - 2), 1 Welch
 *   (Welch-Satterthwaite df); p from the t distribution.  NaN when a group
 *   has fewer than two samples, and for Student when the pooled variance is
 *   zero; Welch with both variances zero gives t = +-inf, p = 0 when the means
 *   differ, NaN when they are equal.
 * napy_anova: the categories of a column are the labels observed anywhere in
 *   it; labels must lie in [0, ncat), 2 <= ncat <= 32.  F = (SSB / (K - 1)) /
 *   (SSW / (N - K)), p from Fisher's F distribution.  NaN when a category is
 *   empty within I(g, h) or the column has one category; when every
 *   within-category variance is zero, F = inf and p = 0 unless all category
 *   means are equal (then NaN).
 * A categorical column with a label outside what the test accepts (not an
 *   integer, negative, >= ncat, or for the t-test not 0 or 1) is not tested:
 *   its statistics and p are NaN and n is 0.
 * Variances and means are decided zero/equal within 1e-10 relative (FP64
 * sums).  The contractions run on FP64 matrix cores.
 * ------------------------------------------------------------------------ */
size_t napy_ttest_workspace(int64_t S, int64_t FC, int64_t FQ, const napy_opts* opts);

int napy_ttest(const float* L, int64_t ldl, const float* X, int64_t ldx, int64_t S, int64_t FC, int64_t FQ,
               int32_t welch, double* t, double* p, int32_t* n, int64_t ldo,
               void* ws, size_t ws_bytes, const napy_opts* opts, void* stream);

size_t napy_anova_workspace(int64_t S, int64_t FC, int64_t FQ, int32_t ncat, const napy_opts* opts);

int napy_anova(const float* L, int64_t ldl, const float* X, int64_t ldx, int64_t S, int64_t FC, int64_t FQ,
               int32_t ncat, double* F, double* p, int32_t* n, int64_t ldo,
               void* ws, size_t ws_bytes, const napy_opts* opts, void* stream);

/* ------------------------------------------------------------------------
 * Rank tests of categorical x continuous pairs with pairwise deletion
 * (Section 3.5): Mann-Whitney U and Kruskal-Wallis H.
 *
 * Inputs, missing values, output layout and the untested-column rule are
 * those of napy_ttest / napy_anova above.  Within I(g, h) the continuous
 * values are ranked 1..n with tied values given the average of their ranks;
 * R_k is the rank sum of label k, n_k its size, T = sum over groups of tied
 * values of t^3 - t.  S <= 65,535 (sorted orders hold 16-bit sample indices;
 * with more than 24,576 the labels are read from global memory when they and
 * the tables do not fit LDS together).
 *
 * napy_mannwhitney: groups are label 0 and label 1; the statistic is
 *   U1 = R_0 - n0 (n0 + 1) / 2.  Two-sided p with U = max(U1, n0 n1 - U1):
 *   asymptotic, z = (U - n0 n1 / 2 - 1/2) / s with
 *   s^2 = n0 n1 / 12 ((n + 1) - T / (n (n - 1))) (continuity and tie
 *   corrections), p = min(1, 2 Q(z)) (Q the standard normal tail; s = 0 gives
 *   p = 1); or exact, p = min(1, 2 P(U' >= U)) under random assignment of the
 *   n ranks.  mode NAPY_MWU_AUTO takes the exact p when I(g, h) has no ties
 *   and a group has fewer than eight samples, NAPY_MWU_ASYMPTOTIC never.  NaN
 *   when a group is empty.
 * napy_kruskal: categories as for napy_anova (labels in [0, ncat),
 *   2 <= ncat <= 32); H = 12 / (n (n + 1)) sum_k (R_k - n_k (n + 1) / 2)^2 /
 *   n_k / (1 - T / (n^3 - n)), p = P(chi2_{K-1} > H).  NaN when a category is
 *   empty within I(g, h), the column has one category, or every value in
 *   I(g, h) is tied.
 * ------------------------------------------------------------------------ */
typedef enum {
    NAPY_MWU_AUTO = 0,
    NAPY_MWU_ASYMPTOTIC = 1
} napy_mwu_mode;

size_t napy_mannwhitney_workspace(int64_t S, int64_t FC, int64_t FQ, const napy_opts* opts);

int napy_mannwhitney(const float* L, int64_t ldl, const float* X, int64_t ldx, int64_t S, int64_t FC, int64_t FQ,
                     int32_t mode, double* U, double* p, int32_t* n, int64_t ldo,
                     void* ws, size_t ws_bytes, const napy_opts* opts, void* stream);

size_t napy_kruskal_workspace(int64_t S, int64_t FC, int64_t FQ, int32_t ncat, const napy_opts* opts);

int napy_kruskal(const float* L, int64_t ldl, const float* X, int64_t ldx, int64_t S, int64_t FC, int64_t FQ,
                 int32_t ncat, double* H, double* p, int32_t* n, int64_t ldo,
                 void* ws, size_t ws_bytes, const napy_opts* opts, void* stream);

/* ------------------------------------------------------------------------
 * Chi-squared test of independence between categorical features with
 * pairwise deletion (Section 3.5), all pairs of one matrix.
 *
 * L is S x F float32 (ldl >= F), label-encoded (Section 3.3), labels in
 * [0, ncat), 2 <= ncat <= 32; missing values as for napy_pearson.  For each
 * pair (g, h) the r x c contingency table on I(g, h) (r, c: the labels
 * observed anywhere in each column) gives chi2 = sum (O - E)^2 / E with
 * E = row sum * column sum / N (no continuity correction), p = P(chi2_df >
 * chi2) with df = (r - 1)(c - 1), Cramer's V = sqrt(chi2 / (N min(r-1, c-1)))
 * (phi for 2 x 2) and n = N = |I(g, h)|.  Outputs chi2, p, v (float64) and n
 * (int32) are full symmetric F x F with ldo >= F, all required; the diagonal
 * is computed like any pair.  NaN everywhere when a category observed in a
 * column is empty within I(g, h) or I(g, h) is empty; p and V NaN when a
 * feature has one category.  A column with a label that is not an integer,
 * negative or >= ncat is not tested (NaN, n = 0).  Counts are exact (FP64
 * matrix cores).  Supported while F * ncat <= 50,000.
 * ------------------------------------------------------------------------ */
size_t napy_chi2_workspace(int64_t S, int64_t F, int32_t ncat, const napy_opts* opts);

int napy_chi2(const float* L, int64_t ldl, int64_t S, int64_t F, int32_t ncat,
              double* chi2, double* p, double* v, int32_t* n, int64_t ldo,
              void* ws, size_t ws_bytes, const napy_opts* opts, void* stream);

/* ------------------------------------------------------------------------
 * Test hooks (not part of the computation path).
 *
 * napy_spearman_pair_ranks: the doubled average ranks 2*rank that the
 * Spearman path assigns inside I(g,h) (Section 3.5.3), scattered to sample
 * order: rank2_g[i], rank2_h[i] (device int32 [S]) for i in I(g,h), -1 for
 * every other sample.  Uses napy_spearman_workspace(S, F) bytes.
 *
 * napy_pvalue_device: evaluates the library's device p-value routine,
 * p[k] = I_{1-r[k]^2}((n[k]-2)/2, 1/2) (NaN for n < 3), on device arrays.
 *
 * napy_pvalue_host: the same routine compiled for the host (host arrays);
 * it lets the p-value arithmetic be checked on a machine without a GPU and
 * is never used by any computation above.
 * ------------------------------------------------------------------------ */
int napy_spearman_pair_ranks(const float* X, int64_t S, int64_t F, int64_t ldx,
                             int32_t g, int32_t h, int32_t* rank2_g, int32_t* rank2_h,
                             void* ws, size_t ws_bytes, const napy_opts* opts, void* stream);

int napy_pvalue_device(const double* r, const int32_t* n, double* p, int64_t count, void* stream);

int napy_pvalue_host(const double* r, const int32_t* n, double* p, int64_t count);

/* napy_fdist_sf_host: the library's F-distribution survival function
 * P(F' > f; d1, d2) (used for the t-test as P(F' > t^2; 1, df) and for ANOVA)
 * compiled for the host, on host arrays; for checking the arithmetic without a
 * GPU. */
int napy_fdist_sf_host(const double* f, const double* d1, const double* d2, double* p, int64_t count);

/* napy_chi2_sf_host: the library's chi-squared survival function
 * P(chi2_df > x) = Q(df/2, x/2) compiled for the host, on host arrays. */
int napy_chi2_sf_host(const double* x, const double* df, double* p, int64_t count);

#ifdef __cplusplus
}
#endif

#endif /* NAPY_H */
