// C ABI of libnapy: argument validation (host only, before any HIP call),
// workspace queries and dispatch to the Pearson and Spearman drivers.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "napy_internal.hpp"
#include "pvalue.hpp"
#include "rankbase.hpp"

namespace napy {

static thread_local char g_last_error[512] = "";

void set_last_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
}

int hip_status(hipError_t e, const char* what)
{
    if (e == hipSuccess) return NAPY_OK;
    set_last_error("%s: %s", what, hipGetErrorString(e));
    return NAPY_E_HIP;
}

int check_launch(const char* what) { return hip_status(hipGetLastError(), what); }

// Spearman drivers (spearman.hip)
size_t spearman_ws_bytes(int64_t S, int64_t F);
int spearman_run(const float* X, int64_t S, int64_t F, int64_t ldx, double* r, double* p, int32_t* n,
                 int64_t ldo, void* ws, const napy_opts* opts, hipStream_t st, void* const* ev);
int spearman_pair_ranks_run(const float* X, int64_t S, int64_t F, int64_t ldx, int g, int h, int32_t* rg,
                            int32_t* rh, void* ws, const napy_opts* opts, hipStream_t st);
size_t spearman_base_bytes(int64_t S, int64_t F);
int spearman_base_prepare_run(const float* X, int64_t S, int64_t F, int64_t ldx, void* base,
                              const napy_opts* opts, hipStream_t st);
size_t spearman_subset_ws_bytes(int64_t S, int64_t Sq, int64_t Fq);
int spearman_subset_run(const void* basebuf, int64_t S, int64_t F, const int32_t* rows, int64_t Sq,
                        const int32_t* cols, int64_t Fq, double* r, double* p, int32_t* n, int64_t ldo,
                        void* ws, hipStream_t st);
// multiple-testing correction (adjust.hip)
size_t adjust_ws_bytes(int64_t F);
int adjust_run(const double* p, int64_t F, int64_t ldp, double* out, int64_t ldo, int method, void* ws,
               hipStream_t st);
// categorical x continuous tests (groups.hip)
size_t groups_ws_bytes(int64_t S, int64_t FC, int64_t FQ, int ncat);
int groups_run(const float* L, int64_t ldl, const float* X, int64_t ldx, int64_t S, int64_t FC, int64_t FQ,
               int test, int ncat, double* stat, double* p, int32_t* n, int64_t ldo, void* ws, const napy_opts* opts,
               hipStream_t st);
// rank tests (ranktests.hip)
size_t ranktests_ws_bytes(int64_t S, int64_t FC, int64_t FQ, bool mwu);
int ranktests_run(const float* L, int64_t ldl, const float* X, int64_t ldx, int64_t S, int64_t FC, int64_t FQ,
                  int test, int ncat, double* stat, double* p, int32_t* n, int64_t ldo, void* ws,
                  const napy_opts* opts, hipStream_t st);
// chi-squared test (chi2.hip)
size_t chi2_ws_bytes(int64_t S, int64_t F, int ncat);
int chi2_run(const float* L, int64_t ldl, int64_t S, int64_t F, int ncat, double* chi, double* p, double* v,
             int32_t* n, int64_t ldo, void* ws, const napy_opts* opts, hipStream_t st);
// backward (backward.hip)
size_t backward_ws_bytes(int64_t S, int64_t F);
int backward_run(const float* X, int64_t S, int64_t F, int64_t ldx, const double* saved, const float* dR,
                 int64_t ldr, float* dX, int64_t lddx, void* ws, const napy_opts* opts, hipStream_t st);

constexpr int64_t MAX_F = 65535;
constexpr int64_t MAX_S = 2147483647;
// Spearman and the rank tests: 16-bit sample indices and sorted positions.
// Query subsets of a resident base compact the base's LDS-sorted orders (tie
// flags in the positions), so the base is limited to the LDS sort's column
// length.
constexpr int64_t MAX_S_SPEARMAN = SPEAR_MAX_S;
constexpr int64_t MAX_S_SUBSET = SORT_LDS_MAX_S;
constexpr int64_t MAX_S_RANKTESTS = SPEAR_MAX_S;

static int check_shape(int64_t S, int64_t F)
{
    if (S < 0 || F < 1) {
        set_last_error("S must be >= 0 and F >= 1 (got S=%lld, F=%lld)", (long long)S, (long long)F);
        return NAPY_E_INVALID;
    }
    if (F > MAX_F || S > MAX_S) {
        set_last_error("shape S=%lld F=%lld outside the supported range", (long long)S, (long long)F);
        return NAPY_E_UNSUPPORTED;
    }
    return NAPY_OK;
}

static int check_common(const float* X, int64_t S, int64_t F, int64_t ldx, int64_t ldo, void* ws,
                        size_t ws_bytes, size_t need, const napy_opts* opts)
{
    NAPY_TRY(check_shape(S, F));
    if (!X && S > 0) return NAPY_E_INVALID;
    if (ldx < F || ldo < F) return NAPY_E_INVALID;
    if (!opts_ok(opts)) return NAPY_E_INVALID;
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255)) return NAPY_E_WORKSPACE;
    return NAPY_OK;
}

}  // namespace napy

using namespace napy;

extern "C" {

const char* napy_strerror(int status)
{
    switch (status) {
    case NAPY_OK: return "success";
    case NAPY_E_INVALID: return "invalid argument";
    case NAPY_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case NAPY_E_UNSUPPORTED: return "shape outside the supported range";
    case NAPY_E_HIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

const char* napy_last_error(void) { return g_last_error; }

const char* napy_version(void) { return "0.1.0"; }

size_t napy_pearson_workspace(int64_t S, int64_t F, const napy_opts* opts)
{
    if (S < 0 || F < 1 || F > MAX_F || !opts_ok(opts)) return 0;
    return pearson_ws_bytes(S, F, opt_prec(opts));
}

int napy_pearson(const float* X, int64_t S, int64_t F, int64_t ldx, double* r, double* p, int32_t* n,
                 int64_t ldo, void* ws, size_t ws_bytes, const napy_opts* opts, void* stream)
{
    if (!opts_ok(opts)) return NAPY_E_INVALID;
    NAPY_TRY(check_shape(S, F));
    NAPY_TRY(check_common(X, S, F, ldx, ldo, ws, ws_bytes, pearson_ws_bytes(S, F, opt_prec(opts)), opts));
    return pearson_run(X, S, F, ldx, r, p, n, ldo, nullptr, ws, ws_bytes, opts, (hipStream_t)stream);
}

int napy_pearson_noalloc(const float* X, int64_t S, int64_t F, int64_t ldx, double* r, double* p, int32_t* n,
                         int64_t ldo, const napy_opts* opts, void* stream)
{
    if (!opts_ok(opts)) return NAPY_E_INVALID;
    NAPY_TRY(check_shape(S, F));
    if (!X && S > 0) return NAPY_E_INVALID;
    if (ldx < F || ldo < F) return NAPY_E_INVALID;
    return pearson_noalloc_run(X, S, F, ldx, r, p, n, ldo, opts, (hipStream_t)stream);
}

int napy_pearson_fwd(const float* X, int64_t S, int64_t F, int64_t ldx, double* r, double* p, int32_t* n,
                     int64_t ldo, double* saved, void* ws, size_t ws_bytes, const napy_opts* opts,
                     void* stream)
{
    if (!opts_ok(opts)) return NAPY_E_INVALID;
    NAPY_TRY(check_shape(S, F));
    NAPY_TRY(check_common(X, S, F, ldx, ldo, ws, ws_bytes, pearson_ws_bytes(S, F, opt_prec(opts)), opts));
    if (!saved) return NAPY_E_INVALID;
    return pearson_run(X, S, F, ldx, r, p, n, ldo, saved, ws, ws_bytes, opts, (hipStream_t)stream);
}

size_t napy_spearman_workspace(int64_t S, int64_t F, const napy_opts* opts)
{
    if (S < 0 || F < 1 || F > MAX_F || S > MAX_S_SPEARMAN || !opts_ok(opts)) return 0;
    return spearman_ws_bytes(S, F);
}

int napy_spearman(const float* X, int64_t S, int64_t F, int64_t ldx, double* r, double* p, int32_t* n,
                  int64_t ldo, void* ws, size_t ws_bytes, const napy_opts* opts, void* stream)
{
    if (!opts_ok(opts)) return NAPY_E_INVALID;
    NAPY_TRY(check_shape(S, F));
    if (S > MAX_S_SPEARMAN) {
        set_last_error("Spearman supports S <= %lld samples (got %lld)", (long long)MAX_S_SPEARMAN,
                       (long long)S);
        return NAPY_E_UNSUPPORTED;
    }
    NAPY_TRY(check_common(X, S, F, ldx, ldo, ws, ws_bytes, spearman_ws_bytes(S, F), opts));
    return spearman_run(X, S, F, ldx, r, p, n, ldo, ws, opts, (hipStream_t)stream, nullptr);
}

int napy_pearson_profiled(const float* X, int64_t S, int64_t F, int64_t ldx, double* r, double* p, int32_t* n,
                          int64_t ldo, void* ws, size_t ws_bytes, const napy_opts* opts, void* stream,
                          void* const* stage_events)
{
    if (!opts_ok(opts)) return NAPY_E_INVALID;
    NAPY_TRY(check_shape(S, F));
    NAPY_TRY(check_common(X, S, F, ldx, ldo, ws, ws_bytes, pearson_ws_bytes(S, F, opt_prec(opts)), opts));
    return pearson_run(X, S, F, ldx, r, p, n, ldo, nullptr, ws, ws_bytes, opts, (hipStream_t)stream,
                       stage_events);
}

int napy_spearman_profiled(const float* X, int64_t S, int64_t F, int64_t ldx, double* r, double* p, int32_t* n,
                           int64_t ldo, void* ws, size_t ws_bytes, const napy_opts* opts, void* stream,
                           void* const* stage_events)
{
    if (!opts_ok(opts)) return NAPY_E_INVALID;
    NAPY_TRY(check_shape(S, F));
    if (S > MAX_S_SPEARMAN) return NAPY_E_UNSUPPORTED;
    NAPY_TRY(check_common(X, S, F, ldx, ldo, ws, ws_bytes, spearman_ws_bytes(S, F), opts));
    return spearman_run(X, S, F, ldx, r, p, n, ldo, ws, opts, (hipStream_t)stream, stage_events);
}

size_t napy_pearson_backward_workspace(int64_t S, int64_t F, const napy_opts* opts)
{
    if (S < 0 || F < 1 || F > MAX_F || !opts_ok(opts)) return 0;
    return backward_ws_bytes(S, F);
}

int napy_pearson_backward(const float* X, int64_t S, int64_t F, int64_t ldx, const double* saved,
                          const float* dR, int64_t ldr, float* dX, int64_t lddx, void* ws, size_t ws_bytes,
                          const napy_opts* opts, void* stream)
{
    if (!opts_ok(opts)) return NAPY_E_INVALID;
    NAPY_TRY(check_shape(S, F));
    if ((!X && S > 0) || !saved || !dR || (!dX && S > 0)) return NAPY_E_INVALID;
    if (ldx < F || ldr < F || lddx < F) return NAPY_E_INVALID;
    if (!ws || ws_bytes < backward_ws_bytes(S, F) || ((uintptr_t)ws & 255)) return NAPY_E_WORKSPACE;
    return backward_run(X, S, F, ldx, saved, dR, ldr, dX, lddx, ws, opts, (hipStream_t)stream);
}

size_t napy_pearson_subset_workspace(int64_t Sq, int64_t Fq, const napy_opts* opts)
{
    if (Sq < 0 || Fq < 1 || Fq > MAX_F || !opts_ok(opts)) return 0;
    Carver c(nullptr);
    c.take<float>((size_t)(Sq > 0 ? Sq : 1) * Fq);
    return c.bytes() + pearson_ws_bytes(Sq, Fq, opt_prec(opts));
}

int napy_pearson_subset(const float* X, int64_t S, int64_t F, int64_t ldx, const int32_t* rows, int64_t Sq,
                        const int32_t* cols, int64_t Fq, double* r, double* p, int32_t* n, int64_t ldo,
                        void* ws, size_t ws_bytes, const napy_opts* opts, void* stream)
{
    if (!opts_ok(opts)) return NAPY_E_INVALID;
    NAPY_TRY(check_shape(S, F));
    NAPY_TRY(check_shape(Sq, Fq));
    if ((!X && S > 0) || (!rows && Sq > 0) || !cols) return NAPY_E_INVALID;
    if (ldx < F || ldo < Fq || Sq > S || Fq > F) return NAPY_E_INVALID;
    const size_t need = napy_pearson_subset_workspace(Sq, Fq, opts);
    if (!ws || ws_bytes < need || ((uintptr_t)ws & 255)) return NAPY_E_WORKSPACE;
    Carver c(ws);
    float* Xq = c.take<float>((size_t)(Sq > 0 ? Sq : 1) * Fq);
    char* rest = (char*)ws + c.bytes();
    hipStream_t st = (hipStream_t)stream;
    if (Sq > 0) NAPY_TRY(gather_launch(X, ldx, rows, Sq, cols, Fq, Xq, st));
    return pearson_run(Xq, Sq, Fq, Fq, r, p, n, ldo, nullptr, rest, ws_bytes - c.bytes(), opts, st);
}

size_t napy_spearman_base_bytes(int64_t S, int64_t F)
{
    if (S < 0 || F < 1 || F > MAX_F || S > MAX_S_SUBSET) return 0;
    return spearman_base_bytes(S, F);
}

int napy_spearman_base_prepare(const float* X, int64_t S, int64_t F, int64_t ldx, void* base,
                               size_t base_bytes, const napy_opts* opts, void* stream)
{
    if (!opts_ok(opts)) return NAPY_E_INVALID;
    NAPY_TRY(check_shape(S, F));
    if (S > MAX_S_SUBSET) return NAPY_E_UNSUPPORTED;
    if ((!X && S > 0) || ldx < F) return NAPY_E_INVALID;
    if (!base || base_bytes < spearman_base_bytes(S, F) || ((uintptr_t)base & 255)) return NAPY_E_WORKSPACE;
    return spearman_base_prepare_run(X, S, F, ldx, base, opts, (hipStream_t)stream);
}

size_t napy_spearman_subset_workspace(int64_t S, int64_t Sq, int64_t Fq, const napy_opts* opts)
{
    if (S < 0 || Sq < 0 || Sq > S || Fq < 1 || Fq > MAX_F || S > MAX_S_SUBSET || !opts_ok(opts)) return 0;
    return spearman_subset_ws_bytes(S, Sq, Fq);
}

int napy_spearman_subset(const void* base, int64_t S, int64_t F, const int32_t* rows, int64_t Sq,
                         const int32_t* cols, int64_t Fq, double* r, double* p, int32_t* n, int64_t ldo,
                         void* ws, size_t ws_bytes, const napy_opts* opts, void* stream)
{
    if (!opts_ok(opts)) return NAPY_E_INVALID;
    NAPY_TRY(check_shape(S, F));
    NAPY_TRY(check_shape(Sq, Fq));
    if (S > MAX_S_SUBSET) return NAPY_E_UNSUPPORTED;
    if (!base || (!rows && Sq > 0) || !cols) return NAPY_E_INVALID;
    if (ldo < Fq || Sq > S || Fq > F) return NAPY_E_INVALID;
    if (!ws || ws_bytes < spearman_subset_ws_bytes(S, Sq, Fq) || ((uintptr_t)ws & 255)) return NAPY_E_WORKSPACE;
    return spearman_subset_run(base, S, F, rows, Sq, cols, Fq, r, p, n, ldo, ws, (hipStream_t)stream);
}

int napy_spearman_pair_ranks(const float* X, int64_t S, int64_t F, int64_t ldx, int32_t g, int32_t h,
                             int32_t* rank2_g, int32_t* rank2_h, void* ws, size_t ws_bytes,
                             const napy_opts* opts, void* stream)
{
    if (!opts_ok(opts)) return NAPY_E_INVALID;
    NAPY_TRY(check_shape(S, F));
    if (S > MAX_S_SPEARMAN) return NAPY_E_UNSUPPORTED;
    if ((!X && S > 0) || ldx < F || g < 0 || h < 0 || g >= F || h >= F) return NAPY_E_INVALID;
    if ((!rank2_g || !rank2_h) && S > 0) return NAPY_E_INVALID;
    if (!ws || ws_bytes < spearman_ws_bytes(S, F) || ((uintptr_t)ws & 255)) return NAPY_E_WORKSPACE;
    return spearman_pair_ranks_run(X, S, F, ldx, g, h, rank2_g, rank2_h, ws, opts, (hipStream_t)stream);
}

static int check_groups(int64_t S, int64_t FC, int64_t FQ, int ncat)
{
    if (S < 0 || FC < 1 || FQ < 1) return NAPY_E_INVALID;
    if (ncat < 2 || ncat > 32) return NAPY_E_INVALID;
    if (FC > MAX_F || FQ > MAX_F || S > MAX_S || FC * ncat * FQ > (int64_t)4000000000LL) {
        set_last_error("shape S=%lld FC=%lld FQ=%lld ncat=%d outside the supported range", (long long)S,
                       (long long)FC, (long long)FQ, ncat);
        return NAPY_E_UNSUPPORTED;
    }
    return NAPY_OK;
}

static int groups_call(const float* L, int64_t ldl, const float* X, int64_t ldx, int64_t S, int64_t FC, int64_t FQ,
                       int test, int ncat, double* stat, double* p, int32_t* n, int64_t ldo, void* ws,
                       size_t ws_bytes, const napy_opts* opts, void* stream)
{
    NAPY_TRY(check_groups(S, FC, FQ, ncat));
    if (S > 0 && (!L || !X)) return NAPY_E_INVALID;
    if (ldl < FC || ldx < FQ || ldo < FQ || !stat || !p || !n) return NAPY_E_INVALID;
    if (!opts_ok(opts)) return NAPY_E_INVALID;
    if (!ws || ws_bytes < groups_ws_bytes(S, FC, FQ, ncat) || ((uintptr_t)ws & 255)) return NAPY_E_WORKSPACE;
    return groups_run(L, ldl, X, ldx, S, FC, FQ, test, ncat, stat, p, n, ldo, ws, opts, (hipStream_t)stream);
}

size_t napy_ttest_workspace(int64_t S, int64_t FC, int64_t FQ, const napy_opts* opts)
{
    if (check_groups(S, FC, FQ, 2) != NAPY_OK || !opts_ok(opts)) return 0;
    return groups_ws_bytes(S, FC, FQ, 2);
}

int napy_ttest(const float* L, int64_t ldl, const float* X, int64_t ldx, int64_t S, int64_t FC, int64_t FQ,
               int32_t welch, double* t, double* p, int32_t* n, int64_t ldo, void* ws, size_t ws_bytes,
               const napy_opts* opts, void* stream)
{
    if (welch != 0 && welch != 1) return NAPY_E_INVALID;
    return groups_call(L, ldl, X, ldx, S, FC, FQ, welch, 2, t, p, n, ldo, ws, ws_bytes, opts, stream);
}

size_t napy_anova_workspace(int64_t S, int64_t FC, int64_t FQ, int32_t ncat, const napy_opts* opts)
{
    if (check_groups(S, FC, FQ, ncat) != NAPY_OK || !opts_ok(opts)) return 0;
    return groups_ws_bytes(S, FC, FQ, ncat);
}

int napy_anova(const float* L, int64_t ldl, const float* X, int64_t ldx, int64_t S, int64_t FC, int64_t FQ,
               int32_t ncat, double* F, double* p, int32_t* n, int64_t ldo, void* ws, size_t ws_bytes,
               const napy_opts* opts, void* stream)
{
    return groups_call(L, ldl, X, ldx, S, FC, FQ, 2, ncat, F, p, n, ldo, ws, ws_bytes, opts, stream);
}

static int check_ranks(int64_t S, int64_t FC, int64_t FQ, int ncat)
{
    NAPY_TRY(check_groups(S, FC, FQ, ncat));
    if (S > MAX_S_RANKTESTS) {
        set_last_error("rank tests support S <= %lld samples (got %lld)", (long long)MAX_S_RANKTESTS, (long long)S);
        return NAPY_E_UNSUPPORTED;
    }
    return NAPY_OK;
}

static int ranks_call(const float* L, int64_t ldl, const float* X, int64_t ldx, int64_t S, int64_t FC, int64_t FQ,
                      int test, int ncat, double* stat, double* p, int32_t* n, int64_t ldo, void* ws,
                      size_t ws_bytes, const napy_opts* opts, void* stream)
{
    NAPY_TRY(check_ranks(S, FC, FQ, ncat));
    if (S > 0 && (!L || !X)) return NAPY_E_INVALID;
    if (ldl < FC || ldx < FQ || ldo < FQ || !stat || !p || !n) return NAPY_E_INVALID;
    if (!opts_ok(opts)) return NAPY_E_INVALID;
    if (!ws || ws_bytes < ranktests_ws_bytes(S, FC, FQ, test <= 1) || ((uintptr_t)ws & 255)) return NAPY_E_WORKSPACE;
    return ranktests_run(L, ldl, X, ldx, S, FC, FQ, test, ncat, stat, p, n, ldo, ws, opts, (hipStream_t)stream);
}

size_t napy_mannwhitney_workspace(int64_t S, int64_t FC, int64_t FQ, const napy_opts* opts)
{
    if (check_ranks(S, FC, FQ, 2) != NAPY_OK || !opts_ok(opts)) return 0;
    return ranktests_ws_bytes(S, FC, FQ, true);
}

int napy_mannwhitney(const float* L, int64_t ldl, const float* X, int64_t ldx, int64_t S, int64_t FC, int64_t FQ,
                     int32_t mode, double* U, double* p, int32_t* n, int64_t ldo, void* ws, size_t ws_bytes,
                     const napy_opts* opts, void* stream)
{
    if (mode != NAPY_MWU_AUTO && mode != NAPY_MWU_ASYMPTOTIC) return NAPY_E_INVALID;
    return ranks_call(L, ldl, X, ldx, S, FC, FQ, mode, 2, U, p, n, ldo, ws, ws_bytes, opts, stream);
}

size_t napy_kruskal_workspace(int64_t S, int64_t FC, int64_t FQ, int32_t ncat, const napy_opts* opts)
{
    if (check_ranks(S, FC, FQ, ncat) != NAPY_OK || !opts_ok(opts)) return 0;
    return ranktests_ws_bytes(S, FC, FQ, false);
}

int napy_kruskal(const float* L, int64_t ldl, const float* X, int64_t ldx, int64_t S, int64_t FC, int64_t FQ,
                 int32_t ncat, double* H, double* p, int32_t* n, int64_t ldo, void* ws, size_t ws_bytes,
                 const napy_opts* opts, void* stream)
{
    return ranks_call(L, ldl, X, ldx, S, FC, FQ, 2, ncat, H, p, n, ldo, ws, ws_bytes, opts, stream);
}

static int check_chi2(int64_t S, int64_t F, int ncat)
{
    if (S < 0 || F < 1 || ncat < 2 || ncat > 32) return NAPY_E_INVALID;
    if (F > MAX_F || S > MAX_S || F * ncat > 50000) {
        set_last_error("shape S=%lld F=%lld ncat=%d outside the supported range", (long long)S, (long long)F, ncat);
        return NAPY_E_UNSUPPORTED;
    }
    return NAPY_OK;
}

size_t napy_chi2_workspace(int64_t S, int64_t F, int32_t ncat, const napy_opts* opts)
{
    if (check_chi2(S, F, ncat) != NAPY_OK || !opts_ok(opts)) return 0;
    return chi2_ws_bytes(S, F, ncat);
}

int napy_chi2(const float* L, int64_t ldl, int64_t S, int64_t F, int32_t ncat, double* chi2, double* p, double* v,
              int32_t* n, int64_t ldo, void* ws, size_t ws_bytes, const napy_opts* opts, void* stream)
{
    NAPY_TRY(check_chi2(S, F, ncat));
    if (S > 0 && !L) return NAPY_E_INVALID;
    if (ldl < F || ldo < F || !chi2 || !p || !v || !n) return NAPY_E_INVALID;
    if (!opts_ok(opts)) return NAPY_E_INVALID;
    if (!ws || ws_bytes < chi2_ws_bytes(S, F, ncat) || ((uintptr_t)ws & 255)) return NAPY_E_WORKSPACE;
    return chi2_run(L, ldl, S, F, ncat, chi2, p, v, n, ldo, ws, opts, (hipStream_t)stream);
}

int napy_chi2_sf_host(const double* x, const double* df, double* p, int64_t count)
{
    if (count < 0 || (count > 0 && (!x || !df || !p))) return NAPY_E_INVALID;
    for (int64_t i = 0; i < count; ++i) p[i] = chi2_sf(x[i], df[i]);
    return NAPY_OK;
}

int napy_fdist_sf_host(const double* f, const double* d1, const double* d2, double* p, int64_t count)
{
    if (count < 0 || (count > 0 && (!f || !d1 || !d2 || !p))) return NAPY_E_INVALID;
    for (int64_t i = 0; i < count; ++i) p[i] = fdist_sf(f[i], d1[i], d2[i]);
    return NAPY_OK;
}

size_t napy_adjust_workspace(int64_t F)
{
    if (F < 1 || F > MAX_F) return 0;
    return adjust_ws_bytes(F);
}

int napy_adjust_pvalues(const double* p, int64_t F, int64_t ldp, double* out, int64_t ldo, int32_t method,
                        void* ws, size_t ws_bytes, void* stream)
{
    if (F < 1) return NAPY_E_INVALID;
    if (F > MAX_F) {
        set_last_error("F=%lld outside the supported range", (long long)F);
        return NAPY_E_UNSUPPORTED;
    }
    if (!p || !out || ldp < F || ldo < F) return NAPY_E_INVALID;
    if (method != NAPY_ADJ_BONFERRONI && method != NAPY_ADJ_BH && method != NAPY_ADJ_BY) return NAPY_E_INVALID;
    if ((const void*)out == (const void*)p) {
        if (ldo != ldp) return NAPY_E_INVALID;
    } else {
        // any other overlap of the two F x F matrices is refused
        const uintptr_t pa = (uintptr_t)p, pb = pa + (uintptr_t)((F - 1) * ldp + F) * sizeof(double);
        const uintptr_t oa = (uintptr_t)out, ob = oa + (uintptr_t)((F - 1) * ldo + F) * sizeof(double);
        if (pa < ob && oa < pb) return NAPY_E_INVALID;
    }
    if (!ws || ws_bytes < adjust_ws_bytes(F) || ((uintptr_t)ws & 255)) return NAPY_E_WORKSPACE;
    return adjust_run(p, F, ldp, out, ldo, method, ws, (hipStream_t)stream);
}

}  // extern "C"

namespace napy {
__global__ void k_pvalue(const double* __restrict__ r, const int32_t* __restrict__ n, double* __restrict__ p,
                         int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) p[i] = corr_pvalue(r[i], (int64_t)n[i]);
}
}  // namespace napy

extern "C" {

int napy_pvalue_device(const double* r, const int32_t* n, double* p, int64_t count, void* stream)
{
    if (count < 0 || (count > 0 && (!r || !n || !p))) return NAPY_E_INVALID;
    if (count == 0) return NAPY_OK;
    hipLaunchKernelGGL(k_pvalue, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, (hipStream_t)stream, r,
                       n, p, count);
    return check_launch("pvalue");
}

int napy_pvalue_host(const double* r, const int32_t* n, double* p, int64_t count)
{
    if (count < 0 || (count > 0 && (!r || !n || !p))) return NAPY_E_INVALID;
    for (int64_t i = 0; i < count; ++i) p[i] = corr_pvalue(r[i], (int64_t)n[i]);
    return NAPY_OK;
}

}  // extern "C"
