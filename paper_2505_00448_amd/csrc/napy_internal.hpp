// Internal helpers shared by the libnapy translation units (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <atomic>

#include "../../include/napy.h"

namespace napy {

// ---- status reporting ------------------------------------------------------
void set_last_error(const char* fmt, ...);
int hip_status(hipError_t e, const char* what);
// Checks the launch just enqueued; returns NAPY_OK or NAPY_E_HIP.
int check_launch(const char* what);

#define NAPY_TRY(expr)                 \
    do {                               \
        int _st = (expr);              \
        if (_st != NAPY_OK) return _st; \
    } while (0)

// ---- kernel attributes ---------------------------------------------------------
// Raises a kernel's dynamic LDS limit to `bytes` on the current device, once
// per device: bit d of `done` (one flag word per kernel) records device d.
// Threads that race here both set the attribute, which is idempotent; a
// device index of 64 or more sets it on every call.
inline int ensure_dyn_lds(std::atomic<uint64_t>& done, const void* fn, int bytes, const char* what)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "hipGetDevice");
    const uint64_t bit = (dev >= 0 && dev < 64) ? (1ull << dev) : 0ull;
    if (bit != 0ull && (done.load(std::memory_order_acquire) & bit) != 0ull) return NAPY_OK;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return hip_status(e, what);
    done.fetch_or(bit, std::memory_order_acq_rel);
    return NAPY_OK;
}

// ---- workspace carving -------------------------------------------------------
// Regions are carved in order from one caller buffer, each 256-byte aligned.
struct Carver {
    char* base;
    size_t off;
    explicit Carver(void* b) : base((char*)b), off(0) {}
    template <class T>
    T* take(size_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? (T*)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t bytes() const { return (off + 255) & ~(size_t)255; }
};

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// ---- option validation -------------------------------------------------------
inline bool opts_ok(const napy_opts* o)
{
    if (!o) return true;  // NULL means defaults
    if (o->precision < 0 || o->precision > 2) return false;
    if (o->use_sentinel != 0 && o->use_sentinel != 1) return false;
    if (o->reserved != 0) return false;
    return true;
}
inline int opt_prec(const napy_opts* o) { return o ? o->precision : NAPY_PREC_FP32; }
inline int opt_use_sent(const napy_opts* o) { return o ? o->use_sentinel : 0; }
inline float opt_sent(const napy_opts* o) { return o ? o->sentinel : 0.0f; }

// ---- device helpers ------------------------------------------------------------
__device__ __forceinline__ bool is_missing(float v, int use_sent, float sent)
{
    return (v != v) || (use_sent && v == sent);
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// number of set bits of `mask` strictly below the calling lane
__device__ __forceinline__ uint32_t mbcnt64(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Inclusive prefix sum within each row of 16 lanes (DPP row shifts; lanes
// shifted in from outside the row read 0).
__device__ __forceinline__ uint32_t row16_incl_scan_u32(uint32_t v)
{
    constexpr int ROW_SHR = 0x110;
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, ROW_SHR + 1, 0xF, 0xF, false);
    x += __builtin_amdgcn_update_dpp(0, x, ROW_SHR + 2, 0xF, 0xF, false);
    x += __builtin_amdgcn_update_dpp(0, x, ROW_SHR + 4, 0xF, 0xF, false);
    x += __builtin_amdgcn_update_dpp(0, x, ROW_SHR + 8, 0xF, 0xF, false);
    return (uint32_t)x;
}

// Inclusive prefix sum over the 64 lanes of a wave, in DPP moves: shifts by
// 1, 2, 4 and 8 lanes within each row of 16 (lanes shifted in from outside
// the row read 0), then lane 15 of rows 0 and 2 added to rows 1 and 3 and
// lane 31 added to rows 2 and 3 (row broadcasts of the GFX9 DPP set).
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v)
{
    constexpr int ROW_SHR = 0x110, ROW_BCAST15 = 0x142, ROW_BCAST31 = 0x143;
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, ROW_SHR + 1, 0xF, 0xF, false);
    x += __builtin_amdgcn_update_dpp(0, x, ROW_SHR + 2, 0xF, 0xF, false);
    x += __builtin_amdgcn_update_dpp(0, x, ROW_SHR + 4, 0xF, 0xF, false);
    x += __builtin_amdgcn_update_dpp(0, x, ROW_SHR + 8, 0xF, 0xF, false);
    x += __builtin_amdgcn_update_dpp(0, x, ROW_BCAST15, 0xA, 0xF, false);
    x += __builtin_amdgcn_update_dpp(0, x, ROW_BCAST31, 0xC, 0xF, false);
    return (uint32_t)x;
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// ---- shared launch helpers ---------------------------------------------------------
// Column statistics: observed count and mean of every column of X (S x F).
struct ColStats {
    int32_t* n;     // [F]
    float* mu32;    // [F] observed mean rounded to float
    double* mu64;   // [F] observed mean in double
    int32_t* pcnt;  // [R][F] partial counts
    double* psum;   // [R][F] partial sums
    int rows_chunks;
};
// observed-label mask (bit k: label k seen) and invalid-label flag of each
// categorical column (groups.hip)
int labels_launch(const float* L, int64_t ldl, int64_t S, int64_t FC, int ncat, int use_sent, float sent,
                  uint64_t* catmask, int32_t* bad, hipStream_t st);

int colstats_plan_chunks(int64_t S, int64_t F);
void colstats_carve(Carver& c, int64_t S, int64_t F, ColStats& cs);
// zero_word (may be null): a 32-bit word the final kernel also sets to zero
// (a counter that a later kernel of the same call starts from)
int colstats_launch(const float* X, int64_t S, int64_t F, int64_t ldx, int use_sent, float sent,
                    const ColStats& cs, hipStream_t st, uint32_t* zero_word = nullptr);

// Row/column gather for subset queries: Xq[i][c] = X[rows[i]][cols[c]].
int gather_launch(const float* X, int64_t ldx, const int32_t* rows, int64_t Sq,
                  const int32_t* cols, int64_t Fq, float* Xq, hipStream_t st);

// Internal Pearson driver; `saved` may be NULL.
// `ev` (may be NULL): up to 4 caller-created events recorded on `st` before
// the first kernel and after each of the three stages.
int pearson_run(const float* X, int64_t S, int64_t F, int64_t ldx, double* r, double* p,
                int32_t* n, int64_t ldo, double* saved, void* ws, size_t ws_bytes,
                const napy_opts* opts, hipStream_t st, void* const* ev = nullptr);

// Pearson with its workspace in a fixed per-device array of the library (no
// allocation by anyone); NAPY_E_UNSUPPORTED when (S, F) needs more.
int pearson_noalloc_run(const float* X, int64_t S, int64_t F, int64_t ldx, double* r, double* p, int32_t* n,
                        int64_t ldo, const napy_opts* opts, hipStream_t st);

inline int record_stage(void* const* ev, int i, hipStream_t st)
{
    if (!ev || !ev[i]) return NAPY_OK;
    return hip_status(hipEventRecord((hipEvent_t)ev[i], st), "hipEventRecord");
}
size_t pearson_ws_bytes(int64_t S, int64_t F, int prec);

}  // namespace napy
