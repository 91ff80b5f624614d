// Pearson correlation with pairwise deletion as masked dense contractions on
// the gfx950 matrix cores (NApy, arXiv 2505.00448, Sections 3.2 and 3.5.2).
//
// For a pair (g, h) with pairwise-complete set I(g,h) and data centred on each
// column's observed mean (r is shift invariant), the six sums
//     n = sum_I 1, Sx = sum_I x_g, Sy = sum_I x_h,
//     Sxx = sum_I x_g^2, Syy = sum_I x_h^2, Sxy = sum_I x_g x_h
// are entries of products of the zero-filled data X0 (S x F), the 0/1
// presence matrix M and Q = X0 o X0:
//     n = M'M, Sx = X0'M, Sy = M'X0, Sxx = Q'M, Syy = M'Q, Sxy = X0'X0.
// Missing values are removed by the zero fill and the partner's mask inside
// every product, so no per-pair subsetting is needed.
//
// Kernels:
//   k_colstats_*     observed count and mean per column (HBM-bound, 1 pass).
//   k_pearson_tiles  one 64 x 64 output tile of the upper triangle over one
//                    range of samples (split-K).  The tile's panels are read
//                    straight from X (row-major, variables contiguous),
//                    centred, converted to the precision's operand planes and
//                    staged through LDS; four waves each own a 32 x 32 block.
//                    FP32 accumulators are flushed into FP64 registers every
//                    FLUSH samples; the FP64 partial sums go to the workspace.
//   k_pearson_combine  sums the split-K partials in FP64, forms
//                    C = n Sxy - Sx Sy, Vx = n Sxx - Sx^2, Vy = n Syy - Sy^2,
//                    r = C / sqrt(Vx Vy) and p, and writes both triangles;
//                    a pair whose complete samples sit far from a column's
//                    mean (or that is constant on I(g,h)) is listed instead.
//   k_pearson_recompute  the listed pairs from the raw values, two passes in
//                    FP64 about the pair's own means, zero variance decided
//                    exactly.
//
// Precisions (napy_opts.precision):
//   FP32    v_mfma_f32_16x16x4_f32, 6 products per pair-sample.
//   BF16X3  v_mfma_f32_32x32x16_bf16 on operands split into three bf16
//           pieces each, x0 = xh + xm + xl and q = qh + qm + ql (exact for
//           float32 inputs); 19 products per pair-sample: n 1, Sx 3, Sy 3,
//           Sxx 3, Syy 3, Sxy 6 (every piece product down to 2^-18 relative:
//           hh, hm, mh, hl, mm, lh).  A two-piece split of x (16 significant
//           bits) perturbs r by more than 1e-6 on short or adversarial
//           columns, so the third piece is kept.
//   FP64    v_mfma_f64_16x16x4_f64 (validation mode).
#include <mutex>
#include <type_traits>

#include "napy_internal.hpp"
#include "pvalue.hpp"
#include "tilefin.hpp"

namespace napy {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int TILE = 64;
constexpr int TILE_ELEMS = TILE * TILE;
constexpr int NSTAT = 6;  // n, Sx, Sy, Sxx, Syy, Sxy

// ---------------------------------------------------------------------------
// K1: column statistics
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_colstats_partial(
    const float* __restrict__ X, int64_t S, int64_t F, int64_t ldx, int use_sent, float sent,
    int64_t rows_per, int32_t* __restrict__ pcnt, double* __restrict__ psum)
{
    __shared__ int32_t sc[4][64];
    __shared__ double ss[4][64];
    const int c = threadIdx.x & 63, rl = threadIdx.x >> 6;
    const int64_t col = (int64_t)blockIdx.x * 64 + c;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per;
    const int64_t r1 = min(S, r0 + rows_per);
    int32_t cnt = 0;
    double sum = 0.0;
    if (col < F) {
        for (int64_t i = r0 + rl; i < r1; i += 4) {
            const float v = X[i * ldx + col];
            if (!is_missing(v, use_sent, sent)) {
                ++cnt;
                sum += (double)v;
            }
        }
    }
    sc[rl][c] = cnt;
    ss[rl][c] = sum;
    __syncthreads();
    if (rl == 0 && col < F) {
        pcnt[(int64_t)blockIdx.y * F + col] = sc[0][c] + sc[1][c] + sc[2][c] + sc[3][c];
        psum[(int64_t)blockIdx.y * F + col] = ((ss[0][c] + ss[1][c]) + ss[2][c]) + ss[3][c];
    }
}

// The same partial sums from 16-byte loads (X 16-byte aligned, ldx a
// multiple of 4): four adjacent columns per thread, 256 per workgroup, four
// rows' loads issued before their adds.  Each column's rows are added in the
// same order as above (rows r0 + rl, r0 + rl + 4, ... per wave, then the four
// waves' sums as ((w0 + w1) + w2) + w3), so the sums are bit-identical.
__global__ __launch_bounds__(256) void k_colstats_partial4(
    const float* __restrict__ X, int64_t S, int64_t F, int64_t ldx, int use_sent, float sent,
    int64_t rows_per, int32_t* __restrict__ pcnt, double* __restrict__ psum)
{
    __shared__ int32_t sc[4][256];
    __shared__ double ss[4][256];
    const int c = threadIdx.x & 63, rl = threadIdx.x >> 6;
    const int64_t col0 = (int64_t)blockIdx.x * 256 + 4 * c;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per;
    const int64_t r1 = min(S, r0 + rows_per);
    int32_t cnt[4] = {0, 0, 0, 0};
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
    const auto add = [&](int q, float v) {
        if (!is_missing(v, use_sent, sent)) {
            ++cnt[q];
            sum[q] += (double)v;
        }
    };
    if (col0 + 3 < F) {
        int64_t i = r0 + rl;
        for (; i + 12 < r1; i += 16) {
            float4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = *(const float4*)(X + (i + 4 * u) * ldx + col0);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                add(0, v[u].x);
                add(1, v[u].y);
                add(2, v[u].z);
                add(3, v[u].w);
            }
        }
        for (; i < r1; i += 4) {
            const float4 v = *(const float4*)(X + i * ldx + col0);
            add(0, v.x);
            add(1, v.y);
            add(2, v.z);
            add(3, v.w);
        }
    } else if (col0 < F) {
        for (int64_t i = r0 + rl; i < r1; i += 4)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (col0 + q < F) add(q, X[i * ldx + col0 + q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        sc[rl][4 * c + q] = cnt[q];
        ss[rl][4 * c + q] = sum[q];
    }
    __syncthreads();
    const int t = threadIdx.x;
    const int64_t col = (int64_t)blockIdx.x * 256 + t;
    if (col < F) {
        pcnt[(int64_t)blockIdx.y * F + col] = sc[0][t] + sc[1][t] + sc[2][t] + sc[3][t];
        psum[(int64_t)blockIdx.y * F + col] = ((ss[0][t] + ss[1][t]) + ss[2][t]) + ss[3][t];
    }
}

// one wave per column: each lane sums the partials r = lane, lane + 64, ...
// and a fixed butterfly adds the lanes (the same order on every call)
__global__ __launch_bounds__(256) void k_colstats_final(
    int R, int64_t F, const int32_t* __restrict__ pcnt, const double* __restrict__ psum,
    int32_t* __restrict__ ncol, float* __restrict__ mu32, double* __restrict__ mu64, uint32_t* __restrict__ zero_word)
{
    if (zero_word && blockIdx.x == 0 && threadIdx.x == 0) *zero_word = 0u;
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= F) return;
    int32_t n = 0;
    double s = 0.0;
    for (int r = lane; r < R; r += 64) {
        n += pcnt[(int64_t)r * F + c];
        s += psum[(int64_t)r * F + c];
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        n += __shfl_xor(n, d, 64);
        s += __shfl_xor(s, d, 64);
    }
    if (lane == 0) {
        const double m = n > 0 ? s / (double)n : 0.0;
        ncol[c] = n;
        mu64[c] = m;
        mu32[c] = (float)m;
    }
}

int colstats_plan_chunks(int64_t S, int64_t F)
{
    const int64_t cb = ceil_div(F, 64);
    int64_t R = ceil_div(2048, cb);
    const int64_t rmax = ceil_div(S, 64);
    if (R > rmax) R = rmax;
    if (R < 1) R = 1;
    return (int)R;
}

void colstats_carve(Carver& c, int64_t S, int64_t F, ColStats& cs)
{
    cs.rows_chunks = colstats_plan_chunks(S, F);
    cs.n = c.take<int32_t>(F);
    cs.mu32 = c.take<float>(F);
    cs.mu64 = c.take<double>(F);
    cs.pcnt = c.take<int32_t>((size_t)cs.rows_chunks * F);
    cs.psum = c.take<double>((size_t)cs.rows_chunks * F);
}

int colstats_launch(const float* X, int64_t S, int64_t F, int64_t ldx, int use_sent, float sent,
                    const ColStats& cs, hipStream_t st, uint32_t* zero_word)
{
    const int R = cs.rows_chunks;
    const int64_t rows_per = ceil_div(S, R);
    if (((uintptr_t)X & 15u) == 0 && (ldx & 3) == 0) {
        dim3 g1((unsigned)ceil_div(F, 256), (unsigned)R);
        hipLaunchKernelGGL(k_colstats_partial4, g1, dim3(256), 0, st, X, S, F, ldx, use_sent, sent,
                           rows_per, cs.pcnt, cs.psum);
    } else {
        dim3 g1((unsigned)ceil_div(F, 64), (unsigned)R);
        hipLaunchKernelGGL(k_colstats_partial, g1, dim3(256), 0, st, X, S, F, ldx, use_sent, sent,
                           rows_per, cs.pcnt, cs.psum);
    }
    NAPY_TRY(check_launch("colstats_partial"));
    hipLaunchKernelGGL(k_colstats_final, dim3((unsigned)ceil_div(F, 4)), dim3(256), 0, st, R, F,
                       cs.pcnt, cs.psum, cs.n, cs.mu32, cs.mu64, zero_word);
    return check_launch("colstats_final");
}

// ---------------------------------------------------------------------------
// gather for subset queries
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gather(const float* __restrict__ X, int64_t ldx,
                                                const int32_t* __restrict__ rows, int64_t Sq,
                                                const int32_t* __restrict__ cols, int64_t Fq,
                                                float* __restrict__ Xq)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= Fq) return;
    const int64_t src_c = cols[c];
    for (int64_t i = blockIdx.y; i < Sq; i += gridDim.y)
        Xq[i * Fq + c] = X[(int64_t)rows[i] * ldx + src_c];
}

int gather_launch(const float* X, int64_t ldx, const int32_t* rows, int64_t Sq, const int32_t* cols,
                  int64_t Fq, float* Xq, hipStream_t st)
{
    int64_t gy = Sq < 1024 ? Sq : 1024;
    if (gy < 1) gy = 1;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)ceil_div(Fq, 256), (unsigned)gy), dim3(256), 0, st,
                       X, ldx, rows, Sq, cols, Fq, Xq);
    return check_launch("gather");
}

// ---------------------------------------------------------------------------
// K2: tile contractions
// ---------------------------------------------------------------------------
template <int PREC>
struct TileCfg;
template <>
struct TileCfg<NAPY_PREC_FP32> {
    static constexpr int BK = 32;     // samples per LDS slab
    static constexpr int LDK = 36;    // LDS row stride (elements)
    static constexpr int FLUSH = 256; // FP32 -> FP64 flush period (samples)
    static constexpr int RPT = 8;     // rows per thread in the staging step
};
template <>
struct TileCfg<NAPY_PREC_FP64> {
    static constexpr int BK = 16;
    static constexpr int LDK = 18;
    static constexpr int FLUSH = 0;
    static constexpr int RPT = 4;
};

// Maps the hardware block index to a logical work index so that every XCD
// (blocks are dealt to the 8 XCDs round-robin) receives a contiguous range of
// logical work, which keeps the rows and panels that neighbouring work items
// read in one L2.
__device__ __forceinline__ int xcd_logical_block(int bid, int nb)
{
    const int x = bid & 7, q = bid >> 3;
    const int base = nb >> 3, rem = nb & 7;
    return x * base + (x < rem ? x : rem) + q;
}

template <int PREC>
struct LdsPlan;
template <>
struct LdsPlan<NAPY_PREC_FP32> {
    static constexpr int ELEMS = 2 * TILE * TileCfg<NAPY_PREC_FP32>::LDK;  // floats per buffer
};
template <>
struct LdsPlan<NAPY_PREC_FP64> {
    static constexpr int ELEMS = 2 * TILE * TileCfg<NAPY_PREC_FP64>::LDK;  // doubles per buffer
};

// FP32 and FP64 forms (the split-BF16 form is k_pearson_bf16 below).
template <int PREC>
__global__ __launch_bounds__(256, 1) void k_pearson_tiles(
    const float* __restrict__ X, int64_t S, int64_t F, int64_t ldx, int use_sent, float sent,
    const float* __restrict__ mu32, const double* __restrict__ mu64, int T, int ntiles, int nsplit,
    int64_t ksplit, double* __restrict__ part)
{
    static_assert(PREC == NAPY_PREC_FP32 || PREC == NAPY_PREC_FP64, "FP32 or FP64 tiles");
    using C = TileCfg<PREC>;
    constexpr int BK = C::BK, LDK = C::LDK, RPT = C::RPT;

    const int lb = xcd_logical_block((int)blockIdx.x, (int)gridDim.x);
    // split-major: an XCD's workgroups are tiles of one sample range, which
    // read the same rows of X at about the same time (one fetch into its L2)
    const int split = lb / ntiles, t = lb % ntiles;
    int tg, th;
    tile_coords(t, T, tg, th);

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wave
    const int wm = wave >> 1, wn = wave & 1;

    const int64_t kbeg = (int64_t)split * ksplit;
    int64_t kend = kbeg + ksplit;
    if (kend > S) kend = S;
    const int nslab = kend > kbeg ? (int)ceil_div(kend - kbeg, BK) : 0;

    // staging coordinates: column c of the panel, rows [kg*RPT, kg*RPT+RPT) of the slab
    const int sc = tid & 63, kg = tid >> 6;
    const int64_t colG = (int64_t)tg * TILE + sc, colH = (int64_t)th * TILE + sc;
    const bool okG = colG < F, okH = colH < F;

    // ---- LDS ----------------------------------------------------------------
    using LT = typename std::conditional<PREC == NAPY_PREC_FP64, double, float>::type;
    constexpr int BUF = LdsPlan<PREC>::ELEMS;
    __shared__ __attribute__((aligned(16))) LT lds[2 * BUF];

    // raw staging registers for the two panels
    float rawG[RPT], rawH[RPT];

    auto load_raw = [&](int slab) {
        const int64_t i0 = kbeg + (int64_t)slab * BK + kg * RPT;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int64_t i = i0 + j;
            const bool in = i < kend;
            rawG[j] = (in && okG) ? X[i * ldx + colG] : __builtin_nanf("");
            rawH[j] = (in && okH) ? X[i * ldx + colH] : __builtin_nanf("");
        }
    };

    const float muG32 = okG ? mu32[colG] : 0.0f, muH32 = okH ? mu32[colH] : 0.0f;
    const double muG64 = okG ? mu64[colG] : 0.0, muH64 = okH ? mu64[colH] : 0.0;

    auto store_lds = [&](int buf) {
        LT* base = lds + buf * BUF;
        if constexpr (PREC == NAPY_PREC_FP32) {
            // layout [side][col][LDK]; missing -> NaN
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                float v[RPT];
#pragma unroll
                for (int j = 0; j < RPT; ++j) {
                    const float raw = side ? rawH[j] : rawG[j];
                    const float mu = side ? muH32 : muG32;
                    v[j] = is_missing(raw, use_sent, sent) ? __builtin_nanf("") : raw - mu;
                }
                float* dst = base + (side * TILE + sc) * LDK + kg * RPT;
                *(f32x4*)(dst) = f32x4{v[0], v[1], v[2], v[3]};
                *(f32x4*)(dst + 4) = f32x4{v[4], v[5], v[6], v[7]};
            }
        } else if constexpr (PREC == NAPY_PREC_FP64) {
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                double v[RPT];
#pragma unroll
                for (int j = 0; j < RPT; ++j) {
                    const float raw = side ? rawH[j] : rawG[j];
                    const double mu = side ? muH64 : muG64;
                    v[j] = is_missing(raw, use_sent, sent) ? __builtin_nan("") : (double)raw - mu;
                }
                double* dst = base + (side * TILE + sc) * LDK + kg * RPT;
#pragma unroll
                for (int j = 0; j < RPT; ++j) dst[j] = v[j];
            }
        }
    };

    // ---- accumulators: four 16x16 sub-blocks per wave, acc[sub][stat] x4 ----
    // FP32 sums are added into FP64 registers every FLUSH samples.
    constexpr int NSUB = 4, NREG = 4, NACC = NSTAT;
    using AccT = typename std::conditional<PREC == NAPY_PREC_FP64, double, float>::type;
    AccT acc[NSUB][NACC][NREG];
    constexpr int N64 = (PREC == NAPY_PREC_FP32) ? NSTAT : 1;  // FP64 sums (unused in FP64 mode)
    double acc64[NSUB][N64][NREG];
#pragma unroll
    for (int a = 0; a < NSUB; ++a) {
#pragma unroll
        for (int s = 0; s < NACC; ++s)
#pragma unroll
            for (int r = 0; r < NREG; ++r) acc[a][s][r] = 0;
#pragma unroll
        for (int s = 0; s < N64; ++s)
#pragma unroll
            for (int r = 0; r < NREG; ++r) acc64[a][s][r] = 0.0;
    }

    auto flush = [&]() {
        if constexpr (PREC == NAPY_PREC_FP32) {
#pragma unroll
            for (int a = 0; a < NSUB; ++a)
#pragma unroll
                for (int s = 0; s < NSTAT; ++s)
#pragma unroll
                    for (int r = 0; r < NREG; ++r) {
                        acc64[a][s][r] += (double)acc[a][s][r];
                        acc[a][s][r] = 0.0f;
                    }
        }
    };

    auto compute = [&](int buf) {
        const LT* base = lds + buf * BUF;
        const int rr = lane & 15, kq = lane >> 4;
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            const int k = kk * 4 + kq;
            AccT xa[2], ma[2], qa[2], xb[2], mb[2], qb[2];
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                const AccT va = base[(0 * TILE + wm * 32 + s2 * 16 + rr) * LDK + k];
                const AccT vb = base[(1 * TILE + wn * 32 + s2 * 16 + rr) * LDK + k];
                const bool pa = va == va, pb = vb == vb;
                xa[s2] = pa ? va : (AccT)0;
                ma[s2] = pa ? (AccT)1 : (AccT)0;
                qa[s2] = xa[s2] * xa[s2];
                xb[s2] = pb ? vb : (AccT)0;
                mb[s2] = pb ? (AccT)1 : (AccT)0;
                qb[s2] = xb[s2] * xb[s2];
            }
#pragma unroll
            for (int ia = 0; ia < 2; ++ia)
#pragma unroll
                for (int ib = 0; ib < 2; ++ib) {
                    const int sub = ia * 2 + ib;
                    if constexpr (PREC == NAPY_PREC_FP32) {
                        f32x4 c[NSTAT];
#pragma unroll
                        for (int s = 0; s < NSTAT; ++s)
                            c[s] = f32x4{acc[sub][s][0], acc[sub][s][1], acc[sub][s][2], acc[sub][s][3]};
                        c[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(ma[ia], mb[ib], c[0], 0, 0, 0);
                        c[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[ia], mb[ib], c[1], 0, 0, 0);
                        c[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(ma[ia], xb[ib], c[2], 0, 0, 0);
                        c[3] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[ia], mb[ib], c[3], 0, 0, 0);
                        c[4] = __builtin_amdgcn_mfma_f32_16x16x4f32(ma[ia], qb[ib], c[4], 0, 0, 0);
                        c[5] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[ia], xb[ib], c[5], 0, 0, 0);
#pragma unroll
                        for (int s = 0; s < NSTAT; ++s)
#pragma unroll
                            for (int r = 0; r < 4; ++r) acc[sub][s][r] = c[s][r];
                    } else {
                        f64x4 c[NSTAT];
#pragma unroll
                        for (int s = 0; s < NSTAT; ++s)
                            c[s] = f64x4{acc[sub][s][0], acc[sub][s][1], acc[sub][s][2], acc[sub][s][3]};
                        c[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ma[ia], mb[ib], c[0], 0, 0, 0);
                        c[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[ia], mb[ib], c[1], 0, 0, 0);
                        c[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(ma[ia], xb[ib], c[2], 0, 0, 0);
                        c[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[ia], mb[ib], c[3], 0, 0, 0);
                        c[4] = __builtin_amdgcn_mfma_f64_16x16x4f64(ma[ia], qb[ib], c[4], 0, 0, 0);
                        c[5] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[ia], xb[ib], c[5], 0, 0, 0);
#pragma unroll
                        for (int s = 0; s < NSTAT; ++s)
#pragma unroll
                            for (int r = 0; r < 4; ++r) acc[sub][s][r] = c[s][r];
                    }
                }
        }
    };

    // ---- main loop: one barrier per slab, staging of slab s+1 overlaps the
    // contractions of slab s ------------------------------------------------------
    constexpr int FLUSH_SLABS = C::FLUSH > 0 ? C::FLUSH / BK : 0;
    if (nslab > 0) {
        load_raw(0);
        store_lds(0);
        __syncthreads();
        for (int s = 0; s < nslab; ++s) {
            const bool more = s + 1 < nslab;
            if (more) load_raw(s + 1);
            compute(s & 1);
            if (more) store_lds((s + 1) & 1);
            if constexpr (FLUSH_SLABS > 0) {
                if ((s + 1) % FLUSH_SLABS == 0) flush();
            }
            __syncthreads();
        }
    }
    flush();

    // ---- epilogue: FP64 partials [split][stat][tile][64][64] -----------------------
#pragma unroll
    for (int s = 0; s < NSTAT; ++s) {
        double* dst = part + (((int64_t)split * NSTAT + s) * ntiles + t) * TILE_ELEMS;
#pragma unroll
        for (int ia = 0; ia < 2; ++ia)
#pragma unroll
            for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    // 16x16 blocks: f32 rows are 4*(lane/16) + r, f64 rows are
                    // lane/16 + 4*r; columns are lane%16 in both
                    const int ri = (PREC == NAPY_PREC_FP64) ? ((lane >> 4) + 4 * r) : (4 * (lane >> 4) + r);
                    const int i = wm * 32 + ia * 16 + ri;
                    const int j = wn * 32 + ib * 16 + (lane & 15);
                    const double v = (PREC == NAPY_PREC_FP64) ? (double)acc[ia * 2 + ib][s][r]
                                                               : acc64[ia * 2 + ib][s][r];
                    dst[i * TILE + j] = v;
                }
    }
}

// ---------------------------------------------------------------------------
// K2, split-BF16 form.  One 64 x 64 output tile over one range of samples,
// 256 threads (four waves, each a 32 x 32 block), slabs of 16 samples = one
// v_mfma_f32_32x32x16_bf16 step, double-buffered in LDS (57 KB, two
// workgroups per CU).  Nine FP32 accumulators stay in place across the loop:
// n; Sx and Sy (all three pieces each); Sxx, Syy, Sxy as a main accumulator
// for the leading piece products and a low one for the trailing ones (the
// matrix cores add each block into the accumulator with one rounding toward
// zero, so tiny trailing products are kept away from the large leading
// sums).  Every 1024 samples the Sxx, Syy and Sxy accumulators are added into
// the workgroup's FP64 partial sums in the workspace and cleared; the sums
// of centred values Sx, Sy stay small and are written once at the end.
// ---------------------------------------------------------------------------
namespace bf3 {
constexpr int BK = 16;
constexpr int NPL = 7;                  // xh, xm, xl, qh, qm, ql, m
constexpr int PLANE = TILE * BK;        // bf16 per plane
constexpr int BUF = 2 * NPL * PLANE;    // one slab, both sides
constexpr int FLUSH_SLABS = 1024 / BK;
static_assert(FLUSH_SLABS % 2 == 0, "blocks of slabs start on an even slab");
}  // namespace bf3

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// two floats to bf16 (round to nearest even) in one conversion
__device__ __forceinline__ bf16x2 to_bf16x2(float a, float b)
{
    return __builtin_convertvector((f32x2){a, b}, bf16x2);
}

template <bool SENT, bool GEN>
__global__ __launch_bounds__(256, 2) void k_pearson_bf16(
    const float* __restrict__ X, int64_t S, int64_t F, int64_t ldx, int use_sent, float sent,
    const float* __restrict__ mu32, int T, int ntiles, int nsplit, int64_t ksplit, double* __restrict__ part)
{
    using namespace bf3;
    const int lb = xcd_logical_block((int)blockIdx.x, (int)gridDim.x);
    // split-major: an XCD's workgroups are tiles of one sample range, which
    // read the same rows of X at about the same time (one fetch into its L2)
    const int split = lb / ntiles, t = lb % ntiles;
    int tg, th;
    tile_coords(t, T, tg, th);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t kbeg = (int64_t)split * ksplit;
    int64_t kend = kbeg + ksplit;
    if (kend > S) kend = S;
    const int nslab = kend > kbeg ? (int)ceil_div(kend - kbeg, BK) : 0;

    // staging: column sc of both panels, samples 4 kq .. 4 kq + 3 of the slab
    const int sc = tid & 63, kq = tid >> 6;
    const int64_t colG = (int64_t)tg * TILE + sc, colH = (int64_t)th * TILE + sc;
    const bool okG = colG < F, okH = colH < F;
    const float muG = okG ? mu32[colG] : 0.0f, muH = okH ? mu32[colH] : 0.0f;

    __shared__ __attribute__((aligned(16))) __bf16 lds[2 * BUF];
    // raw values of two slabs in flight (sets A and B, alternating).  Every
    // slab is read as 16 whole rows from a row pointer (uniform) plus 32-bit
    // byte offsets fixed per thread, one instruction sequence for all slabs
    // (so the wait for a slab's values does not also wait for the loads of
    // the slab after it): a slab that would run past kend is moved back to
    // end at kend, and its rows before the slab's own start, counted already
    // (or belonging to the previous split), are staged as missing.  A column
    // past F is read as column 0 and counted missing in store_lds.  GEN (S
    // below one slab, or rows too long for 32-bit offsets) clamps each row
    // index instead.
    float rawG[4], rawH[4], nxtG[4], nxtH[4];
    const int64_t cG = okG ? colG : 0, cH = okH ? colH : 0;
    uint32_t offG[4], offH[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        offG[j] = ((uint32_t)(kq * 4 + j) * (uint32_t)ldx + (uint32_t)cG) * 4u;
        offH[j] = ((uint32_t)(kq * 4 + j) * (uint32_t)ldx + (uint32_t)cH) * 4u;
    }
    // first row of the 16 that slab `slab` reads (uniform)
    auto slab_base = [&](int slab) -> int64_t {
        const int64_t s0 = kbeg + (int64_t)slab * BK;
        return s0 < kend - BK ? s0 : kend - BK;
    };
    // leading rows of the slab read as missing
    auto lead_missing = [&](int slab) -> int {
        if constexpr (GEN) return 0;
        return (int)(kbeg + (int64_t)slab * BK - slab_base(slab));
    };
    auto load_raw = [&](int slab, float (&rg)[4], float (&rh)[4]) {
        if constexpr (!GEN) {
            const char* row = (const char*)(X + slab_base(slab) * ldx);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                rg[j] = *(const float*)(row + offG[j]);
                rh[j] = *(const float*)(row + offH[j]);
            }
        } else {
            const int64_t i0 = kbeg + (int64_t)slab * BK + kq * 4;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t i = i0 + j;
                const int64_t ic = i < kend ? i : kend - 1;
                rg[j] = X[ic * ldx + cG];
                rh[j] = X[ic * ldx + cH];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool in = i0 + j < kend;
                rg[j] = in ? rg[j] : __builtin_nanf("");
                rh[j] = in ? rh[j] : __builtin_nanf("");
            }
        }
    };
    // LDS rows are 32 B (16 samples); the two 16-B halves of row c are
    // swapped when bit 3 of c is set, so that the 16-lane phases of the
    // row-wise 16-B reads below hit distinct banks
    // (lo: leading rows of the slab read as missing; a comparison per sample
    // rather than a branch, which would make the wait for this slab's values
    // also wait for the loads issued after them)
    auto store_lds = [&](int buf, const float (&rG)[4], const float (&rH)[4], int lo) {
        __bf16* base = lds + buf * BUF;
        const int slot = (kq ^ (((sc >> 3) & 1) << 1)) * 4;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            bf16x4 pl[NPL];
#pragma unroll
            for (int jp = 0; jp < 2; ++jp) {
                float x[2], q[2];
                bool miss[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const float raw = side ? rH[2 * jp + u] : rG[2 * jp + u];
                    // bitwise, not short-circuit: no control flow in the loop
                    // body, so the contractions and the staging interleave
                    miss[u] = (raw != raw) | (SENT & (raw == sent)) | !(side ? okH : okG) |
                              (kq * 4 + 2 * jp + u < lo);
                    x[u] = miss[u] ? 0.0f : raw - (side ? muH : muG);
                    q[u] = x[u] * x[u];
                }
                // x = xh + xm + xl and q = qh + qm + ql exactly, two samples
                // per conversion
                const bf16x2 xh = to_bf16x2(x[0], x[1]);
                const float x10 = x[0] - (float)xh[0], x11 = x[1] - (float)xh[1];
                const bf16x2 xm = to_bf16x2(x10, x11);
                const bf16x2 xl = to_bf16x2(x10 - (float)xm[0], x11 - (float)xm[1]);
                const bf16x2 qh = to_bf16x2(q[0], q[1]);
                const float q10 = q[0] - (float)qh[0], q11 = q[1] - (float)qh[1];
                const bf16x2 qm = to_bf16x2(q10, q11);
                const bf16x2 ql = to_bf16x2(q10 - (float)qm[0], q11 - (float)qm[1]);
                const bf16x2 mk = to_bf16x2(miss[0] ? 0.0f : 1.0f, miss[1] ? 0.0f : 1.0f);
                const bf16x2 v[NPL] = {xh, xm, xl, qh, qm, ql, mk};
#pragma unroll
                for (int pp = 0; pp < NPL; ++pp) {
                    pl[pp][2 * jp] = v[pp][0];
                    pl[pp][2 * jp + 1] = v[pp][1];
                }
            }
#pragma unroll
            for (int pp = 0; pp < NPL; ++pp)
                *(bf16x4*)(base + ((side * NPL + pp) * TILE + sc) * BK + slot) = pl[pp];
        }
    };

    f32x16 aN, aSx, aSy, aSxx, aSxxL, aSyy, aSyyL, aSxy, aSxyL;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        aN[r] = 0.f; aSx[r] = 0.f; aSy[r] = 0.f;
        aSxx[r] = 0.f; aSxxL[r] = 0.f; aSyy[r] = 0.f; aSyyL[r] = 0.f; aSxy[r] = 0.f; aSxyL[r] = 0.f;
    }
    auto compute = [&](int buf) {
        const __bf16* base = lds + buf * BUF;
        const int rr = lane & 31, kk = ((lane >> 5) ^ ((rr >> 3) & 1)) * 8;  // swizzled half
        // all seven planes of the G side; the H side's planes one at a time
        bf16x8 a[NPL];
#pragma unroll
        for (int pp = 0; pp < NPL; ++pp)
            a[pp] = *(const bf16x8*)(base + ((0 * NPL + pp) * TILE + wm * 32 + rr) * BK + kk);
        auto bpl = [&](int pp) -> bf16x8 {
            return *(const bf16x8*)(base + ((1 * NPL + pp) * TILE + wn * 32 + rr) * BK + kk);
        };
        // planes: 0 xh, 1 xm, 2 xl, 3 qh, 4 qm, 5 ql, 6 m
#define NAPY_MF(acc, x, y) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, acc, 0, 0, 0)
        {
            const bf16x8 b = bpl(6);
            NAPY_MF(aN, a[6], b);
            NAPY_MF(aSx, a[0], b);
            NAPY_MF(aSxx, a[3], b);
            NAPY_MF(aSx, a[1], b);
            NAPY_MF(aSxxL, a[4], b);
            NAPY_MF(aSx, a[2], b);
            NAPY_MF(aSxxL, a[5], b);
        }
        {
            const bf16x8 b = bpl(0);
            NAPY_MF(aSy, a[6], b);
            NAPY_MF(aSxy, a[0], b);
            NAPY_MF(aSxyL, a[1], b);
            NAPY_MF(aSxyL, a[2], b);
        }
        {
            const bf16x8 b = bpl(1);
            NAPY_MF(aSy, a[6], b);
            NAPY_MF(aSxyL, a[0], b);
            NAPY_MF(aSxyL, a[1], b);
        }
        {
            const bf16x8 b = bpl(2);
            NAPY_MF(aSy, a[6], b);
            NAPY_MF(aSxyL, a[0], b);
        }
        NAPY_MF(aSyy, a[6], bpl(3));
        NAPY_MF(aSyyL, a[6], bpl(4));
        NAPY_MF(aSyyL, a[6], bpl(5));
#undef NAPY_MF
    };

    // output element of accumulator register r (32 x 32 block layout): the
    // lane's base element plus a constant offset per register
    const int ebase = (wm * 32 + 4 * (lane >> 5)) * TILE + wn * 32 + (lane & 31);
    auto eoff = [](int r) -> int { return (8 * (r >> 2) + (r & 3)) * TILE; };
    auto slice = [&](int s) -> double* {
        return part + (((int64_t)split * NSTAT + s) * ntiles + t) * TILE_ELEMS + ebase;
    };
    bool flushed = false;
    auto flush = [&]() {
        double* d3 = slice(3);
        double* d4 = slice(4);
        double* d5 = slice(5);
        // keep the addresses from being computed ahead of the loop (they
        // would occupy registers for its whole length)
        asm volatile("" : "+v"(d3), "+v"(d4), "+v"(d5));
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int e = eoff(r);
            const double v3 = (double)aSxx[r] + (double)aSxxL[r];
            const double v4 = (double)aSyy[r] + (double)aSyyL[r];
            const double v5 = (double)aSxy[r] + (double)aSxyL[r];
            d3[e] = flushed ? d3[e] + v3 : v3;
            d4[e] = flushed ? d4[e] + v4 : v4;
            d5[e] = flushed ? d5[e] + v5 : v5;
            aSxx[r] = 0.f; aSxxL[r] = 0.f; aSyy[r] = 0.f; aSyyL[r] = 0.f; aSxy[r] = 0.f; aSxyL[r] = 0.f;
        }
        flushed = true;
    };

    // main loop, one barrier per slab: the contractions of slab s overlap the
    // staging of slab s+1, whose raw values were loaded one slab earlier
    // (global latency is longer than one slab's contractions); the
    // scheduling hints interleave the staging's VALU work with the MFMAs
    auto step = [&](int sl, const float (&cG)[4], const float (&cH)[4], float (&lG)[4], float (&lH)[4]) {
        load_raw(sl + 2, lG, lH);
        compute(sl & 1);
        store_lds((sl + 1) & 1, cG, cH, lead_missing(sl + 1));
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 6, 0);  // six VALU
        }
        __syncthreads();
    };
    // blocks of FLUSH_SLABS slabs (an even count, so every block starts with
    // the next slab's values in rawG / rawH), the flush between blocks: the
    // inner loop holds no global access but the raw loads, and its body is
    // one block of code
    if (nslab > 0) {
        load_raw(0, rawG, rawH);
        store_lds(0, rawG, rawH, lead_missing(0));
        load_raw(1, rawG, rawH);
        __syncthreads();
        int sl = 0;
        for (;;) {
            const int be = min(nslab, sl + FLUSH_SLABS);
            for (; sl + 1 < be; sl += 2) {
                step(sl, rawG, rawH, nxtG, nxtH);
                step(sl + 1, nxtG, nxtH, rawG, rawH);
            }
            if (sl < be) {  // an odd count: the last block
                step(sl, rawG, rawH, nxtG, nxtH);
                ++sl;
            }
            if (sl >= nslab) break;
            flush();
            // every global access complete (vmcnt 0): the next block starts
            // in the state its own loop leaves, so its waits stay exact
            __builtin_amdgcn_s_waitcnt(0x0F70);
        }
    }
    flush();
    double* d0 = slice(0);
    double* d1 = slice(1);
    double* d2 = slice(2);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int e = eoff(r);
        d0[e] = (double)aN[r];
        d1[e] = (double)aSx[r];
        d2[e] = (double)aSy[r];
    }
}

// ---------------------------------------------------------------------------
// K3: combine split-K partials, r, p, n; both triangles
// ---------------------------------------------------------------------------
// A pair is combined from its sums when, on both sides, the variance about
// the pair's own mean is at least WELL_CENTRED of the second moment about the
// column mean (n Sxx - Sx^2 >= WELL_CENTRED n Sxx): the rounding error of the
// accumulated sums then reaches r amplified by at most 1 / WELL_CENTRED.
// Every other pair with n >= 2 -- complete samples far from the column mean,
// and every pair that is constant on I(g,h) -- goes to a list and is
// recomputed from the raw values by k_pearson_recompute.
constexpr double WELL_CENTRED = 0.9;
constexpr int NSAVED = NSTAT + 1;  // saved sums n, Sx, Sy, Sxx, Syy, Sxy, then r

__device__ __forceinline__ void write_pair(int64_t g, int64_t h, int64_t ldo, double rv, double pv, int64_t ni,
                                           double* __restrict__ r, double* __restrict__ p,
                                           int32_t* __restrict__ n)
{
    if (r) {
        r[g * ldo + h] = rv;
        r[h * ldo + g] = rv;
    }
    if (p) {
        p[g * ldo + h] = pv;
        p[h * ldo + g] = pv;
    }
    if (n) {
        n[g * ldo + h] = (int32_t)ni;
        n[h * ldo + g] = (int32_t)ni;
    }
}

// saved[s][g][h] for the ordered pair (g, h) and its mirror (h, g), whose x
// and y sides swap
__device__ __forceinline__ void write_saved(double* __restrict__ saved, int64_t F, int64_t g, int64_t h,
                                            const double (&st)[NSTAT], double rv)
{
    const int64_t FF = F * F;
    const double vgh[NSAVED] = {st[0], st[1], st[2], st[3], st[4], st[5], rv};
    const double vhg[NSAVED] = {st[0], st[2], st[1], st[4], st[3], st[5], rv};
#pragma unroll
    for (int s = 0; s < NSAVED; ++s) {
        saved[s * FF + g * F + h] = vgh[s];
        saved[s * FF + h * F + g] = vhg[s];
    }
}

// One workgroup per 32 x 32 tile of the upper triangle (a quarter of one
// 64 x 64 contraction tile): the split-K partials summed in FP64, r, n and
// the redo list, then p and both triangles.
__global__ __launch_bounds__(FT_THREADS) void k_pearson_combine(
    const double* __restrict__ part, int T, int ntiles, int nsplit, int64_t F, int T32,
    double* __restrict__ r, double* __restrict__ p, int32_t* __restrict__ n, int64_t ldo,
    double* __restrict__ saved, uint32_t* __restrict__ redo_count, uint32_t* __restrict__ redo)
{
    __shared__ FinSmem f;
    int tg, th;
    finish_tile_coords((int)blockIdx.x, T32, tg, th);
    const int64_t g0 = (int64_t)tg * FT, h0 = (int64_t)th * FT;
    const int t = tile_index(tg >> 1, th >> 1, T);
    const int ro = (tg & 1) * FT, co = (th & 1) * FT;  // the quarter inside the 64 x 64 tile
    const int j = ft_col();
    bool valid[FT_K];
#pragma unroll
    for (int k = 0; k < FT_K; ++k) {
        valid[k] = ft_valid(g0, h0, F, k);
        if (!valid[k]) continue;
        const int i = ft_row(k);
        const int64_t g = g0 + i, h = h0 + j;
        const int e = (ro + i) * TILE + co + j;
        double st[NSTAT];
#pragma unroll
        for (int s = 0; s < NSTAT; ++s) st[s] = 0.0;
        for (int sp = 0; sp < nsplit; ++sp)
#pragma unroll
            for (int s = 0; s < NSTAT; ++s)
                st[s] += part[(((int64_t)sp * NSTAT + s) * ntiles + t) * TILE_ELEMS + e];
        const double cn = st[0], sx = st[1], sy = st[2], sxx = st[3], syy = st[4], sxy = st[5];
        const int64_t ni = (int64_t)(cn + 0.5);
        double rv = __builtin_nan("");
        if (ni >= 2) {
            const double vx = cn * sxx - sx * sx;
            const double vy = cn * syy - sy * sy;
            if (vx >= WELL_CENTRED * cn * sxx && vy >= WELL_CENTRED * cn * syy && vx > 0.0 && vy > 0.0) {
                const double cxy = cn * sxy - sx * sy;
                rv = cxy / sqrt(vx * vy);
                rv = rv > 1.0 ? 1.0 : (rv < -1.0 ? -1.0 : rv);
            } else {
                const uint32_t slot = atomicAdd(redo_count, 1u);
                redo[slot] = (uint32_t)(g * F + h);
            }
        }
        f.r[i][j] = rv;
        f.n[i][j] = (int32_t)ni;
        if (saved) write_saved(saved, F, g, h, st, rv);
    }
    ft_pvalues(f, valid, true);  // n = 2: p = 1 (listed pairs get theirs from the recomputation)
    __syncthreads();
    ft_write(f, g0, h0, F, r, p, n, ldo);
}

// Recomputation of the listed pairs from the raw values in FP64, one
// workgroup per pair: a first pass over the samples takes n, the sums of
// both sides and their minima and maxima over I(g,h); a second pass the
// centred sums about the pair's own means (two-pass Pearson).  Zero variance
// is decided exactly: the minimum equals the maximum on I(g,h).  With
// `saved`, the six sums about the column means (the centring of the
// contractions: mu32 in float arithmetic, or mu64 in the FP64 mode) are
// recomputed in FP64 too.
constexpr int RC_THREADS = 256;

__device__ __forceinline__ double block_sum_f64(double v, double* red)
{
    v = wave_sum_f64(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < RC_THREADS / 64; ++w) t += red[w];
    return t;
}

__global__ __launch_bounds__(RC_THREADS) void k_pearson_recompute(
    const float* __restrict__ X, int64_t S, int64_t F, int64_t ldx, int use_sent, float sent,
    const float* __restrict__ mu32, const double* __restrict__ mu64, int center64,
    const uint32_t* __restrict__ redo_count, const uint32_t* __restrict__ redo,
    double* __restrict__ r, double* __restrict__ p, int64_t ldo, double* __restrict__ saved)
{
    __shared__ double red[RC_THREADS / 64];
    __shared__ float mred[4][RC_THREADS / 64];
    const uint32_t count = *redo_count;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (uint32_t k = blockIdx.x; k < count; k += gridDim.x) {
        const uint32_t code = redo[k];
        const int64_t g = code / (uint32_t)F, h = code % (uint32_t)F;
        // pass 1: n, sums, extremes
        double cnt = 0.0, s1x = 0.0, s1y = 0.0;
        float mnx = __builtin_inff(), mxx = -__builtin_inff(), mny = __builtin_inff(), mxy = -__builtin_inff();
        for (int64_t i = threadIdx.x; i < S; i += RC_THREADS) {
            const float x = X[i * ldx + g], y = X[i * ldx + h];
            if (!is_missing(x, use_sent, sent) && !is_missing(y, use_sent, sent)) {
                cnt += 1.0;
                s1x += (double)x;
                s1y += (double)y;
                mnx = fminf(mnx, x);
                mxx = fmaxf(mxx, x);
                mny = fminf(mny, y);
                mxy = fmaxf(mxy, y);
            }
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            mnx = fminf(mnx, __shfl_xor(mnx, d, 64));
            mxx = fmaxf(mxx, __shfl_xor(mxx, d, 64));
            mny = fminf(mny, __shfl_xor(mny, d, 64));
            mxy = fmaxf(mxy, __shfl_xor(mxy, d, 64));
        }
        if (lane == 0) {
            mred[0][wave] = mnx;
            mred[1][wave] = mxx;
            mred[2][wave] = mny;
            mred[3][wave] = mxy;
        }
        const double nn = block_sum_f64(cnt, red);
        const double sumx = block_sum_f64(s1x, red);
        const double sumy = block_sum_f64(s1y, red);
#pragma unroll
        for (int w = 0; w < RC_THREADS / 64; ++w) {
            mnx = fminf(mnx, mred[0][w]);
            mxx = fmaxf(mxx, mred[1][w]);
            mny = fminf(mny, mred[2][w]);
            mxy = fmaxf(mxy, mred[3][w]);
        }
        const double mx = sumx / nn, my = sumy / nn;
        const float cx32 = mu32[g], cy32 = mu32[h];
        const double cx64 = mu64[g], cy64 = mu64[h];
        // pass 2: centred sums about the pair means (r), and about the column
        // means (the saved sums)
        double sdd = 0.0, see = 0.0, sde = 0.0;
        double tx = 0.0, ty = 0.0, txx = 0.0, tyy = 0.0, txy = 0.0;
        for (int64_t i = threadIdx.x; i < S; i += RC_THREADS) {
            const float x = X[i * ldx + g], y = X[i * ldx + h];
            if (!is_missing(x, use_sent, sent) && !is_missing(y, use_sent, sent)) {
                const double d = (double)x - mx, e = (double)y - my;
                sdd += d * d;
                see += e * e;
                sde += d * e;
                if (saved) {
                    const double u = center64 ? (double)x - cx64 : (double)(x - cx32);
                    const double v = center64 ? (double)y - cy64 : (double)(y - cy32);
                    tx += u;
                    ty += v;
                    txx += u * u;
                    tyy += v * v;
                    txy += u * v;
                }
            }
        }
        const double Sdd = block_sum_f64(sdd, red);
        const double See = block_sum_f64(see, red);
        const double Sde = block_sum_f64(sde, red);
        double st[NSTAT] = {nn, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (saved) {
            st[1] = block_sum_f64(tx, red);
            st[2] = block_sum_f64(ty, red);
            st[3] = block_sum_f64(txx, red);
            st[4] = block_sum_f64(tyy, red);
            st[5] = block_sum_f64(txy, red);
        }
        if (threadIdx.x == 0) {
            const int64_t ni = (int64_t)(nn + 0.5);
            double rv = __builtin_nan(""), pv = __builtin_nan("");
            if (ni >= 2 && mnx != mxx && mny != mxy && Sdd > 0.0 && See > 0.0) {
                rv = Sde / sqrt(Sdd * See);
                rv = rv > 1.0 ? 1.0 : (rv < -1.0 ? -1.0 : rv);
                pv = (ni == 2) ? 1.0 : corr_pvalue(rv, ni);
            }
            write_pair(g, h, ldo, rv, pv, ni, r, p, nullptr);
            if (saved) write_saved(saved, F, g, h, st, rv);
        }
        __syncthreads();  // red / mred reused by the next pair
    }
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
struct PearsonPlan {
    int T, ntiles, nsplit;
    int64_t ksplit;
};

static PearsonPlan pearson_plan(int64_t S, int64_t F, int prec)
{
    PearsonPlan pl;
    pl.T = (int)ceil_div(F, TILE);
    pl.ntiles = pl.T * (pl.T + 1) / 2;
    if (prec == NAPY_PREC_BF16X3) {
        // 512 workgroup slots (two per CU): the smallest number of full
        // rounds of workgroups that is at least 90% occupied
        const int64_t BK = bf3::BK;
        int64_t want = 1;
        if (pl.ntiles < 512) {
            for (int64_t w = 1; w <= 4; ++w) {
                want = (512 * w) / pl.ntiles;
                if (want >= 1 && (double)(want * pl.ntiles) >= 0.9 * 512.0 * (double)w) break;
            }
        }
        int64_t maxs = S / 512;
        if (maxs < 1) maxs = 1;
        if (want > maxs) want = maxs;
        if (want < 1) want = 1;
        pl.ksplit = round_up(ceil_div(S, want), BK);
        if (pl.ksplit < BK) pl.ksplit = BK;
        pl.nsplit = (int)ceil_div(S, pl.ksplit);
        if (pl.nsplit < 1) pl.nsplit = 1;
        return pl;
    }
    const int BK = (prec == NAPY_PREC_FP64) ? 16 : 32;
    int64_t want = ceil_div(512, pl.ntiles);
    int64_t maxs = S / 512;
    if (maxs < 1) maxs = 1;
    if (want > maxs) want = maxs;
    if (want < 1) want = 1;
    pl.ksplit = round_up(ceil_div(S, want), BK);
    if (pl.ksplit < BK) pl.ksplit = BK;
    pl.nsplit = (int)ceil_div(S, pl.ksplit);
    if (pl.nsplit < 1) pl.nsplit = 1;
    return pl;
}

struct PearsonWs {
    ColStats cs;
    double* part;          // [nsplit][6][ntiles][64 x 64] split-K partial sums
    uint32_t* redo_count;  // pairs listed for recomputation
    uint32_t* redo;        // [F (F + 1) / 2] their codes g F + h
};

static void pearson_carve(Carver& c, int64_t S, int64_t F, const PearsonPlan& pl, PearsonWs& w)
{
    colstats_carve(c, S, F, w.cs);
    w.part = c.take<double>((size_t)pl.nsplit * NSTAT * pl.ntiles * TILE_ELEMS);
    w.redo_count = c.take<uint32_t>(1);
    w.redo = c.take<uint32_t>((size_t)(F * (F + 1) / 2));
}

static size_t plan_bytes(int64_t S, int64_t F, const PearsonPlan& pl)
{
    Carver c(nullptr);
    PearsonWs w;
    pearson_carve(c, S, F, pl, w);
    return c.bytes();
}

size_t pearson_ws_bytes(int64_t S, int64_t F, int prec)
{
    return plan_bytes(S, F, pearson_plan(S, F, prec));
}

static int pearson_run_plan(const float* X, int64_t S, int64_t F, int64_t ldx, double* r, double* p,
                            int32_t* n, int64_t ldo, double* saved, void* ws, const PearsonPlan& pl,
                            const napy_opts* opts, hipStream_t st, void* const* ev)
{
    const int prec = opt_prec(opts);
    const int us = opt_use_sent(opts);
    const float sv = opt_sent(opts);
    Carver c(ws);
    PearsonWs w;
    pearson_carve(c, S, F, pl, w);
    const ColStats& cs = w.cs;
    double* part = w.part;

    NAPY_TRY(record_stage(ev, 0, st));
    // (the final column-statistics kernel also clears the recomputation
    // list's counter, which the combine appends to)
    NAPY_TRY(colstats_launch(X, S, F, ldx, us, sv, cs, st, w.redo_count));
    NAPY_TRY(record_stage(ev, 1, st));
    const unsigned nb = (unsigned)(pl.ntiles * pl.nsplit);
    switch (prec) {
    case NAPY_PREC_FP32:
        hipLaunchKernelGGL(k_pearson_tiles<NAPY_PREC_FP32>, dim3(nb), dim3(256), 0, st, X, S, F, ldx, us, sv,
                           cs.mu32, cs.mu64, pl.T, pl.ntiles, pl.nsplit, pl.ksplit, part);
        break;
    case NAPY_PREC_BF16X3:
    {
        // 16 rows of ldx floats must be addressable with 32-bit byte offsets
        const bool gen = S < bf3::BK || ldx >= ((int64_t)1 << 26);
        auto kern = us ? (gen ? k_pearson_bf16<true, true> : k_pearson_bf16<true, false>)
                       : (gen ? k_pearson_bf16<false, true> : k_pearson_bf16<false, false>);
        hipLaunchKernelGGL(kern, dim3(nb), dim3(256), 0, st, X, S, F, ldx, us, sv, cs.mu32, pl.T, pl.ntiles,
                           pl.nsplit, pl.ksplit, part);
        break;
    }
    default:
        hipLaunchKernelGGL(k_pearson_tiles<NAPY_PREC_FP64>, dim3(nb), dim3(256), 0, st, X, S, F, ldx, us, sv,
                           cs.mu32, cs.mu64, pl.T, pl.ntiles, pl.nsplit, pl.ksplit, part);
        break;
    }
    NAPY_TRY(check_launch("pearson_tiles"));
    NAPY_TRY(record_stage(ev, 2, st));
    const int T32 = (int)ceil_div(F, FT);
    hipLaunchKernelGGL(k_pearson_combine, dim3((unsigned)(T32 * (T32 + 1) / 2)), dim3(FT_THREADS), 0, st, part,
                       pl.T, pl.ntiles, pl.nsplit, F, T32, r, p, n, ldo, saved, w.redo_count, w.redo);
    NAPY_TRY(check_launch("pearson_combine"));
    // a fixed grid: workgroups whose index is at least the listed count
    // return at once
    const int64_t npairs = F * (F + 1) / 2;
    const unsigned nrc = (unsigned)(npairs < 1024 ? npairs : 1024);
    hipLaunchKernelGGL(k_pearson_recompute, dim3(nrc), dim3(RC_THREADS), 0, st, X, S, F, ldx, us, sv, cs.mu32,
                       cs.mu64, prec == NAPY_PREC_FP64 ? 1 : 0, w.redo_count, w.redo, r, p, ldo, saved);
    NAPY_TRY(check_launch("pearson_recompute"));
    return record_stage(ev, 3, st);
}

int pearson_run(const float* X, int64_t S, int64_t F, int64_t ldx, double* r, double* p,
                int32_t* n, int64_t ldo, double* saved, void* ws, size_t ws_bytes,
                const napy_opts* opts, hipStream_t st, void* const* ev)
{
    (void)ws_bytes;
    return pearson_run_plan(X, S, F, ldx, r, p, n, ldo, saved, ws, pearson_plan(S, F, opt_prec(opts)), opts, st,
                            ev);
}

// ---------------------------------------------------------------------------
// allocation-free Pearson: the workspace is a fixed device array
// ---------------------------------------------------------------------------
// Each device that loads the library holds its own copy of `scratch` until
// the process ends.  Host code never passes the array's name to a kernel (in
// host code it is a host-side stand-in): the device address is looked up
// once per device with hipGetSymbolAddress and kept in scratch_dev.
constexpr size_t PEARSON_NOALLOC_BYTES = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[PEARSON_NOALLOC_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex scratch_mu;
static void* scratch_dev[SCRATCH_MAX_DEVICES] = {};

static int scratch_address(void** out)
{
    int dev = 0;
    NAPY_TRY(hip_status(hipGetDevice(&dev), "hipGetDevice"));
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) {
        set_last_error("device %d: the allocation-free entry point supports devices 0..%d", dev,
                       SCRATCH_MAX_DEVICES - 1);
        return NAPY_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void* ptr = nullptr;
        NAPY_TRY(hip_status(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"));
        if (!ptr || ((uintptr_t)ptr & 255)) {
            set_last_error("scratch array of device %d has no usable address", dev);
            return NAPY_E_HIP;
        }
        scratch_dev[dev] = ptr;
    }
    *out = scratch_dev[dev];
    return NAPY_OK;
}

// The default plan when its workspace fits the array, else the same plan with
// fewer sample splits (the split count only changes the order of the FP64
// partial additions).
static PearsonPlan noalloc_plan(int64_t S, int64_t F, int prec)
{
    PearsonPlan pl = pearson_plan(S, F, prec);
    const int64_t BK = (prec == NAPY_PREC_BF16X3) ? bf3::BK : (prec == NAPY_PREC_FP64 ? 16 : 32);
    while (plan_bytes(S, F, pl) > PEARSON_NOALLOC_BYTES && pl.nsplit > 1) {
        pl.ksplit = round_up(ceil_div(S, (int64_t)pl.nsplit - 1), BK);
        pl.nsplit = (int)ceil_div(S, pl.ksplit);
        if (pl.nsplit < 1) pl.nsplit = 1;
    }
    return pl;
}

int pearson_noalloc_run(const float* X, int64_t S, int64_t F, int64_t ldx, double* r, double* p, int32_t* n,
                        int64_t ldo, const napy_opts* opts, hipStream_t st)
{
    const PearsonPlan pl = noalloc_plan(S, F, opt_prec(opts));
    const size_t need = plan_bytes(S, F, pl);
    if (need > PEARSON_NOALLOC_BYTES) {
        set_last_error("S=%lld F=%lld needs %zu bytes of scratch; the allocation-free Pearson holds %zu",
                       (long long)S, (long long)F, need, (size_t)PEARSON_NOALLOC_BYTES);
        return NAPY_E_UNSUPPORTED;
    }
    void* ws = nullptr;
    NAPY_TRY(scratch_address(&ws));
    return pearson_run_plan(X, S, F, ldx, r, p, n, ldo, nullptr, ws, pl, opts, st, nullptr);
}

}  // namespace napy
