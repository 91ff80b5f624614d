// Rank tests of categorical x continuous pairs with pairwise deletion (NApy,
// Section 3.5): Mann-Whitney U (labels 0 and 1) and Kruskal-Wallis H.
//
// Every continuous column is sorted once (the Spearman sort, with its tie
// runs).  For a pair (g, h) the ranks within I(g, h) follow from one walk of
// h's sorted order: a position is kept when g's label at its sample is
// present, and a kept untied sample has doubled rank 2 C1 with C1 = 1 + (kept
// samples at earlier positions).  A tie run [s, e) of h's order gives its kept
// samples the doubled average rank C(s) + C(e) + 1 (C(x): kept samples before
// position x) and adds t^3 - t, t = C(e) - C(s), to the tie term; for columns
// with ties, C(x) comes from a table of kept bits and prefix counts along h's
// order built by a first walk.  The doubled ranks are summed per label.
//
// Kernels:
//   labels_launch (shared)  observed-label mask and invalid flag per column.
//   k_rank_labels           labels transposed to bytes per column (0xFF:
//                           missing or not a label of the test).
//   k_rank_walk<NW>         one categorical column g and 8 continuous columns
//                           per workgroup, one wave per pair: the walk, the
//                           group rank sums and counts, then U or H, p and n.
//                           Two labels: label 0 summed with selects; more:
//                           windows of four labels, each position's doubled
//                           rank added by one LDS atomic to its lane's slot
//                           of its label.
//   k_mwu_exact             pairs whose p is exact (no ties within I and a
//                           group below eight samples): the distribution of U
//                           from the generating function
//                           prod_{i=1}^{m} (1 - q^(M+i)) / (1 - q^i), m <= 7,
//                           one workgroup per pair with two coefficient
//                           buffers in the workspace: each factor is a
//                           shifted difference, then i interleaved prefix
//                           sums (stride i), both in parallel.
#include "napy_internal.hpp"
#include "pvalue.hpp"
#include "rankbase.hpp"

namespace napy {

constexpr int RK_WAVES = 8;
constexpr int RK_THREADS = 64 * RK_WAVES;
constexpr int RK_U = 4;  // chunks of 64 sorted positions per pipelined step
constexpr int RK_EX_THREADS = 256;
constexpr int RK_EX_BLOCKS = 64;  // concurrent exact-p computations
constexpr int RK_EXACT_MAXM = 7;  // exact mode: the smaller group below eight

struct RankWs {
    SpearBase base;      // sorted continuous columns (then the sort's keys buffer)
    uint8_t* lab;        // [FC][ld] labels as bytes
    uint64_t* catmask;   // [FC]
    int32_t* bad;        // [FC]
    uint32_t* nexact;    // [1]
    int4* exact;         // [FC * FQ] (g, h, U, m | M << 16 as packed ints)
    double* slab;        // [RK_EX_BLOCKS][2][dmax + 1]
    int64_t dmax;
};

static int64_t rk_dmax(int64_t S) { return (int64_t)RK_EXACT_MAXM * (S > 0 ? S : 1) / 2 + 1; }

static void rk_carve(Carver& c, int64_t S, int64_t FC, int64_t FQ, bool mwu, RankWs& w)
{
    base_carve(c, S, FQ, w.base);
    c.take<uint32_t>((size_t)sort_keys_words(S, FQ));  // keys buffer of the sort
    w.lab = c.take<uint8_t>((size_t)FC * spear_ld(S));
    w.catmask = c.take<uint64_t>(FC);
    w.bad = c.take<int32_t>(FC);
    w.nexact = c.take<uint32_t>(1);
    w.exact = c.take<int4>(mwu ? (size_t)FC * FQ : 1);
    w.dmax = rk_dmax(S);
    w.slab = c.take<double>(mwu ? (size_t)RK_EX_BLOCKS * 2 * (w.dmax + 1) : 1);
}

size_t ranktests_ws_bytes(int64_t S, int64_t FC, int64_t FQ, bool mwu)
{
    Carver c(nullptr);
    RankWs w;
    rk_carve(c, S, FC, FQ, mwu, w);
    return c.bytes();
}

// L (S x FC) -> lab[g][i] bytes through a 64 x 64 tile; 0xFF for a missing
// value or a value that is not an integer label in [0, ncat); samples S .. ld
// (the sorted orders' dummy sample and padding) get 0xFF as well
__global__ __launch_bounds__(256) void k_rank_labels(const float* __restrict__ L, int64_t ldl, int64_t S,
                                                     int64_t FC, int ncat, int use_sent, float sent, int64_t ld,
                                                     uint8_t* __restrict__ lab, uint32_t* __restrict__ nexact)
{
    __shared__ uint8_t tile[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t i0 = (int64_t)blockIdx.y * 64, g0 = (int64_t)blockIdx.x * 64;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *nexact = 0u;
    for (int r = ty; r < 64; r += 4) {
        const int64_t i = i0 + r, g = g0 + tx;
        uint8_t b = 0xFF;
        if (i < S && g < FC) {
            const float v = L[i * ldl + g];
            if (!is_missing(v, use_sent, sent) && v >= 0.0f && v < (float)ncat && v == floorf(v)) b = (uint8_t)v;
        }
        tile[r][tx] = b;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t g = g0 + r, i = i0 + tx;
        if (g < FC && i < ld) lab[g * ld + i] = tile[tx][r];
    }
}

// kept samples at positions < x (table: per 32 positions the kept bits and the
// count before them)
__device__ __forceinline__ uint32_t rk_count(const uint2* tab, uint32_t x)
{
    const uint2 e = tab[x >> 5];
    return e.y + (uint32_t)__popc(__builtin_amdgcn_ubfe(e.x, 0u, x));
}

__device__ __forceinline__ double normal_sf(double z) { return 0.5 * erfc(z * 0.70710678118654752440); }

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
    // DPP scan read at lane 63: no LDS traffic; the result is uniform
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan_u32(v), 63);
}

template <int CTRL, int RMASK>
__device__ __forceinline__ uint64_t rk_dpp_step_u64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, RMASK, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, RMASK, 0xF, false);
    return v + (((uint64_t)hi << 32) | lo);
}

// 64-bit wave total by DPP scans (modulo 2^64); uniform
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
    constexpr int ROW_SHR = 0x110, ROW_BCAST15 = 0x142, ROW_BCAST31 = 0x143;
    v = rk_dpp_step_u64<ROW_SHR + 1, 0xF>(v);
    v = rk_dpp_step_u64<ROW_SHR + 2, 0xF>(v);
    v = rk_dpp_step_u64<ROW_SHR + 4, 0xF>(v);
    v = rk_dpp_step_u64<ROW_SHR + 8, 0xF>(v);
    v = rk_dpp_step_u64<ROW_BCAST15, 0xA>(v);
    v = rk_dpp_step_u64<ROW_BCAST31, 0xC>(v);
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
}

// One walk of h's sorted order for the labels g0 .. g0 + NA - 1: every kept
// position gets its doubled rank 2 C1 (C1 = kept positions before it + 1), or
// with TABLE the tied average C(s) + C(e) + 1; summed per label (acc, per
// lane) and counted (cnt, wave-uniform) with selects and ballots, or with
// LDSACC added with one LDS atomic per position into the lane's slot of its
// label in accw (sum in the low 40 bits, count above).  Returns the kept count.  Chunks are
// processed RK_U at a time with the next group's sorted orders in flight;
// chunks from nch up to the group's end hold the dummy sample (never kept),
// and reads past the column stay inside the ord allocation.
template <int NA, bool TABLE, bool LDSACC>
__device__ __forceinline__ uint32_t rank_walk(const uint16_t* __restrict__ ordH, const uint32_t* __restrict__ runsH,
                                              const uint64_t* __restrict__ tbH, const uint8_t* labL,
                                              const uint2* tab, int nch, int g0, int lane, uint32_t (&acc)[NA],
                                              uint32_t (&cnt)[NA], unsigned long long* accw)
{
    uint32_t carry = 0;  // kept samples before the chunk (wave-uniform)
    uint32_t nxt[RK_U];
#pragma unroll
    for (int j = 0; j < RK_U; ++j) nxt[j] = ordH[j * 64 + lane];
    for (int c0 = 0; c0 < nch; c0 += RK_U) {
        uint64_t tbw[RK_U];
        uint32_t rr[RK_U];
        if (TABLE) {
            // tie bits of the group (ld / 64 is a multiple of RK_U) and the run
            // bounds of its tied positions, loaded before the next group's
            // orders so that waiting for them leaves those in flight
#pragma unroll
            for (int j = 0; j < RK_U; ++j) tbw[j] = tbH[c0 + j];
#pragma unroll
            for (int j = 0; j < RK_U; ++j) rr[j] = ((tbw[j] >> lane) & 1ull) ? runsH[(c0 + j) * 64 + lane] : 0u;
        }
        uint32_t lbs[RK_U];
#pragma unroll
        for (int j = 0; j < RK_U; ++j) lbs[j] = labL[nxt[j]];
#pragma unroll
        for (int j = 0; j < RK_U; ++j) nxt[j] = ordH[(c0 + RK_U + j) * 64 + lane];
#pragma unroll
        for (int j = 0; j < RK_U; ++j) {
            const uint32_t lb = lbs[j];
            const uint64_t m = __ballot(lb != 0xFFu);
            uint32_t r2 = 2u * __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, carry)) + 2u;
            if (TABLE && ((tbw[j] >> lane) & 1ull)) {
                const uint32_t s = rr[j] & 0xFFFFu, e = rr[j] >> 16;
                r2 = rk_count(tab, s) + rk_count(tab, e) + 1u;
            }
            if constexpr (LDSACC) {
                // this lane's slot of the sample's label: count in bits 40 and up
                const uint32_t kk = lb - (uint32_t)g0;
                if (kk < (uint32_t)NA) atomicAdd(&accw[kk * 64u + (uint32_t)lane], (1ull << 40) | r2);
            } else {
#pragma unroll
                for (int k = 0; k < NA; ++k) {
                    const bool in = lb == (uint32_t)(g0 + k);
                    acc[k] += in ? r2 : 0u;
                    cnt[k] += (uint32_t)__popcll(__ballot(in));
                }
            }
            carry += (uint32_t)__popcll(m);
        }
    }
    return carry;
}

// Short tie runs, one lane per run: the walk gave the t kept members of a run
// the doubled ranks 2 (C(s) + j), j = 1 .. t, their average is C(s) + C(e) + 1
// = 2 C(s) + t + 1, so a member with label k changes label k's sum by
// t + 1 - 2 j.  Adds t^3 - t per run to `tie` when `tieterm`.
template <int NA>
__device__ __forceinline__ void rank_short_runs(const uint16_t* __restrict__ ordH, const uint32_t* __restrict__ rl,
                                                int nr, const uint8_t* labL, int g0, int lane, int64_t (&corr)[NA],
                                                bool tieterm, double& tie)
{
    for (int r = lane; r < nr; r += 64) {
        const uint32_t rr = rl[r];
        const uint32_t s = rr & 0xFFFFu, e = rr >> 16;
        uint32_t t = 0;
        uint32_t nkr[NA], jsum[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k) nkr[k] = jsum[k] = 0u;
        for (uint32_t q = s; q < e; ++q) {
            const uint32_t lb = labL[ordH[q]];
            if (lb != 0xFFu) {
                ++t;
#pragma unroll
                for (int k = 0; k < NA; ++k)
                    if (lb == (uint32_t)(g0 + k)) {
                        ++nkr[k];
                        jsum[k] += t;
                    }
            }
        }
#pragma unroll
        for (int k = 0; k < NA; ++k) corr[k] += (int64_t)nkr[k] * (t + 1u) - 2 * (int64_t)jsum[k];
        if (tieterm) {
            const double td = (double)t;
            tie += td * td * td - td;
        }
    }
}

// test: 0 Mann-Whitney (auto), 1 Mann-Whitney (asymptotic), 2 Kruskal-Wallis.
// The labels are summed in windows of NW (one walk per window), which bounds
// the per-lane accumulators (in LDS for NW > 2) for up to 32 categories.  With two labels only
// label 0 is summed: label 1 holds the rest of n (n + 1) and of n.
template <int NW, bool LABG>
__global__ __launch_bounds__(RK_THREADS) void k_rank_walk(SpearBase bs, const uint8_t* __restrict__ lab, int64_t S,
                                                          int64_t FC, int64_t FQ, int test, int ncat,
                                                          const uint64_t* __restrict__ catmask,
                                                          const int32_t* __restrict__ bad, double* __restrict__ stat,
                                                          double* __restrict__ pval, int32_t* __restrict__ nout,
                                                          int64_t ldo, uint32_t* __restrict__ nexact,
                                                          int4* __restrict__ exact)
{
    constexpr int NA = NW == 2 ? 1 : NW;
    constexpr bool LDSACC = NW > 2;
    extern __shared__ __attribute__((aligned(16))) unsigned char rk_smem[];
    __shared__ double res[RK_WAVES][2][32];  // per wave: doubled rank sums, counts
    const int64_t ld = bs.ld;
    const int nwp = (int)((S + 1 + 31) / 32) + 1;  // table entries per wave
    const int64_t g = blockIdx.x;
    // labels: copied to LDS, or read from global memory when the tables of
    // long columns leave no room for them (LABG)
    const uint8_t* labL = LABG ? lab + g * ld : rk_smem;
    uint2* tabs = (uint2*)(rk_smem + (LABG ? 0 : round_up(ld, 16)));
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    if constexpr (!LABG) {
        const uint4* src = (const uint4*)(lab + g * ld);
        uint4* dst = (uint4*)rk_smem;
        for (int64_t k = threadIdx.x; k < ld / 16; k += RK_THREADS) dst[k] = src[k];
    }
    __syncthreads();

    const int64_t h = (int64_t)blockIdx.y * RK_WAVES + wave;
    if (h >= FQ) return;
    const int nh = bs.ncol[h];
    const uint16_t* ordH = bs.ord + h * ld;
    const uint32_t* runsH = bs.runs + h * ld;
    const uint64_t* tbH = bs.tbits + h * (ld / 64);
    const uint32_t* rl = bs.rlist + h * (ld / 2);
    const int nr = bs.nruns[h];
    const int mode = bs.tcls[h];  // tie class: 0 none, 1 few short runs, 2 otherwise
    const int nch = (nh + 63) >> 6;
    uint2* tab = tabs + (size_t)wave * nwp;
    unsigned long long* accw = (unsigned long long*)(tabs + (size_t)RK_WAVES * nwp) + (size_t)wave * NA * 64;

    double tie = 0.0;  // sum of t^3 - t, exact below 2^53
    if (mode == 2) {
        // kept bits along h's order (positions from nh on hold the dummy sample)
        const int NWD = (nh + 1 + 31) >> 5;
        for (int c = 0; c < (NWD + 1) / 2; ++c) {
            const uint32_t iv = ordH[c * 64 + lane];
            const uint64_t m = __ballot(labL[iv] != 0xFF);
            if (lane == 0) {
                tab[2 * c].x = (uint32_t)m;
                if (2 * c + 1 < NWD) tab[2 * c + 1].x = (uint32_t)(m >> 32);
            }
        }
        wave_sync_lds();
        uint32_t run = 0;
        for (int w0 = 0; w0 < NWD; w0 += 64) {
            const int w = w0 + lane;
            const uint32_t v = w < NWD ? (uint32_t)__popc(tab[w].x) : 0u;
            const uint32_t incl = wave_incl_scan_u32(v);
            if (w < NWD) tab[w].y = run + incl - v;
            run += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        }
        wave_sync_lds();
        for (int r = lane; r < nr; r += 64) {
            const uint32_t rr = rl[r];
            const double t = (double)(rk_count(tab, rr >> 16) - rk_count(tab, rr & 0xFFFFu));
            tie += t * t * t - t;
        }
    }

    uint32_t ntot = 0;
    for (int g0 = 0; g0 < ncat; g0 += NW) {
        uint32_t acc[NA];   // doubled rank sums of this lane (each below 2^32)
        int64_t corr[NA];   // this lane's corrections for short tie runs
        uint32_t cnt[NA];   // wave-uniform counts
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            acc[k] = cnt[k] = 0u;
            corr[k] = 0;
        }
        if constexpr (LDSACC) {
#pragma unroll
            for (int k = 0; k < NA; ++k) accw[k * 64 + lane] = 0ull;
            wave_sync_lds();
        }
        if (mode == 2) {
            ntot = rank_walk<NA, true, LDSACC>(ordH, runsH, tbH, labL, tab, nch, g0, lane, acc, cnt, accw);
        } else {
            ntot = rank_walk<NA, false, LDSACC>(ordH, runsH, tbH, labL, tab, nch, g0, lane, acc, cnt, accw);
            if (mode == 1) rank_short_runs<NA>(ordH, rl, nr, labL, g0, lane, corr, g0 == 0, tie);
        }
        if constexpr (LDSACC) {
            wave_sync_lds();
#pragma unroll
            for (int k = 0; k < NA; ++k) {
                const unsigned long long v = accw[k * 64 + lane];
                acc[k] += (uint32_t)(v & ((1ull << 40) - 1ull));
                cnt[k] = wave_sum_u32((uint32_t)(v >> 40));
            }
        }
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            // 64-bit totals (the corrections may be negative: modulo 2^64)
            const uint64_t r2sum = wave_sum_u64((uint64_t)acc[k]) + wave_sum_u64((uint64_t)corr[k]);
            if (lane == 0 && g0 + k < 32) {
                res[wave][0][g0 + k] = (double)r2sum;
                res[wave][1][g0 + k] = (double)cnt[k];
            }
        }
        if (NW == 2 && lane == 0) {
            const double n = (double)ntot;
            res[wave][0][1] = n * (n + 1.0) - res[wave][0][0];
            res[wave][1][1] = n - res[wave][1][0];
        }
    }
    const double T = wave_sum_f64(tie);
    if (lane != 0) return;

    const double* R2 = res[wave][0];
    const double* nk = res[wave][1];
    double st = NAN, p = NAN;
    const bool ok = bad[g] == 0;
    if (ok && test <= 1) {
        const double n0 = nk[0], n1 = nk[1];
        if (n0 > 0.5 && n1 > 0.5) {
            const double n = n0 + n1;
            const double U1 = 0.5 * R2[0] - n0 * (n0 + 1.0) * 0.5;
            const double U = fmax(U1, n0 * n1 - U1);
            st = U1;
            if (test == 0 && T == 0.0 && fmin(n0, n1) < 8.0) {
                // exact p from k_mwu_exact; the entry carries U and the sizes
                const uint32_t slot = atomicAdd(nexact, 1u);
                exact[slot] = make_int4((int)g, (int)h, (int)U, (int)n0 | ((int)n1 << 16));
            } else {
                const double s2 = n0 * n1 / 12.0 * ((n + 1.0) - T / (n * (n - 1.0)));
                const double z = s2 > 0.0 ? (U - n0 * n1 * 0.5 - 0.5) / sqrt(s2) : -INFINITY;
                p = fmin(1.0, 2.0 * normal_sf(z));
            }
        }
    } else if (ok) {
        // sum_k R_k^2 / n_k - n (n + 1)^2 / 4 = sum_k (R_k - n_k (n + 1) / 2)^2 / n_k
        // (the R_k add up to n (n + 1) / 2): no cancellation for small H
        const uint64_t cm = catmask[g];
        const int K = __popcll(cm);
        const double n = (double)ntot;
        bool empty = false;
        double s = 0.0;
        for (int k = 0; k < ncat; ++k) {
            if (!((cm >> k) & 1ull)) continue;
            if (nk[k] < 0.5) {
                empty = true;
                continue;
            }
            const double dk = 0.5 * (R2[k] - nk[k] * (n + 1.0));  // exact: half-integers
            s += dk * dk / nk[k];
        }
        if (!empty && K >= 2) {
            const double denom = 1.0 - T / (n * n * n - n);
            if (denom > 0.0) {
                st = 12.0 / (n * (n + 1.0)) * s / denom;
                p = chi2_sf(st, (double)(K - 1));
            }
        }
    }
    stat[g * ldo + h] = st;
    pval[g * ldo + h] = p;
    nout[g * ldo + h] = ok ? (int32_t)ntot : 0;
}

// two-sided exact p = min(1, 2 P(U' >= U)) = min(1, 2 P(U' <= m M - U)) (the
// distribution is symmetric), U = max(U1, U2): the generating function's
// coefficients up to degree D = m M - U <= m M / 2, m the smaller group, over
// the total C(m + M, m).  Per factor i: B = A (1 - q^(M+i)) (a shifted
// difference), then A = B / (1 - q^i), i.e. prefix sums along d = r + i j for
// each residue r < i: every thread sums a block of rows j per residue, the
// block totals are scanned in LDS, and each thread rewrites its rows.
__global__ __launch_bounds__(RK_EX_THREADS) void k_mwu_exact(const uint32_t* __restrict__ nexact,
                                                             const int4* __restrict__ exact,
                                                             double* __restrict__ slab, int64_t dmax,
                                                             double* __restrict__ pval, int64_t ldo)
{
    __shared__ double part[RK_EXACT_MAXM][RK_EX_THREADS];
    __shared__ double red[RK_EX_THREADS / 64];
    const uint32_t count = *nexact;
    const int t = threadIdx.x;
    double* A = slab + (int64_t)blockIdx.x * 2 * (dmax + 1);
    double* B = A + (dmax + 1);
    for (uint32_t e = blockIdx.x; e < count; e += gridDim.x) {
        const int4 q = exact[e];
        const int64_t n0 = q.w & 0xFFFF, n1 = (uint32_t)q.w >> 16;
        const int64_t m = min(n0, n1), M = max(n0, n1);
        const int64_t D = m * M - (int64_t)q.z;
        for (int64_t d = t; d <= D; d += RK_EX_THREADS) A[d] = d == 0 ? 1.0 : 0.0;
        __syncthreads();
        for (int i = 1; i <= (int)m; ++i) {
            const int64_t k = M + i;
            for (int64_t d = t; d <= D; d += RK_EX_THREADS) B[d] = A[d] - (d >= k ? A[d - k] : 0.0);
            __syncthreads();
            const int64_t rows = D / i + 1;
            const int64_t per = ceil_div(rows, RK_EX_THREADS);
            const int64_t j0 = min(rows, (int64_t)t * per), j1 = min(rows, j0 + per);
            double v[RK_EXACT_MAXM];
#pragma unroll
            for (int r = 0; r < RK_EXACT_MAXM; ++r) {
                double sr = 0.0;
                if (r < i)
                    for (int64_t j = j0; j < j1; ++j) {
                        const int64_t d = j * i + r;
                        if (d <= D) sr += B[d];
                    }
                v[r] = sr;
                part[r][t] = sr;
            }
            __syncthreads();
            // inclusive scan over the threads (Hillis-Steele), per residue
            for (int off = 1; off < RK_EX_THREADS; off <<= 1) {
#pragma unroll
                for (int r = 0; r < RK_EXACT_MAXM; ++r)
                    if (r < i && t >= off) v[r] += part[r][t - off];
                __syncthreads();
#pragma unroll
                for (int r = 0; r < RK_EXACT_MAXM; ++r)
                    if (r < i) part[r][t] = v[r];
                __syncthreads();
            }
#pragma unroll
            for (int r = 0; r < RK_EXACT_MAXM; ++r) {
                if (r >= i) continue;
                double run = t > 0 ? part[r][t - 1] : 0.0;
                for (int64_t j = j0; j < j1; ++j) {
                    const int64_t d = j * i + r;
                    if (d <= D) {
                        run += B[d];
                        A[d] = run;
                    }
                }
            }
            __syncthreads();
        }
        double cdf = 0.0;
        for (int64_t d = t; d <= D; d += RK_EX_THREADS) cdf += A[d];
        cdf = wave_sum_f64(cdf);
        if ((t & 63) == 0) red[t >> 6] = cdf;
        __syncthreads();
        if (t == 0) {
            double tot = 0.0;
            for (int w = 0; w < RK_EX_THREADS / 64; ++w) tot += red[w];
            double total = 1.0;  // C(m + M, m)
            for (int64_t j = 1; j <= m; ++j) total = total * (double)(M + j) / (double)j;
            pval[(int64_t)q.x * ldo + q.y] = fmin(1.0, 2.0 * tot / total);
        }
        __syncthreads();  // A and red reused by the next pair
    }
}

template <int NW, bool LABG>
static int walk_launch_t(const RankWs& w, int64_t S, int64_t FC, int64_t FQ, int test, int ncat, double* stat,
                         double* p, int32_t* n, int64_t ldo, size_t smem, hipStream_t st)
{
    static std::atomic<uint64_t> attr_done{0};
    NAPY_TRY(ensure_dyn_lds(attr_done, (const void*)k_rank_walk<NW, LABG>,
                            (int)(160 * 1024 - sizeof(double) * RK_WAVES * 64), "hipFuncSetAttribute(k_rank_walk)"));
    hipLaunchKernelGGL((k_rank_walk<NW, LABG>), dim3((unsigned)FC, (unsigned)ceil_div(FQ, RK_WAVES)), dim3(RK_THREADS),
                       smem, st, w.base, w.lab, S, FC, FQ, test, ncat, w.catmask, w.bad, stat, p, n, ldo, w.nexact,
                       w.exact);
    return check_launch("rank walk");
}

template <int NW>
static int walk_launch(const RankWs& w, int64_t S, int64_t FC, int64_t FQ, int test, int ncat, double* stat,
                       double* p, int32_t* n, int64_t ldo, hipStream_t st)
{
    const size_t tables =
        (size_t)RK_WAVES * ((S + 1 + 31) / 32 + 1) * 8 + (NW > 2 ? (size_t)RK_WAVES * NW * 64 * 8 : 0);
    const size_t with_labels = (size_t)round_up(w.base.ld, 16) + tables;
    const size_t limit = 160 * 1024 - sizeof(double) * RK_WAVES * 64;
    if (with_labels <= limit)
        return walk_launch_t<NW, false>(w, S, FC, FQ, test, ncat, stat, p, n, ldo, with_labels, st);
    if (tables > limit) return NAPY_E_UNSUPPORTED;
    return walk_launch_t<NW, true>(w, S, FC, FQ, test, ncat, stat, p, n, ldo, tables, st);
}

int ranktests_run(const float* L, int64_t ldl, const float* X, int64_t ldx, int64_t S, int64_t FC, int64_t FQ,
                  int test, int ncat, double* stat, double* p, int32_t* n, int64_t ldo, void* ws,
                  const napy_opts* opts, hipStream_t st)
{
    const int us = opt_use_sent(opts);
    const float sv = opt_sent(opts);
    const bool mwu = test <= 1;
    Carver c(ws);
    RankWs w;
    rk_carve(c, S, FC, FQ, mwu, w);
    NAPY_TRY(labels_launch(L, ldl, S, FC, ncat, us, sv, w.catmask, w.bad, st));
    NAPY_TRY(spearman_base_prepare_run(X, S, FQ, ldx, ws, opts, st));  // the base is carved first
    hipLaunchKernelGGL(k_rank_labels, dim3((unsigned)ceil_div(FC, 64), (unsigned)ceil_div(w.base.ld, 64)), dim3(256),
                       0, st, L, ldl, S, FC, ncat, us, sv, w.base.ld, w.lab, w.nexact);
    NAPY_TRY(check_launch("rank labels"));
    if (ncat <= 2) NAPY_TRY(walk_launch<2>(w, S, FC, FQ, test, ncat, stat, p, n, ldo, st));
    else NAPY_TRY(walk_launch<4>(w, S, FC, FQ, test, ncat, stat, p, n, ldo, st));
    if (mwu) {
        hipLaunchKernelGGL(k_mwu_exact, dim3(RK_EX_BLOCKS), dim3(RK_EX_THREADS), 0, st, w.nexact, w.exact, w.slab,
                           w.dmax, p, ldo);
        NAPY_TRY(check_launch("mwu exact"));
    }
    return NAPY_OK;
}

}  // namespace napy
