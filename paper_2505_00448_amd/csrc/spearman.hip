// Spearman correlation with pairwise deletion (NApy, arXiv 2505.00448,
// Sections 3.2 and 3.5.3): each variable is sorted once; for every pair the
// ranks inside the pairwise-complete set I(g,h) are re-derived from that
// sorted order by counting the partner's present samples, with tied values
// given the average of their ranks.
//
// Doubled ranks keep everything in integers.  Along column a's sorted order,
// let C(x) be the number of pairwise-complete samples at sorted positions
// below x.  A sample in a run of tied values spanning positions [s, e) then
// has doubled average rank  R = C(s) + C(e) + 1  (for an untied sample
// R = 2 C(x) + 2).  With R_a, R_b the doubled ranks of both sides,
//     A = sum_I R_a R_b,  B_a = sum_I R_a^2,  B_b = sum_I R_b^2,
//     K = n (n + 1)^2,
//     rho = (A - K) / sqrt((B_a - K)(B_b - K)),
// all sums being exact integers (held in FP64 below 2^53).
//
// Kernels:
//   k_sort_keys      transposes X into per-column order-preserving uint32 keys
//                    (-0 canonicalised to +0; missing -> 0xFFFFFFFF).
//   k_colsort        one 1024-thread workgroup per column: LSD radix sort of
//                    the keys in LDS (8 passes of 4 bits), then
//                    ord[c][k] (sample at sorted position k), pos[c][i]
//                    (sorted position of sample i, 0xFFFF if missing),
//                    runs[c][k] = s | e << 16 (tie run of position k), n_c and
//                    a has-ties flag.
//   k_spearman_pairs one workgroup per (column a, block of 16 partners b);
//                    pos_a lives in LDS, each wave takes one partner at a
//                    time.  Walk 1 streams b's sorted order, looks up a's
//                    position of every sample, ballots the complete ones
//                    (b-side presence mask per 64 positions plus prefix) and
//                    sets their bits in an a-side bitmap; a prefix over the
//                    bitmap words follows; walk 2 streams b's order again and
//                    forms both doubled ranks from popcounts and the sums.
//   k_spearman_final one thread per pair: rho, p, n into both triangles.
#include "napy_internal.hpp"
#include "pvalue.hpp"

namespace napy {

constexpr int SORT_THREADS = 1024;
constexpr int SORT_EPT = 24;  // elements per thread
constexpr int SPEARMAN_MAX_S = SORT_THREADS * SORT_EPT;  // 24576
constexpr int PAIR_BLOCK = 16;  // partners per workgroup
constexpr int PAIR_WAVES = 4;

struct SpearBase {
    uint16_t* ord;     // [F][ld]
    uint16_t* pos;     // [F][ld]
    uint32_t* runs;    // [F][ld]
    int32_t* ncol;     // [F]
    int32_t* hasties;  // [F]
    int64_t ld;
};

static inline int64_t spear_ld(int64_t S) { return round_up(S > 0 ? S : 1, 64); }

static void base_carve(Carver& c, int64_t S, int64_t F, SpearBase& b)
{
    b.ld = spear_ld(S);
    b.ord = c.take<uint16_t>((size_t)F * b.ld);
    b.pos = c.take<uint16_t>((size_t)F * b.ld);
    b.runs = c.take<uint32_t>((size_t)F * b.ld);
    b.ncol = c.take<int32_t>(F);
    b.hasties = c.take<int32_t>(F);
}

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t order_key(float v, int use_sent, float sent)
{
    if (is_missing(v, use_sent, sent)) return 0xFFFFFFFFu;
    uint32_t u = __float_as_uint(v);
    if (u == 0x80000000u) u = 0u;  // -0 ties +0
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// X (S x F row-major) -> keys [F][ld] through a 64 x 64 LDS tile.
__global__ __launch_bounds__(256) void k_sort_keys(const float* __restrict__ X, int64_t S, int64_t F,
                                                   int64_t ldx, int use_sent, float sent,
                                                   uint32_t* __restrict__ keys, int64_t ld)
{
    __shared__ uint32_t tile[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t i0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    for (int r = ty; r < 64; r += 4) {
        const int64_t i = i0 + r, c = c0 + tx;
        tile[r][tx] = (i < S && c < F) ? order_key(X[i * ldx + c], use_sent, sent) : 0xFFFFFFFFu;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t c = c0 + r, i = i0 + tx;
        if (c < F && i < ld) keys[c * ld + i] = tile[tx][r];
    }
}

// ---------------------------------------------------------------------------
// per-column sort
// ---------------------------------------------------------------------------
struct SortSmem {
    uint32_t key[SPEARMAN_MAX_S];
    uint16_t idx[SPEARMAN_MAX_S];
    uint32_t wtot[16][8];   // per-wave totals of the packed digit counts
    uint32_t dbase[16];     // exclusive offset of each digit
    int32_t red[16];
};

// 16 digit counters packed as 8-bit fields in four words.
__device__ __forceinline__ uint32_t cnt_get(const uint32_t c[4], uint32_t d)
{
    const uint32_t w = (d >> 2) == 0 ? c[0] : (d >> 2) == 1 ? c[1] : (d >> 2) == 2 ? c[2] : c[3];
    return (w >> (8 * (d & 3))) & 0xFFu;
}
__device__ __forceinline__ void cnt_inc(uint32_t c[4], uint32_t d)
{
    const uint32_t inc = 1u << (8 * (d & 3));
    const uint32_t q = d >> 2;
    c[0] += q == 0 ? inc : 0u;
    c[1] += q == 1 ? inc : 0u;
    c[2] += q == 2 ? inc : 0u;
    c[3] += q == 3 ? inc : 0u;
}

__device__ __forceinline__ uint32_t sel8(const uint32_t w[8], uint32_t q)
{
    const uint32_t a = (q & 1) ? w[1] : w[0];
    const uint32_t b = (q & 1) ? w[3] : w[2];
    const uint32_t c = (q & 1) ? w[5] : w[4];
    const uint32_t d = (q & 1) ? w[7] : w[6];
    const uint32_t ab = (q & 2) ? b : a;
    const uint32_t cd = (q & 2) ? d : c;
    return (q & 4) ? cd : ab;
}

__global__ __launch_bounds__(SORT_THREADS) void k_colsort(const uint32_t* __restrict__ keys, int64_t S,
                                                          int64_t ld, SpearBase out)
{
    __shared__ SortSmem sm;
    const int col = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int E = (int)ceil_div(S, SORT_THREADS);  // <= SORT_EPT
    const uint32_t* kc = keys + (int64_t)col * ld;

    uint32_t key[SORT_EPT];
    uint16_t idx[SORT_EPT];
    int present = 0;
#pragma unroll
    for (int e = 0; e < SORT_EPT; ++e) {
        if (e < E) {
            const int64_t j = (int64_t)e * SORT_THREADS + t;  // striped load, coalesced
            key[e] = j < S ? kc[j] : 0xFFFFFFFFu;
            idx[e] = (uint16_t)(j < S ? j : 0xFFFF);
            present += key[e] != 0xFFFFFFFFu;
        }
    }
    // n_c
    {
        int v = present;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
        if (lane == 0) sm.red[wave] = v;
    }
    __syncthreads();
    int ncount = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) ncount += sm.red[w];

    // The initial order is arbitrary (order among equal keys does not affect
    // average ranks); each pass below is stable with respect to the sequence
    // in which thread t holds positions t*E .. t*E+E-1.
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 4 * pass;
        uint32_t c[4] = {0u, 0u, 0u, 0u};
        uint8_t lr[SORT_EPT];
#pragma unroll
        for (int e = 0; e < SORT_EPT; ++e) {
            if (e < E) {
                const uint32_t d = (key[e] >> shift) & 15u;
                lr[e] = (uint8_t)cnt_get(c, d);
                cnt_inc(c, d);
            }
        }
        // pack into 16-bit fields: w[k] = count(2k) | count(2k+1) << 16
        uint32_t w[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t lo = (c[k >> 1] >> (16 * (k & 1))) & 0xFFu;
            const uint32_t hi = (c[k >> 1] >> (16 * (k & 1) + 8)) & 0xFFu;
            w[k] = lo | (hi << 16);
        }
        uint32_t incl[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) incl[k] = wave_incl_scan_u32(w[k]);
        if (lane == 63) {
#pragma unroll
            for (int k = 0; k < 8; ++k) sm.wtot[wave][k] = incl[k];
        }
        __syncthreads();
        if (t < 16) {
            // digit totals -> exclusive digit bases
            uint32_t tot = 0;
            for (int ww = 0; ww < 16; ++ww) tot += (sm.wtot[ww][t >> 1] >> (16 * (t & 1))) & 0xFFFFu;
            sm.red[t] = (int32_t)tot;
        }
        __syncthreads();
        if (t == 0) {
            uint32_t run = 0;
            for (int d = 0; d < 16; ++d) {
                sm.dbase[d] = run;
                run += (uint32_t)sm.red[d];
            }
        }
        uint32_t wpre[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            uint32_t s = 0;
            for (int ww = 0; ww < wave; ++ww) s += sm.wtot[ww][k];
            wpre[k] = s + incl[k] - w[k];  // exclusive prefix over threads, packed
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < SORT_EPT; ++e) {
            if (e < E) {
                const uint32_t d = (key[e] >> shift) & 15u;
                const uint32_t pw = sel8(wpre, d >> 1);
                const uint32_t pre = (pw >> (16 * (d & 1))) & 0xFFFFu;
                const uint32_t dst = sm.dbase[d] + pre + lr[e];
                sm.key[dst] = key[e];
                sm.idx[dst] = idx[e];
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < SORT_EPT; ++e) {
            if (e < E) {
                key[e] = sm.key[t * E + e];
                idx[e] = sm.idx[t * E + e];
            }
        }
        __syncthreads();
    }

    // ---- outputs: positions are t*E + e (blocked), keys in registers ----------
    uint16_t* ordc = out.ord + (int64_t)col * ld;
    uint16_t* posc = out.pos + (int64_t)col * ld;
    uint32_t* runc = out.runs + (int64_t)col * ld;
    // run starts: s(k) = max{j <= k : j == 0 or key[j] != key[j-1]}; the
    // sorted keys are still in sm.key
    int last = -1;
    int rs[SORT_EPT];
#pragma unroll
    for (int e = 0; e < SORT_EPT; ++e) {
        if (e < E) {
            const int k = t * E + e;
            const bool start = (k == 0) || (k < ncount && key[e] != sm.key[k - 1]);
            if (k < ncount && start) last = k;
            rs[e] = last;  // -1 if the start lies in an earlier thread
        }
    }
    // block exclusive max-scan of `last`
    int v = last;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(v, d, 64);
        if (lane >= d) v = max(v, o);
    }
    __syncthreads();
    if (lane == 63) sm.red[wave] = v;
    __syncthreads();
    int before = -1;
    for (int ww = 0; ww < wave; ++ww) before = max(before, sm.red[ww]);
    int excl = __shfl_up(v, 1, 64);
    if (lane == 0) excl = -1;
    before = max(before, excl);
#pragma unroll
    for (int e = 0; e < SORT_EPT; ++e)
        if (e < E && rs[e] < 0) rs[e] = before;
    __syncthreads();
    uint32_t* END = sm.key;  // reused: END[run start] = run end
    bool tie_here = false;
    // A run ends at k when k+1 == ncount or rs(k+1) != rs(k).  rs of the
    // successor is held by the same thread (e+1) or by thread t+1 (e = 0).
    int rs_next_first = __shfl_down(rs[0], 1, 64);
    __syncthreads();
    if (lane == 0) sm.red[wave] = rs[0];
    __syncthreads();
    if (lane == 63) rs_next_first = (wave + 1 < 16) ? sm.red[wave + 1] : -2;
#pragma unroll
    for (int e = 0; e < SORT_EPT; ++e) {
        if (e < E) {
            const int k = t * E + e;
            if (k < ncount) {
                const int rn = (k + 1 == ncount) ? -2 : (e + 1 < E ? rs[e + 1] : rs_next_first);
                if (rn != rs[e]) {
                    END[rs[e]] = (uint32_t)(k + 1);
                    if (k > rs[e]) tie_here = true;
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < SORT_EPT; ++e) {
        if (e < E) {
            const int k = t * E + e;
            if (k < ncount) {
                ordc[k] = idx[e];
                posc[idx[e]] = (uint16_t)k;
                runc[k] = (uint32_t)rs[e] | (END[rs[e]] << 16);
            } else if (idx[e] != 0xFFFF) {
                posc[idx[e]] = 0xFFFF;  // missing sample
            }
        }
    }
    const int anytie = __syncthreads_or(tie_here ? 1 : 0);
    if (t == 0) {
        out.ncol[col] = ncount;
        out.hasties[col] = anytie ? 1 : 0;
    }
}

// ---------------------------------------------------------------------------
// per-pair re-ranking scan
// ---------------------------------------------------------------------------
struct PairOut {
    double4* sums;  // [npairs] (n, A, B_a, B_b)
    int2* ab;       // [npairs]
    int32_t* dbg_ra;
    int32_t* dbg_rb;
    int dbg_a, dbg_b;
};

__device__ __forceinline__ int64_t pair_index(int64_t a, int64_t b, int64_t F)
{
    return a * F - a * (a - 1) / 2 + (b - a);
}

__device__ __forceinline__ int64_t sum_sq_doubled_untied(int64_t n)
{
    // sum_{m=1..n} (2m)^2 = 4 n (n+1) (2n+1) / 6
    return (n * (n + 1) * (2 * n + 1) / 6) * 4;
}

__global__ __launch_bounds__(256) void k_spearman_pairs(SpearBase bs, int64_t S, int64_t F, PairOut po)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool dbg = po.dbg_ra != nullptr;
    const int64_t a = dbg ? po.dbg_a : (int64_t)blockIdx.y;
    const int64_t b0 = dbg ? po.dbg_b : (int64_t)blockIdx.x * PAIR_BLOCK;
    const int nb_here = dbg ? 1 : PAIR_BLOCK;
    if (a >= F) return;
    if (!dbg && b0 + PAIR_BLOCK - 1 < a) return;
    if (b0 >= F) return;

    const int64_t ld = bs.ld;
    const int nwa_max = (int)ceil_div(S, 32) + 1;
    const int ncb_max = (int)ceil_div(S, 64) + 1;
    uint16_t* posA = (uint16_t*)smem_raw;
    unsigned char* wbase = smem_raw + round_up(ld * 2, 16);
    const size_t per_wave = round_up((size_t)nwa_max * 8 + (size_t)ncb_max * 12, 16);
    unsigned char* wmem = wbase + per_wave * wave;
    uint64_t* KB = (uint64_t*)wmem;                       // [ncb_max]
    uint32_t* KA = (uint32_t*)(wmem + (size_t)ncb_max * 8);  // [nwa_max]
    uint32_t* PA = KA + nwa_max;                          // [nwa_max]
    uint32_t* PB = PA + nwa_max;                          // [ncb_max]

    // stage pos_a
    {
        const uint32_t* src = (const uint32_t*)(bs.pos + a * ld);
        uint32_t* dst = (uint32_t*)posA;
        for (int64_t w = threadIdx.x; w < ld / 2; w += 256) dst[w] = src[w];
    }
    __syncthreads();

    const int na = bs.ncol[a];
    const int tA = bs.hasties[a];
    const uint32_t* runsA = bs.runs + a * ld;
    const int nwa = (na + 31) >> 5;

    for (int q = wave; q < nb_here; q += PAIR_WAVES) {
        const int64_t b = b0 + q;
        if (b >= F || (!dbg && b < a)) continue;
        const int nbv = bs.ncol[b];
        const int tB = bs.hasties[b];
        const uint16_t* ordB = bs.ord + b * ld;
        const uint32_t* runsB = bs.runs + b * ld;
        const int ncb = (nbv + 63) >> 6;

        for (int w = lane; w <= nwa; w += 64) KA[w] = 0u;
        wave_sync_lds();

        // walk 1: b's presence mask along b's order, a-side bitmap
        uint32_t carry = 0;
        for (int c = 0; c < ncb; ++c) {
            const int k = c * 64 + lane;
            const bool valid = k < nbv;
            const uint32_t i = valid ? ordB[k] : 0u;
            const uint32_t p = valid ? posA[i] : 0xFFFFu;
            const bool kept = p != 0xFFFFu;
            const uint64_t mask = __ballot(kept);
            if (lane == 0) {
                KB[c] = mask;
                PB[c] = carry;
            }
            carry += (uint32_t)__popcll(mask);
            if (kept) atomicOr(&KA[p >> 5], 1u << (p & 31));
        }
        if (lane == 0) {
            KB[ncb] = 0ull;
            PB[ncb] = carry;
        }
        const uint32_t n = carry;
        wave_sync_lds();

        // prefix over the a-side bitmap words (one extra word past the end)
        uint32_t run = 0;
        for (int w0 = 0; w0 <= nwa; w0 += 64) {
            const int w = w0 + lane;
            const uint32_t v = (w <= nwa) ? (uint32_t)__popc(KA[w]) : 0u;
            const uint32_t incl = wave_incl_scan_u32(v);
            if (w <= nwa) PA[w] = run + incl - v;
            run += __shfl(incl, 63, 64);
        }
        wave_sync_lds();

        // walk 2: doubled ranks and sums
        double sA = 0.0, sBa = 0.0, sBb = 0.0;
        for (int c = 0; c < ncb; ++c) {
            const int k = c * 64 + lane;
            const bool valid = k < nbv;
            const uint32_t i = valid ? ordB[k] : 0u;
            const uint32_t p = valid ? posA[i] : 0xFFFFu;
            const bool kept = p != 0xFFFFu;
            const uint64_t mask = KB[c];
            const uint32_t cb = PB[c] + mbcnt64(mask);
            if (kept) {
                uint32_t Rb;
                if (tB) {
                    const uint32_t rr = runsB[k];
                    const uint32_t x0 = rr & 0xFFFFu, x1 = rr >> 16;
                    const uint32_t c0 = PB[x0 >> 6] + (uint32_t)__popcll(KB[x0 >> 6] & ((1ull << (x0 & 63)) - 1ull));
                    const uint32_t c1 = PB[x1 >> 6] + (uint32_t)__popcll(KB[x1 >> 6] & ((1ull << (x1 & 63)) - 1ull));
                    Rb = c0 + c1 + 1u;
                } else {
                    Rb = 2u * cb + 2u;
                }
                uint32_t Ra;
                if (tA) {
                    const uint32_t rr = runsA[p];
                    const uint32_t x0 = rr & 0xFFFFu, x1 = rr >> 16;
                    const uint32_t c0 = PA[x0 >> 5] + (uint32_t)__popc(KA[x0 >> 5] & ((1u << (x0 & 31)) - 1u));
                    const uint32_t c1 = PA[x1 >> 5] + (uint32_t)__popc(KA[x1 >> 5] & ((1u << (x1 & 31)) - 1u));
                    Ra = c0 + c1 + 1u;
                } else {
                    const uint32_t ca = PA[p >> 5] + (uint32_t)__popc(KA[p >> 5] & ((1u << (p & 31)) - 1u));
                    Ra = 2u * ca + 2u;
                }
                sA += (double)(Ra * Rb);
                if (tA) sBa += (double)(Ra * Ra);
                if (tB) sBb += (double)(Rb * Rb);
                if (dbg) {
                    po.dbg_ra[i] = (int32_t)Ra;
                    po.dbg_rb[i] = (int32_t)Rb;
                }
            }
        }
        sA = wave_sum_f64(sA);
        sBa = wave_sum_f64(sBa);
        sBb = wave_sum_f64(sBb);
        if (lane == 0 && !dbg) {
            const int64_t nn = (int64_t)n;
            const double Ba = tA ? sBa : (double)sum_sq_doubled_untied(nn);
            const double Bb = tB ? sBb : (double)sum_sq_doubled_untied(nn);
            const int64_t pid = pair_index(a, b, F);
            po.sums[pid] = make_double4((double)nn, sA, Ba, Bb);
            po.ab[pid] = make_int2((int)a, (int)b);
        }
        wave_sync_lds();
    }
}

__global__ __launch_bounds__(256) void k_spearman_final(const double4* __restrict__ sums,
                                                        const int2* __restrict__ ab, int64_t npairs,
                                                        double* __restrict__ r, double* __restrict__ p,
                                                        int32_t* __restrict__ n, int64_t ldo)
{
    const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (id >= npairs) return;
    const double4 s = sums[id];
    const int2 q = ab[id];
    const int64_t nn = (int64_t)s.x;
    const int64_t A = (int64_t)s.y, Ba = (int64_t)s.z, Bb = (int64_t)s.w;
    const int64_t K = nn * (nn + 1) * (nn + 1);
    const int64_t num = A - K, Da = Ba - K, Db = Bb - K;
    double rho = __builtin_nan(""), pv = __builtin_nan("");
    if (nn >= 2 && Da > 0 && Db > 0) {
        // sqrt of the product (not the product of roots) so that identical
        // rank vectors give exactly 1
        rho = (double)num / sqrt((double)Da * (double)Db);
        rho = rho > 1.0 ? 1.0 : (rho < -1.0 ? -1.0 : rho);
        if (nn >= 3) pv = corr_pvalue(rho, nn);
    }
    const int64_t g = q.x, h = q.y;
    if (r) {
        r[g * ldo + h] = rho;
        r[h * ldo + g] = rho;
    }
    if (p) {
        p[g * ldo + h] = pv;
        p[h * ldo + g] = pv;
    }
    if (n) {
        n[g * ldo + h] = (int32_t)nn;
        n[h * ldo + g] = (int32_t)nn;
    }
}

// ---------------------------------------------------------------------------
// subset compaction: a query's rows and columns from a prepared base
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_rowmap(const int32_t* __restrict__ rows, int64_t Sq, int64_t S,
                                                int32_t* __restrict__ rowmap)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < S) rowmap[i] = -1;
}
__global__ __launch_bounds__(256) void k_rowmap_set(const int32_t* __restrict__ rows, int64_t Sq,
                                                    int32_t* __restrict__ rowmap)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < Sq) rowmap[rows[j]] = (int32_t)j;
}

// One 1024-thread workgroup per query column: keeps the base column's sorted
// order restricted to the query rows (order preserved), renumbers samples and
// positions, and maps tie runs through the prefix count of kept positions.
__global__ __launch_bounds__(SORT_THREADS) void k_compact(SpearBase base, const int32_t* __restrict__ cols,
                                                          const int32_t* __restrict__ rowmap, int64_t Sq,
                                                          SpearBase q)
{
    __shared__ uint16_t P[SPEARMAN_MAX_S + 1];  // kept positions below k
    __shared__ uint32_t wsum[16];
    const int qc = blockIdx.x;
    const int64_t c = cols[qc];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int nc = base.ncol[c];
    const uint16_t* ord = base.ord + c * base.ld;
    const uint32_t* runs = base.runs + c * base.ld;
    uint16_t* qord = q.ord + (int64_t)qc * q.ld;
    uint16_t* qpos = q.pos + (int64_t)qc * q.ld;
    uint32_t* qruns = q.runs + (int64_t)qc * q.ld;
    for (int64_t j = t; j < Sq; j += SORT_THREADS) qpos[j] = 0xFFFF;
    __syncthreads();
    uint32_t carry = 0;
    for (int k0 = 0; k0 < nc; k0 += SORT_THREADS) {
        const int k = k0 + t;
        int32_t nr = -1;
        if (k < nc) nr = rowmap[ord[k]];
        const bool kept = nr >= 0;
        const uint64_t m = __ballot(kept);
        if (lane == 0) wsum[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = carry;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        uint32_t tot = 0;
        for (int w = 0; w < 16; ++w) tot += wsum[w];
        const uint32_t kp = before + mbcnt64(m);
        if (k < nc) P[k] = (uint16_t)kp;
        if (kept) {
            qord[kp] = (uint16_t)nr;
            qpos[nr] = (uint16_t)kp;
        }
        carry += tot;
        __syncthreads();
    }
    if (t == 0) P[nc] = (uint16_t)carry;
    __syncthreads();
    int tie = 0;
    for (int k0 = 0; k0 < nc; k0 += SORT_THREADS) {
        const int k = k0 + t;
        if (k < nc) {
            const int32_t nr = rowmap[ord[k]];
            if (nr >= 0) {
                const uint32_t rr = runs[k];
                const uint32_t s0 = P[rr & 0xFFFFu], e0 = P[rr >> 16];
                qruns[P[k]] = s0 | (e0 << 16);
                tie |= (e0 - s0) > 1u;
            }
        }
    }
    const int anytie = __syncthreads_or(tie);
    if (t == 0) {
        q.ncol[qc] = (int32_t)carry;
        q.hasties[qc] = anytie;
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static size_t pair_smem_bytes(int64_t S)
{
    const int64_t ld = spear_ld(S);
    const int nwa_max = (int)ceil_div(S, 32) + 1;
    const int ncb_max = (int)ceil_div(S, 64) + 1;
    const size_t per_wave = round_up((size_t)nwa_max * 8 + (size_t)ncb_max * 12, 16);
    return (size_t)round_up(ld * 2, 16) + per_wave * PAIR_WAVES;
}

static int pairs_launch(const SpearBase& bs, int64_t S, int64_t F, PairOut po, hipStream_t st)
{
    const size_t smem = pair_smem_bytes(S);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_spearman_pairs,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return hip_status(e, "hipFuncSetAttribute(k_spearman_pairs)");
        attr_set = true;
    }
    dim3 grid;
    if (po.dbg_ra) {
        grid = dim3(1, 1);
    } else {
        // pad the partner-block count to a multiple of 8 so that a partner
        // block always lands on the same XCD (its sorted orders stay in L2)
        grid = dim3((unsigned)round_up(ceil_div(F, PAIR_BLOCK), 8), (unsigned)F);
    }
    hipLaunchKernelGGL(k_spearman_pairs, grid, dim3(256), smem, st, bs, S, F, po);
    return check_launch("spearman_pairs");
}

struct SpearWs {
    uint32_t* keys;
    SpearBase base;
    double4* sums;
    int2* ab;
};

static void spear_carve(Carver& c, int64_t S, int64_t F, SpearWs& w)
{
    const int64_t ld = spear_ld(S);
    w.keys = c.take<uint32_t>((size_t)F * ld);
    base_carve(c, S, F, w.base);
    const int64_t npairs = F * (F + 1) / 2;
    w.sums = c.take<double4>(npairs);
    w.ab = c.take<int2>(npairs);
}

static int sort_launch(const float* X, int64_t S, int64_t F, int64_t ldx, int us, float sv,
                       uint32_t* keys, const SpearBase& base, hipStream_t st)
{
    dim3 gk((unsigned)ceil_div(F, 64), (unsigned)ceil_div(base.ld, 64));
    hipLaunchKernelGGL(k_sort_keys, gk, dim3(256), 0, st, X, S, F, ldx, us, sv, keys, base.ld);
    NAPY_TRY(check_launch("sort_keys"));
    hipLaunchKernelGGL(k_colsort, dim3((unsigned)F), dim3(SORT_THREADS), 0, st, keys, S, base.ld, base);
    return check_launch("colsort");
}

static int final_launch(const SpearWs& w, int64_t F, double* r, double* p, int32_t* n, int64_t ldo,
                        hipStream_t st)
{
    const int64_t npairs = F * (F + 1) / 2;
    hipLaunchKernelGGL(k_spearman_final, dim3((unsigned)ceil_div(npairs, 256)), dim3(256), 0, st, w.sums,
                       w.ab, npairs, r, p, n, ldo);
    return check_launch("spearman_final");
}

size_t spearman_ws_bytes(int64_t S, int64_t F)
{
    Carver c(nullptr);
    SpearWs w;
    spear_carve(c, S, F, w);
    return c.bytes();
}

int spearman_run(const float* X, int64_t S, int64_t F, int64_t ldx, double* r, double* p, int32_t* n,
                 int64_t ldo, void* ws, const napy_opts* opts, hipStream_t st, void* const* ev)
{
    Carver c(ws);
    SpearWs w;
    spear_carve(c, S, F, w);
    NAPY_TRY(record_stage(ev, 0, st));
    NAPY_TRY(sort_launch(X, S, F, ldx, opt_use_sent(opts), opt_sent(opts), w.keys, w.base, st));
    NAPY_TRY(record_stage(ev, 1, st));
    PairOut po{w.sums, w.ab, nullptr, nullptr, 0, 0};
    NAPY_TRY(pairs_launch(w.base, S, F, po, st));
    NAPY_TRY(record_stage(ev, 2, st));
    NAPY_TRY(final_launch(w, F, r, p, n, ldo, st));
    return record_stage(ev, 3, st);
}

__global__ void k_fill_i32(int32_t* __restrict__ a, int64_t count, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) a[i] = v;
}

int spearman_pair_ranks_run(const float* X, int64_t S, int64_t F, int64_t ldx, int g, int h, int32_t* rg,
                            int32_t* rh, void* ws, const napy_opts* opts, hipStream_t st)
{
    Carver c(ws);
    SpearWs w;
    spear_carve(c, S, F, w);
    NAPY_TRY(sort_launch(X, S, F, ldx, opt_use_sent(opts), opt_sent(opts), w.keys, w.base, st));
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)ceil_div(S, 256)), dim3(256), 0, st, rg, S, -1);
    NAPY_TRY(check_launch("fill"));
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)ceil_div(S, 256)), dim3(256), 0, st, rh, S, -1);
    NAPY_TRY(check_launch("fill"));
    PairOut po{w.sums, w.ab, rg, rh, g, h};
    return pairs_launch(w.base, S, F, po, st);
}

size_t spearman_base_bytes(int64_t S, int64_t F)
{
    Carver c(nullptr);
    SpearBase b;
    base_carve(c, S, F, b);
    // the keys buffer used while sorting is carved after the base
    c.take<uint32_t>((size_t)F * spear_ld(S));
    return c.bytes();
}

int spearman_base_prepare_run(const float* X, int64_t S, int64_t F, int64_t ldx, void* base,
                              const napy_opts* opts, hipStream_t st)
{
    Carver c(base);
    SpearBase b;
    base_carve(c, S, F, b);
    uint32_t* keys = c.take<uint32_t>((size_t)F * spear_ld(S));
    return sort_launch(X, S, F, ldx, opt_use_sent(opts), opt_sent(opts), keys, b, st);
}

size_t spearman_subset_ws_bytes(int64_t S, int64_t Sq, int64_t Fq)
{
    Carver c(nullptr);
    c.take<int32_t>(S > 0 ? S : 1);
    SpearBase q;
    base_carve(c, Sq, Fq, q);
    const int64_t npairs = Fq * (Fq + 1) / 2;
    c.take<double4>(npairs);
    c.take<int2>(npairs);
    return c.bytes();
}

int spearman_subset_run(const void* basebuf, int64_t S, int64_t F, const int32_t* rows, int64_t Sq,
                        const int32_t* cols, int64_t Fq, double* r, double* p, int32_t* n, int64_t ldo,
                        void* ws, hipStream_t st)
{
    Carver cb((void*)basebuf);
    SpearBase b;
    base_carve(cb, S, F, b);
    Carver c(ws);
    int32_t* rowmap = c.take<int32_t>(S > 0 ? S : 1);
    SpearWs w;
    base_carve(c, Sq, Fq, w.base);
    const int64_t npairs = Fq * (Fq + 1) / 2;
    w.sums = c.take<double4>(npairs);
    w.ab = c.take<int2>(npairs);
    w.keys = nullptr;
    hipLaunchKernelGGL(k_rowmap, dim3((unsigned)ceil_div(S, 256)), dim3(256), 0, st, rows, Sq, S, rowmap);
    NAPY_TRY(check_launch("rowmap"));
    hipLaunchKernelGGL(k_rowmap_set, dim3((unsigned)ceil_div(Sq, 256)), dim3(256), 0, st, rows, Sq, rowmap);
    NAPY_TRY(check_launch("rowmap_set"));
    hipLaunchKernelGGL(k_compact, dim3((unsigned)Fq), dim3(SORT_THREADS), 0, st, b, cols, rowmap, Sq, w.base);
    NAPY_TRY(check_launch("compact"));
    PairOut po{w.sums, w.ab, nullptr, nullptr, 0, 0};
    NAPY_TRY(pairs_launch(w.base, Sq, Fq, po, st));
    return final_launch(w, Fq, r, p, n, ldo, st);
}

}  // namespace napy
