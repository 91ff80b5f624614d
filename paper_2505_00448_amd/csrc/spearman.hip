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
//                    the keys in LDS (4 passes of 8 bits; k_colsort_big
//                    over global memory for columns past 24,576), then
//                    ord[c][k] (sample at sorted position k), pos[c][i]
//                    (sorted position of sample i, 0xFFFF if missing),
//                    runs[c][k] = s | e << 16 (tie run of position k), n_c and
//                    a has-ties flag.
//   k_presence       presence bytes: bit j of presb[q][i] = sample i present
//                    in column 8 q + j of the processing order.
//   k_spearman_pairs one workgroup per (column a, block of 8 partners b).
//                    Step 1 copies the block's presence bytes to LDS and
//                    builds, for all 8 partners at once, a table along a's
//                    sorted order: the partner's presence bits per 32
//                    positions and the count before them (one LDS byte
//                    gather per position, one ballot per partner), plus the
//                    tie defects of a's runs; pos_a then replaces the
//                    presence bytes in LDS.  Step 2:
//                    each wave walks one partner's sorted order once; b's
//                    count of complete samples below each position comes from
//                    ballot + mbcnt, a's from the table by popcount; the
//                    rank products and b's tie defects follow.
//   k_spearman_final one thread per pair: rho, p, n into both triangles.
#include "napy_internal.hpp"
#include "pvalue.hpp"
#include "rankbase.hpp"
#include "tilefin.hpp"

namespace napy {

constexpr int SPEARMAN_MAX_S = (int)SORT_LDS_MAX_S;  // longest column of the LDS sort
// column sort: 1024 threads (16 waves) and up to CS_EPT_MAX keys per thread
constexpr int CS_THREADS = 1024;
constexpr int CS_WAVES = CS_THREADS / 64;
constexpr int CS_EPT_MAX = SPEARMAN_MAX_S / CS_THREADS;  // 24

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

// X (S x F row-major) -> keys [F][ld] through a 64 x 64 LDS tile.  Lane
// groups of 16 take a tile row as 16 runs of 4 columns (one 16-byte load per
// lane when VEC: ldx a multiple of 4 and X 16-byte aligned, and the 4
// columns inside the matrix), and write a tile column as 16 runs of 4
// samples (one 16-byte store).  The tile rows are 65 words apart, so both
// the stores into the tile and the column reads out of it fall on distinct
// banks.
template <bool VEC>
__global__ __launch_bounds__(256) void k_sort_keys(const float* __restrict__ X, int64_t S, int64_t F,
                                                   int64_t ldx, int use_sent, float sent,
                                                   uint32_t* __restrict__ keys, int64_t ld)
{
    __shared__ uint32_t tile[64][65];
    const int q = threadIdx.x & 15, g = threadIdx.x >> 4;  // run of 4, lane group
    const int64_t i0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int r = g + 16 * u;
        const int64_t i = i0 + r, c = c0 + 4 * q;
        float v[4];
        if (VEC && i < S && c + 3 < F) {
            const float4 x4 = *(const float4*)(X + i * ldx + c);
            v[0] = x4.x;
            v[1] = x4.y;
            v[2] = x4.z;
            v[3] = x4.w;
#pragma unroll
            for (int k = 0; k < 4; ++k) tile[r][4 * q + k] = order_key(v[k], use_sent, sent);
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                tile[r][4 * q + k] =
                    (i < S && c + k < F) ? order_key(X[i * ldx + c + k], use_sent, sent) : 0xFFFFFFFFu;
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int cc = g + 16 * u;
        const int64_t c = c0 + cc, i = i0 + 4 * q;  // ld is a multiple of 4: i < ld covers i + 3
        if (c < F && i < ld)
            *(uint4*)(keys + c * ld + i) =
                make_uint4(tile[4 * q][cc], tile[4 * q + 1][cc], tile[4 * q + 2][cc], tile[4 * q + 3][cc]);
    }
}

// ---------------------------------------------------------------------------
// per-column sort
// ---------------------------------------------------------------------------
// LDS of the column sort for E keys per thread: the keys and sample indices
// of CS_THREADS * E slots, each wave's 256 digit counters (16-bit), and the
// per-wave values of the block scans.
struct SortSmem {
    uint32_t* key;    // [CS_THREADS * E]
    uint16_t* idx;    // [CS_THREADS * E]
    uint16_t* wcnt;   // [CS_WAVES][256]
    uint32_t* red;    // [4][CS_WAVES]
};

__host__ __device__ inline size_t sort_smem_bytes(int E)
{
    const size_t cap = (size_t)CS_THREADS * (size_t)E;
    return (size_t)round_up((int64_t)(cap * 4), 16) + (size_t)round_up((int64_t)(cap * 2), 16) +
           (size_t)CS_WAVES * 256 * 2 + 4 * CS_WAVES * 4;
}

__device__ inline SortSmem sort_smem(unsigned char* raw, int E)
{
    const size_t cap = (size_t)CS_THREADS * (size_t)E;
    SortSmem m;
    m.key = (uint32_t*)raw;
    unsigned char* p = raw + round_up((int64_t)(cap * 4), 16);
    m.idx = (uint16_t*)p;
    p += round_up((int64_t)(cap * 2), 16);
    m.wcnt = (uint16_t*)p;
    m.red = (uint32_t*)(p + CS_WAVES * 256 * 2);
    return m;
}

// lanes whose 8-bit digit equals this lane's: the complement of the lanes
// that differ in some bit, where lanes differing in bit b are the ballot of
// bit b XOR (this lane's bit b, spread over all 32 bits)
__device__ __forceinline__ uint64_t match_digit8(uint32_t d)
{
    uint32_t nlo = 0u, nhi = 0u;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint32_t sb = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);  // 0 or all ones
        // the lane mask of sb != 0 as a compare of sb itself (33: not equal;
        // written as a ballot, the compare is rebuilt from a shift of d)
        const uint64_t bl = __builtin_amdgcn_uicmp(sb, 0u, 33);
        // the lanes that differ from this one in bit b: n |= bl ^ sb, one
        // three-input bit operation per half (0xF6: a | (b ^ c))
        nlo = __builtin_amdgcn_bitop3_b32(nlo, (uint32_t)bl, sb, 0xF6);
        nhi = __builtin_amdgcn_bitop3_b32(nhi, (uint32_t)(bl >> 32), sb, 0xF6);
    }
    return ((uint64_t)~nhi << 32) | (uint64_t)~nlo;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// inclusive max-scan over the 64 lanes (values >= 0)
__device__ __forceinline__ int wave_incl_max_scan(int x)
{
    constexpr int ROW_SHR = 0x110, ROW_BCAST15 = 0x142, ROW_BCAST31 = 0x143;
    x = max(x, __builtin_amdgcn_update_dpp(0, x, ROW_SHR + 1, 0xF, 0xF, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, ROW_SHR + 2, 0xF, 0xF, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, ROW_SHR + 4, 0xF, 0xF, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, ROW_SHR + 8, 0xF, 0xF, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, ROW_BCAST15, 0xA, 0xF, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, ROW_BCAST31, 0xC, 0xF, false));
    return x;
}

// One column per workgroup.  The observed keys (sample index as payload) are
// compacted, then sorted by an LSD radix sort in LDS: 4 stable passes of
// 8-bit digits.  Wave w holds sorted slots w 64 E' .. (w + 1) 64 E' - 1,
// lane l at step e slot w 64 E' + 64 e + l (E' = observed keys per thread,
// rounded up), so within a wave the slots run in (step, lane) order.  A
// pass ranks each step's keys among the wave's equal digits (lanes matched
// on the digit by ballots; a 16-bit counter per digit and wave carries the
// count across steps), scans the 256 x 16 counters in (digit, wave) order
// into destinations, scatters the keys in LDS and reloads them.  The tail
// derives tie runs from the sorted keys: ord, pos, runs, the tie-run list,
// tie bits and counts.
// Sum (op 0) or maximum (op 1) over the waves of the sort block of one value
// per wave, stored at w[0 .. CS_WAVES): lane v reads wave v's value and a
// scan over the first row of 16 lanes (four DPP row shifts) gives, by lane
// reads, the part over the waves before this one and the whole (both
// wave-uniform), instead of every thread looping over the 16 values
template <int OP>
__device__ __forceinline__ void cs_wave_prefix(const uint32_t* w, int lane, int wave, uint32_t& before,
                                               uint32_t& total)
{
    static_assert(CS_WAVES == 16, "one row of 16 lanes");
    constexpr int ROW_SHR = 0x110;
    int x = lane < CS_WAVES ? (int)w[lane] : 0;
    // (values are non-negative: 0, shifted in, is the identity of both)
    const auto op = [](int a, int b) { return OP == 0 ? a + b : max(a, b); };
    x = op(x, __builtin_amdgcn_update_dpp(0, x, ROW_SHR + 1, 0xF, 0xF, false));
    x = op(x, __builtin_amdgcn_update_dpp(0, x, ROW_SHR + 2, 0xF, 0xF, false));
    x = op(x, __builtin_amdgcn_update_dpp(0, x, ROW_SHR + 4, 0xF, 0xF, false));
    x = op(x, __builtin_amdgcn_update_dpp(0, x, ROW_SHR + 8, 0xF, 0xF, false));
    total = (uint32_t)__builtin_amdgcn_readlane(x, CS_WAVES - 1);
    before = wave > 0 ? (uint32_t)__builtin_amdgcn_readlane(x, wave - 1) : 0u;
}

template <int EPT>
__global__ __launch_bounds__(CS_THREADS, EPT <= 10 ? 8 : 4) void k_colsort(const uint32_t* __restrict__ keys, int64_t S,
                                                          int64_t ld, SpearBase out)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char sort_raw[];
    constexpr int E = EPT;
    const int col = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const SortSmem sm = sort_smem(sort_raw, E);
    const uint32_t* kc = keys + (int64_t)col * ld;
    uint16_t* ordc = out.ord + (int64_t)col * ld;
    uint16_t* ord2c = out.ord2 + (int64_t)col * ld;
    uint16_t* posc = out.pos + (int64_t)col * ld;
    uint32_t* runc = out.runs + (int64_t)col * ld;

    // ---- compaction of the observed keys (striped, coalesced loads) ------
    uint32_t key[E], pk[E];  // pk: sample index (low 16 bits) | rank in the wave (high 16)
    uint32_t nobs = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int64_t j = (int64_t)e * CS_THREADS + t;
        key[e] = j < S ? kc[j] : 0xFFFFFFFFu;
        const bool obs = key[e] != 0xFFFFFFFFu;
        if (!obs && j < S) posc[j] = 0xFFFF;  // missing sample
        nobs += obs;
    }
    const uint32_t oincl = wave_incl_scan_u32(nobs);
    if (lane == 63) sm.red[wave] = oincl;
    __syncthreads();
    uint32_t obase, ncount;
    cs_wave_prefix<0>(sm.red, lane, wave, obase, ncount);
    obase += oincl - nobs;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (key[e] != 0xFFFFFFFFu) {
            sm.key[obase] = key[e];
            sm.idx[obase] = (uint16_t)(e * CS_THREADS + t);
            ++obase;
        }
    }
    const int Ee = (int)((ncount + CS_THREADS - 1) / CS_THREADS);  // steps per wave
    const int slots = Ee * CS_THREADS;
    for (int k = (int)ncount + t; k < slots; k += CS_THREADS) {
        sm.key[k] = 0xFFFFFFFFu;  // padding sorts last
        sm.idx[k] = 0xFFFF;
    }
    __syncthreads();
    const int wbase = wave * 64 * Ee;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (e < Ee) {
            key[e] = sm.key[wbase + 64 * e + lane];
            pk[e] = sm.idx[wbase + 64 * e + lane];
        }
    }

    // bits in which some observed key differs from the first: a pass whose
    // digit is the same for every observed key leaves the order as it is
    // (integer-valued columns have zero low mantissa bytes)
    uint32_t diff = 0u;
    {
        const uint32_t k0 = ncount > 0 ? sm.key[0] : 0u;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (e < Ee && wbase + 64 * e + lane < (int)ncount) diff |= key[e] ^ k0;
#pragma unroll
        for (int dd = 32; dd >= 1; dd >>= 1) diff |= (uint32_t)__shfl_xor((int)diff, dd, 64);
        // (slots CS_WAVES.. are next written after a pass's first barrier)
        if (lane == 0) sm.red[CS_WAVES + wave] = diff;
        __syncthreads();
#pragma unroll
        for (int v = 0; v < CS_WAVES; ++v) diff |= sm.red[CS_WAVES + v];
    }

    // ---- 4 passes of 8-bit digits ------------------------------------------
    uint16_t* wc = sm.wcnt + wave * 256;
    for (int pass = 0; pass < 4 && Ee > 0; ++pass) {
        const int shift = 8 * pass;
        if (((diff >> shift) & 255u) == 0u) continue;  // uniform over the block
#pragma unroll
        for (int q = 0; q < 4; ++q) wc[q * 64 + lane] = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (e < Ee) {
                const uint32_t d = (key[e] >> shift) & 255u;
                const uint64_t peers = match_digit8(d);
                const uint32_t below = lanes_below(peers);
                const uint32_t cnt = (uint32_t)__popcll(peers);
                const uint32_t b = wc[d];
                if (below + 1u == cnt) wc[d] = (uint16_t)(b + cnt);  // last of the peers
                pk[e] = (pk[e] & 0xFFFFu) | ((b + below) << 16);
            }
        }
        __syncthreads();
        // thread t: digit t / 4, waves 4 (t % 4) .. 4 (t % 4) + 3
        {
            const int dd = t >> 2, q = t & 3;
            uint32_t c4[4], sum = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                c4[i] = sm.wcnt[(4 * q + i) * 256 + dd];
                sum += c4[i];
            }
            const uint32_t incl = wave_incl_scan_u32(sum);
            if (lane == 63) sm.red[CS_WAVES + wave] = incl;
            __syncthreads();
            uint32_t before, all;
            cs_wave_prefix<0>(sm.red + CS_WAVES, lane, wave, before, all);
            uint32_t run = incl - sum + before;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                sm.wcnt[(4 * q + i) * 256 + dd] = (uint16_t)run;
                run += c4[i];
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (e < Ee) {
                const uint32_t d = (key[e] >> shift) & 255u;
                const uint32_t dst = (uint32_t)wc[d] + (pk[e] >> 16);
                sm.key[dst] = key[e];
                sm.idx[dst] = (uint16_t)pk[e];
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (e < Ee) {
                key[e] = sm.key[wbase + 64 * e + lane];
                pk[e] = sm.idx[wbase + 64 * e + lane];
            }
        }
    }

    // ---- tie runs ------------------------------------------------------------
    // start: the key differs from its predecessor; last: from its successor.
    // s(k) = the latest start <= k (a max-scan: within the wave, carried
    // across steps, then across waves); a tie run is a start that is not also
    // a last, and tie runs are numbered in position order (within a wave:
    // by step, then lane).  The last of each run records its end at the
    // run's start.
    // From here key[e] holds the element's run start (low 30 bits) and its
    // flags (bit 30: start, bit 31: last).
    const int nc = (int)ncount;
    int carry = 0;
    uint32_t ntr = 0;  // tie runs starting in the wave's slots (wave-uniform)
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (e < Ee) {
            const int k = wbase + 64 * e + lane;
            uint32_t f = 0;
            if (k < nc) {
                const bool st = k == 0 || sm.key[k - 1] != key[e];
                const bool ls = k + 1 == nc || sm.key[k + 1] != key[e];
                f = (st ? 1u : 0u) | (ls ? 2u : 0u);
            }
            ntr += (uint32_t)__popcll(__ballot(f == 1u));
            const int x = max(wave_incl_max_scan((f & 1u) ? k : 0), carry);
            carry = __builtin_amdgcn_readlane(x, 63);
            key[e] = (uint32_t)x | (f << 30);
        }
    }
    if (lane == 0) {
        sm.red[2 * CS_WAVES + wave] = (uint32_t)carry;
        sm.red[3 * CS_WAVES + wave] = ntr;
    }
    __syncthreads();  // also: every neighbour key has been read
    uint32_t cin_u, cmax, rid, nrun;
    cs_wave_prefix<1>(sm.red + 2 * CS_WAVES, lane, wave, cin_u, cmax);
    cs_wave_prefix<0>(sm.red + 3 * CS_WAVES, lane, wave, rid, nrun);
    int cin = (int)cin_u;
    uint16_t* END = sm.idx;             // END[s] = end of the run starting at s
    uint16_t* RID = (uint16_t*)sm.key;  // RID[s] = index of the tie run starting at s
    uint32_t* rlc = out.rlist + (int64_t)col * (ld / 2);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (e < Ee) {
            const uint32_t f = key[e] >> 30;
            const int sp = max((int)(key[e] & 0x3FFFFFFFu), cin);
            key[e] = (uint32_t)sp;
            const int k = wbase + 64 * e + lane;
            if (f & 2u) END[sp] = (uint16_t)(k + 1);
            const uint64_t m = __ballot(f == 1u);
            if (f == 1u) RID[k] = (uint16_t)(rid + lanes_below(m));
            rid += (uint32_t)__popcll(m);
        }
    }
    __syncthreads();
    uint32_t ntied = 0;
    const int64_t nwords = ld / 64;
    uint64_t* tbc = out.tbits + (int64_t)col * nwords;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (e < Ee) {
            const int k = wbase + 64 * e + lane;
            bool tied = false;
            if (k < nc) {
                const uint32_t s0 = key[e], e0 = END[s0];
                tied = e0 - s0 > 1u;
                ordc[k] = (uint16_t)pk[e];
                ord2c[k] = (uint16_t)(2u * (pk[e] & 0xFFFFu));
                // a tied sample's position entry holds the flag bit and its
                // run index instead of the sorted position
                const uint32_t r0 = tied ? (uint32_t)RID[s0] : 0u;
                posc[pk[e]] = (uint16_t)(tied ? (0x8000u | r0) : (uint32_t)k);
                runc[k] = s0 | (e0 << 16);
                if (tied && (uint32_t)k == s0) rlc[r0] = s0 | (e0 << 16);
            }
            const uint64_t m = __ballot(tied);
            // (the slots may run past the row's words; tied positions never do)
            if (lane == 0 && (wbase >> 6) + e < nwords) tbc[(wbase >> 6) + e] = m;
            ntied += (uint32_t)__popcll(m);
        }
    }
    // padding: sorted positions past the observed count hold the dummy
    // sample S, whose position is "missing"; tie-bit words past the slots
    // are zero
    for (int64_t k = nc + t; k < ld; k += CS_THREADS) {
        ordc[k] = (uint16_t)S;
        ord2c[k] = (uint16_t)(2 * S);
    }
    for (int64_t i = S + t; i < ld; i += CS_THREADS) posc[i] = 0xFFFF;
    for (int64_t w = (int64_t)(slots >> 6) + t; w < nwords; w += CS_THREADS) tbc[w] = 0ull;
    if (col == (int)gridDim.x - 1)
        for (int64_t k = t; k < ORD_TAIL; k += CS_THREADS) {
            ordc[ld + k] = (uint16_t)S;
            ord2c[ld + k] = (uint16_t)(2 * S);
        }
    if (lane == 0) sm.red[wave] = ntied;
    __syncthreads();
    if (t == 0) {
        uint32_t tc = 0;
        for (int v = 0; v < CS_WAVES; ++v) tc += sm.red[v];
        out.ncol[col] = nc;
        out.hasties[col] = tc > 0 ? 1 : 0;
        out.nruns[col] = (int32_t)nrun;
        out.tcount[col] = (int32_t)tc;
    }
}

// ---------------------------------------------------------------------------
// per-column sort of long columns (more than SPEARMAN_MAX_S samples)
// ---------------------------------------------------------------------------
// The same LSD radix sort (4 stable passes of 8-bit digits, keys ranked
// within each wave by ballot digit matching) over global memory, one
// workgroup per column, in tiles of BS_TILE sorted slots taken in order:
// a key's destination is its digit's base in the whole column (from the
// column's histograms of all four digits, taken while the observed keys are
// compacted), plus the keys of that digit in earlier tiles, plus those in
// earlier waves of its tile, plus its rank in its wave.  Keys and sample
// indices alternate between two buffers (u32 each: the keys buffer's four
// planes A, B, I, J).  The tail takes two sweeps: the first finds each
// position's run start (a max-scan carried across steps, waves and tiles),
// records each run's end at its start and numbers the tie runs in position
// order; the second writes ord, pos (positions only: no tie flag, which the
// 16-bit positions of these lengths need all their bits for), runs, the
// tie-run list and the tie bits.  Between phases each thread's global
// writes are made visible to the workgroup's later reads (device fence).
constexpr int BS_ET = 8;                     // sorted slots per thread and tile
constexpr int BS_TILE = CS_THREADS * BS_ET;  // 8192

__global__ __launch_bounds__(CS_THREADS) void k_colsort_big(uint32_t* __restrict__ keys, int64_t S, int64_t ld,
                                                            int64_t F, SpearBase out)
{
    __shared__ uint16_t wcnt[CS_WAVES][256];
    __shared__ uint32_t hist[4][256];  // digit counts, then each pass's digit bases
    __shared__ uint32_t run[256];
    __shared__ uint32_t red[4][CS_WAVES];
    const int col = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int64_t plane = F * ld;
    uint32_t* kA = keys + (int64_t)col * ld;  // raw keys, then the compacted keys
    uint32_t* kB = kA + plane;
    uint32_t* iA = kA + 2 * plane;
    uint32_t* iB = kA + 3 * plane;
    uint16_t* ordc = out.ord + (int64_t)col * ld;
    uint16_t* posc = out.pos + (int64_t)col * ld;
    uint32_t* runc = out.runs + (int64_t)col * ld;
    uint32_t* rlc = out.rlist + (int64_t)col * (ld / 2);
    const int64_t nwords = ld / 64;
    uint64_t* tbc = out.tbits + (int64_t)col * nwords;

    for (int i = t; i < 4 * 256; i += CS_THREADS) (&hist[0][0])[i] = 0u;
    __syncthreads();
    // ---- compaction (in place: a tile's keys are read before any of its
    // compacted keys are written, and those land below the tile's end) ----
    uint32_t n = 0u, kor = 0u, kand = 0xFFFFFFFFu;
    for (int64_t t0 = 0; t0 < S; t0 += BS_TILE) {
        uint32_t key[BS_ET];
        uint32_t nobs = 0u;
#pragma unroll
        for (int e = 0; e < BS_ET; ++e) {
            const int64_t j = t0 + (int64_t)e * CS_THREADS + t;
            key[e] = j < S ? kA[j] : 0xFFFFFFFFu;
            const bool obs = key[e] != 0xFFFFFFFFu;
            if (!obs && j < S) posc[j] = 0xFFFF;  // missing sample
            if (obs) {
                ++nobs;
                kor |= key[e];
                kand &= key[e];
#pragma unroll
                for (int p = 0; p < 4; ++p) atomicAdd(&hist[p][(key[e] >> (8 * p)) & 255u], 1u);
            }
        }
        const uint32_t incl = wave_incl_scan_u32(nobs);
        if (lane == 63) red[0][wave] = incl;
        __syncthreads();
        uint32_t base = n + incl - nobs, tot = 0u;
#pragma unroll
        for (int v = 0; v < CS_WAVES; ++v) {
            const uint32_t tv = red[0][v];
            base += v < wave ? tv : 0u;
            tot += tv;
        }
#pragma unroll
        for (int e = 0; e < BS_ET; ++e) {
            if (key[e] != 0xFFFFFFFFu) {
                kA[base] = key[e];
                iA[base] = (uint32_t)(t0 + (int64_t)e * CS_THREADS + t);
                ++base;
            }
        }
        n += tot;
        __syncthreads();  // red reused
    }
    // bits in which some observed key differs (all observed keys agree on the
    // others): a pass over a constant digit is skipped
#pragma unroll
    for (int dd = 32; dd >= 1; dd >>= 1) {
        kor |= (uint32_t)__shfl_xor((int)kor, dd, 64);
        kand &= (uint32_t)__shfl_xor((int)kand, dd, 64);
    }
    if (lane == 0) {
        red[1][wave] = kor;
        red[2][wave] = kand;
    }
    // digit bases: exclusive scans of the four histograms (four waves)
    __syncthreads();
    if (wave < 4) {
        uint32_t c4[4], sum = 0u;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            c4[i] = hist[wave][4 * lane + i];
            sum += c4[i];
        }
        uint32_t acc = wave_incl_scan_u32(sum) - sum;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            hist[wave][4 * lane + i] = acc;
            acc += c4[i];
        }
    }
    uint32_t vor = 0u, vand = 0xFFFFFFFFu;
#pragma unroll
    for (int v = 0; v < CS_WAVES; ++v) {
        vor |= red[1][v];
        vand &= red[2][v];
    }
    const uint32_t diff = n > 0u ? (vor ^ vand) : 0u;
    __threadfence();
    __syncthreads();

    // ---- 4 passes ------------------------------------------------------------
    uint16_t* wc = &wcnt[wave][0];
    int cur = 0;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 8 * pass;
        if (((diff >> shift) & 255u) == 0u) continue;  // uniform
        const uint32_t* sk = cur ? kB : kA;
        const uint32_t* si = cur ? iB : iA;
        uint32_t* dk = cur ? kA : kB;
        uint32_t* di = cur ? iA : iB;
        if (t < 256) run[t] = 0u;
        for (int64_t t0 = 0; t0 < (int64_t)n; t0 += BS_TILE) {
#pragma unroll
            for (int q = 0; q < 4; ++q) wc[q * 64 + lane] = 0;
            uint32_t key[BS_ET], ix[BS_ET], rk[BS_ET];
#pragma unroll
            for (int e = 0; e < BS_ET; ++e) {
                const int64_t k = t0 + (int64_t)wave * 64 * BS_ET + 64 * e + lane;
                const bool valid = k < (int64_t)n;
                key[e] = valid ? sk[k] : 0u;
                ix[e] = valid ? si[k] : 0u;
                const uint64_t vm = __ballot(valid);
                if (vm == 0ull) continue;  // uniform
                const uint32_t d = (key[e] >> shift) & 255u;
                const uint64_t peers = match_digit8(d) & vm;
                const uint32_t below = lanes_below(peers);
                const uint32_t cnt = (uint32_t)__popcll(peers);
                if (valid) {
                    const uint32_t b = wc[d];
                    if (below + 1u == cnt) wc[d] = (uint16_t)(b + cnt);  // last of the peers
                    rk[e] = b + below;
                }
            }
            __syncthreads();
            // destinations per (digit, wave): the digit's base, its keys in
            // earlier tiles and in earlier waves of this tile
            if (t < 256) {
                uint32_t acc = hist[pass][t] + run[t];
#pragma unroll
                for (int v = 0; v < CS_WAVES; ++v) {
                    const uint32_t c = wcnt[v][t];
                    wcnt[v][t] = (uint16_t)acc;
                    acc += c;
                }
                run[t] = acc - hist[pass][t];
            }
            __syncthreads();
#pragma unroll
            for (int e = 0; e < BS_ET; ++e) {
                const int64_t k = t0 + (int64_t)wave * 64 * BS_ET + 64 * e + lane;
                if (k < (int64_t)n) {
                    const uint32_t dst = (uint32_t)wc[(key[e] >> shift) & 255u] + rk[e];
                    dk[dst] = key[e];
                    di[dst] = ix[e];
                }
            }
            __syncthreads();  // wcnt read by the destinations above
        }
        __threadfence();
        __syncthreads();
        cur ^= 1;
    }
    const uint32_t* sk = cur ? kB : kA;  // sorted keys
    const uint32_t* si = cur ? iB : iA;  // their sample indices
    uint32_t* END = cur ? kA : kB;       // END[s]: end of the run starting at s
    uint32_t* RID = cur ? iA : iB;       // RID[s]: index of the tie run starting at s

    // ---- tail, sweep 1: run starts (into runc for now), ends, tie-run numbers
    int tcarry = 0;       // latest run start so far (uniform)
    uint32_t trid = 0u;   // tie runs so far (uniform)
    for (int64_t t0 = 0; t0 < (int64_t)n; t0 += BS_TILE) {
        int sp[BS_ET];
        uint32_t fl[BS_ET];
        int carry = 0;
        uint32_t ntr = 0u;
#pragma unroll
        for (int e = 0; e < BS_ET; ++e) {
            const int64_t k = t0 + (int64_t)wave * 64 * BS_ET + 64 * e + lane;
            uint32_t f = 0u;
            if (k < (int64_t)n) {
                const uint32_t key = sk[k];
                const bool st = k == 0 || sk[k - 1] != key;
                const bool ls = k + 1 == (int64_t)n || sk[k + 1] != key;
                f = (st ? 1u : 0u) | (ls ? 2u : 0u);
            }
            fl[e] = f;
            ntr += (uint32_t)__popcll(__ballot(f == 1u));
            const int x = max(wave_incl_max_scan((f & 1u) ? (int)k : 0), carry);
            carry = __builtin_amdgcn_readlane(x, 63);
            sp[e] = x;
        }
        if (lane == 0) {
            red[0][wave] = (uint32_t)carry;
            red[1][wave] = ntr;
        }
        __syncthreads();
        int cin = tcarry;
        uint32_t rid = trid, tmax = (uint32_t)tcarry, ttot = 0u;
#pragma unroll
        for (int v = 0; v < CS_WAVES; ++v) {
            const uint32_t c = red[0][v], r = red[1][v];
            if (v < wave) {
                cin = max(cin, (int)c);
                rid += r;
            }
            tmax = max(tmax, c);
            ttot += r;
        }
#pragma unroll
        for (int e = 0; e < BS_ET; ++e) {
            const int64_t k = t0 + (int64_t)wave * 64 * BS_ET + 64 * e + lane;
            const int s0 = max(sp[e], cin);
            if (k < (int64_t)n) {
                runc[k] = (uint32_t)s0;
                if (fl[e] & 2u) END[s0] = (uint32_t)(k + 1);
            }
            const uint64_t m = __ballot(fl[e] == 1u);
            if (fl[e] == 1u) RID[k] = rid + lanes_below(m);
            rid += (uint32_t)__popcll(m);
        }
        tcarry = (int)tmax;
        trid += ttot;
        __syncthreads();  // red reused
    }
    __threadfence();
    __syncthreads();
    // ---- tail, sweep 2 --------------------------------------------------------
    uint32_t ntied = 0u;
    for (int64_t t0 = 0; t0 < (int64_t)n; t0 += BS_TILE) {
#pragma unroll
        for (int e = 0; e < BS_ET; ++e) {
            const int64_t k = t0 + (int64_t)wave * 64 * BS_ET + 64 * e + lane;
            bool tied = false;
            if (k < (int64_t)n) {
                const uint32_t s0 = runc[k], e0 = END[s0];
                tied = e0 - s0 > 1u;
                const uint32_t ix = si[k];
                ordc[k] = (uint16_t)ix;
                posc[ix] = (uint16_t)k;
                runc[k] = s0 | (e0 << 16);
                if (tied && (uint32_t)k == s0) rlc[RID[s0]] = s0 | (e0 << 16);
            }
            const uint64_t m = __ballot(tied);
            const int64_t w0 = (t0 + (int64_t)wave * 64 * BS_ET + 64 * e) >> 6;
            if (lane == 0 && w0 < nwords && w0 * 64 < (int64_t)n) tbc[w0] = m;
            ntied += (uint32_t)__popcll(m);
        }
    }
    for (int64_t k = (int64_t)n + t; k < ld; k += CS_THREADS) ordc[k] = (uint16_t)S;
    for (int64_t i = S + t; i < ld; i += CS_THREADS) posc[i] = 0xFFFF;
    for (int64_t w = ((int64_t)n + 63) / 64 + t; w < nwords; w += CS_THREADS) tbc[w] = 0ull;
    if (col == (int)gridDim.x - 1)
        for (int64_t k = t; k < ORD_TAIL; k += CS_THREADS) ordc[ld + k] = (uint16_t)S;
    if (lane == 0) red[2][wave] = ntied;
    __syncthreads();
    if (t == 0) {
        uint32_t tc = 0u;
        for (int v = 0; v < CS_WAVES; ++v) tc += red[2][v];
        out.ncol[col] = (int32_t)n;
        out.hasties[col] = tc > 0u ? 1 : 0;
        out.nruns[col] = (int32_t)trid;
        out.tcount[col] = (int32_t)tc;
    }
}

// ---------------------------------------------------------------------------
// per-pair re-ranking scan
// ---------------------------------------------------------------------------
struct PairOut {
    double4* sums;  // [npairs] (n, A, B_a, B_b)
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

// Tie bits: bit k of tbits[c][k / 64] is set when sorted position k of column
// c belongs to a run of two or more equal values.
__global__ __launch_bounds__(256) void k_tiebits(SpearBase bs)
{
    const int64_t c = blockIdx.y;
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int nc = bs.ncol[c];
    bool tie = false;
    if (k < nc) {
        const uint32_t rr = bs.runs[c * bs.ld + k];
        tie = (rr >> 16) - (rr & 0xFFFFu) > 1u;
    }
    const uint64_t m = __ballot(tie);
    if ((threadIdx.x & 63) == 0 && k < bs.ld) {
        bs.tbits[c * (bs.ld / 64) + (k >> 6)] = m;
        if (m) atomicAdd(&bs.tcount[c], (int32_t)__popcll(m));
    }
}

__global__ void k_fill_zero_i32(int32_t* __restrict__ a, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) a[i] = 0;
}

// Wave total of a 64-bit value: an inclusive scan by DPP row shifts and
// broadcasts, read at lane 63 (no LDS traffic, unlike lane shuffles).  Each
// step is one add of the low halves with carry-out and one add of the high
// halves with that carry, both taking their first operand from the lane the
// DPP control selects.  With the bound control off, a lane with no such
// source (first lanes of a row, rows masked off) does not execute the adds
// and keeps its value, which is what a scan step adds to it (nothing).  The
// compiler does not fuse the row moves into 64-bit adds, so the two adds are
// written out; the leading s_nop covers the two wait states a DPP read needs
// after a VALU write of its source (the other step's or the caller's).
#define NAPY_DPP_ADD64_STEP(CTRL)                                          \
    asm volatile("s_nop 1\n\t"                                            \
                 "v_add_co_u32_dpp %0, vcc, %0, %0 " CTRL "\n\t"         \
                 "v_addc_co_u32_dpp %1, vcc, %1, %1, vcc " CTRL            \
                 : "+v"(lo), "+v"(hi)                                      \
                 :                                                          \
                 : "vcc")

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    NAPY_DPP_ADD64_STEP("row_shr:1 row_mask:0xf bank_mask:0xf");
    NAPY_DPP_ADD64_STEP("row_shr:2 row_mask:0xf bank_mask:0xf");
    NAPY_DPP_ADD64_STEP("row_shr:4 row_mask:0xf bank_mask:0xf");
    NAPY_DPP_ADD64_STEP("row_shr:8 row_mask:0xf bank_mask:0xf");
    NAPY_DPP_ADD64_STEP("row_bcast:15 row_mask:0xa bank_mask:0xf");
    NAPY_DPP_ADD64_STEP("row_bcast:31 row_mask:0xc bank_mask:0xf");
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)hi, 63) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)lo, 63);
}
#undef NAPY_DPP_ADD64_STEP

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan_u32(v), 63);
}

// Tie class of each column, from its run list: 0 no ties; 1 few short runs
// (one lane per run can settle them after a walk that treats them as
// untied: ceil(runs / 64) * longest run, times 8, at most the column's
// 64-position chunks); 2 otherwise.  A densely tied column (more than 1/8 of
// its observed positions in runs) whose runs and untied positions number at
// most RUN_GROUPS_MAX also gets the list of its untied positions (nsing; -1
// for every other column).
__global__ __launch_bounds__(256) void k_tcls(SpearBase bs, int64_t F)
{
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= F) return;
    const int nr = bs.nruns[c];
    const int nc = bs.ncol[c];
    const uint32_t* rl = bs.rlist + c * (bs.ld / 2);
    uint32_t mx = 0;
    for (int r = lane; r < nr; r += 64) {
        const uint32_t rr = rl[r];
        mx = max(mx, (rr >> 16) - (rr & 0xFFFFu));
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, d, 64));
    const int nsg = nc - bs.tcount[c];
    const bool grouped = nr > 0 && bs.tcount[c] * 8 > nc && nr + nsg <= RUN_GROUPS_MAX;
    if (grouped) {
        // untied positions below nc: clear tie bits, one 64-bit word per lane
        const uint64_t* tb = bs.tbits + c * (bs.ld / 64);
        uint16_t* sg = bs.sing + c * RUN_GROUPS_MAX;
        uint32_t base = 0;
        for (int w0 = 0; w0 * 64 < nc; w0 += 64) {
            const int w = w0 + lane;
            uint64_t word = 0;
            if (w * 64 < nc) {
                word = ~tb[w];
                const int valid = nc - w * 64;
                if (valid < 64) word &= (1ull << valid) - 1ull;
            }
            const uint32_t cnt = (uint32_t)__popcll(word);
            const uint32_t incl = wave_incl_scan_u32(cnt);
            uint32_t at = base + incl - cnt;
            while (word) {
                const int bit = __builtin_ctzll(word);
                sg[at++] = (uint16_t)(w * 64 + bit);
                word &= word - 1ull;
            }
            base += (uint32_t)__shfl((int)incl, 63, 64);
        }
    }
    if (lane == 0) {
        const int64_t nch = (nc + 63) / 64;
        const int64_t serial = ceil_div(nr, 64) * (int64_t)mx;
        bs.tcls[c] = nr == 0 ? 0 : (serial * 8 <= nch ? 1 : 2);
        bs.nsing[c] = grouped ? nsg : -1;
    }
}

// Processing order of the columns: first the columns whose ties are dense
// (more than 1/8 of the observed positions in tie runs) or otherwise not few
// and short, then the others; each group by decreasing observed count in
// steps of 256, and within a step the untied columns before those with a few
// short runs.  Pairs are walked along the later column of this order: the
// walked side is the shorter one (to within a step), a column with dense or
// long runs is (nearly always) the fixed side, whose tie runs are looked up
// per sample, and a column with a few short runs is preferably the walked
// side, whose runs are settled after the walk.
__device__ __forceinline__ uint32_t perm_key(const SpearBase& bs, int64_t c)
{
    const int32_t n = bs.ncol[c];
    const int cls = bs.tcls[c];
    const bool fixed_side = bs.tcount[c] * 8 > n || cls == 2;
    return ((fixed_side ? 0u : 1u) << 20) | (((uint32_t)(65535 - n) >> 8) << 1) | (cls == 1 ? 1u : 0u);
}

// rank of each column's key (ties by column index), one wave per column
// comparing against all keys, then the column goes to that place of perm
__global__ __launch_bounds__(256) void k_perm(SpearBase bs, int64_t F)
{
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= F) return;
    const uint32_t kc = perm_key(bs, c);
    uint32_t rank = 0;
    for (int64_t d = lane; d < F; d += 64) {
        const uint32_t kd = perm_key(bs, d);
        rank += (kd < kc) || (kd == kc && d < c);
    }
    rank = wave_sum_u32(rank);
    if (lane == 0) bs.perm[rank] = (int32_t)c;
}

// Tie classes and processing order; with_bits: first the tie bits and counts
// from the run arrays (the column sort writes them itself)
static int tiebits_launch(const SpearBase& bs, int64_t F, hipStream_t st, bool with_bits = true)
{
    if (with_bits) {
        hipLaunchKernelGGL(k_fill_zero_i32, dim3((unsigned)ceil_div(F, 256)), dim3(256), 0, st, bs.tcount, F);
        NAPY_TRY(check_launch("fill"));
        hipLaunchKernelGGL(k_tiebits, dim3((unsigned)ceil_div(bs.ld, 256), (unsigned)F), dim3(256), 0, st, bs);
        NAPY_TRY(check_launch("tiebits"));
    }
    hipLaunchKernelGGL(k_tcls, dim3((unsigned)ceil_div(F, 4)), dim3(256), 0, st, bs, F);
    NAPY_TRY(check_launch("tie classes"));
    hipLaunchKernelGGL(k_perm, dim3((unsigned)ceil_div(F, 4)), dim3(256), 0, st, bs, F);
    return check_launch("perm");
}

// Presence bytes in processing order, one plane per block of 8 columns:
// bit j of presb[q][i] = sample i present in column perm[8 q + j].  A pair
// workgroup copies its partner block's plane (S bytes) into LDS.  Each
// thread makes four consecutive bytes (ld is a multiple of 256), from eight
// 8-byte loads issued together.
__global__ __launch_bounds__(256) void k_presence(SpearBase bs, int64_t S, int64_t F, uint8_t* __restrict__ presb)
{
    const int64_t i0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    const int64_t q = blockIdx.y;
    if (i0 >= bs.ld) return;
    const int64_t c0 = q * 8;
    uint2 v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        // a column past F reads column perm[c0] and is masked below
        const int64_t col = bs.perm[c0 + j < F ? c0 + j : c0];
        v[j] = *(const uint2*)(bs.pos + col * bs.ld + i0);
    }
    uint32_t word = 0u;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (c0 + j >= F) continue;
        const uint32_t h[4] = {v[j].x & 0xFFFFu, v[j].x >> 16, v[j].y & 0xFFFFu, v[j].y >> 16};
#pragma unroll
        for (int u = 0; u < 4; ++u) word |= (uint32_t)(h[u] != 0xFFFFu) << (8 * u + j);
    }
    // samples from S on are absent (their positions hold 0xFFFF, but the
    // bytes are cleared explicitly)
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (i0 + u >= S) word &= ~(0xFFu << (8 * u));
    *(uint32_t*)(presb + q * bs.ld + i0) = word;
}

constexpr int PAIR_THREADS = 512;
constexpr int PAIR_WAVES = PAIR_THREADS / 64;

// bits of `mask` at lanes below x (x in 0..64)
__device__ __forceinline__ uint64_t bits_below(uint64_t mask, uint32_t x)
{
    return x >= 64u ? mask : (mask & ((1ull << x) - 1ull));
}

constexpr uint32_t POS_TIED = 0x8000u;  // position flag: the sample's value is tied
constexpr uint32_t POS_MASK = 0x7FFFu;

// Partner table of one partner along column a's sorted order, one entry per
// 32 positions: x = presence bits of the partner at positions 32w..32w+31,
// y = 1 + number of partner-present positions before 32w.  Entry NW (just
// past the words covering positions 0..n_a) is {0, 0}: looking up any
// position >= 32 NW gives 0.
__device__ __forceinline__ uint32_t cnt1(const uint2* tab, uint32_t x)
{
    // the word index is kept opaque so that its address is one shift-add
    // (the compiler would otherwise rewrite (x >> 5) << 3 as shift + mask)
    uint32_t w = x >> 5;
    asm("" : "+v"(w));
    const uint2 e = tab[w];
    // the field width of the bit-field extract is taken modulo 32 by the
    // hardware: the low x mod 32 bits
    return e.y + (uint32_t)__popc(__builtin_amdgcn_ubfe(e.x, 0u, x));
}

// doubled average rank of a sample in a's tie run [s, e): C(s) + C(e) + 1
__device__ __forceinline__ uint32_t ra_run(const uint2* tab, uint32_t rr)
{
    return cnt1(tab, rr & 0xFFFFu) + cnt1(tab, rr >> 16) - 1u;
}

// t^3 - t: a tie run of t complete samples lowers the sum of squared doubled
// ranks by (t^3 - t) / 3 relative to untied ranks 2, 4, ..., 2n; the sums of
// t^3 - t are divided by 3 once (each term is a multiple of 3)
__device__ __forceinline__ uint64_t cube_minus(uint32_t t)
{
    return (uint64_t)(t * t) * t - t;
}

struct WalkSums {
    uint32_t n;
    uint64_t A4;   // per lane: sum of C1_a * C1_b over untied complete samples
    uint64_t At;   // per lane: sum of R_a * C1_b over complete samples tied in a
    uint64_t Af;   // per lane: sum of R_a * R_b over complete samples in b's tie runs
    uint64_t d3B;  // per lane: sum of t^3 - t over b's tie runs
    uint64_t Au;   // wave-uniform: deferred tie runs of b
};

constexpr int WALK_U = 4;  // chunks of 64 positions per group; rows are padded to 64 * WALK_U
static_assert(WALK_U == 4, "the grouped walk of a with ties ORs four chunk masks");

// a's tied samples: their stored position is the flag bit plus the index of
// their tie run in a's run list.  With at most RUN_TABLE_MAX runs each run's
// doubled average rank for the partner sits in LDS; with more, it comes from
// the run's bounds (run list, global) and two table lookups.  A grouped a
// (its runs and untied positions at most RUN_GROUPS_MAX) has its untied
// samples flagged as one-sample runs numbered after the runs, so every
// sample's rank comes from the table; entry RUN_TABLE_MAX of a partner's
// table is 0 (missing samples).
constexpr int RUN_TABLE_MAX = RUN_GROUPS_MAX;
constexpr int RUN_TABLE_STRIDE = RUN_TABLE_MAX + 1;

// rank of a tied a-sample: from the run-rank table when a has at most
// RUN_TABLE_MAX runs (rrun != nullptr), else from the run list
__device__ __forceinline__ uint32_t ra_of_tied(const uint2* tab, const uint32_t* __restrict__ rlA,
                                               const uint32_t* rrun, uint32_t pv)
{
    if (rrun) return rrun[pv & POS_MASK];
    return ra_run(tab, rlA[pv & POS_MASK]);
}

// a's samples in LDS, and the code `miss` of a missing one: a grouped a
// stores for every sample its index in the run-rank table (no flag bit),
// miss = RUN_TABLE_MAX (the table's zero entry); an untied a stores
// positions, miss = XS = 32 NW (the partner table's zero entry); a tied a
// stores positions, a tied one with the flag bit, miss = 0xFFFF (clamped to
// XS for a table lookup).
constexpr uint32_t MISS_GROUPED = (uint32_t)RUN_TABLE_MAX;

// Doubled rank R_a of a complete sample from a's stored code pv (not the
// missing code).  TA 0: a untied, pv the position; 1: a tied, a tied
// sample's pv is POS_TIED plus its run's number; 2: pv an index into the
// run-rank table; 3 and 4 (columns longer than the LDS sort handles): pv the
// position, a untied (3) or tied (4), a tied sample found by its run in a's
// runs array by position (rlA then points at that array).
template <int TA>
__device__ __forceinline__ uint32_t a_rank(uint32_t pv, const uint2* tab, const uint32_t* __restrict__ rlA,
                                           const uint32_t* rrun)
{
    if constexpr (TA == 2) return rrun[pv];
    if constexpr (TA == 1) {
        if (pv & POS_TIED) return ra_of_tied(tab, rlA, rrun, pv);
    }
    if constexpr (TA == 4) {
        const uint32_t rr = rlA[pv];
        if ((rr >> 16) - (rr & 0xFFFFu) > 1u) return ra_run(tab, rr);
    }
    return 2u * cnt1(tab, pv);
}

// One chunk of 64 positions of b's sorted order without tied b-positions.
// b's C1 = carry1 + (complete samples at lower lanes) by mbcnt; a sample is
// complete when its a-position is not `miss`.  TA = 0 (a untied) or 1 (a
// with ties): a's C1 from the partner table, 0 for missing or tied
// a-positions (TA = 1 clamps both to XS), whose products are added
// separately; C1_a C1_b goes to t32.  TA = 2 (a grouped): every sample's R_a
// from the run-rank table, no partner-table lookup and no branch; R_a C1_b
// (below 2^31) goes to t32, which the caller empties every two chunks.
// A wave-uniform pointer computed where it stands: the lane read is
// convergent, so the compiler does not sink the address arithmetic into the
// divergent blocks that use it (which would keep the base's pointers live
// through the walk loops, spilled and reloaded there)
// (the lane-read builtin takes and returns 32 bits: the two halves of the
// address are read separately; the result is rebuilt as a global-memory
// pointer, so that its loads stay global loads, not flat ones)
template <class T>
__device__ __forceinline__ T* pin_uniform(T* p)
{
    typedef __attribute__((address_space(1))) T GT;
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (T*)(GT*)(((uint64_t)hi << 32) | (uint64_t)lo);
}

// The walks of columns sorted in LDS (TA <= 2) read b's order doubled
// (2 x sample index): a's positions sit at the start of the kernel's LDS,
// which is its dynamic block alone (the launcher checks that the kernel has
// no static LDS), so the code is the LDS byte address of the sample's
// a-position and feeds the load with no address arithmetic.  Long columns
// (TA >= 3) read plain sample indices into a's positions in global memory.
template <int TA>
__device__ __forceinline__ uint32_t pos_at(const uint16_t* posA, uint32_t code)
{
    if constexpr (TA <= 2) return *(const __attribute__((address_space(3))) uint16_t*)(uintptr_t)code;
    else return posA[code];
}
template <int TA>
__device__ __forceinline__ uint32_t sample_at(uint32_t code) { return TA <= 2 ? code >> 1 : code; }

template <int TA, bool DBG>
__device__ __forceinline__ void walk_chunk_untied(uint32_t iv, uint32_t pv, const uint2* tab, uint32_t XS,
                                                  uint32_t miss, const uint32_t* __restrict__ rlA,
                                                  const uint32_t* rrun, uint32_t& carry1, uint32_t& t32,
                                                  uint64_t& sAt, int32_t* dbg_ra, int32_t* dbg_rb)
{
    const bool kept = pv != miss;
    const uint64_t mask = __ballot(kept);
    const uint32_t cb1 = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, carry1));
    if constexpr (TA == 2) {
        t32 += __umul24(rrun[pv], cb1);
    } else if constexpr (TA >= 3) {
        // long columns: positions up to 65534 (C1 and R up to 2^17), so the
        // products go straight into 64 bits, the untied ones doubled (R_a R_b
        // = 4 C1_a C1_b, and sAt carries weight 2)
        bool tied = false;
        uint32_t rr = 0u;
        if constexpr (TA == 4) {
            if (kept) {
                rr = rlA[pv];
                tied = (rr >> 16) - (rr & 0xFFFFu) > 1u;
            }
        }
        const uint32_t ca1 = (kept && !tied) ? cnt1(tab, pv) : 0u;
        sAt += 2ull * ((uint64_t)ca1 * cb1);
        uint32_t ra = 0u;
        if (tied) {
            ra = ra_run(tab, rr);
            sAt += (uint64_t)ra * cb1;
        }
        if constexpr (DBG) {
            if (kept) {
                dbg_ra[iv] = (int32_t)(tied ? ra : 2u * ca1);
                dbg_rb[iv] = (int32_t)(2u * cb1);
            }
        }
    } else {
        const uint32_t ca1 = cnt1(tab, TA == 0 ? pv : min(pv, XS));
        t32 += __umul24(ca1, cb1);
        bool tied = false;
        if constexpr (TA == 1) {
            tied = kept && (pv & POS_TIED);
            // R_a * C1_b < 2^31: one 32-bit product per sample
            if (tied) sAt += __umul24(ra_of_tied(tab, rlA, rrun, pv), cb1);
        }
        if constexpr (DBG) {
            if (kept) {
                dbg_ra[iv] = (int32_t)(tied ? ra_of_tied(tab, rlA, rrun, pv) : 2u * ca1);
                dbg_rb[iv] = (int32_t)(2u * cb1);
            }
        }
    }
    carry1 += (uint32_t)__popcll(mask);
}

// Walk of partner b's sorted order for the pair (a, b).  The complete
// samples are those with an a-position.  With C1 = 1 + (complete samples at
// earlier positions), an untied complete sample has doubled ranks 2 C1 on
// each side; the products C1_a C1_b of four chunks are summed in 32 bits
// (each is below 2^30) before entering a 64-bit sum.  Tied a-positions (flag
// bit in the stored position) are added with their run's average rank.  A
// chunk holding tied b-positions (tbB bit word nonzero) resolves the runs
// inside it from its ballot mask; the one run that may continue into the
// next chunk is carried as wave-uniform state (its start count, plus per
// lane the a-ranks of its complete samples so far) and settled where it
// ends, and the lane at each run's last position records t^3 - t for it.
template <int TA, bool TB, bool DBG>
__device__ __forceinline__ void pair_walk(const uint16_t* __restrict__ ordB, const uint32_t* __restrict__ runsB,
                                          const uint64_t* __restrict__ tbB, const uint32_t* __restrict__ rlA,
                                          int nbv, const uint16_t* posA, const uint2* tab, const uint32_t* rrun,
                                          uint32_t XS, uint32_t miss, int lane, int32_t* dbg_ra, int32_t* dbg_rb,
                                          WalkSums& ws)
{
    constexpr int U = WALK_U;
    const int ncb = (nbv + 63) >> 6;
    const int ngrp = (ncb + U - 1) / U;
    uint32_t carry1 = 1;  // wave-uniform
    uint64_t sA4 = 0, sAt = 0, sAf = 0, d3B = 0, uA = 0;
    uint32_t open_cs = 0, pend_lane = 0;
    bool open = false;
    uint32_t ivn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) ivn[u] = ngrp > 0 ? ordB[u * 64 + lane] : 0u;
    // chunks holding tied b-positions, 64 chunks per window: bit c of dmask
    // for chunk 64 w + c of the current window w (wave-uniform), built by one
    // ballot over the window's tie-bit words, the next window's words loaded
    // one window ahead
    const int nwords = ngrp * U;  // tie-bit words of b's row that the walk covers
    uint64_t dmask = 0, tbnext = 0;
    if constexpr (TB) {
        const uint64_t w0 = lane < nwords ? tbB[lane] : 0ull;
        dmask = __ballot(w0 != 0ull);
        tbnext = 64 + lane < nwords ? tbB[64 + lane] : 0ull;
    }
    for (int g = 0; g < ngrp; ++g) {
        const int c0 = g * U;
        uint32_t iv[U] = {}, pv[U];  // iv: sample indices, kept for the debug output only
#pragma unroll
        for (int u = 0; u < U; ++u) pv[u] = pos_at<TA>(posA, ivn[u]);
        if constexpr (DBG) {
#pragma unroll
            for (int u = 0; u < U; ++u) iv[u] = sample_at<TA>(ivn[u]);
        }
        // prefetch the next group's sample indices into the same registers
        // (rows are padded, so a whole group is always inside the row); the
        // last group reloads its own, which keeps the loop body one block
        {
            // (a scalar base pinned per group and an unsigned lane offset: the
            // loads take the scalar-base form, with no 64-bit address add)
            const uint16_t* nx = pin_uniform(ordB + (size_t)((g + 1 < ngrp) ? c0 + U : c0) * 64);
#pragma unroll
            for (int u = 0; u < U; ++u) ivn[u] = nx[(uint32_t)lane + 64u * (uint32_t)u];
        }
        uint32_t dbits = 0;  // bit u: chunk c0 + u holds tied b-positions
        if constexpr (TB) {
            if ((c0 & 63) == 0 && c0 > 0) {
                dmask = __ballot(tbnext != 0ull);
                const int nw = c0 + 64 + lane;
                tbnext = nw < nwords ? tbB[nw] : 0ull;
            }
            dbits = (uint32_t)(dmask >> (c0 & 63)) & ((1u << U) - 1u);
        }
        const bool dirty = dbits != 0u;
        uint32_t t32 = 0;
        if constexpr (TA == 1 && !DBG) {
            if (!dirty) {
                // a with ties, most of them rare: the four chunks as untied
                // (a tied or missing a-position is clamped to XS, whose
                // table entry gives 0), one block of code; the tied lanes'
                // products after them, in a branch taken only by a group
                // that holds tied a-positions
                // (only the group's first carry and one OR of the tied-lane
                // ballots stay live; the rare branch rebuilds the chunks'
                // ballots from the positions)
                const uint32_t cg = carry1;
                uint64_t anyt = 0ull;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const bool kept = pv[u] != miss;
                    const uint64_t km = __ballot(kept);
                    anyt |= __ballot((pv[u] & POS_TIED) != 0u) & km;
                    const uint32_t cb1 = __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)km, carry1));
                    t32 += __umul24(cnt1(tab, min(pv[u], XS)), cb1);
                    carry1 += (uint32_t)__popcll(km);
                }
                sA4 += t32;
                if (anyt != 0ull) {
                    uint32_t c = cg;
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const bool kept = pv[u] != miss;
                        const uint64_t km = __ballot(kept);
                        if (kept && (pv[u] & POS_TIED)) {
                            const uint32_t cb1 = __builtin_amdgcn_mbcnt_hi(
                                (uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, c));
                            sAt += __umul24(ra_of_tied(tab, rlA, rrun, pv[u]), cb1);
                        }
                        c += (uint32_t)__popcll(km);
                    }
                }
                continue;
            }
        }
        if (!dirty) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                walk_chunk_untied<TA, DBG>(iv[u], pv[u], tab, XS, miss, rlA, rrun, carry1, t32, sAt, dbg_ra, dbg_rb);
                if constexpr (TA == 2) {
                    if (u & 1) {
                        sAt += t32;
                        t32 = 0;
                    }
                }
            }
            sA4 += t32;
            continue;
        }
        if constexpr (TB) {
            // a group with tied b-positions: one chunk at a time (the code of
            // this rarely taken path exists once), sample indices reloaded
#pragma unroll 1
            for (int u = 0; u < U; ++u) {
                const int c = c0 + u;
                const uint32_t k = (uint32_t)(c * 64 + lane);
                const uint32_t ivu = sample_at<TA>(ordB[k]);
                const uint32_t pvu = pos_at<TA>(posA, ordB[k]);
                if (((dbits >> u) & 1u) == 0u) {
                    // no tied b-position here, and no run crosses into this chunk
                    walk_chunk_untied<TA, DBG>(ivu, pvu, tab, XS, miss, rlA, rrun, carry1, t32, sAt, dbg_ra, dbg_rb);
                    if constexpr (TA == 2) {
                        sAt += t32;
                        t32 = 0;
                    }
                    continue;
                }
                const uint32_t rb = ((int)k < nbv) ? runsB[k] : (k | ((k + 1u) << 16));
                const bool kept = pvu != miss;
                const uint64_t mask = __ballot(kept);
                const uint32_t carry = carry1 - 1u;
                uint32_t Ra;
                if constexpr (TA == 2) {
                    Ra = rrun[pvu];
                } else if constexpr (TA >= 3) {
                    Ra = kept ? a_rank<TA>(pvu, tab, rlA, rrun) : 0u;
                } else {
                    Ra = 2u * cnt1(tab, min(pvu, XS));
                    if constexpr (TA == 1) {
                        if (kept && (pvu & POS_TIED)) Ra = ra_of_tied(tab, rlA, rrun, pvu);
                    }
                }
                const uint32_t lo = (uint32_t)c * 64u;
                const uint32_t rs = rb & 0xFFFFu, re = rb >> 16;
                const uint32_t cs = (rs >= lo) ? carry + (uint32_t)__popcll(bits_below(mask, rs - lo)) : open_cs;
                const bool ends = re <= lo + 64u;
                const uint32_t ce = carry + (uint32_t)__popcll(bits_below(mask, ends ? re - lo : 64u));
                const uint32_t Rb = cs + ce + 1u;
                if (ends && k + 1u == re && re - rs > 1u) d3B += cube_minus(ce - cs);
                // settle the run carried in from earlier chunks (lane 0
                // belongs to it) if it ends here
                if (open) {
                    const uint32_t e0 = __builtin_amdgcn_readlane(re, 0);
                    if (e0 <= lo + 64u) {
                        const uint32_t r_open = __builtin_amdgcn_readlane(Rb, 0);
                        uA += (uint64_t)r_open * (TA >= 3 ? wave_sum_u64((uint64_t)pend_lane) : (uint64_t)wave_sum_u32(pend_lane));
                        if constexpr (DBG) {
                            // report the settled rank of every complete sample of the run
                            const uint32_t s0 = __builtin_amdgcn_readlane(rs, 0);
                            for (uint32_t kk = s0 + (uint32_t)lane; kk < e0; kk += 64u) {
                                if (pos_at<TA>(posA, ordB[kk]) != miss) dbg_rb[sample_at<TA>(ordB[kk])] = (int32_t)r_open;
                            }
                        }
                        pend_lane = 0;
                        open = false;
                    }
                }
                const bool defer = kept && !ends;
                const bool direct = kept && ends;
                const uint64_t dm = __ballot(defer);
                if (dm) {
                    pend_lane += defer ? Ra : 0u;
                    open = true;
                    open_cs = __builtin_amdgcn_readlane(cs, 63);
                } else if (!open) {
                    // a run can also continue with no complete sample yet
                    const uint32_t e63 = __builtin_amdgcn_readlane(re, 63);
                    const bool v63 = (c * 64 + 63) < nbv;
                    if (v63 && e63 > lo + 64u) {
                        open = true;
                        open_cs = __builtin_amdgcn_readlane(cs, 63);
                    }
                }
                carry1 += (uint32_t)__popcll(mask);
                if (direct) sAf += (uint64_t)Ra * Rb;
                if constexpr (DBG) {
                    if (kept) {
                        dbg_ra[ivu] = (int32_t)Ra;
                        if (direct) dbg_rb[ivu] = (int32_t)Rb;
                    }
                }
            }
            sA4 += t32;
        }
    }
    ws.n = carry1 - 1u;
    ws.A4 = sA4;
    ws.At = sAt;
    ws.Af = sAf;
    ws.d3B = d3B;
    ws.Au = uA;
}

// Partner b with a few short tie runs, walked as untied: the t complete
// samples of a run [s, e) got the doubled ranks 2 (C(s) + j), j = 1..t, whose
// average is 2 C(s) + t + 1, so the sum of R_a R_b changes by
// sum_j R_a,j (t + 1 - 2 j).  One lane per run; adds that to corr and
// t^3 - t to d3B.
template <int TA>
__device__ __forceinline__ void settle_short_runs_b(const uint16_t* __restrict__ ordB, const uint32_t* __restrict__ rlB,
                                                    int nrb, const uint16_t* posA, const uint2* tab,
                                                    const uint32_t* __restrict__ rlA, const uint32_t* rrun,
                                                    uint32_t miss, int lane, int64_t& corr, uint64_t& d3B)
{
    for (int r = lane; r < nrb; r += 64) {
        const uint32_t rr = rlB[r];
        const uint32_t s = rr & 0xFFFFu, e = rr >> 16;
        uint32_t t = 0;
        uint64_t sra = 0, sraj = 0;
        for (uint32_t k = s; k < e; ++k) {
            const uint32_t pv = pos_at<TA>(posA, ordB[k]);
            if (pv == miss) continue;
            ++t;
            const uint32_t Ra = a_rank<TA>(pv, tab, rlA, rrun);
            sra += Ra;
            sraj += (uint64_t)Ra * t;
        }
        corr += (int64_t)((uint64_t)(t + 1u) * sra) - 2 * (int64_t)sraj;
        if (t > 1u) d3B += cube_minus(t);
    }
}

// Walk of a grouped partner b (its tie runs and untied positions, at most
// RUN_GROUPS_MAX groups, partition its observed positions): every complete
// sample of a group has the group's doubled average rank 2 C + t + 1 (C
// complete samples before the group, t in it), so the sum of R_a R_b is
// sum over groups of that rank times the group's sum of R_a.  One pass over
// b's order, four chunks in flight; each lane sums R_a of its samples in the
// open group, which is closed (one wave sum) at its end.  Returns the sum,
// n and the tie defect sum of t^3 - t.
template <int TA>
__device__ __forceinline__ void grouped_b_walk(const uint16_t* __restrict__ ordB, int nbv,
                                               const uint32_t* __restrict__ rlB, int nrb,
                                               const uint16_t* __restrict__ sgB, int nsgB, const uint16_t* posA,
                                               const uint2* tab, const uint32_t* __restrict__ rlA,
                                               const uint32_t* rrun, uint32_t XS, uint32_t miss, int lane,
                                               uint64_t& sum,
                                               uint32_t& n, uint64_t& d3B)
{
    constexpr int U = WALK_U;
    // group starts in position order: lane g holds the start of group g,
    // lane G (the group count) holds nbv, lanes above it all ones
    const uint32_t rsv = lane < nrb ? rlB[lane] & 0xFFFFu : 0xFFFFFFFFu;
    const uint32_t sgv = lane < nsgB ? (uint32_t)sgB[lane] : 0xFFFFFFFFu;
    const int G = nrb + nsgB;
    uint32_t bnd = lane == G ? (uint32_t)nbv : 0xFFFFFFFFu;
    {
        int ir = 0, is = 0;
        for (int g = 0; g < G; ++g) {
            const uint32_t r = ir < nrb ? (uint32_t)__builtin_amdgcn_readlane((int)rsv, ir) : 0xFFFFFFFFu;
            const uint32_t q = is < nsgB ? (uint32_t)__builtin_amdgcn_readlane((int)sgv, is) : 0xFFFFFFFFu;
            const uint32_t st = r < q ? r : q;
            if (r < q) ++ir;
            else ++is;
            if (lane == g) bnd = st;
        }
    }
    int gcur = 0;
    uint32_t gnext = (uint32_t)__builtin_amdgcn_readlane((int)bnd, 1);
    uint32_t carry = 0, t = 0, acc = 0;
    uint64_t tot = 0, d3 = 0;
    const int ngrp = (((nbv + 63) >> 6) + U - 1) / U;
    uint32_t ivn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) ivn[u] = ordB[u * 64 + lane];
    for (int gi = 0; gi < ngrp; ++gi) {
        uint32_t pv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) pv[u] = pos_at<TA>(posA, ivn[u]);
        // rows are padded to whole groups of U chunks; the read past the
        // last group stays inside the ord allocation
        {
            const uint16_t* nx = pin_uniform(ordB + (size_t)(gi + 1) * U * 64);
#pragma unroll
            for (int u = 0; u < U; ++u) ivn[u] = nx[(uint32_t)lane + 64u * (uint32_t)u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t c0 = (uint32_t)((gi * U + u) * 64);
            const uint32_t k = c0 + (uint32_t)lane;
            const uint32_t p = pv[u];
            const bool kept = p != miss;  // positions from nbv on hold the dummy sample
            uint32_t Ra;
            if constexpr (TA == 2) {
                Ra = rrun[p];  // 0 for a missing sample
            } else if constexpr (TA >= 3) {
                Ra = kept ? a_rank<TA>(p, tab, rlA, rrun) : 0u;
            } else {
                Ra = 2u * cnt1(tab, min(p, XS));
                if constexpr (TA == 1)
                    if (kept && (p & POS_TIED)) Ra = ra_of_tied(tab, rlA, rrun, p);
            }
            uint32_t val = kept ? Ra : 0u;  // R_a >= 1 for a complete sample
            while (gnext < c0 + 64u) {
                // the open group ends inside this chunk
                const bool in = k < gnext;
                const uint32_t v = in ? val : 0u;
                acc += v;
                t += (uint32_t)__popcll(__ballot(v != 0u));
                val = in ? 0u : val;
                // below t (2 S + 1): 32 bits for the LDS-sorted lengths
                const uint64_t sra = TA >= 3 ? wave_sum_u64((uint64_t)acc) : (uint64_t)wave_sum_u32(acc);
                tot += (uint64_t)(2u * carry + t + 1u) * sra;
                if (t > 1u) d3 += cube_minus(t);
                carry += t;
                acc = 0u;
                t = 0u;
                ++gcur;
                gnext = (uint32_t)__builtin_amdgcn_readlane((int)bnd, gcur + 1);
            }
            acc += val;
            t += (uint32_t)__popcll(__ballot(val != 0u));
        }
    }
    if (gcur < G) {
        // the last group ends with the walked chunks (nbv a multiple of 64 U)
        const uint64_t sra = TA >= 3 ? wave_sum_u64((uint64_t)acc) : (uint64_t)wave_sum_u32(acc);
        tot += (uint64_t)(2u * carry + t + 1u) * sra;
        if (t > 1u) d3 += cube_minus(t);
        carry += t;
    }
    sum = tot;
    n = carry;
    d3B = d3;
}

// LDS layout of the pair kernel for S samples and PB partners
// llvm.amdgcn.writelane: old with one lane replaced by a wave-uniform value
// (v_writelane_b32).  Declared through the intrinsic so that the compiler
// sees the instruction and inserts the wait states after the VALU write of
// the scalar register it reads.
// 8 x 8 bit transpose of a 64-bit block held as (lo, hi): bit 8 t + j (byte
// t, bit j) moves to bit 8 j + t, by three rounds of masked delta swaps
// (distances 7, 14 and 28 bits)
__device__ __forceinline__ void bit_transpose8(uint32_t& lo, uint32_t& hi)
{
    uint32_t t;
    t = ((lo >> 7) ^ lo) & 0x00AA00AAu;
    lo ^= t ^ (t << 7);
    t = ((hi >> 7) ^ hi) & 0x00AA00AAu;
    hi ^= t ^ (t << 7);
    t = ((lo >> 14) ^ lo) & 0x0000CCCCu;
    lo ^= t ^ (t << 14);
    t = ((hi >> 14) ^ hi) & 0x0000CCCCu;
    hi ^= t ^ (t << 14);
    t = ((hi << 4) ^ lo) & 0xF0F0F0F0u;
    lo ^= t;
    hi ^= t >> 4;
}

// b0 | b1 << 8 | b2 << 16 | b3 << 24 for bytes b0..b3 (values below 256):
// the pairs (b0, b2) and (b1, b3) as two 16-bit lanes each, then one
// shift-or (three instructions instead of a shift and an or per byte)
__device__ __forceinline__ uint32_t join_bytes(uint32_t b0, uint32_t b1, uint32_t b2, uint32_t b3)
{
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    u16x2 e, o;
    e.x = (unsigned short)b0;
    e.y = (unsigned short)b2;
    o.x = (unsigned short)b1;
    o.y = (unsigned short)b3;
    return __builtin_bit_cast(uint32_t, e) | (__builtin_bit_cast(uint32_t, o) << 8);
}

// Presence of the block's 8 partners at a's sorted positions k0 .. k0 + 31
// (k0 = 32 w), as one 32-bit word per partner: bit t of x[j] = partner j
// present at position k0 + t.  Each position's presence byte (bit j =
// partner j) is gathered from LDS; four 8 x 8 bit transposes give 8 bits per
// partner and 8 positions, and two 4 x 4 byte transposes (byte permutes)
// assemble each partner's word.  The debug form takes the single partner's
// presence (bit 0) from its positions in global memory.
template <bool DBG>
__device__ __forceinline__ void presence_words(const uint16_t* __restrict__ ordw, const uint8_t* presL,
                                               const uint16_t* __restrict__ posDbg, int k0, int na, uint32_t x[8])
{
    uint32_t blk[4][2];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint4 iv = ((const uint4*)ordw)[q];
        const uint32_t iw[4] = {iv.x, iv.y, iv.z, iv.w};
        uint32_t by[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const uint32_t idx = (iw[t >> 1] >> (16 * (t & 1))) & 0xFFFFu;
            if constexpr (DBG)
                by[t] = (k0 + 8 * q + t < na) ? (uint32_t)(posDbg[idx] != 0xFFFF) : 0u;
            else
                by[t] = presL[idx];
        }
        // bytes 0 and 2, then 1 and 3, as 16-bit halves; one shift-or joins them
        uint32_t lo = join_bytes(by[0], by[1], by[2], by[3]);
        uint32_t hi = join_bytes(by[4], by[5], by[6], by[7]);
        bit_transpose8(lo, hi);
        blk[q][0] = lo;
        blk[q][1] = hi;
    }
    // v_perm: selector byte values 0-3 pick bytes of the second operand, 4-7
    // of the first
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t u0 = __builtin_amdgcn_perm(blk[1][h], blk[0][h], 0x05010400u);
        const uint32_t u1 = __builtin_amdgcn_perm(blk[1][h], blk[0][h], 0x07030602u);
        const uint32_t v0 = __builtin_amdgcn_perm(blk[3][h], blk[2][h], 0x05010400u);
        const uint32_t v1 = __builtin_amdgcn_perm(blk[3][h], blk[2][h], 0x07030602u);
        x[4 * h + 0] = __builtin_amdgcn_perm(v0, u0, 0x05040100u);
        x[4 * h + 1] = __builtin_amdgcn_perm(v0, u0, 0x07060302u);
        x[4 * h + 2] = __builtin_amdgcn_perm(v1, u1, 0x05040100u);
        x[4 * h + 3] = __builtin_amdgcn_perm(v1, u1, 0x07060302u);
    }
}

// Block-wide copy of n16 16-byte words from global memory to LDS, every load
// of a thread issued before its stores.  Loads come from a clamped index
// (always inside the source) so the words stay in registers; only the stores
// are predicated.
__device__ __forceinline__ void copy16_to_lds(uint4* dst, const uint4* __restrict__ src, int n16)
{
    constexpr int CU = 2;
    for (int w0 = 0; w0 < n16; w0 += PAIR_THREADS * CU) {
        uint4 v[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            const int w = w0 + u * PAIR_THREADS + (int)threadIdx.x;
            v[u] = src[w < n16 ? w : n16 - 1];
        }
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            const int w = w0 + u * PAIR_THREADS + (int)threadIdx.x;
            if (w < n16) dst[w] = v[u];
        }
    }
}

// copy16_to_lds for a column's sorted positions (u16, 0xFFFF for a missing
// sample), each u16 v written as min(v & keep, clamp) (two u16 per packed
// 16-bit min).  The first POS_PRE x PAIR_THREADS words are loaded ahead by
// pos_prefetch (so that their latency passes during the table build) and
// handed in as pre; the rest are loaded here.
constexpr int POS_PRE = 3;

__device__ __forceinline__ void pos_prefetch(const uint4* __restrict__ src, int n16, uint4 (&pre)[POS_PRE])
{
#pragma unroll
    for (int u = 0; u < POS_PRE; ++u) {
        const int w = u * PAIR_THREADS + (int)threadIdx.x;
        pre[u] = src[w < n16 ? w : n16 - 1];
    }
}

__device__ __forceinline__ void copy_pos_to_lds(uint4* dst, const uint4* __restrict__ src, int n16, uint32_t keep,
                                                uint32_t clamp, const uint4 (&pre)[POS_PRE])
{
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    constexpr int CU = 3;
    const u16x2 c2 = __builtin_bit_cast(u16x2, clamp | (clamp << 16));
    const uint32_t k2 = keep | (keep << 16);
    const auto fix = [c2, k2](uint32_t w) {
        return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, w & k2), c2));
    };
#pragma unroll
    for (int u = 0; u < POS_PRE; ++u) {
        const int w = u * PAIR_THREADS + (int)threadIdx.x;
        if (w < n16) dst[w] = make_uint4(fix(pre[u].x), fix(pre[u].y), fix(pre[u].z), fix(pre[u].w));
    }
    for (int w0 = POS_PRE * PAIR_THREADS; w0 < n16; w0 += PAIR_THREADS * CU) {
        uint4 v[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            const int w = w0 + u * PAIR_THREADS + (int)threadIdx.x;
            v[u] = src[w < n16 ? w : n16 - 1];
        }
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            const int w = w0 + u * PAIR_THREADS + (int)threadIdx.x;
            if (w < n16) dst[w] = make_uint4(fix(v[u].x), fix(v[u].y), fix(v[u].z), fix(v[u].w));
        }
    }
}

struct PairSmem {
    size_t off_tab, off_corr, off_rrun, bytes;
    int nwp;  // table entries per partner
};

// posA: positions of samples 0..S (S is the dummy; not in LDS for long
// columns, big); tab: PB partner tables; corr: PB tie-defect sums; rrun:
// [PB][RUN_TABLE_STRIDE] run ranks
__host__ __device__ inline PairSmem pair_smem(int64_t ld, int64_t S, int PB, bool big = false)
{
    (void)ld;
    PairSmem m;
    m.nwp = (int)((S + 1 + 31) / 32) + 1;
    m.off_tab = big ? 0 : (size_t)round_up(2 * (S + 1), 16);
    m.off_corr = m.off_tab + (size_t)PB * m.nwp * 8;
    m.off_rrun = m.off_corr + (size_t)PB * 8;
    m.bytes = m.off_rrun + (size_t)PB * RUN_TABLE_STRIDE * 4;
    return m;
}

// Work list of the pair kernel.  Rows la of the processing order come in
// bands of 8 PB rows; band g holds partner blocks 8g .. nbp-1 (nbp = number of
// partner blocks padded to a multiple of 8), which covers every block that
// pairs with a row of the band (block q pairs with row la when q >= la / PB).
// Each band's row length is a multiple of 8, so a workgroup index and its
// partner block are congruent mod 8: a partner block always runs on the same
// XCD (workgroups are dealt to the 8 XCDs round-robin) and its sorted orders
// stay in that XCD's L2.
__host__ __device__ inline int64_t pair_band_start(int64_t g, int64_t nbp, int PB)
{
    return 8 * (int64_t)PB * (g * nbp - 4 * g * (g - 1));
}

__host__ inline int64_t pair_grid_size(int64_t F, int64_t nbp, int PB)
{
    const int64_t rows = 8 * (int64_t)PB;
    const int64_t G = ceil_div(F, rows);
    return pair_band_start(G - 1, nbp, PB) + (F - rows * (G - 1)) * (nbp - 8 * (G - 1));
}

// BIG (columns longer than the LDS sort handles): only the partner tables
// live in LDS; a's positions (no tie flag) and the partner block's presence
// bytes are read from global memory, a tied a-sample is recognised by its
// run (TA 4), and products are summed in 64 bits.
template <int PB, bool DBG, bool BIG>
__global__ __launch_bounds__(PAIR_THREADS, 8) void k_spearman_pairs(SpearBase bs, const uint8_t* __restrict__ presb,
                                                                 int64_t S, int64_t F, int64_t nbp, PairOut po)
{
    static_assert(PB == 8, "a partner block is one plane of presence bytes");
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    // the wave index is the same in every lane: readfirstlane lets the
    // compiler keep everything derived from it in scalar registers
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int64_t la = 0, b0 = 0;
    if constexpr (!DBG) {
        const int64_t id = (int64_t)blockIdx.x;
        // band g: the last band (8 g < nbp) with pair_band_start(g) <= id;
        // the band starts rise with g, so a binary search on the scalar
        // unit finds it (integer work on uniform values, no vector FP64)
        int64_t g = 0, ghi = nbp / 8;
        while (ghi - g > 1) {
            const int64_t mid = (g + ghi) >> 1;
            if (pair_band_start(mid, nbp, PB) <= id) g = mid;
            else ghi = mid;
        }
        // the offset in the band and the band's row length are below 2^31
        // (the grid is), so the division is a 32-bit one
        const uint32_t r = (uint32_t)(id - pair_band_start(g, nbp, PB));
        const uint32_t len = (uint32_t)(nbp - 8 * g);
        la = 8 * (int64_t)PB * g + (int64_t)(r / len);
        b0 = (8 * g + (int64_t)(r % len)) * PB;
        if (la >= F || b0 >= F || b0 + PB - 1 < la) return;
    }
    const int64_t a = DBG ? po.dbg_a : bs.perm[la];

    const int64_t ld = bs.ld;
    const PairSmem L = pair_smem(ld, S, PB, BIG);
    uint16_t* posA = BIG ? pin_uniform(bs.pos + a * ld) : (uint16_t*)smem_raw;
    uint2* tab = (uint2*)(smem_raw + L.off_tab);                               // [PB][nwp]
    unsigned long long* corrA = (unsigned long long*)(smem_raw + L.off_corr);  // [PB]
    uint32_t* rrun = (uint32_t*)(smem_raw + L.off_rrun);                       // [PB][RUN_TABLE_STRIDE]

    const int na = bs.ncol[a];
    const int tA = bs.hasties[a];
    const uint16_t* ordA = pin_uniform(bs.ord + a * ld);
    const uint32_t* rlA = pin_uniform(bs.rlist + a * (ld / 2));
    const uint32_t* runsA = pin_uniform(bs.runs + a * ld);  // a's runs by position (long columns)
    const int nra = tA ? bs.nruns[a] : 0;
    const bool rtab = !BIG && tA && nra <= RUN_TABLE_MAX;  // run-rank table in LDS
    const int nsg = (!DBG && !BIG && tA) ? bs.nsing[a] : -1;
    const bool grouped = nsg >= 0;  // implies rtab (runs + untied positions <= RUN_TABLE_MAX)
    const uint16_t* sgA = pin_uniform(bs.sing + a * RUN_GROUPS_MAX);
    const uint16_t* posAg = pin_uniform(bs.pos + a * ld);

    // this wave's partner j = wave (one partner per wave; the debug form has
    // one partner, on wave 0): its column and pointers are read here, so
    // that the base's pointers die before the tables are built
    static_assert(PB <= PAIR_WAVES, "one partner per wave");
    const int j = wave;
    const int64_t lb = b0 + j;
    const bool jact = DBG ? j == 0 : (j < PB && lb < F && lb >= la);
    const int64_t b = DBG ? (int64_t)po.dbg_b : (jact ? (int64_t)bs.perm[lb] : 0);
    const int nbv = jact ? bs.ncol[b] : 0;
    const int tB = jact ? bs.hasties[b] : 0;
    // b's tie runs resolved in the walk (class 2), or settled after an
    // untied walk (class 1; the debug walk reports every rank, so it
    // resolves them in the walk)
    const int cB = DBG ? (tB ? 2 : 0) : (jact ? bs.tcls[b] : 0);
    const int nsgB = DBG ? -1 : (jact ? bs.nsing[b] : -1);
    const int nrb = jact ? bs.nruns[b] : 0;
    const uint16_t* ordB = pin_uniform((BIG ? bs.ord : bs.ord2) + b * ld);  // doubled for the LDS path
    const uint32_t* runsB = pin_uniform(bs.runs + b * ld);
    const uint64_t* tbB = pin_uniform(bs.tbits + b * (ld / 64));
    const uint32_t* rlB = pin_uniform(bs.rlist + b * (ld / 2));
    const uint16_t* sgB = pin_uniform(bs.sing + b * RUN_GROUPS_MAX);
    const int NW = (na + 1 + 31) >> 5;  // words covering positions 0..na
    // the partner block's presence bytes go where a's positions will be
    // (they are needed only while the tables are built); lane-wise gathers
    // from LDS instead of global memory
    const uint8_t* presL = BIG ? presb + (b0 / PB) * ld : (const uint8_t*)smem_raw;
    // a's positions: the first words loaded now, stored after the table build
    uint4 pos_pre[POS_PRE];
    if constexpr (!BIG) pos_prefetch((const uint4*)posAg, (int)((S + 1 + 7) / 8), pos_pre);
    // bytes 0..S: byte S is zero (the sentinel sample of a's padded order)
    if constexpr (!DBG && !BIG)
        copy16_to_lds((uint4*)smem_raw, (const uint4*)(presb + (b0 / PB) * ld), (int)((S + 16) / 16));
    if (threadIdx.x < PB) corrA[threadIdx.x] = 0ull;
    __syncthreads();

    // ---- step 1: partner tables along a's order, PB partners at once --------
    // Thread t builds table word w = t (+ PAIR_THREADS per pass) of all PB
    // partners: the masks from presence_words, the counts y by a block scan
    // of the masks' popcounts (two partners' counts per 32-bit value, each
    // half at most na < 2^16).  Positions below 32 NW <= round_up(na + 1, 64) <= ld stay
    // inside a's padded order, and positions from na on hold the sentinel S,
    // whose presence byte is zero; lanes past NW read word NW - 1 and store
    // nothing.  The run-rank table's space holds the per-wave scan totals.
    static_assert(PAIR_WAVES == 8, "the wave totals fill two rows of 16 lanes");
    const uint16_t* posDbg = pin_uniform(bs.pos + (int64_t)po.dbg_b * ld);
    uint32_t* wtot = rrun;  // [PAIR_WAVES][4]
    uint32_t carry[4] = {0u, 0u, 0u, 0u};
    for (int w0 = 0; w0 < NW; w0 += PAIR_THREADS) {
        const int w = w0 + (int)threadIdx.x;
        const bool valid = w < NW;
        // a wave past the last word has no masks and zero counts
        uint32_t x[8] = {}, pc[4] = {}, incl[4] = {};
        if (w0 + wave * 64 < NW) {  // wave-uniform
            const int wl = valid ? w : NW - 1;
            presence_words<DBG>(ordA + 32 * wl, presL, posDbg, 32 * wl, na, x);
            if (!valid) {
#pragma unroll
                for (int j = 0; j < 8; ++j) x[j] = 0u;
            }
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                pc[h] = (uint32_t)__popc(x[2 * h]) | ((uint32_t)__popc(x[2 * h + 1]) << 16);
                incl[h] = wave_incl_scan_u32(pc[h]);
            }
        }
        if (lane == 63) {
#pragma unroll
            for (int h = 0; h < 4; ++h) wtot[wave * 4 + h] = incl[h];
        }
        __syncthreads();
        // the wave totals, lane 4 v + h holding wave v's for pair h, summed
        // over the waves of each row of 16 lanes (waves 0-3 and 4-7) by two
        // row shifts; this wave's base and the pass total are then read
        // from the row ends and the lane of the wave before it
        uint32_t base[4];
        {
            constexpr int ROW_SHR = 0x110;
            int sv = lane < 4 * PAIR_WAVES ? (int)wtot[lane] : 0;
            sv += __builtin_amdgcn_update_dpp(0, sv, ROW_SHR + 4, 0xF, 0xF, false);
            sv += __builtin_amdgcn_update_dpp(0, sv, ROW_SHR + 8, 0xF, 0xF, false);
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const uint32_t row0 = (uint32_t)__builtin_amdgcn_readlane(sv, 12 + h);
                const uint32_t row1 = (uint32_t)__builtin_amdgcn_readlane(sv, 28 + h);
                const uint32_t prev = wave > 0 ? (uint32_t)__builtin_amdgcn_readlane(sv, 4 * (wave - 1) + h) : 0u;
                base[h] = carry[h] + prev + (wave > 4 ? row0 : 0u);
                carry[h] += row0 + row1;
            }
        }
        if (valid) {
#pragma unroll
            for (int j = 0; j < PB; ++j) {
                const uint32_t ex = base[j >> 1] + incl[j >> 1] - pc[j >> 1];
                tab[(size_t)j * L.nwp + w] = make_uint2(x[j], 1u + ((ex >> (16 * (j & 1))) & 0xFFFFu));
            }
        }
        __syncthreads();  // wtot is rewritten by the next pass
    }
    if (threadIdx.x < PB) tab[(size_t)threadIdx.x * L.nwp + NW] = make_uint2(0u, 0u);
    // a's positions 0..S (S is the dummy) over the presence bytes, with the
    // missing code of a's class: untied, min(v, XS) turns 0xFFFF into XS;
    // grouped, min(v & POS_MASK, RUN_TABLE_MAX) turns a tied sample's flagged
    // run number into the run number and 0xFFFF into RUN_TABLE_MAX (untied
    // samples get theirs below); tied, unchanged
    const uint32_t XS = 32u * (uint32_t)NW;
    const uint32_t miss = BIG ? 0xFFFFu : grouped ? MISS_GROUPED : tA ? 0xFFFFu : XS;
    if constexpr (!BIG)
        copy_pos_to_lds((uint4*)posA, (const uint4*)posAg, (int)((S + 1 + 7) / 8),
                        grouped ? POS_MASK : 0xFFFFu, grouped ? MISS_GROUPED : tA ? 0xFFFFu : XS, pos_pre);
    __syncthreads();
    if (tA) {
        // per tie run [s, e) of a and partner: C(e) - C(s) complete samples
        // (tie defect) with doubled average rank C(s) + C(e) + 1 (run-rank
        // table); a grouped a adds its untied positions as runs [s, s + 1)
        // after the runs, and its untied samples' positions become those
        // runs' numbers (its tied samples' became their runs' numbers in
        // the copy)
        // one thread per (run, partner): a's few runs are spread over the
        // block instead of taking the partners one after another
        constexpr int LNJ = DBG ? 0 : 3;
        static_assert(DBG || PB == (1 << LNJ), "partners per block");
        const int ngr = grouped ? nra + nsg : nra;
        for (int q = threadIdx.x; q < (ngr << LNJ); q += PAIR_THREADS) {
            const int r = q >> LNJ, jr = q & ((1 << LNJ) - 1);
            uint32_t s, e;
            if (r < nra) {
                const uint32_t rr = rlA[r];
                s = rr & 0xFFFFu;
                e = rr >> 16;
            } else {
                s = sgA[r - nra];
                e = s + 1u;
                if (jr == 0) posA[ordA[s]] = (uint16_t)r;
            }
            const uint2* tj = tab + (size_t)jr * L.nwp;
            const uint32_t c1s = cnt1(tj, s), c1e = cnt1(tj, e);
            if (rtab) rrun[jr * RUN_TABLE_STRIDE + r] = c1s + c1e - 1u;
            const uint32_t tt = c1e - c1s;
            if (tt > 1u) atomicAdd(&corrA[jr], (unsigned long long)cube_minus(tt));
        }
        if (rtab && threadIdx.x < (1 << LNJ)) rrun[threadIdx.x * RUN_TABLE_STRIDE + RUN_TABLE_MAX] = 0u;
        __syncthreads();
    }

    // ---- step 2: one walk of each partner's sorted order ---------------------
    if (jact) {
        const uint2* tj = tab + (size_t)j * L.nwp;
        const uint32_t* rj = rtab ? rrun + j * RUN_TABLE_STRIDE : nullptr;
        WalkSums w;
        uint64_t sA, d3B;
        if (nsgB >= 0) {
            // b grouped: one pass by value groups
            uint32_t ng;
            if constexpr (BIG) {
                if (tA) grouped_b_walk<4>(ordB, nbv, rlB, nrb, sgB, nsgB, posA, tj, runsA, rj, XS, miss, lane, sA, ng, d3B);
                else grouped_b_walk<3>(ordB, nbv, rlB, nrb, sgB, nsgB, posA, tj, runsA, rj, XS, miss, lane, sA, ng, d3B);
            } else if (grouped) grouped_b_walk<2>(ordB, nbv, rlB, nrb, sgB, nsgB, posA, tj, rlA, rj, XS, miss, lane, sA, ng, d3B);
            else if (tA) grouped_b_walk<1>(ordB, nbv, rlB, nrb, sgB, nsgB, posA, tj, rlA, rj, XS, miss, lane, sA, ng, d3B);
            else grouped_b_walk<0>(ordB, nbv, rlB, nrb, sgB, nsgB, posA, tj, rlA, rj, XS, miss, lane, sA, ng, d3B);
            w.n = ng;
        } else {
#define NAPY_WALK(A, B) pair_walk<A, B, DBG>(ordB, runsB, tbB, A >= 3 ? runsA : rlA, nbv, posA, tj, rj, XS, miss, lane, po.dbg_ra, po.dbg_rb, w)
            if constexpr (BIG) {
                if (tA) {
                    if (cB == 2) NAPY_WALK(4, true);
                    else NAPY_WALK(4, false);
                } else {
                    if (cB == 2) NAPY_WALK(3, true);
                    else NAPY_WALK(3, false);
                }
            } else if (grouped) {
                if (cB == 2) NAPY_WALK(2, true);
                else NAPY_WALK(2, false);
            } else if (tA) {
                if (cB == 2) NAPY_WALK(1, true);
                else NAPY_WALK(1, false);
            } else {
                if (cB == 2) NAPY_WALK(0, true);
                else NAPY_WALK(0, false);
            }
#undef NAPY_WALK
            int64_t corr = 0;
            uint64_t d3s = 0;
            if (!DBG && cB == 1) {
                if constexpr (BIG) {
                    if (tA) settle_short_runs_b<4>(ordB, rlB, nrb, posA, tj, runsA, rj, miss, lane, corr, d3s);
                    else settle_short_runs_b<3>(ordB, rlB, nrb, posA, tj, runsA, rj, miss, lane, corr, d3s);
                } else if (grouped) settle_short_runs_b<2>(ordB, rlB, nrb, posA, tj, rlA, rj, miss, lane, corr, d3s);
                else if (tA) settle_short_runs_b<1>(ordB, rlB, nrb, posA, tj, rlA, rj, miss, lane, corr, d3s);
                else settle_short_runs_b<0>(ordB, rlB, nrb, posA, tj, rlA, rj, miss, lane, corr, d3s);
            }
            // one reduction of the lane's combined sums (the tie corrections
            // may be negative: the sum is taken modulo 2^64)
            sA = wave_sum_u64(4ull * w.A4 + 2ull * w.At + w.Af + (uint64_t)corr) + w.Au;
            d3B = tB ? wave_sum_u64(w.d3B + d3s) : 0ull;
        }
        if (lane == 0 && !DBG) {
            const int64_t nn = (int64_t)w.n;
            const int64_t closed = sum_sq_doubled_untied(nn);
            const double Ba = (double)(closed - (int64_t)((tA ? corrA[j] : 0ull) / 3u));
            const double Bb = (double)(closed - (int64_t)(d3B / 3u));
            const int64_t g = a < b ? a : b, h = a < b ? b : a;
            const int64_t pid = pair_index(g, h, F);
            po.sums[pid] = make_double4((double)nn, (double)sA, Ba, Bb);
        }
    }
}

// One workgroup per 32 x 32 tile of the upper triangle: rho and n from the
// exact integer sums of each pair (g <= h), then p and both triangles.
__global__ __launch_bounds__(FT_THREADS) void k_spearman_final(const double4* __restrict__ sums, int64_t F, int T32,
                                                              double* __restrict__ r, double* __restrict__ p,
                                                              int32_t* __restrict__ n, int64_t ldo)
{
    __shared__ FinSmem f;
    int tg, th;
    finish_tile_coords((int)blockIdx.x, T32, tg, th);
    const int64_t g0 = (int64_t)tg * FT, h0 = (int64_t)th * FT;
    const int j = ft_col();
    bool valid[FT_K];
#pragma unroll
    for (int k = 0; k < FT_K; ++k) {
        valid[k] = ft_valid(g0, h0, F, k);
        if (!valid[k]) continue;
        const int i = ft_row(k);
        const double4 s = sums[pair_index(g0 + i, h0 + j, F)];
        const int64_t nn = (int64_t)s.x;
        const int64_t A = (int64_t)s.y, Ba = (int64_t)s.z, Bb = (int64_t)s.w;
        const int64_t K = nn * (nn + 1) * (nn + 1);
        const int64_t num = A - K, Da = Ba - K, Db = Bb - K;
        double rho = __builtin_nan("");
        if (nn >= 2 && Da > 0 && Db > 0) {
            // sqrt of the product (not the product of roots) so that identical
            // rank vectors give exactly 1
            rho = (double)num / sqrt((double)Da * (double)Db);
            rho = rho > 1.0 ? 1.0 : (rho < -1.0 ? -1.0 : rho);
        }
        f.r[i][j] = rho;
        f.n[i][j] = (int32_t)nn;
    }
    ft_pvalues(f, valid, false);  // n = 2: p undefined
    __syncthreads();
    ft_write(f, g0, h0, F, r, p, n, ldo);
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

// Exclusive prefix sum of v over the 1024 threads of a workgroup; *total
// gets the sum.  wtot: 16 words of LDS.
__device__ __forceinline__ uint32_t block1024_excl_scan(uint32_t v, uint32_t* wtot, uint32_t* total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan_u32(v);
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();
    const uint32_t wincl = wave_incl_scan_u32(lane < 16 ? wtot[lane] : 0u);
    const uint32_t before = wave > 0 ? (uint32_t)__shfl((int)wincl, wave - 1, 64) : 0u;
    *total = (uint32_t)__shfl((int)wincl, 15, 64);
    __syncthreads();  // wtot may be reused
    return before + incl - v;
}

constexpr int CP_THREADS = 1024;
constexpr int CP_BATCH = 8;  // gathers in flight per thread

__host__ __device__ inline size_t compact_smem_bytes(int64_t base_ld) { return (size_t)round_up(4 * base_ld + 2, 16); }

// One 1024-thread workgroup per query column: keeps the base column's sorted
// order restricted to the query rows (order preserved), renumbers samples and
// positions, and maps tie runs through the prefix count of kept positions.
//   A  X[k] = query row of the sample at base position k (0xFFFF: not in the
//      query), gathers batched CP_BATCH per thread.
//   B  P[k] = kept positions below k, one block scan with every thread owning
//      a consecutive range of positions; the kept samples' new order and
//      positions.
//   C  the query's tie runs are the base runs keeping two or more samples,
//      numbered in position order by a block scan over the base run list;
//      QR[base run] = query run number (in X's place).
//   D  run bounds of every kept position; a sample in a query tie run gets
//      the flag and its run's number (through its base run index).
__global__ __launch_bounds__(CP_THREADS) void k_compact(SpearBase base, const int32_t* __restrict__ cols,
                                                         const int32_t* __restrict__ rowmap, int64_t Sq,
                                                         SpearBase q)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char cp_smem[];
    __shared__ uint32_t wtot[16];
    uint16_t* X = (uint16_t*)cp_smem;  // [base.ld]
    uint16_t* P = X + base.ld;         // [base.ld + 1]
    const int qc = blockIdx.x;
    const int t = threadIdx.x;
    const int64_t c = cols[qc];
    const int nc = base.ncol[c];
    const uint16_t* ord = base.ord + c * base.ld;
    const uint32_t* runs = base.runs + c * base.ld;
    const uint16_t* bpos = base.pos + c * base.ld;
    const uint32_t* brl = base.rlist + c * (base.ld / 2);
    const int nrb = base.nruns[c];
    uint16_t* qord = q.ord + (int64_t)qc * q.ld;
    uint16_t* qord2 = q.ord2 + (int64_t)qc * q.ld;
    uint16_t* qpos = q.pos + (int64_t)qc * q.ld;
    uint32_t* qruns = q.runs + (int64_t)qc * q.ld;
    uint32_t* qrl = q.rlist + (int64_t)qc * (q.ld / 2);
    for (int64_t j = t; j < q.ld; j += CP_THREADS) qpos[j] = 0xFFFF;

    // A
    for (int k0 = 0; k0 < nc; k0 += CP_BATCH * CP_THREADS) {
        uint32_t iv[CP_BATCH];
        int32_t nr[CP_BATCH];
#pragma unroll
        for (int u = 0; u < CP_BATCH; ++u) {
            const int k = k0 + u * CP_THREADS + t;
            iv[u] = ord[k < nc ? k : 0];
        }
#pragma unroll
        for (int u = 0; u < CP_BATCH; ++u) nr[u] = (k0 + u * CP_THREADS + t < nc) ? rowmap[iv[u]] : -1;
#pragma unroll
        for (int u = 0; u < CP_BATCH; ++u) {
            const int k = k0 + u * CP_THREADS + t;
            if (k < nc) X[k] = nr[u] >= 0 ? (uint16_t)nr[u] : (uint16_t)0xFFFF;
        }
    }
    __syncthreads();

    // B
    const int E = (nc + CP_THREADS - 1) / CP_THREADS;
    const int ka = min(t * E, nc), kb = min(ka + E, nc);
    uint32_t cnt = 0;
    for (int k = ka; k < kb; ++k) cnt += X[k] != 0xFFFF ? 1u : 0u;
    uint32_t total;
    uint32_t kp = block1024_excl_scan(cnt, wtot, &total);
    for (int k = ka; k < kb; ++k) {
        P[k] = (uint16_t)kp;
        const uint32_t x = X[k];
        if (x != 0xFFFFu) {
            qord[kp] = (uint16_t)x;
            qord2[kp] = (uint16_t)(2u * x);
            qpos[x] = (uint16_t)kp;
            ++kp;
        }
    }
    if (t == 0) P[nc] = (uint16_t)total;
    for (int64_t k = total + t; k < q.ld; k += CP_THREADS) {
        qord[k] = (uint16_t)Sq;
        qord2[k] = (uint16_t)(2 * Sq);
    }
    if (qc == (int)gridDim.x - 1)
        for (int64_t k = t; k < ORD_TAIL; k += CP_THREADS) {
            qord[q.ld + k] = (uint16_t)Sq;
            qord2[q.ld + k] = (uint16_t)(2 * Sq);
        }
    __syncthreads();

    // C
    uint16_t* QR = X;
    const int Er = (nrb + CP_THREADS - 1) / CP_THREADS;
    const int ra = min(t * Er, nrb), rz = min(ra + Er, nrb);
    uint32_t nt = 0;
    for (int r = ra; r < rz; ++r) {
        const uint32_t rr = brl[r];
        nt += (uint32_t)P[rr >> 16] - (uint32_t)P[rr & 0xFFFFu] > 1u ? 1u : 0u;
    }
    uint32_t nq;
    uint32_t rid = block1024_excl_scan(nt, wtot, &nq);
    for (int r = ra; r < rz; ++r) {
        const uint32_t rr = brl[r];
        const uint32_t s0 = P[rr & 0xFFFFu], e0 = P[rr >> 16];
        if (e0 - s0 > 1u) {
            QR[r] = (uint16_t)rid;
            qrl[rid] = s0 | (e0 << 16);
            ++rid;
        }
    }
    __syncthreads();

    // D
    for (int k0 = 0; k0 < nc; k0 += CP_BATCH * CP_THREADS) {
        uint32_t iv[CP_BATCH], rr[CP_BATCH];
        int32_t nr[CP_BATCH];
#pragma unroll
        for (int u = 0; u < CP_BATCH; ++u) {
            const int k = k0 + u * CP_THREADS + t;
            iv[u] = ord[k < nc ? k : 0];
            rr[u] = runs[k < nc ? k : 0];
        }
#pragma unroll
        for (int u = 0; u < CP_BATCH; ++u) nr[u] = (k0 + u * CP_THREADS + t < nc) ? rowmap[iv[u]] : -1;
#pragma unroll
        for (int u = 0; u < CP_BATCH; ++u) {
            const int k = k0 + u * CP_THREADS + t;
            if (k >= nc || nr[u] < 0) continue;
            const uint32_t kpk = P[k];
            const uint32_t s = rr[u] & 0xFFFFu, e = rr[u] >> 16;
            if (e - s == 1u) {
                qruns[kpk] = kpk | ((kpk + 1u) << 16);
            } else {
                const uint32_t s0 = P[s], e0 = P[e];
                qruns[kpk] = s0 | (e0 << 16);
                if (e0 - s0 > 1u) qpos[nr[u]] = (uint16_t)(POS_TIED | QR[bpos[iv[u]] & POS_MASK]);
            }
        }
    }
    if (t == 0) {
        q.ncol[qc] = (int32_t)total;
        q.hasties[qc] = nq > 0u ? 1 : 0;
        q.nruns[qc] = (int32_t)nq;
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// partners per workgroup, one per wave: 8 keeps a workgroup's LDS (a's
// positions plus 8 partner tables) near 40 KB, so four workgroups (32 waves)
// share a CU
constexpr int PAIR_PB = 8;
static_assert(PAIR_PB * 64 == PAIR_THREADS, "one partner per wave");

template <bool DBG, bool BIG>
static int pairs_launch_t(const SpearBase& bs, const uint8_t* presb, int64_t S, int64_t F, PairOut po,
                          hipStream_t st)
{
    const size_t smem = pair_smem(bs.ld, S, PAIR_PB, BIG).bytes;
    static std::atomic<uint64_t> attr_done{0};
    NAPY_TRY(ensure_dyn_lds(attr_done, (const void*)k_spearman_pairs<PAIR_PB, DBG, BIG>, 160 * 1024,
                            "hipFuncSetAttribute(k_spearman_pairs)"));
    if constexpr (!BIG) {
        // the walks take a doubled sample index as the LDS address of its
        // a-position: the dynamic block (a's positions first) must begin at
        // LDS address 0, so the kernel may hold no static LDS
        static std::atomic<int> lds_at0{-1};
        int v = lds_at0.load(std::memory_order_acquire);
        if (v < 0) {
            hipFuncAttributes fa;
            const hipError_t e = hipFuncGetAttributes(&fa, (const void*)k_spearman_pairs<PAIR_PB, DBG, BIG>);
            if (e != hipSuccess) return hip_status(e, "hipFuncGetAttributes(k_spearman_pairs)");
            v = fa.sharedSizeBytes == 0 ? 1 : 0;
            lds_at0.store(v, std::memory_order_release);
        }
        if (v == 0) {
            set_last_error("k_spearman_pairs holds static LDS: its dynamic block does not begin at address 0");
            return NAPY_E_HIP;
        }
    }
    if (smem > 160 * 1024) return NAPY_E_UNSUPPORTED;
    const int64_t nbp = round_up(ceil_div(F, PAIR_PB), 8);
    const int64_t nblk = DBG ? 1 : pair_grid_size(F, nbp, PAIR_PB);
    if (nblk > 0x7FFFFFFFLL) return NAPY_E_UNSUPPORTED;
    hipLaunchKernelGGL((k_spearman_pairs<PAIR_PB, DBG, BIG>), dim3((unsigned)nblk), dim3(PAIR_THREADS), smem, st, bs,
                       presb, S, F, nbp, po);
    return check_launch("spearman_pairs");
}

// the partner blocks' presence planes (input of the pair scan)
static int presence_launch(const SpearBase& bs, uint32_t* pres, int64_t S, int64_t F, hipStream_t st)
{
    const int64_t nq = ceil_div(F, 8);
    hipLaunchKernelGGL(k_presence, dim3((unsigned)ceil_div(bs.ld, 1024), (unsigned)nq), dim3(256), 0, st, bs, S, F,
                       (uint8_t*)pres);
    return check_launch("presence");
}

// presence planes, then the pair scan
static int pairs_launch(const SpearBase& bs, uint32_t* pres, int64_t S, int64_t F, PairOut po, hipStream_t st,
                        bool with_presence = true)
{
    uint8_t* presb = (uint8_t*)pres;
    if (with_presence) NAPY_TRY(presence_launch(bs, pres, S, F, st));
    // columns longer than the LDS sort handles carry no tie flag in their
    // positions (and would not fit a's positions in LDS next to the tables)
    if (S > SORT_LDS_MAX_S) {
        if (po.dbg_ra) return pairs_launch_t<true, true>(bs, presb, S, F, po, st);
        return pairs_launch_t<false, true>(bs, presb, S, F, po, st);
    }
    if (po.dbg_ra) return pairs_launch_t<true, false>(bs, presb, S, F, po, st);
    return pairs_launch_t<false, false>(bs, presb, S, F, po, st);
}

struct SpearWs {
    uint32_t* keys;
    SpearBase base;
    uint32_t* pres;  // ceil(F/32) * ld words: ceil(F/8) planes of ld presence bytes
    double4* sums;
};

static void spear_carve(Carver& c, int64_t S, int64_t F, SpearWs& w)
{
    const int64_t ld = spear_ld(S);
    w.keys = c.take<uint32_t>((size_t)sort_keys_words(S, F));
    base_carve(c, S, F, w.base);
    w.pres = c.take<uint32_t>((size_t)ceil_div(F, 32) * ld);
    const int64_t npairs = F * (F + 1) / 2;
    w.sums = c.take<double4>(npairs);
}

template <int EPT>
static int colsort_launch(const uint32_t* keys, int64_t S, int64_t F, const SpearBase& base, hipStream_t st)
{
    static std::atomic<uint64_t> attr_done{0};
    NAPY_TRY(ensure_dyn_lds(attr_done, (const void*)k_colsort<EPT>, (int)sort_smem_bytes(EPT),
                            "hipFuncSetAttribute(k_colsort)"));
    hipLaunchKernelGGL(k_colsort<EPT>, dim3((unsigned)F), dim3(CS_THREADS), sort_smem_bytes(EPT), st, keys, S,
                       base.ld, base);
    return check_launch("colsort");
}

static int sort_launch(const float* X, int64_t S, int64_t F, int64_t ldx, int us, float sv,
                       uint32_t* keys, const SpearBase& base, hipStream_t st)
{
    dim3 gk((unsigned)ceil_div(F, 64), (unsigned)ceil_div(base.ld, 64));
    // (the key rows are 16-byte aligned: the workspace's carve aligns them and ld is a multiple of 256)
    if (base.ld % 4 != 0 || ((uintptr_t)keys & 15u) != 0u) {
        set_last_error("sort keys: key rows not 16-byte aligned");
        return NAPY_E_INVALID;
    }
    if (ldx % 4 == 0 && ((uintptr_t)X & 15u) == 0u)
        hipLaunchKernelGGL(k_sort_keys<true>, gk, dim3(256), 0, st, X, S, F, ldx, us, sv, keys, base.ld);
    else
        hipLaunchKernelGGL(k_sort_keys<false>, gk, dim3(256), 0, st, X, S, F, ldx, us, sv, keys, base.ld);
    NAPY_TRY(check_launch("sort_keys"));
    if (S > SORT_LDS_MAX_S) {
        hipLaunchKernelGGL(k_colsort_big, dim3((unsigned)F), dim3(CS_THREADS), 0, st, keys, S, base.ld, F, base);
        NAPY_TRY(check_launch("colsort_big"));
        return tiebits_launch(base, F, st, false);
    }
    const int64_t E = ceil_div(S, CS_THREADS);
    if (E <= 2) NAPY_TRY(colsort_launch<2>(keys, S, F, base, st));
    else if (E <= 4) NAPY_TRY(colsort_launch<4>(keys, S, F, base, st));
    else if (E <= 6) NAPY_TRY(colsort_launch<6>(keys, S, F, base, st));
    else if (E <= 8) NAPY_TRY(colsort_launch<8>(keys, S, F, base, st));
    else if (E <= 10) NAPY_TRY(colsort_launch<10>(keys, S, F, base, st));
    else if (E <= 12) NAPY_TRY(colsort_launch<12>(keys, S, F, base, st));
    else if (E <= 16) NAPY_TRY(colsort_launch<16>(keys, S, F, base, st));
    else if (E <= 20) NAPY_TRY(colsort_launch<20>(keys, S, F, base, st));
    else NAPY_TRY(colsort_launch<CS_EPT_MAX>(keys, S, F, base, st));
    return tiebits_launch(base, F, st, false);
}

static int final_launch(const SpearWs& w, int64_t F, double* r, double* p, int32_t* n, int64_t ldo,
                        hipStream_t st)
{
    const int T32 = (int)ceil_div(F, FT);
    hipLaunchKernelGGL(k_spearman_final, dim3((unsigned)(T32 * (T32 + 1) / 2)), dim3(FT_THREADS), 0, st, w.sums, F,
                       T32, r, p, n, ldo);
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
    // the presence planes close the first stage, so that the second is the
    // pair scan kernel alone
    NAPY_TRY(presence_launch(w.base, w.pres, S, F, st));
    NAPY_TRY(record_stage(ev, 1, st));
    PairOut po{w.sums, nullptr, nullptr, 0, 0};
    NAPY_TRY(pairs_launch(w.base, w.pres, S, F, po, st, false));
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
    PairOut po{w.sums, rg, rh, g, h};
    return pairs_launch(w.base, w.pres, S, F, po, st);
}

size_t spearman_base_bytes(int64_t S, int64_t F)
{
    Carver c(nullptr);
    SpearBase b;
    base_carve(c, S, F, b);
    // the keys buffer used while sorting is carved after the base
    c.take<uint32_t>((size_t)sort_keys_words(S, F));
    return c.bytes();
}

int spearman_base_prepare_run(const float* X, int64_t S, int64_t F, int64_t ldx, void* base,
                              const napy_opts* opts, hipStream_t st)
{
    Carver c(base);
    SpearBase b;
    base_carve(c, S, F, b);
    uint32_t* keys = c.take<uint32_t>((size_t)sort_keys_words(S, F));
    return sort_launch(X, S, F, ldx, opt_use_sent(opts), opt_sent(opts), keys, b, st);
}

size_t spearman_subset_ws_bytes(int64_t S, int64_t Sq, int64_t Fq)
{
    Carver c(nullptr);
    c.take<int32_t>(S > 0 ? S : 1);
    SpearBase q;
    base_carve(c, Sq, Fq, q);
    c.take<uint32_t>((size_t)ceil_div(Fq, 32) * spear_ld(Sq));
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
    w.pres = c.take<uint32_t>((size_t)ceil_div(Fq, 32) * spear_ld(Sq));
    const int64_t npairs = Fq * (Fq + 1) / 2;
    w.sums = c.take<double4>(npairs);
    w.keys = nullptr;
    if (S > 0) {
        hipLaunchKernelGGL(k_rowmap, dim3((unsigned)ceil_div(S, 256)), dim3(256), 0, st, rows, Sq, S, rowmap);
        NAPY_TRY(check_launch("rowmap"));
    }
    if (Sq > 0) {
        hipLaunchKernelGGL(k_rowmap_set, dim3((unsigned)ceil_div(Sq, 256)), dim3(256), 0, st, rows, Sq, rowmap);
        NAPY_TRY(check_launch("rowmap_set"));
    }
    {
        const size_t smem = compact_smem_bytes(b.ld);
        static std::atomic<uint64_t> attr_done{0};
        NAPY_TRY(ensure_dyn_lds(attr_done, (const void*)k_compact, (int)compact_smem_bytes(spear_ld(SPEARMAN_MAX_S)),
                                "hipFuncSetAttribute(k_compact)"));
        hipLaunchKernelGGL(k_compact, dim3((unsigned)Fq), dim3(CP_THREADS), smem, st, b, cols, rowmap, Sq, w.base);
        NAPY_TRY(check_launch("compact"));
    }
    NAPY_TRY(tiebits_launch(w.base, Fq, st));
    PairOut po{w.sums, nullptr, nullptr, 0, 0};
    NAPY_TRY(pairs_launch(w.base, w.pres, Sq, Fq, po, st));
    return final_launch(w, Fq, r, p, n, ldo, st);
}

}  // namespace napy
