// Multiple-testing correction of an all-pairs p matrix (NApy, Section 3.4):
// Bonferroni, Benjamini-Hochberg (step-up) and Benjamini-Yekutieli.
//
// The tests are the unordered pairs i < j with a defined p-value (m of them);
// the diagonal self-tests are not tests and are NaN in the result, as are
// pairs whose p is NaN.  The upper triangle is read and both triangles are
// written.  With the m defined p-values in ascending order p_(1..m):
//   Bonferroni  min(1, m p)
//   BH          min(1, min_{l >= k} m p_(l) / l)      for p = p_(k)
//   BY          the same with m c(m), c(m) = sum_{i <= m} 1 / i
// Equal p-values get equal adjusted values whatever their order in the sort,
// so an unstable sort serves.
//
// Kernels, in stream order:
//   k_adj_pad / k_adj_gather  keys (the IEEE bits of p: order-preserving for
//                    p >= 0; NaN -> all ones but the last bit, padding -> all
//                    ones, so they sort after every p and padding last) and
//                    pair indices i * F + j of the upper triangle, padded to
//                    a power of two N >= ADJ_TILE; one workgroup per row,
//                    which also counts the row's defined p-values.
//   k_adj_factor     m (the sum of the row counts), and the factor m or m c(m).
//   bitonic sort     k_bitonic_tile (LDS tiles of ADJ_TILE elements, every
//                    step with a stride below the tile), k_bitonic_multi (up
//                    to three larger strides per global pass).
//   k_adj_scale      q_k = factor p_(k) / k and its suffix minimum within
//                    each block of ADJ_SCAN elements, plus the block minima.
//   k_adj_blocks     suffix minimum over the block minima (one workgroup).
//   k_adj_scatter    min(1, min(q suffix, later blocks)) to (i, j) and (j, i).
#include "napy_internal.hpp"

namespace napy {

constexpr int ADJ_TILE = 4096;        // bitonic LDS tile (12 B per element)
constexpr int ADJ_TILE_THREADS = 1024;
constexpr int ADJ_SCAN = 4096;        // elements per suffix-scan block
constexpr int ADJ_SCAN_THREADS = 1024;
constexpr uint64_t ADJ_KEY_PAD = ~0ull;
constexpr uint64_t ADJ_KEY_NAN = ~0ull - 1ull;
constexpr uint32_t ADJ_NO_PAIR = 0xFFFFFFFFu;  // above any i * F + j for F <= 65535
constexpr long long ADJ_NAN_BITS = 0x7FF8000000000000LL;

struct AdjWs {
    uint64_t* keys;  // [N]; after the sort, q as double
    uint32_t* vals;  // [N]
    double* bmin;    // [N / ADJ_SCAN] block minima, then their exclusive suffix minima
    uint32_t* rowm;  // [F] defined p-values per row of the upper triangle
    uint32_t* m;     // [1]
    double* factor;  // [1]
};

static int64_t adj_npairs(int64_t F) { return F * (F - 1) / 2; }

static int64_t adj_n(int64_t F)
{
    int64_t n = ADJ_TILE;
    while (n < adj_npairs(F)) n <<= 1;
    return n;
}

static void adj_carve(Carver& c, int64_t F, AdjWs& w)
{
    const int64_t N = adj_n(F);
    w.keys = c.take<uint64_t>(N);
    w.vals = c.take<uint32_t>(N);
    w.bmin = c.take<double>(N / ADJ_SCAN);
    w.rowm = c.take<uint32_t>(F);
    w.m = c.take<uint32_t>(1);
    w.factor = c.take<double>(1);
}

size_t adjust_ws_bytes(int64_t F)
{
    Carver c(nullptr);
    AdjWs w;
    adj_carve(c, F, w);
    return c.bytes();
}

__global__ __launch_bounds__(256) void k_adj_pad(uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                 int64_t from, int64_t N)
{
    const int64_t k = from + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < N) {
        keys[k] = ADJ_KEY_PAD;
        vals[k] = ADJ_NO_PAIR;
    }
}

__device__ __forceinline__ uint32_t block256_sum_u32(uint32_t v)
{
    __shared__ uint32_t part[4];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    return part[0] + part[1] + part[2] + part[3];
}

// one workgroup per row i of the upper triangle: columns j > i
__global__ __launch_bounds__(256) void k_adj_gather(const double* __restrict__ p, int64_t F, int64_t ldp,
                                                    uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                    uint32_t* __restrict__ rowm)
{
    const int64_t i = blockIdx.x;
    const int64_t u0 = i * (2 * F - i - 1) / 2 - (i + 1);  // pair index u0 + j
    uint32_t c = 0;
    for (int64_t j = i + 1 + threadIdx.x; j < F; j += 256) {
        const double v = p[i * ldp + j];
        const bool defined = !isnan(v);
        // + 0.0 turns -0 into +0, whose bits sort first
        keys[u0 + j] = defined ? (uint64_t)__double_as_longlong(v + 0.0) : ADJ_KEY_NAN;
        vals[u0 + j] = (uint32_t)(i * F + j);
        c += defined ? 1u : 0u;
    }
    c = block256_sum_u32(c);
    if (threadIdx.x == 0) rowm[i] = c;
}

// c(m) = sum_{i <= m} 1/i: summed from the small end below 1024 terms, else
// the asymptotic expansion ln m + gamma + 1/(2m) - 1/(12 m^2) + 1/(120 m^4)
// - 1/(252 m^6) (next term below 1e-22 at m = 1024).
__device__ double harmonic_number(uint32_t m)
{
    if (m < 1024u) {
        double s = 0.0;
        for (uint32_t i = m; i >= 1u; --i) s += 1.0 / (double)i;
        return s;
    }
    const double x = (double)m, x2 = 1.0 / (x * x);
    const double euler_gamma = 0.57721566490153286061;
    return log(x) + euler_gamma + 0.5 / x - x2 * (1.0 / 12.0 - x2 * (1.0 / 120.0 - x2 * (1.0 / 252.0)));
}

__global__ __launch_bounds__(256) void k_adj_factor(const uint32_t* __restrict__ rowm, int64_t rows, int method,
                                                    uint32_t* __restrict__ m, double* __restrict__ factor)
{
    uint32_t c = 0;
    for (int64_t i = threadIdx.x; i < rows; i += 256) c += rowm[i];
    const uint32_t mm = block256_sum_u32(c);
    if (threadIdx.x == 0) {
        *m = mm;
        *factor = method == NAPY_ADJ_BY ? (double)mm * harmonic_number(mm) : (double)mm;
    }
}

__device__ __forceinline__ void cmp_swap(uint64_t& ka, uint32_t& va, uint64_t& kb, uint32_t& vb, bool ascending)
{
    if ((ka > kb) == ascending) {
        const uint64_t tk = ka;
        ka = kb;
        kb = tk;
        const uint32_t tv = va;
        va = vb;
        vb = tv;
    }
}

// One tile of ADJ_TILE elements in LDS.  kmax == 0: sort the tile (all
// bitonic stages k = 2 .. ADJ_TILE).  Otherwise: the steps with strides
// ADJ_TILE/2 .. 1 of stage kmax (> ADJ_TILE).  The direction of a pair
// follows its global index, so the tiles fit the global bitonic network.
__global__ __launch_bounds__(ADJ_TILE_THREADS) void k_bitonic_tile(uint64_t* __restrict__ keys,
                                                                     uint32_t* __restrict__ vals, int64_t kmax)
{
    __shared__ uint64_t sk[ADJ_TILE];
    __shared__ uint32_t sv[ADJ_TILE];
    const int64_t base = (int64_t)blockIdx.x * ADJ_TILE;
    const int t = threadIdx.x;
    for (int e = t; e < ADJ_TILE; e += ADJ_TILE_THREADS) {
        sk[e] = keys[base + e];
        sv[e] = vals[base + e];
    }
    __syncthreads();
    const int64_t k0 = kmax == 0 ? 2 : kmax;
    const int64_t k1 = kmax == 0 ? ADJ_TILE : kmax;
    for (int64_t k = k0; k <= k1; k <<= 1) {
        for (int j = (int)min(k >> 1, (int64_t)(ADJ_TILE >> 1)); j >= 1; j >>= 1) {
            for (int q = t; q < ADJ_TILE / 2; q += ADJ_TILE_THREADS) {
                const int lo = ((q / j) * 2 * j) + (q % j);
                const int hi = lo + j;
                const bool asc = ((base + lo) & k) == 0;
                uint64_t ka = sk[lo], kb = sk[hi];
                uint32_t va = sv[lo], vb = sv[hi];
                cmp_swap(ka, va, kb, vb, asc);
                sk[lo] = ka;
                sk[hi] = kb;
                sv[lo] = va;
                sv[hi] = vb;
            }
            __syncthreads();
        }
    }
    for (int e = t; e < ADJ_TILE; e += ADJ_TILE_THREADS) {
        keys[base + e] = sk[e];
        vals[base + e] = sv[e];
    }
}

// one global step of stage k with stride j = 2^lj >= ADJ_TILE: thread per pair

// R consecutive global strides j, j/2, .., j/2^(R-1) (lj = log2 j, all at
// least ADJ_TILE) of merge level k in one pass: a thread holds the 2^R
// elements b + m j / 2^(R-1) (b: its index with zero bits at the R stride
// positions), which all lie in one k-block and take one direction, and does
// the R compare-exchange rounds in registers.
template <int R>
__global__ __launch_bounds__(256) void k_bitonic_multi(uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                       int lj, int64_t k, int64_t ngroups)
{
    constexpr int E = 1 << R;
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= ngroups) return;
    const int lo = lj - R + 1;  // lowest stride bit
    const int64_t low = q & (((int64_t)1 << lo) - 1);
    const int64_t b = ((q >> lo) << (lj + 1)) | low;
    const int64_t step = (int64_t)1 << lo;
    const bool asc = (b & k) == 0;
    uint64_t kk[E];
    uint32_t vv[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        kk[m] = keys[b + m * step];
        vv[m] = vals[b + m * step];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int h = 1 << (R - 1 - r);  // partner distance in m for stride j >> r
#pragma unroll
        for (int m = 0; m < E; ++m)
            if ((m & h) == 0) cmp_swap(kk[m], vv[m], kk[m + h], vv[m + h], asc);
    }
#pragma unroll
    for (int m = 0; m < E; ++m) {
        keys[b + m * step] = kk[m];
        vals[b + m * step] = vv[m];
    }
}

// Minimum of v over the threads after this one in a workgroup of
// ADJ_SCAN_THREADS (exclusive suffix; +inf for the last thread); *incl gets
// the inclusive one.
__device__ double block_suffix_min_excl(double v, double* red, double* incl)
{
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    constexpr int NWAVES = ADJ_SCAN_THREADS / 64;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double o = __shfl_down(v, d, 64);
        if (lane + d < 64) v = fmin(v, o);
    }
    // v: minimum over lanes >= lane of the wave
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double later = INFINITY;  // later waves
    for (int w = wave + 1; w < NWAVES; ++w) later = fmin(later, red[w]);
    __syncthreads();
    const double next = __shfl_down(v, 1, 64);
    *incl = fmin(v, later);
    return lane < 63 ? fmin(next, later) : later;
}

// q_k = factor p_(k) / k (1-based k; +inf from position m on) and its suffix
// minimum within the block (written over the key), plus the block minimum
__global__ __launch_bounds__(ADJ_SCAN_THREADS) void k_adj_scale(uint64_t* __restrict__ keys,
                                                                  const uint32_t* __restrict__ m,
                                                                  const double* __restrict__ factor,
                                                                  double* __restrict__ bmin)
{
    __shared__ double red[ADJ_SCAN_THREADS / 64];
    constexpr int PER = ADJ_SCAN / ADJ_SCAN_THREADS;
    const int64_t base = (int64_t)blockIdx.x * ADJ_SCAN + (int64_t)threadIdx.x * PER;
    const int64_t mm = *m;
    const double f = *factor;
    double q[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int64_t k = base + e;
        q[e] = k < mm ? f * __longlong_as_double((long long)keys[k]) / (double)(k + 1) : INFINITY;
    }
#pragma unroll
    for (int e = PER - 2; e >= 0; --e) q[e] = fmin(q[e], q[e + 1]);
    double incl;
    const double later = block_suffix_min_excl(q[0], red, &incl);
#pragma unroll
    for (int e = 0; e < PER; ++e) keys[base + e] = (uint64_t)__double_as_longlong(fmin(q[e], later));
    if (threadIdx.x == 0) bmin[blockIdx.x] = incl;
}

// exclusive suffix minima over nb block minima, in place (one workgroup)
__global__ __launch_bounds__(ADJ_SCAN_THREADS) void k_adj_blocks(double* __restrict__ bmin, int64_t nb)
{
    __shared__ double red[ADJ_SCAN_THREADS / 64];
    const int64_t per = ceil_div(nb, ADJ_SCAN_THREADS);
    const int64_t b0 = min(nb, (int64_t)threadIdx.x * per), b1 = min(nb, b0 + per);
    double mine = INFINITY;
    for (int64_t b = b0; b < b1; ++b) mine = fmin(mine, bmin[b]);
    double incl;
    double run = block_suffix_min_excl(mine, red, &incl);
    // the own chunk from its end: each block's exclusive suffix
    for (int64_t b = b1 - 1; b >= b0; --b) {
        const double v = bmin[b];
        bmin[b] = run;
        run = fmin(run, v);
    }
}

__global__ __launch_bounds__(256) void k_adj_scatter(const uint64_t* __restrict__ q, const uint32_t* __restrict__ vals,
                                                     const double* __restrict__ bafter, const uint32_t* __restrict__ m,
                                                     int64_t count, int64_t F, double* __restrict__ out, int64_t ldo)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= count) return;
    const uint32_t v = vals[k];
    if (v == ADJ_NO_PAIR) return;
    const int64_t i = (int64_t)(v / (uint32_t)F), j = (int64_t)(v % (uint32_t)F);
    double a = __longlong_as_double(ADJ_NAN_BITS);
    if (k < (int64_t)*m) a = fmin(1.0, fmin(__longlong_as_double((long long)q[k]), bafter[k / ADJ_SCAN]));
    out[i * ldo + j] = a;
    out[j * ldo + i] = a;
}

// Bonferroni on the gathered (unsorted) keys
__global__ __launch_bounds__(256) void k_adj_bonferroni(const uint64_t* __restrict__ keys,
                                                        const uint32_t* __restrict__ vals,
                                                        const double* __restrict__ factor, int64_t count, int64_t F,
                                                        double* __restrict__ out, int64_t ldo)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= count) return;
    const uint32_t v = vals[k];
    const int64_t i = (int64_t)(v / (uint32_t)F), j = (int64_t)(v % (uint32_t)F);
    const uint64_t key = keys[k];
    const double a = key == ADJ_KEY_NAN ? __longlong_as_double(ADJ_NAN_BITS)
                                         : fmin(1.0, *factor * __longlong_as_double((long long)key));
    out[i * ldo + j] = a;
    out[j * ldo + i] = a;
}

__global__ __launch_bounds__(256) void k_adj_diag(double* __restrict__ out, int64_t F, int64_t ldo)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < F) out[i * ldo + i] = __longlong_as_double(ADJ_NAN_BITS);
}

int adjust_run(const double* p, int64_t F, int64_t ldp, double* out, int64_t ldo, int method, void* ws,
               hipStream_t st)
{
    Carver c(ws);
    AdjWs w;
    adj_carve(c, F, w);
    const int64_t np = adj_npairs(F), N = adj_n(F);
    hipLaunchKernelGGL(k_adj_pad, dim3((unsigned)ceil_div(N - np, 256) + 1), dim3(256), 0, st, w.keys, w.vals, np,
                       N);
    NAPY_TRY(check_launch("adjust pad"));
    if (F > 1) {
        hipLaunchKernelGGL(k_adj_gather, dim3((unsigned)(F - 1)), dim3(256), 0, st, p, F, ldp, w.keys, w.vals,
                           w.rowm);
        NAPY_TRY(check_launch("adjust gather"));
    }
    hipLaunchKernelGGL(k_adj_factor, dim3(1), dim3(256), 0, st, w.rowm, F - 1, method, w.m, w.factor);
    NAPY_TRY(check_launch("adjust factor"));
    if (np > 0) {
        if (method == NAPY_ADJ_BONFERRONI) {
            hipLaunchKernelGGL(k_adj_bonferroni, dim3((unsigned)ceil_div(np, 256)), dim3(256), 0, st, w.keys, w.vals,
                               w.factor, np, F, out, ldo);
            NAPY_TRY(check_launch("adjust bonferroni"));
        } else {
            const unsigned ntiles = (unsigned)(N / ADJ_TILE);
            hipLaunchKernelGGL(k_bitonic_tile, dim3(ntiles), dim3(ADJ_TILE_THREADS), 0, st, w.keys, w.vals,
                               (int64_t)0);
            NAPY_TRY(check_launch("adjust sort tiles"));
            for (int64_t k = 2 * (int64_t)ADJ_TILE; k <= N; k <<= 1) {
                // global strides k/2 .. ADJ_TILE, up to three per pass
                int lj = 0;
                while (((int64_t)1 << lj) < (k >> 1)) ++lj;
                int ltile = 0;
                while (((int64_t)1 << ltile) < ADJ_TILE) ++ltile;
                while (lj >= ltile) {
                    const int R = lj - ltile + 1 >= 3 ? 3 : lj - ltile + 1;
                    const int64_t ng = N >> R;
                    const unsigned nb = (unsigned)ceil_div(ng, 256);
                    if (R == 3) hipLaunchKernelGGL(k_bitonic_multi<3>, dim3(nb), dim3(256), 0, st, w.keys, w.vals, lj, k, ng);
                    else if (R == 2) hipLaunchKernelGGL(k_bitonic_multi<2>, dim3(nb), dim3(256), 0, st, w.keys, w.vals, lj, k, ng);
                    else hipLaunchKernelGGL(k_bitonic_multi<1>, dim3(nb), dim3(256), 0, st, w.keys, w.vals, lj, k, ng);
                    NAPY_TRY(check_launch("adjust sort step"));
                    lj -= R;
                }
                hipLaunchKernelGGL(k_bitonic_tile, dim3(ntiles), dim3(ADJ_TILE_THREADS), 0, st, w.keys, w.vals, k);
                NAPY_TRY(check_launch("adjust sort merge"));
            }
            const int64_t nb = N / ADJ_SCAN;
            hipLaunchKernelGGL(k_adj_scale, dim3((unsigned)nb), dim3(ADJ_SCAN_THREADS), 0, st, w.keys, w.m, w.factor,
                               w.bmin);
            NAPY_TRY(check_launch("adjust scale"));
            hipLaunchKernelGGL(k_adj_blocks, dim3(1), dim3(ADJ_SCAN_THREADS), 0, st, w.bmin, nb);
            NAPY_TRY(check_launch("adjust blocks"));
            hipLaunchKernelGGL(k_adj_scatter, dim3((unsigned)ceil_div(np, 256)), dim3(256), 0, st, w.keys, w.vals,
                               w.bmin, w.m, np, F, out, ldo);
            NAPY_TRY(check_launch("adjust scatter"));
        }
    }
    hipLaunchKernelGGL(k_adj_diag, dim3((unsigned)ceil_div(F, 256)), dim3(256), 0, st, out, F, ldo);
    return check_launch("adjust diagonal");
}

}  // namespace napy
