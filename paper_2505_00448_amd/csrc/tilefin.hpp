// Output tiles of the correlation matrices: r, p and n of 32 x 32 pairs per
// workgroup, the p-value (NApy, arXiv 2505.00448, Sections 3.5.2 and 3.5.3)
// of every pair, and both triangles of the symmetric outputs.
//
// A workgroup of FT_THREADS threads owns the pairs (g0 + i, h0 + j) of one
// tile on or above the diagonal; thread t holds the pair (i, j) = (t / 32,
// t mod 32) for r and n.  The p-values' continued fractions take from 2 to
// about 28 steps, and a wave runs its slowest lane's count: the tile's
// pairs are therefore handed to the threads for p grouped by the expected
// count (a counting sort on six classes of the tail and of r^2 (a + 2.5)),
// so that a wave's lanes take similar counts.  The tile (row g0 + i) is
// written directly and its mirror (row h0 + j) through a transpose in LDS,
// so both writes are whole rows of 32 values.
#pragma once

#include "napy_internal.hpp"
#include "pvalue.hpp"

namespace napy {

constexpr int FT = 32;
constexpr int FT_THREADS = 1024;
constexpr int FT_K = FT * FT / FT_THREADS;  // pairs per thread

struct FinSmem {
    double r[FT][FT + 1];
    double v[FT][FT + 1];  // p
    int32_t n[FT][FT + 1];
    uint16_t order[FT * FT];  // pairs i * FT + j grouped by class
    uint32_t cls[8];          // per class: count, then first slot
};

static_assert(FT_THREADS == FT * FT, "one pair per thread");

// tile index -> (tg, th), tg <= th, row-major over the upper triangle of T x T
__host__ __device__ inline void tile_coords(int t, int T, int& tg, int& th)
{
    // start(g) = g*T - g*(g-1)/2
    int g = (int)((2.0f * T + 1.0f - sqrtf((2.0f * T + 1.0f) * (2.0f * T + 1.0f) - 8.0f * t)) * 0.5f);
    if (g < 0) g = 0;
    if (g > T - 1) g = T - 1;
    while (g > 0 && g * T - g * (g - 1) / 2 > t) --g;
    while (g + 1 < T && (g + 1) * T - (g + 1) * g / 2 <= t) ++g;
    tg = g;
    th = g + (t - (g * T - g * (g - 1) / 2));
}

// (tg, th), tg <= th -> tile index
__host__ __device__ inline int tile_index(int tg, int th, int T)
{
    return tg * T - tg * (tg - 1) / 2 + (th - tg);
}

// Launch order of the finish kernels' T (T + 1) / 2 tiles: the T (T - 1) / 2
// tiles off the diagonal first (row-major over tg < th), the T diagonal
// tiles last.  A diagonal tile holds about half the pairs, so when the tile
// count slightly exceeds the workgroups the GPU runs at once (528 tiles at
// T = 32 against 512 slots), the short second round is made of half tiles.
__device__ inline void finish_tile_coords(int b, int T, int& tg, int& th)
{
    const int noff = T * (T - 1) / 2;
    if (b >= noff) {
        tg = th = b - noff;
        return;
    }
    // off-diagonal tile b of the triangle of a (T - 1) x (T - 1) grid whose
    // row g holds the tiles (g, g + 1 .. T - 1)
    int g, hh;
    tile_coords(b, T - 1, g, hh);
    tg = g;
    th = hh + 1;
}

__device__ __forceinline__ int ft_row(int k) { return (int)(threadIdx.x >> 5) + (FT_THREADS / 32) * k; }
__device__ __forceinline__ int ft_col() { return (int)(threadIdx.x & 31); }

// pair k of the thread lies in the matrix and on or above the diagonal
__device__ __forceinline__ bool ft_valid(int64_t g0, int64_t h0, int64_t F, int k)
{
    const int64_t g = g0 + ft_row(k), h = h0 + ft_col();
    return g < F && h < F && (g0 != h0 || ft_row(k) <= ft_col());
}

// class of the continued fraction's expected step count: 0 none, 1-2 the
// complement tail (r^2 (a + 2.5) below or above 1.5), 3-5 the direct tail
// (above 10, 6 to 10, below 6)
__device__ __forceinline__ uint32_t ft_class(double r, int64_t n, bool n2one)
{
    if (n2one && n == 2 && r == r) return 0u;
    const CorrPSetup q = corr_p_params(r, n);
    if (q.done) return 0u;
    const double u = r * r * (0.5 * (double)(n - 2) + 2.5);
    if (!q.direct) return u < 1.5 ? 1u : 2u;
    return u >= 10.0 ? 3u : (u >= 6.0 ? 4u : 5u);
}

// p-values of the tile's valid pairs, from r and n in f (n2one: a pair of
// two samples with a defined r has p = 1, the Pearson rule; otherwise NaN),
// left in f.v.  Every thread of the workgroup calls it after writing its
// pair's r and n; it contains barriers, the caller synchronises again
// before reading f.v.
__device__ inline void ft_pvalues(FinSmem& f, const bool (&valid)[FT_K], bool n2one)
{
    const int t = threadIdx.x, i = ft_row(0), j = ft_col();
    if (t < 8) f.cls[t] = 0u;
    __syncthreads();
    uint32_t c = 7u, rank = 0u;  // class 7: invalid pair
    if (valid[0]) {
        c = ft_class(f.r[i][j], (int64_t)f.n[i][j], n2one);
        rank = atomicAdd(&f.cls[c], 1u);
    }
    __syncthreads();
    if (t == 0) {
        uint32_t run = 0u;
        for (int k = 0; k < 8; ++k) {
            const uint32_t cnt = f.cls[k];
            f.cls[k] = run;
            run += cnt;
        }
    }
    __syncthreads();
    if (valid[0]) f.order[f.cls[c] + rank] = (uint16_t)(i * FT + j);
    const uint32_t nvalid = f.cls[7];
    __syncthreads();
    if ((uint32_t)t < nvalid) {
        const int at = f.order[t], ii = at / FT, jj = at % FT;
        const int64_t n = f.n[ii][jj];
        const double rv = f.r[ii][jj];
        f.v[ii][jj] = (n2one && n == 2 && rv == rv) ? 1.0 : corr_pvalue(rv, n);
    }
}

// Writes r (f.r), p (f.v) and n (f.n) of the tile and of its mirror.  Call
// after a barrier that follows every thread's last write of f.
__device__ inline void ft_write(const FinSmem& f, int64_t g0, int64_t h0, int64_t F, double* __restrict__ r,
                                double* __restrict__ p, int32_t* __restrict__ n, int64_t ldo)
{
    const int j = ft_col();
#pragma unroll
    for (int k = 0; k < FT_K; ++k) {
        const int i = ft_row(k);
        // the tile: pair (i, j) at (g0 + i, h0 + j)
        if (ft_valid(g0, h0, F, k)) {
            const int64_t o = (g0 + i) * ldo + h0 + j;
            if (r) r[o] = f.r[i][j];
            if (p) p[o] = f.v[i][j];
            if (n) n[o] = f.n[i][j];
        }
        // the mirror: pair (j, i) at (h0 + i, g0 + j); on a diagonal tile
        // only below the diagonal
        const int64_t hm = h0 + i, gm = g0 + j;
        if (hm < F && gm < F && (g0 != h0 || j < i)) {
            const int64_t o = hm * ldo + gm;
            if (r) r[o] = f.r[j][i];
            if (p) p[o] = f.v[j][i];
            if (n) n[o] = f.n[j][i];
        }
    }
}

}  // namespace napy
