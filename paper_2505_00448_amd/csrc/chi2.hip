// Chi-squared test of independence between categorical features with
// pairwise deletion (NApy, Section 3.5), all pairs of one label-encoded
// matrix, with Cramer's V (phi for 2 x 2 tables, Table 2).
//
// The contingency table of a pair (g, h) on I(g, h) has the counts
//   O_kl(g, h) = sum_i [L_ig = k] [L_ih = l],
// a contraction over the samples of the 0/1 category indicators of both
// features (one "expanded" column e = g ncat + k per feature and label, zero
// where the label is missing).  The counts run on FP64 MFMA
// (v_mfma_f64_16x16x4f64, exact integers) as 64 x 64 tiles of the upper
// triangle of the expanded columns (the counts are symmetric, so entry
// (e1, e2) is read at (min, max)).  One thread per pair then forms
// the table's margins, chi2 = sum (O - E)^2 / E, p = Q(df/2, chi2/2), V and n,
// and writes both (g, h) and (h, g).
#include "napy_internal.hpp"
#include "pvalue.hpp"

namespace napy {

typedef double cf64x4 __attribute__((ext_vector_type(4)));

constexpr int CHI_TILE = 64;
constexpr int CHI_BK = 16;
constexpr int CHI_LDK = 18;
constexpr int CHI_RPT = 4;

struct ChiPlan {
    int64_t E;  // F * ncat
    int T;      // tiles per side
    int ntiles; // T (T + 1) / 2
    int nsplit;
    int64_t ksplit;
};

struct ChiWs {
    uint64_t* catmask;  // [F]
    int32_t* bad;       // [F]
    double* part;       // [nsplit][E][E] (upper-triangle tiles written)
};

static ChiPlan chi_plan(int64_t S, int64_t F, int ncat)
{
    ChiPlan p;
    p.E = F * ncat;
    p.T = (int)ceil_div(p.E, CHI_TILE);
    p.ntiles = p.T * (p.T + 1) / 2;
    int64_t ns = ceil_div(1024, p.ntiles);
    const int64_t nmax = S / 256 > 1 ? S / 256 : 1;
    if (ns > nmax) ns = nmax;
    if (ns > 16) ns = 16;
    if (ns < 1) ns = 1;
    p.nsplit = (int)ns;
    p.ksplit = round_up(ceil_div(S > 0 ? S : 1, ns), CHI_BK);
    return p;
}

static void chi_carve(Carver& c, int64_t S, int64_t F, int ncat, ChiWs& w)
{
    const ChiPlan p = chi_plan(S, F, ncat);
    w.catmask = c.take<uint64_t>(F);
    w.bad = c.take<int32_t>(F);
    w.part = c.take<double>((size_t)p.nsplit * p.E * p.E);
}

size_t chi2_ws_bytes(int64_t S, int64_t F, int ncat)
{
    Carver c(nullptr);
    ChiWs w;
    chi_carve(c, S, F, ncat, w);
    return c.bytes();
}

// tile index t -> (tg, th), tg <= th, row-major over the upper triangle of T x T
__device__ __forceinline__ void chi_tile_coords(int t, int T, int& tg, int& th)
{
    int g = (int)((2.0 * T + 1.0 - sqrt((2.0 * T + 1.0) * (2.0 * T + 1.0) - 8.0 * t)) * 0.5);
    if (g < 0) g = 0;
    if (g > T - 1) g = T - 1;
    while (g > 0 && g * T - g * (g - 1) / 2 > t) --g;
    while (g + 1 < T && (g + 1) * T - (g + 1) * g / 2 <= t) ++g;
    tg = g;
    th = g + (t - (g * T - g * (g - 1) / 2));
}

__global__ __launch_bounds__(256) void k_chi2_tiles(const float* __restrict__ L, int64_t ldl, int64_t S, int ncat,
                                                    int use_sent, float sent, ChiPlan plan, double* __restrict__ part)
{
    const int nb = (int)gridDim.x;
    int lb = (int)blockIdx.x;
    {
        const int x = lb & 7, q = lb >> 3, base = nb >> 3, rem = nb & 7;
        lb = x * base + (x < rem ? x : rem) + q;
    }
    const int split = lb % plan.nsplit, t = lb / plan.nsplit;
    int tg, th;
    chi_tile_coords(t, plan.T, tg, th);
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;

    const int64_t kbeg = (int64_t)split * plan.ksplit;
    const int64_t kend = min(S, kbeg + plan.ksplit);
    const int nslab = kend > kbeg ? (int)ceil_div(kend - kbeg, CHI_BK) : 0;

    const int sc = tid & 63, kg = tid >> 6;
    int64_t col[2];
    float kcat[2];
    bool ok[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int64_t e = (int64_t)(side ? th : tg) * CHI_TILE + sc;
        ok[side] = e < plan.E;
        col[side] = ok[side] ? e / ncat : 0;
        kcat[side] = ok[side] ? (float)(e % ncat) : -1.0f;
    }

    __shared__ __attribute__((aligned(16))) double lds[2][2][CHI_TILE * CHI_LDK];
    float raw[2][CHI_RPT];
    auto load_raw = [&](int slab) {
        const int64_t i0 = kbeg + (int64_t)slab * CHI_BK + kg * CHI_RPT;
#pragma unroll
        for (int side = 0; side < 2; ++side)
#pragma unroll
            for (int j = 0; j < CHI_RPT; ++j) {
                const int64_t i = i0 + j;
                raw[side][j] = (i < kend && ok[side]) ? L[i * ldl + col[side]] : __builtin_nanf("");
            }
    };
    auto store_lds = [&](int buf) {
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            double* d = &lds[buf][side][sc * CHI_LDK + kg * CHI_RPT];
#pragma unroll
            for (int j = 0; j < CHI_RPT; ++j)
                d[j] = (!is_missing(raw[side][j], use_sent, sent) && raw[side][j] == kcat[side]) ? 1.0 : 0.0;
        }
    };

    cf64x4 acc[4];
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) acc[s4] = cf64x4{0.0, 0.0, 0.0, 0.0};
    auto compute = [&](int buf) {
        const int rr = lane & 15, kq = lane >> 4;
#pragma unroll
        for (int kk = 0; kk < CHI_BK / 4; ++kk) {
            const int k = kk * 4 + kq;
            double a[2], b[2];
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                a[s2] = lds[buf][0][(wm * 32 + s2 * 16 + rr) * CHI_LDK + k];
                b[s2] = lds[buf][1][(wn * 32 + s2 * 16 + rr) * CHI_LDK + k];
            }
#pragma unroll
            for (int ia = 0; ia < 2; ++ia)
#pragma unroll
                for (int ib = 0; ib < 2; ++ib)
                    acc[ia * 2 + ib] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ia], b[ib], acc[ia * 2 + ib], 0, 0, 0);
        }
    };

    if (nslab > 0) {
        load_raw(0);
        store_lds(0);
        __syncthreads();
        for (int s = 0; s < nslab; ++s) {
            const bool more = s + 1 < nslab;
            if (more) load_raw(s + 1);
            compute(s & 1);
            if (more) store_lds((s + 1) & 1);
            __syncthreads();
        }
    }
    double* dst = part + (int64_t)split * plan.E * plan.E;
#pragma unroll
    for (int ia = 0; ia < 2; ++ia)
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t e1 = (int64_t)tg * CHI_TILE + wm * 32 + ia * 16 + (lane >> 4) + 4 * r;
                const int64_t e2 = (int64_t)th * CHI_TILE + wn * 32 + ib * 16 + (lane & 15);
                if (e1 < plan.E && e2 < plan.E) dst[e1 * plan.E + e2] = acc[ia * 2 + ib][r];
            }
}

// pair (g, h), g <= h: h = blockIdx.x * 256 + threadIdx.x, g = blockIdx.y
__global__ __launch_bounds__(256) void k_chi2_combine(const double* __restrict__ part, ChiPlan plan, int64_t F,
                                                      int ncat, const uint64_t* __restrict__ catmask,
                                                      const int32_t* __restrict__ bad, double* __restrict__ chi,
                                                      double* __restrict__ pv, double* __restrict__ cv,
                                                      int32_t* __restrict__ nout, int64_t ldo)
{
    const int64_t h = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t g = blockIdx.y;
    if (h >= F || h < g) return;
    double c2 = NAN, p = NAN, v = NAN;
    int64_t nn = 0;
    if (bad[g] == 0 && bad[h] == 0) {
        const uint64_t mg = catmask[g], mh = catmask[h];
        const int r = __popcll(mg), c = __popcll(mh);
        auto O = [&](int k, int l) {
            // counts are symmetric; only e1 <= e2 is stored (a feature's own
            // expanded columns may straddle two tiles)
            const int64_t ea = g * ncat + k, eb = h * ncat + l;
            const int64_t e1 = min(ea, eb), e2 = max(ea, eb);
            double s = 0.0;
            for (int sp = 0; sp < plan.nsplit; ++sp) s += part[(int64_t)sp * plan.E * plan.E + e1 * plan.E + e2];
            return s;
        };
        double R[32], C[32];
        for (int k = 0; k < ncat; ++k) R[k] = C[k] = 0.0;
        double N = 0.0;
        for (int k = 0; k < ncat; ++k)
            for (int l = 0; l < ncat; ++l) {
                if (!((mg >> k) & 1ull) || !((mh >> l) & 1ull)) continue;
                const double o = O(k, l);
                R[k] += o;
                C[l] += o;
                N += o;
            }
        nn = (int64_t)N;
        bool empty = false;
        for (int k = 0; k < ncat; ++k) {
            if (((mg >> k) & 1ull) && R[k] < 0.5) empty = true;
            if (((mh >> k) & 1ull) && C[k] < 0.5) empty = true;
        }
        if (!empty && N > 0.5) {
            double s = 0.0;
            for (int k = 0; k < ncat; ++k)
                for (int l = 0; l < ncat; ++l) {
                    if (!((mg >> k) & 1ull) || !((mh >> l) & 1ull)) continue;
                    const double E = R[k] * C[l] / N;
                    const double d = O(k, l) - E;
                    s += d * d / E;
                }
            c2 = s;
            if (r >= 2 && c >= 2) {
                p = chi2_sf(c2, (double)((r - 1) * (c - 1)));
                v = sqrt(c2 / (N * (double)min(r - 1, c - 1)));
            }
        }
    }
    chi[g * ldo + h] = c2;
    chi[h * ldo + g] = c2;
    pv[g * ldo + h] = p;
    pv[h * ldo + g] = p;
    cv[g * ldo + h] = v;
    cv[h * ldo + g] = v;
    nout[g * ldo + h] = (int32_t)nn;
    nout[h * ldo + g] = (int32_t)nn;
}

int chi2_run(const float* L, int64_t ldl, int64_t S, int64_t F, int ncat, double* chi, double* p, double* v,
             int32_t* n, int64_t ldo, void* ws, const napy_opts* opts, hipStream_t st)
{
    const int us = opt_use_sent(opts);
    const float sv = opt_sent(opts);
    Carver c(ws);
    ChiWs w;
    chi_carve(c, S, F, ncat, w);
    const ChiPlan plan = chi_plan(S, F, ncat);
    NAPY_TRY(labels_launch(L, ldl, S, F, ncat, us, sv, w.catmask, w.bad, st));
    hipLaunchKernelGGL(k_chi2_tiles, dim3((unsigned)((int64_t)plan.ntiles * plan.nsplit)), dim3(256), 0, st, L, ldl,
                       S, ncat, us, sv, plan, w.part);
    NAPY_TRY(check_launch("chi2 tiles"));
    hipLaunchKernelGGL(k_chi2_combine, dim3((unsigned)ceil_div(F, 256), (unsigned)F), dim3(256), 0, st, w.part,
                       plan, F, ncat, w.catmask, w.bad, chi, p, v, n, ldo);
    return check_launch("chi2 combine");
}

}  // namespace napy
