// Categorical x continuous tests with pairwise deletion (NApy, Section 3.5):
// two-sample t-test (Student or Welch) and one-way ANOVA.
//
// For a categorical column g with labels 0 .. ncat-1 and a continuous column
// h, the pair's samples I(g, h) fall into groups by label; every test needs,
// per group k, the count n_k, the sum s1_k and the sum of squares s2_k of
// the values, taken here about the column's observed mean mu_h (shifting the
// values changes no statistic and keeps s2_k - s1_k^2 / n_k well
// conditioned).  These are contractions over the samples:
//   n_k(g, h)  = sum_i [L_ig = k] m_ih
//   s1_k(g, h) = sum_i [L_ig = k] (x_ih - mu_h) m_ih
//   s2_k(g, h) = sum_i [L_ig = k] (x_ih - mu_h)^2 m_ih
// with the 0/1 group indicator of an "expanded" categorical column e =
// g ncat + k (zero where L_ig is missing) and the presence m_ih of x_ih.  They
// run on FP64 MFMA (v_mfma_f64_16x16x4f64): the indicator products are
// exact, and the sums keep FP64 accuracy, so the undefined cases can be
// decided with FP64 thresholds.
//
// Kernels, in stream order:
//   colstats (shared)  observed mean of each continuous column.
//   k_grp_labels       per categorical column: the observed labels (bit mask)
//                      and whether every label is an integer in [0, ncat).
//   k_grp_tiles        64 expanded columns x 64 continuous columns per
//                      workgroup over a range of samples (split over the
//                      samples to fill the GPU): FP64 partial sums.
//   k_grp_combine      per (g, h): sums over the splits, then the statistic,
//                      its p-value and n = |I(g, h)|.
#include "napy_internal.hpp"
#include "pvalue.hpp"

namespace napy {

typedef double gf64x4 __attribute__((ext_vector_type(4)));

constexpr int GRP_TILE = 64;
constexpr int GRP_BK = 16;   // samples per LDS slab (four MFMA k-steps)
constexpr int GRP_LDK = 18;  // LDS row stride in doubles
constexpr int GRP_RPT = 4;   // rows per thread in the staging step
constexpr int GRP_NSTAT = 3; // n, s1, s2

// Zero-variance and equal-mean decisions on FP64 sums: a group's sum of
// squared deviations is zero when it is at most GRP_TAU times its sum of
// squares about mu_h, and two means are equal when they differ by at most
// GRP_TAU of their size.  A constant group of n samples leaves a rounding
// residue of at most about n * 1.1e-16 of its sum of squares (linear error
// growth of the FP64 sums), so 1e-10 decides correctly up to about 1e6
// samples per group.
constexpr double GRP_TAU = 1e-10;

struct GrpPlan {
    int64_t E;        // expanded categorical columns FC * ncat
    int tiles_e, tiles_h, nsplit;
    int64_t ksplit;   // samples per split
};

struct GrpWs {
    ColStats cs;
    uint64_t* catmask;  // [FC]
    int32_t* bad;       // [FC]
    double* part;       // [nsplit][3][E][FQ]
};

static GrpPlan grp_plan(int64_t S, int64_t FC, int64_t FQ, int ncat)
{
    GrpPlan p;
    p.E = FC * ncat;
    p.tiles_e = (int)ceil_div(p.E, GRP_TILE);
    p.tiles_h = (int)ceil_div(FQ, GRP_TILE);
    const int64_t tiles = (int64_t)p.tiles_e * p.tiles_h;
    // about 1024 workgroups (four per CU), at least 256 samples each
    int64_t ns = ceil_div(1024, tiles);
    const int64_t nmax = S / 256 > 1 ? S / 256 : 1;
    if (ns > nmax) ns = nmax;
    if (ns > 16) ns = 16;
    if (ns < 1) ns = 1;
    p.nsplit = (int)ns;
    p.ksplit = round_up(ceil_div(S > 0 ? S : 1, ns), GRP_BK);
    return p;
}

static void grp_carve(Carver& c, int64_t S, int64_t FC, int64_t FQ, int ncat, GrpWs& w)
{
    const GrpPlan p = grp_plan(S, FC, FQ, ncat);
    colstats_carve(c, S, FQ, w.cs);
    w.catmask = c.take<uint64_t>(FC);
    w.bad = c.take<int32_t>(FC);
    w.part = c.take<double>((size_t)p.nsplit * GRP_NSTAT * p.E * FQ);
}

size_t groups_ws_bytes(int64_t S, int64_t FC, int64_t FQ, int ncat)
{
    Carver c(nullptr);
    GrpWs w;
    grp_carve(c, S, FC, FQ, ncat, w);
    return c.bytes();
}

__global__ __launch_bounds__(256) void k_grp_zero(uint64_t* __restrict__ catmask, int32_t* __restrict__ bad,
                                                  int64_t FC)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g < FC) {
        catmask[g] = 0ull;
        bad[g] = 0;
    }
}

// 64 columns x 4 row lanes per workgroup, blockIdx.y: a range of 256 rows
__global__ __launch_bounds__(256) void k_grp_labels(const float* __restrict__ L, int64_t S, int64_t FC,
                                                    int64_t ldl, int ncat, int use_sent, float sent,
                                                    uint64_t* __restrict__ catmask, int32_t* __restrict__ bad)
{
    const int c = threadIdx.x & 63, rl = threadIdx.x >> 6;
    const int64_t g = (int64_t)blockIdx.x * 64 + c;
    if (g >= FC) return;
    const int64_t r0 = (int64_t)blockIdx.y * 256, r1 = min(S, r0 + 256);
    uint64_t mask = 0ull;
    int nb = 0;
    for (int64_t i = r0 + rl; i < r1; i += 4) {
        const float v = L[i * ldl + g];
        if (is_missing(v, use_sent, sent)) continue;
        if (v >= 0.0f && v < (float)ncat && v == floorf(v))
            mask |= 1ull << (int)v;
        else
            nb = 1;
    }
    if (mask) atomicOr((unsigned long long*)&catmask[g], (unsigned long long)mask);
    if (nb) atomicOr(&bad[g], 1);
}

// One 64 x 64 block of (expanded categorical column e, continuous column h)
// over one range of samples; four waves, each a 32 x 32 quadrant of 16 x 16
// MFMA blocks.  LDS holds one slab per side: the indicators of the 64
// expanded columns and the centred values of the 64 continuous columns
// (NaN where missing), double-buffered.
__global__ __launch_bounds__(256) void k_grp_tiles(const float* __restrict__ L, int64_t ldl,
                                                    const float* __restrict__ X, int64_t ldx, int64_t S,
                                                    int64_t FC, int64_t FQ, int ncat, int use_sent, float sent,
                                                    const double* __restrict__ mu, GrpPlan plan,
                                                    double* __restrict__ part)
{
    const int nb = (int)gridDim.x;
    int lb = (int)blockIdx.x;
    {
        // every XCD (blocks are dealt round-robin) takes a contiguous range
        const int x = lb & 7, q = lb >> 3, base = nb >> 3, rem = nb & 7;
        lb = x * base + (x < rem ? x : rem) + q;
    }
    const int split = lb % plan.nsplit, t = lb / plan.nsplit;
    const int te = t / plan.tiles_h, th = t % plan.tiles_h;
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;

    const int64_t kbeg = (int64_t)split * plan.ksplit;
    const int64_t kend = min(S, kbeg + plan.ksplit);
    const int nslab = kend > kbeg ? (int)ceil_div(kend - kbeg, GRP_BK) : 0;

    // staging: column sc of each panel, rows kg*RPT .. +RPT of the slab
    const int sc = tid & 63, kg = tid >> 6;
    const int64_t e = (int64_t)te * GRP_TILE + sc;
    const bool okE = e < plan.E;
    const int64_t g = okE ? e / ncat : 0;
    const float kcat = okE ? (float)(e % ncat) : -1.0f;
    const int64_t h = (int64_t)th * GRP_TILE + sc;
    const bool okH = h < FQ;
    const double muh = okH ? mu[h] : 0.0;

    __shared__ __attribute__((aligned(16))) double lds[2][2][GRP_TILE * GRP_LDK];
    float rawA[GRP_RPT], rawB[GRP_RPT];

    auto load_raw = [&](int slab) {
        const int64_t i0 = kbeg + (int64_t)slab * GRP_BK + kg * GRP_RPT;
#pragma unroll
        for (int j = 0; j < GRP_RPT; ++j) {
            const int64_t i = i0 + j;
            const bool in = i < kend;
            rawA[j] = (in && okE) ? L[i * ldl + g] : __builtin_nanf("");
            rawB[j] = (in && okH) ? X[i * ldx + h] : __builtin_nanf("");
        }
    };
    auto store_lds = [&](int buf) {
        double* a = &lds[buf][0][sc * GRP_LDK + kg * GRP_RPT];
        double* b = &lds[buf][1][sc * GRP_LDK + kg * GRP_RPT];
#pragma unroll
        for (int j = 0; j < GRP_RPT; ++j) {
            const bool ia = !is_missing(rawA[j], use_sent, sent) && rawA[j] == kcat;
            a[j] = ia ? 1.0 : 0.0;
            b[j] = is_missing(rawB[j], use_sent, sent) ? __builtin_nan("") : (double)rawB[j] - muh;
        }
    };

    gf64x4 acc[4][GRP_NSTAT];
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int s = 0; s < GRP_NSTAT; ++s) acc[s4][s] = gf64x4{0.0, 0.0, 0.0, 0.0};

    auto compute = [&](int buf) {
        const int rr = lane & 15, kq = lane >> 4;
#pragma unroll
        for (int kk = 0; kk < GRP_BK / 4; ++kk) {
            const int k = kk * 4 + kq;
            double av[2], mb[2], xb[2], qb[2];
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                av[s2] = lds[buf][0][(wm * 32 + s2 * 16 + rr) * GRP_LDK + k];
                const double vb = lds[buf][1][(wn * 32 + s2 * 16 + rr) * GRP_LDK + k];
                const bool pb = vb == vb;
                mb[s2] = pb ? 1.0 : 0.0;
                xb[s2] = pb ? vb : 0.0;
                qb[s2] = xb[s2] * xb[s2];
            }
#pragma unroll
            for (int ia = 0; ia < 2; ++ia)
#pragma unroll
                for (int ib = 0; ib < 2; ++ib) {
                    gf64x4* c = acc[ia * 2 + ib];
                    c[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ia], mb[ib], c[0], 0, 0, 0);
                    c[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ia], xb[ib], c[1], 0, 0, 0);
                    c[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ia], qb[ib], c[2], 0, 0, 0);
                }
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

    // FP64 partials [split][stat][e][h]; f64 16x16 blocks: rows lane/16 + 4r,
    // columns lane%16
#pragma unroll
    for (int s = 0; s < GRP_NSTAT; ++s) {
        double* dst = part + ((int64_t)split * GRP_NSTAT + s) * plan.E * FQ;
#pragma unroll
        for (int ia = 0; ia < 2; ++ia)
#pragma unroll
            for (int ib = 0; ib < 2; ++ib)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t ee = (int64_t)te * GRP_TILE + wm * 32 + ia * 16 + (lane >> 4) + 4 * r;
                    const int64_t hh = (int64_t)th * GRP_TILE + wn * 32 + ib * 16 + (lane & 15);
                    if (ee < plan.E && hh < FQ) dst[ee * FQ + hh] = acc[ia * 2 + ib][s][r];
                }
    }
}

struct GroupSums {
    double n, s1, s2;
};

__device__ inline GroupSums grp_sums(const double* __restrict__ part, const GrpPlan& plan, int64_t FQ, int64_t e,
                                     int64_t h)
{
    GroupSums r{0.0, 0.0, 0.0};
    for (int sp = 0; sp < plan.nsplit; ++sp) {
        const double* b = part + (int64_t)sp * GRP_NSTAT * plan.E * FQ + e * FQ + h;
        r.n += b[0];
        r.s1 += b[plan.E * FQ];
        r.s2 += b[2 * plan.E * FQ];
    }
    return r;
}

// sum of squared deviations about the group mean, with the zero decision
__device__ inline double grp_ss(const GroupSums& s, bool& zero)
{
    double ss = s.s2 - s.s1 * (s.s1 / s.n);
    if (ss < 0.0) ss = 0.0;
    zero = ss <= GRP_TAU * s.s2;
    return zero ? 0.0 : ss;
}

__device__ inline bool grp_means_equal(double a, double b)
{
    return fabs(a - b) <= GRP_TAU * fmax(fabs(a), fabs(b));
}

// test: 0 Student, 1 Welch, 2 ANOVA
__global__ __launch_bounds__(256) void k_grp_combine(const double* __restrict__ part, GrpPlan plan, int64_t FC,
                                                     int64_t FQ, int ncat, int test,
                                                     const uint64_t* __restrict__ catmask,
                                                     const int32_t* __restrict__ bad, double* __restrict__ stat,
                                                     double* __restrict__ pval, int32_t* __restrict__ nout,
                                                     int64_t ldo)
{
    const int64_t h = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t g = blockIdx.y;
    if (h >= FQ) return;
    double st = NAN, p = NAN;
    int64_t ntot = 0;
    const bool ok = bad[g] == 0;
    if (ok && test <= 1) {
        const GroupSums a = grp_sums(part, plan, FQ, g * ncat + 0, h);
        const GroupSums b = grp_sums(part, plan, FQ, g * ncat + 1, h);
        ntot = (int64_t)a.n + (int64_t)b.n;
        if (a.n >= 2.0 && b.n >= 2.0) {
            bool za, zb;
            const double ssa = grp_ss(a, za), ssb = grp_ss(b, zb);
            const double ma = a.s1 / a.n, mb = b.s1 / b.n;  // means about mu_h
            const double d = ma - mb;
            if (test == 0) {
                if (!(za && zb)) {
                    const double df = a.n + b.n - 2.0;
                    const double sp2 = (ssa + ssb) / df;
                    st = d / sqrt(sp2 * (1.0 / a.n + 1.0 / b.n));
                    p = fdist_sf(st * st, 1.0, df);
                }
            } else if (za && zb) {
                if (!grp_means_equal(ma, mb)) {
                    st = d > 0.0 ? INFINITY : -INFINITY;
                    p = 0.0;
                }
            } else {
                const double va = ssa / (a.n - 1.0) / a.n, vb = ssb / (b.n - 1.0) / b.n;
                st = d / sqrt(va + vb);
                const double df = (va + vb) * (va + vb) / (va * va / (a.n - 1.0) + vb * vb / (b.n - 1.0));
                p = fdist_sf(st * st, 1.0, df);
            }
        }
    } else if (ok) {
        const uint64_t cm = catmask[g];
        const int K = __popcll(cm);
        double N = 0.0, S1 = 0.0, ssw = 0.0, sq = 0.0;
        bool empty = false, allzero = true;
        double m0 = 0.0;
        bool first = true, alleq = true;
        for (int k = 0; k < ncat; ++k) {
            const GroupSums s = grp_sums(part, plan, FQ, g * ncat + k, h);
            ntot += (int64_t)s.n;
            if (!((cm >> k) & 1ull)) continue;  // not a category of this column
            if (s.n < 0.5) {
                empty = true;
                continue;
            }
            bool z;
            ssw += grp_ss(s, z);
            allzero = allzero && z;
            const double mk = s.s1 / s.n;
            if (first) {
                m0 = mk;
                first = false;
            } else if (!grp_means_equal(mk, m0)) {
                alleq = false;
            }
            N += s.n;
            S1 += s.s1;
            sq += s.s1 * (s.s1 / s.n);  // n_k m_k^2
        }
        if (!empty && K >= 2) {
            if (allzero) {
                if (!alleq) {
                    st = INFINITY;
                    p = 0.0;
                }
            } else {
                double ssb = sq - S1 * (S1 / N);
                if (ssb < 0.0) ssb = 0.0;
                const double df1 = (double)(K - 1), df2 = N - (double)K;
                st = (ssb / df1) / (ssw / df2);
                p = fdist_sf(st, df1, df2);
            }
        }
    }
    stat[g * ldo + h] = st;
    pval[g * ldo + h] = p;
    nout[g * ldo + h] = ok ? (int32_t)ntot : 0;
}

// per categorical column: observed-label mask and invalid-label flag
int labels_launch(const float* L, int64_t ldl, int64_t S, int64_t FC, int ncat, int use_sent, float sent,
                  uint64_t* catmask, int32_t* bad, hipStream_t st)
{
    hipLaunchKernelGGL(k_grp_zero, dim3((unsigned)ceil_div(FC, 256)), dim3(256), 0, st, catmask, bad, FC);
    NAPY_TRY(check_launch("labels zero"));
    if (S > 0) {
        hipLaunchKernelGGL(k_grp_labels, dim3((unsigned)ceil_div(FC, 64), (unsigned)ceil_div(S, 256)), dim3(256), 0,
                           st, L, S, FC, ldl, ncat, use_sent, sent, catmask, bad);
        NAPY_TRY(check_launch("labels"));
    }
    return NAPY_OK;
}

int groups_run(const float* L, int64_t ldl, const float* X, int64_t ldx, int64_t S, int64_t FC, int64_t FQ,
               int test, int ncat, double* stat, double* p, int32_t* n, int64_t ldo, void* ws, const napy_opts* opts,
               hipStream_t st)
{
    const int us = opt_use_sent(opts);
    const float sv = opt_sent(opts);
    Carver c(ws);
    GrpWs w;
    grp_carve(c, S, FC, FQ, ncat, w);
    const GrpPlan plan = grp_plan(S, FC, FQ, ncat);
    NAPY_TRY(colstats_launch(X, S, FQ, ldx, us, sv, w.cs, st));
    NAPY_TRY(labels_launch(L, ldl, S, FC, ncat, us, sv, w.catmask, w.bad, st));
    const int64_t nblk = (int64_t)plan.tiles_e * plan.tiles_h * plan.nsplit;
    hipLaunchKernelGGL(k_grp_tiles, dim3((unsigned)nblk), dim3(256), 0, st, L, ldl, X, ldx, S, FC, FQ, ncat, us, sv,
                       w.cs.mu64, plan, w.part);
    NAPY_TRY(check_launch("groups tiles"));
    hipLaunchKernelGGL(k_grp_combine, dim3((unsigned)ceil_div(FQ, 256), (unsigned)FC), dim3(256), 0, st, w.part,
                       plan, FC, FQ, ncat, test, w.catmask, w.bad, stat, p, n, ldo);
    return check_launch("groups combine");
}

}  // namespace napy
