// Backward of the pairwise-deletion Pearson matrix (the derivative of the
// Section 3.5.2 definition of NApy, arXiv 2505.00448; the paper itself has no
// gradient).
//
// For a pair (g, h) with sums over I(g,h) on centred data (n, Sx, Sy, Sxx,
// Syy, Sxy), C = n Sxy - Sx Sy, Vx = n Sxx - Sx^2, Vy = n Syy - Sy^2 and
// r = C / sqrt(Vx Vy), the derivative for a sample i in I(g,h) is
//     dr/dx_ig = (n x_ih - Sy) / sqrt(Vx Vy) - r (n x_ig - Sx) / Vx .
// With G = dR + dR' (diagonal excluded: r_gg is constant) and per ordered pair
//     A_gh = G_gh n / sqrt(Vx Vy)
//     B_gh = G_gh (-Sy / sqrt(Vx Vy) + r Sx / Vx)
//     Q_gh = -G_gh r n / Vx
// the gradient is
//     dX = M o (X0 A' + M B' + X0 o (M Q'))
// with X0 the zero-filled centred data and M the presence mask: three
// [S x F] x [F x F] products and an elementwise epilogue.  Because r is
// invariant to the per-column centring, this is also the gradient for the raw
// data.  Pairs whose forward r is undefined (NaN) contribute nothing; missing
// entries get 0.
//
//   k_bwd_coef   FP64 per-pair coefficients from the saved forward sums and
//                the forward's r, stored as FP32 [F][F] matrices.
//   k_bwd_mfma   64 x 64 (samples x variables) output tiles on
//                v_mfma_f32_16x16x4_f32, contraction over partners h.
#include "napy_internal.hpp"

namespace napy {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_bwd_coef(const double* __restrict__ saved, const float* __restrict__ dR,
                                                  int64_t ldr, int64_t F, float* __restrict__ Ac,
                                                  float* __restrict__ Bc, float* __restrict__ Qc)
{
    const int64_t h = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t g = blockIdx.y;
    if (h >= F) return;
    const int64_t FF = F * F, e = g * F + h;
    float a = 0.f, b = 0.f, q = 0.f;
    if (g != h) {
        const double n = saved[e], sx = saved[FF + e], sy = saved[2 * FF + e];
        const double sxx = saved[3 * FF + e], syy = saved[4 * FF + e];
        const double r = saved[6 * FF + e];  // the forward's r (NaN: undefined)
        const double vx = n * sxx - sx * sx, vy = n * syy - sy * sy;
        if (r == r && vx > 0.0 && vy > 0.0) {
            const double G = (double)dR[g * ldr + h] + (double)dR[h * ldr + g];
            const double rs = sqrt(vx * vy);
            a = (float)(G * n / rs);
            b = (float)(G * (-sy / rs + r * sx / vx));
            q = (float)(-G * r * n / vx);
        }
    }
    Ac[e] = a;
    Bc[e] = b;
    Qc[e] = q;
}

constexpr int BT = 64;   // output tile
constexpr int BKH = 32;  // partners per slab
constexpr int LDH = 36;

__global__ __launch_bounds__(256) void k_bwd_mfma(const float* __restrict__ X, int64_t S, int64_t F,
                                                  int64_t ldx, int use_sent, float sent,
                                                  const float* __restrict__ mu32, const double* __restrict__ mu64,
                                                  int center64, const float* __restrict__ Ac,
                                                  const float* __restrict__ Bc, const float* __restrict__ Qc,
                                                  float* __restrict__ dX, int64_t lddx)
{
    __shared__ __attribute__((aligned(16))) float sx[BT * LDH];      // x0 with NaN for missing: [i][h]
    __shared__ __attribute__((aligned(16))) float sc[3][BT * LDH];   // coefficients: [g][h]
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t i0 = (int64_t)blockIdx.x * BT, g0 = (int64_t)blockIdx.y * BT;
    // centring must match the forward's: float mean for FP32/BF16X3, double
    // mean (then rounded) for FP64
    auto centre = [&](float raw, int64_t c) -> float {
        return center64 ? (float)((double)raw - mu64[c]) : raw - mu32[c];
    };

    f32x4 acc[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[s][k] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int hh = tid & 31, rr0 = tid >> 5;  // staging: column hh, rows rr0 + 8 j
    for (int64_t h0 = 0; h0 < F; h0 += BKH) {
        const int64_t h = h0 + hh;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int rr = rr0 + 8 * j;
            const int64_t i = i0 + rr, g = g0 + rr;
            float v = __builtin_nanf("");
            if (i < S && h < F) {
                const float raw = X[i * ldx + h];
                if (!is_missing(raw, use_sent, sent)) v = centre(raw, h);
            }
            sx[rr * LDH + hh] = v;
            const bool okc = (g < F && h < F);
            sc[0][rr * LDH + hh] = okc ? Ac[g * F + h] : 0.f;
            sc[1][rr * LDH + hh] = okc ? Bc[g * F + h] : 0.f;
            sc[2][rr * LDH + hh] = okc ? Qc[g * F + h] : 0.f;
        }
        __syncthreads();
        const int r16 = lane & 15, kq = lane >> 4;
#pragma unroll
        for (int kk = 0; kk < BKH / 4; ++kk) {
            const int k = kk * 4 + kq;
            float xa[2], ma[2], cb[2][3];
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                const float v = sx[(wm * 32 + s2 * 16 + r16) * LDH + k];
                const bool pr = v == v;
                xa[s2] = pr ? v : 0.f;
                ma[s2] = pr ? 1.f : 0.f;
#pragma unroll
                for (int c = 0; c < 3; ++c) cb[s2][c] = sc[c][(wn * 32 + s2 * 16 + r16) * LDH + k];
            }
#pragma unroll
            for (int ia = 0; ia < 2; ++ia)
#pragma unroll
                for (int ib = 0; ib < 2; ++ib) {
                    const int s = ia * 2 + ib;
                    acc[s][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[ia], cb[ib][0], acc[s][0], 0, 0, 0);
                    acc[s][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(ma[ia], cb[ib][1], acc[s][1], 0, 0, 0);
                    acc[s][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(ma[ia], cb[ib][2], acc[s][2], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    // epilogue: dX[i][g] = m_ig (P1 + P2 + x0_ig P3)
#pragma unroll
    for (int ia = 0; ia < 2; ++ia)
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + wm * 32 + ia * 16 + 4 * (lane >> 4) + r;
                const int64_t g = g0 + wn * 32 + ib * 16 + (lane & 15);
                if (i < S && g < F) {
                    const float raw = X[i * ldx + g];
                    float out = 0.f;
                    if (!is_missing(raw, use_sent, sent)) {
                        const float x0 = centre(raw, g);
                        const int s = ia * 2 + ib;
                        out = acc[s][0][r] + acc[s][1][r] + x0 * acc[s][2][r];
                    }
                    dX[i * lddx + g] = out;
                }
            }
}

struct BwdWs {
    ColStats cs;
    float *Ac, *Bc, *Qc;
};

static void bwd_carve(Carver& c, int64_t S, int64_t F, BwdWs& w)
{
    colstats_carve(c, S, F, w.cs);
    w.Ac = c.take<float>((size_t)F * F);
    w.Bc = c.take<float>((size_t)F * F);
    w.Qc = c.take<float>((size_t)F * F);
}

size_t backward_ws_bytes(int64_t S, int64_t F)
{
    Carver c(nullptr);
    BwdWs w;
    bwd_carve(c, S, F, w);
    return c.bytes();
}

int backward_run(const float* X, int64_t S, int64_t F, int64_t ldx, const double* saved, const float* dR,
                 int64_t ldr, float* dX, int64_t lddx, void* ws, const napy_opts* opts, hipStream_t st)
{
    Carver c(ws);
    BwdWs w;
    bwd_carve(c, S, F, w);
    const int us = opt_use_sent(opts);
    const float sv = opt_sent(opts);
    NAPY_TRY(colstats_launch(X, S, F, ldx, us, sv, w.cs, st));
    hipLaunchKernelGGL(k_bwd_coef, dim3((unsigned)ceil_div(F, 256), (unsigned)F), dim3(256), 0, st, saved, dR,
                       ldr, F, w.Ac, w.Bc, w.Qc);
    NAPY_TRY(check_launch("bwd_coef"));
    if (S == 0) return NAPY_OK;
    hipLaunchKernelGGL(k_bwd_mfma, dim3((unsigned)ceil_div(S, BT), (unsigned)ceil_div(F, BT)), dim3(256), 0, st,
                       X, S, F, ldx, us, sv, w.cs.mu32, w.cs.mu64, opt_prec(opts) == NAPY_PREC_FP64 ? 1 : 0,
                       w.Ac, w.Bc, w.Qc, dX, lddx);
    return check_launch("bwd_mfma");
}

}  // namespace napy
