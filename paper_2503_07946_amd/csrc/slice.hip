// Conditional slicing of 7D Gaussians (Sec. 4.2; Algorithm 1 steps 3-6) and
// its reverse.  One lane per (frame, Gaussian); FP32 in and out, FP64 inside.
//
// Forward, per Gaussian, with P = (x, y, z), Q = (t, dx, dy, dz):
//   Sigma = L L^T (only the blocks needed are formed),
//   C = chol(Sigma_QQ), V = Sigma_PQ C^{-T}, u = C^{-1} r, r = (t - mu_t, d - mu_d),
//   mu_c = mu_p + V u                       (eq. cond_mean)
//   Sigma_c = Sigma_PP - V V^T              (eq. cond_cov)
//   alpha_c = alpha exp(-(lambda_t r_t^2 / Sigma_t + lambda_d delta^T Sigma_d^{-1} delta) / 2)
//                                           (eq. temp_mod x eq. dir_mod, marginal blocks)
// Loads are coalesced: each of the 36 input planes is read with consecutive
// lanes on consecutive Gaussians.
#include "common.h"
#include "gload.h"

namespace sd7 {

__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Sigma entry (a, b), a >= b, from the packed factor.
__device__ __forceinline__ double sig(const double* L, int a, int b)
{
    double s = 0.0;
#pragma unroll
    for (int k = 0; k <= b; ++k) s = fma(L[tri(a, k)], L[tri(b, k)], s);
    return s;
}

// View-independent part of the slice: Sigma blocks, chol(Sigma_QQ), V, and
// chol of the marginal direction block.
struct SliceFixed {
    double SPP[3][3];
    double SPQ[3][4];
    double C[4][4];     // chol(Sigma_QQ), lower
    double rC[4];       // 1 / C[k][k]
    double V[3][4];     // Sigma_PQ C^{-T}
    double CD[3][3];    // chol(Sigma_DD), lower
    double rCD[3];      // 1 / CD[k][k]
    double s_tt;        // Sigma_t
    bool ok;
};

// Per-view part: the residual r = (t - mu_t, d - mu_d) and what follows from it.
struct SliceView {
    double u[4];        // C^{-1} r
    double r[4];
    double y[3];        // Sigma_DD^{-1} delta (reverse pass only)
    double d[3];        // the direction conditioned on
    double rn;          // 1 / |mu_p - c| when d = unit(mu_p - c)
    double q_d;         // delta^T Sigma_DD^{-1} delta
    double e_t, e_d;    // exponents lambda_t r_t^2 / Sigma_t and lambda_d delta^T Sigma_d^{-1} delta
};

struct SliceState : SliceFixed, SliceView {
    double L[28];
};

__device__ __forceinline__ void load_L(const float* __restrict__ Lp, uint32_t n, uint32_t i, double L[28])
{
#pragma unroll
    for (int k = 0; k < 28; ++k) L[k] = (double)gload(Lp, (size_t)k * n + i);
}

__device__ __forceinline__ void slice_fixed(const double L[28], SliceFixed& S, uint32_t& flag)
{
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 7; ++k)
        if (!(L[tri(k, k)] > 0.0)) ok = false;
    if (!ok) flag |= SD7_FLAG_NONPOS_DIAG;

#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) S.SPP[a][b] = S.SPP[b][a] = sig(L, a, b);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q) S.SPQ[a][q] = sig(L, 3 + q, a);
    double SQQ[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) SQQ[a][b] = SQQ[b][a] = sig(L, 3 + a, 3 + b);
    S.s_tt = SQQ[0][0];

    // Cholesky of Sigma_QQ
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            double s = SQQ[a][b];
#pragma unroll
            for (int k = 0; k < b; ++k) s = fma(-S.C[a][k], S.C[b][k], s);
            if (a == b) {
                if (!(s > 0.0)) { ok = false; s = 1.0; }
                S.C[a][a] = sqrt(s);
                S.rC[a] = 1.0 / S.C[a][a];
            } else {
                S.C[a][b] = s * S.rC[b];
            }
        }
#pragma unroll
        for (int b = a + 1; b < 4; ++b) S.C[a][b] = 0.0;
    }
    // V rows: solve C v = Sigma_Q,a
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double s = S.SPQ[a][k];
#pragma unroll
            for (int m = 0; m < k; ++m) s = fma(-S.C[k][m], S.V[a][m], s);
            S.V[a][k] = s * S.rC[k];
        }
    // Cholesky of the marginal direction block Sigma_DD = SQQ[1:4, 1:4]
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            double s = SQQ[1 + a][1 + b];
#pragma unroll
            for (int k = 0; k < b; ++k) s = fma(-S.CD[a][k], S.CD[b][k], s);
            if (a == b) {
                if (!(s > 0.0)) { ok = false; s = 1.0; }
                S.CD[a][a] = sqrt(s);
                S.rCD[a] = 1.0 / S.CD[a][a];
            } else {
                S.CD[a][b] = s * S.rCD[b];
            }
        }
#pragma unroll
        for (int b = a + 1; b < 3; ++b) S.CD[a][b] = 0.0;
    }
    if (!(S.s_tt > 0.0)) ok = false;
    S.ok = ok;
}

// The direction Gaussian i is conditioned on: the view's d, or unit(mu_p - c)
// when the frame asks for one direction per Gaussian (then rn = 1/|mu_p - c|).
__device__ __forceinline__ void view_direction(const FrameDev& F, const float mu_p[3], double d[3], double& rn)
{
    if (F.d_mode) {
        double e[3], s = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            e[k] = (double)mu_p[k] - (double)F.c[k];
            s = fma(e[k], e[k], s);
        }
        rn = 1.0 / sqrt(s);
#pragma unroll
        for (int k = 0; k < 3; ++k) d[k] = e[k] * rn;
    } else {
        rn = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) d[k] = (double)F.d[k];
    }
}

// mu_t and mu_d of the Gaussian, t of the view, d from view_direction; y only
// if WITH_Y.
template <bool WITH_Y>
__device__ __forceinline__ void slice_view(const SliceFixed& S, double t, const double d[3], double rn,
                                           double mu_t, const double mu_d[3], float lambda_t, float lambda_d,
                                           SliceView& W)
{
#pragma unroll
    for (int k = 0; k < 3; ++k) W.d[k] = d[k];
    W.rn = rn;
    W.r[0] = t - mu_t;
#pragma unroll
    for (int k = 0; k < 3; ++k) W.r[1 + k] = d[k] - mu_d[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double s = W.r[k];
#pragma unroll
        for (int m = 0; m < k; ++m) s = fma(-S.C[k][m], W.u[m], s);
        W.u[k] = s * S.rC[k];
    }
    double z[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double s = W.r[1 + k];
#pragma unroll
        for (int m = 0; m < k; ++m) s = fma(-S.CD[k][m], z[m], s);
        z[k] = s * S.rCD[k];
    }
    W.q_d = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
    W.e_d = (double)lambda_d * W.q_d;
    if (WITH_Y) {
#pragma unroll
        for (int k = 2; k >= 0; --k) {  // y = CD^{-T} z = Sigma_DD^{-1} delta
            double s = z[k];
#pragma unroll
            for (int m = k + 1; m < 3; ++m) s = fma(-S.CD[m][k], W.y[m], s);
            W.y[k] = s * S.rCD[k];
        }
    }
    W.e_t = (double)lambda_t * W.r[0] * W.r[0] / S.s_tt;
}

template <bool WITH_Y>
__device__ __forceinline__ void slice_state(const FrameDev& F, uint32_t i, SliceState& S, uint32_t& flag)
{
    const uint32_t n = F.n;
    load_L(F.L, n, i, S.L);
    slice_fixed(S.L, S, flag);
    double mu_d[3], d[3], rn;
#pragma unroll
    for (int k = 0; k < 3; ++k) mu_d[k] = (double)gload(F.mu_d, (size_t)k * n + i);
    float mu_p[3] = {0.f, 0.f, 0.f};
    if (F.d_mode) {
#pragma unroll
        for (int k = 0; k < 3; ++k) mu_p[k] = gload(F.mu_p, (size_t)k * n + i);
    }
    view_direction(F, mu_p, d, rn);
    slice_view<WITH_Y>(S, (double)F.t, d, rn, (double)gload(F.mu_t, i), mu_d, F.lambda_t, F.lambda_d, S);
}

// Sigma_c = Sigma_PP - V V^T (eq. cond_cov), packed (xx, xy, xz, yy, yz, zz),
// rounded to FP32; returns whether every entry is finite.
__device__ __forceinline__ bool slice_cov(const SliceFixed& S, float cv[6])
{
    const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
    bool fin = true;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        double s = S.SPP[pa[e]][pb[e]];
#pragma unroll
        for (int k = 0; k < 4; ++k) s = fma(-S.V[pa[e]][k], S.V[pb[e]][k], s);
        fin = fin && isfinite(s);
        cv[e] = (float)s;
    }
    return fin;
}

// The FP32 outputs of one (frame, Gaussian): mu_c (eq. cond_mean), the packed
// Sigma_c, alpha_c; zeros (and a device flag) when the slice is undefined.
__device__ __forceinline__ void slice_outputs(const SliceFixed& S, const SliceView& W, const float mu_p[3],
                                              const float cv32[6], bool cv_fin, float alpha, float mc[3],
                                              float cv[6], float& ac, uint32_t& flag)
{
    double m[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double s = (double)mu_p[a];
#pragma unroll
        for (int k = 0; k < 4; ++k) s = fma(S.V[a][k], W.u[k], s);
        m[a] = s;
    }
    // e^{-(e_t + e_d)/2} = 2^t = 2^n 2^f with n = floor(t) and f = t - n in
    // [0, 1) exact in FP64; 2^f from the hardware exp2 in FP32 (relative
    // error about 1e-7, below the FP32 rounding of alpha_c); NaN passes on.
    const double t = -0.5 * 1.4426950408889634 * (W.e_t + W.e_d);
    double a_c = t;
    if (t == t) {
        const double n = floor(fmin(fmax(t, -1100.0), 1100.0));
        const float f = (float)(fmin(fmax(t, -1100.0), 1100.0) - n);
        a_c = ldexp((double)alpha * (double)__builtin_amdgcn_exp2f(f), (int)n);
    }
    const bool fin = isfinite(m[0]) && isfinite(m[1]) && isfinite(m[2]) && isfinite(a_c) && cv_fin;
    if (S.ok && !fin) flag |= SD7_FLAG_NONFINITE;
    if (!S.ok && !(flag & SD7_FLAG_NONPOS_DIAG)) flag |= SD7_FLAG_NONFINITE;
    const bool good = S.ok && fin;
#pragma unroll
    for (int a = 0; a < 3; ++a) mc[a] = good ? (float)m[a] : 0.0f;
#pragma unroll
    for (int e = 0; e < 6; ++e) cv[e] = good ? cv32[e] : 0.0f;
    ac = good ? (float)a_c : 0.0f;
}

// One atomic per wave for a frame's device flags.
__device__ __forceinline__ void wave_flags(uint32_t flag, uint32_t* __restrict__ counts, int f)
{
    const uint64_t any = __ballot(flag != 0);
    if (any) {
        uint32_t fl = flag;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) fl |= __shfl_xor(fl, off);
        if (__lane_id() == 0) atomicOr(&counts[f * SD7_CNT_WORDS + SD7_CNT_FLAGS], fl);
    }
}

__global__ __launch_bounds__(kBlock) void k_slice(const FrameDev* __restrict__ tab, BlockMap bm,
                                                  float* __restrict__ mu_c, float* __restrict__ cov_c,
                                                  float* __restrict__ alpha_c, uint32_t* __restrict__ counts)
{
    const int f = frame_of_block(bm, blockIdx.x);
    const FrameDev& F = tab[f];
    if (F.agr) return;  // uniform: refined and sliced by k_agr_slice
    const uint32_t i = (blockIdx.x - bm.start[f]) * kBlock + threadIdx.x;
    uint32_t flag = 0;
    if (i < F.n) {
        const uint32_t n = F.n;
        SliceState S;
        slice_state<false>(F, i, S, flag);
        float mu_p[3], cv32[6];
#pragma unroll
        for (int a = 0; a < 3; ++a) mu_p[a] = gload(F.mu_p, (size_t)a * n + i);
        const bool cv_fin = slice_cov(S, cv32);
        float mc[3], cv[6], ac;
        slice_outputs(S, S, mu_p, cv32, cv_fin, gload(F.alpha, i), mc, cv, ac, flag);
        const size_t g0 = F.g0;
#pragma unroll
        for (int a = 0; a < 3; ++a) mu_c[3 * g0 + (size_t)a * n + i] = mc[a];
#pragma unroll
        for (int e = 0; e < 6; ++e) cov_c[6 * g0 + (size_t)e * n + i] = cv[e];
        alpha_c[g0 + i] = ac;
    }
    wave_flags(flag, counts, f);
}

// Reverse of k_slice.  Inputs d_mu_c [3], d_cov_c [6] (packed symmetric: the
// off-diagonal value sets both entries), d_alpha_c; outputs the gradients of
// mu_p, mu_t, mu_d, L (packed, lower triangle) and alpha.
__global__ __launch_bounds__(kBlock) void k_slice_bwd(const FrameDev* __restrict__ tab, BlockMap bm,
                                                      const float* __restrict__ d_mu_c,
                                                      const float* __restrict__ d_cov_c,
                                                      const float* __restrict__ d_alpha_c)
{
    const int f = frame_of_block(bm, blockIdx.x);
    const FrameDev& F = tab[f];
    const uint32_t i0 = (blockIdx.x - bm.start[f]) * kBlock + threadIdx.x;
    const bool valid = i0 < F.n;
    const uint32_t i = valid ? i0 : 0;  // invalid lanes compute on Gaussian 0 and write nothing
    const uint32_t n = F.n;
    const size_t g0 = F.g0;
    double gl_t = 0.0, gl_d = 0.0;      // this lane's dL/dlambda_t, dL/dlambda_d
    double gm[3], Gc[3][3], ga;
#pragma unroll
    for (int a = 0; a < 3; ++a) gm[a] = (double)d_mu_c[3 * g0 + (size_t)a * n + i];
    {
        const double xx = d_cov_c[6 * g0 + 0 * (size_t)n + i], xy = d_cov_c[6 * g0 + 1 * (size_t)n + i];
        const double xz = d_cov_c[6 * g0 + 2 * (size_t)n + i], yy = d_cov_c[6 * g0 + 3 * (size_t)n + i];
        const double yz = d_cov_c[6 * g0 + 4 * (size_t)n + i], zz = d_cov_c[6 * g0 + 5 * (size_t)n + i];
        Gc[0][0] = xx; Gc[1][1] = yy; Gc[2][2] = zz;
        Gc[0][1] = Gc[1][0] = 0.5 * xy;
        Gc[0][2] = Gc[2][0] = 0.5 * xz;
        Gc[1][2] = Gc[2][1] = 0.5 * yz;
    }
    ga = (double)d_alpha_c[g0 + i];

    uint32_t flag = 0;
    SliceState S;
    slice_state<true>(F, i, S, flag);
    double out_mu_p[3] = {0, 0, 0}, out_mu_t = 0, out_mu_d[3] = {0, 0, 0}, out_alpha = 0;
    double dL[28];
#pragma unroll
    for (int k = 0; k < 28; ++k) dL[k] = 0.0;
    bool any_grad = ga != 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) any_grad = any_grad || gm[a] != 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) any_grad = any_grad || Gc[a][b] != 0.0;

    if (S.ok && any_grad) {
        // K = Sigma_PQ Sigma_QQ^{-1} = V C^{-1}  (rows: solve C^T k = v)
        double K[3][4], w[4];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int k = 3; k >= 0; --k) {
                double s = S.V[a][k];
#pragma unroll
                for (int m = k + 1; m < 4; ++m) s = fma(-S.C[m][k], K[a][m], s);
                K[a][k] = s / S.C[k][k];
            }
#pragma unroll
        for (int k = 3; k >= 0; --k) {  // w = Sigma_QQ^{-1} r = C^{-T} u
            double s = S.u[k];
#pragma unroll
            for (int m = k + 1; m < 4; ++m) s = fma(-S.C[m][k], w[m], s);
            w[k] = s / S.C[k][k];
        }
        // Gradient w.r.t. the symmetric 7x7 Sigma, G (blocks PP, PQ, QQ).
        double GPQ[3][4], GQQ[4][4];
        // dB = -2 Gc K + gm w^T ; G_PQ = dB / 2
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double s = gm[a] * w[q];
#pragma unroll
                for (int b = 0; b < 3; ++b) s = fma(-2.0 * Gc[a][b], K[b][q], s);
                GPQ[a][q] = 0.5 * s;
            }
        // dC = K^T Gc K - sym(K^T gm w^T)
        double Kg[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) Kg[q] = K[0][q] * gm[0] + K[1][q] * gm[1] + K[2][q] * gm[2];
        double GK[3][4];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) GK[a][q] = Gc[a][0] * K[0][q] + Gc[a][1] * K[1][q] + Gc[a][2] * K[2][q];
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double s = K[0][p] * GK[0][q] + K[1][p] * GK[1][q] + K[2][p] * GK[2][q];
                GQQ[p][q] = s - 0.5 * (Kg[p] * w[q] + w[p] * Kg[q]);
            }
        // mean: d mu_p = gm, d r = K^T gm
#pragma unroll
        for (int a = 0; a < 3; ++a) out_mu_p[a] = gm[a];
        out_mu_t = -Kg[0];
#pragma unroll
        for (int k = 0; k < 3; ++k) out_mu_d[k] = -Kg[1 + k];
        // modulation: alpha_c = alpha exp(-(e_t + e_d)/2)
        const double fmod = exp(-0.5 * (S.e_t + S.e_d));
        const double alpha = (double)gload(F.alpha, i);
        out_alpha = ga * fmod;
        const double s = ga * alpha * fmod;  // dl/d(ln alpha_c)
        const double lt = (double)F.lambda_t, ld = (double)F.lambda_d;
        out_mu_t += s * lt * S.r[0] / S.s_tt;
        GQQ[0][0] += s * 0.5 * lt * S.r[0] * S.r[0] / (S.s_tt * S.s_tt);
#pragma unroll
        for (int k = 0; k < 3; ++k) out_mu_d[k] += s * ld * S.y[k];
        // lambda: d ln alpha_c / d lambda_t = -r_t^2 / (2 Sigma_t), / d lambda_d = -q_d / 2
        gl_t = -0.5 * s * S.r[0] * S.r[0] / S.s_tt;
        gl_d = -0.5 * s * S.q_d;
        // d = unit(mu_p - c): dL/dd = -dL/dmu_d, d d / d mu_p = (I - d d^T) / |mu_p - c|
        if (F.d_mode) {
            const double dd = -(S.d[0] * out_mu_d[0] + S.d[1] * out_mu_d[1] + S.d[2] * out_mu_d[2]);
#pragma unroll
            for (int a = 0; a < 3; ++a) out_mu_p[a] += S.rn * (-out_mu_d[a] - S.d[a] * dd);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) GQQ[1 + a][1 + b] += s * 0.5 * ld * S.y[a] * S.y[b];
        // dL = 2 G L (lower triangle)
        auto Gat = [&](int a, int b) -> double {
            if (a < 3 && b < 3) return Gc[a][b];
            if (a < 3) return GPQ[a][b - 3];
            if (b < 3) return GPQ[b][a - 3];
            return GQQ[a - 3][b - 3];
        };
#pragma unroll
        for (int a = 0; a < 7; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b) {
                double acc = 0.0;
#pragma unroll
                for (int k = b; k < 7; ++k) acc = fma(Gat(a, k), S.L[tri(k, b)], acc);
                dL[tri(a, b)] = 2.0 * acc;
            }
    }
    if (valid) {
#pragma unroll
        for (int a = 0; a < 3; ++a) F.g_mu_p[(size_t)a * n + i] = (float)out_mu_p[a];
        F.g_mu_t[i] = (float)out_mu_t;
#pragma unroll
        for (int a = 0; a < 3; ++a) F.g_mu_d[(size_t)a * n + i] = (float)out_mu_d[a];
#pragma unroll
        for (int k = 0; k < 28; ++k) F.g_L[(size_t)k * n + i] = (float)dL[k];
        F.g_alpha[i] = (float)out_alpha;
    } else {
        gl_t = gl_d = 0.0;
    }
    if (F.g_lambda) {  // uniform over the block (one frame)
        // wave sums, the block's sum of them in LDS, then one atomic per
        // block and value: same-address atomics serialize in L2, and one
        // per wave and value made up most of this kernel's time
        __shared__ double s_gl[kBlock / 64][2];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            gl_t += __shfl_xor(gl_t, off);
            gl_d += __shfl_xor(gl_d, off);
        }
        if (__lane_id() == 0) {
            s_gl[threadIdx.x / 64][0] = gl_t;
            s_gl[threadIdx.x / 64][1] = gl_d;
        }
        __syncthreads();
        if (threadIdx.x < 2) {
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) sum += s_gl[w][threadIdx.x];
            atomicAdd(&F.g_lambda[threadIdx.x], (float)sum);
        }
    }
}

}  // namespace sd7
