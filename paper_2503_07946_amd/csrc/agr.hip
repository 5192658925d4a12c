// Adaptive Gaussian refinement (Sec. 4.3; Algorithm 1 steps 1-2) fused with
// the slice.  One lane per (frame, Gaussian), one frame per block.
//
// f = mu_p (+) mu_t (+) mu_d (+) gamma(t) feeds four two-layer MLPs
// (27 -> 64 -> C_out, ReLU) whose outputs are added to mu_p, mu_t, mu_d and
// the packed factor L; the refined parameters are then sliced exactly as by
// k_slice.  gamma(t) is the same for every Gaussian of a frame, so the block
// folds W1[:, 7:27] gamma(t) into the first-layer bias once (FP64 sines of
// 2^k pi t, k <= 9); each lane then needs 7 multiply-adds per hidden unit and
// C_out per hidden unit for the second layer, 4032 FP32 multiply-adds in
// all, with the weights read from LDS as broadcasts.
#include "common.h"
#include "gload.h"

namespace sd7 {

constexpr int kAgrIn = 27, kAgrHidden = 64, kAgrK = 10;
__constant__ const int kAgrOut[4] = {3, 1, 3, 28};
// LDS row strides of the transposed second layer (multiples of 4 floats)
constexpr int kW2Stride[4] = {4, 4, 4, 28};
constexpr int kW2Off[4] = {0, 4 * 64, 8 * 64, 12 * 64};
constexpr int kW2Floats = 40 * 64;
constexpr int kAgrWeights = SD7_AGR_WEIGHTS;

// Offset of MLP m's block (W1, b1, W2, b2) in the packed weights.
__host__ __device__ constexpr int agr_base(int m)
{
    int off = 0;
    const int c[4] = {3, 1, 3, 28};
    for (int k = 0; k < m; ++k) off += kAgrHidden * kAgrIn + kAgrHidden + c[k] * kAgrHidden + c[k];
    return off;
}
static_assert(agr_base(4) == kAgrWeights, "AGR weight count");

template <int C>
__device__ __forceinline__ void mlp_layer2(const float* __restrict__ s_hid, const float* __restrict__ s_w2, int m,
                                           const float x[7], float out[C])
{
#pragma unroll 4
    for (int j = 0; j < kAgrHidden; ++j) {
        const float4 w0 = *reinterpret_cast<const float4*>(s_hid + (m * kAgrHidden + j) * 8);
        const float4 w1 = *reinterpret_cast<const float4*>(s_hid + (m * kAgrHidden + j) * 8 + 4);
        float a = w1.w;  // b1 + W1[:, 7:27] gamma(t)
        a = fmaf(w0.x, x[0], a);
        a = fmaf(w0.y, x[1], a);
        a = fmaf(w0.z, x[2], a);
        a = fmaf(w0.w, x[3], a);
        a = fmaf(w1.x, x[4], a);
        a = fmaf(w1.y, x[5], a);
        a = fmaf(w1.z, x[6], a);
        const float h = fmaxf(a, 0.0f);
        const float* w2 = s_w2 + kW2Off[m] + j * kW2Stride[m];
#pragma unroll
        for (int o = 0; o < C; ++o) out[o] = fmaf(w2[o], h, out[o]);
    }
}

__global__ __launch_bounds__(kBlock, 4) void k_agr_slice(const FrameDev* __restrict__ tab, BlockMap bm,
                                                      float* __restrict__ mu_c, float* __restrict__ cov_c,
                                                      float* __restrict__ alpha_c, uint32_t* __restrict__ counts)
{
    const int f = frame_of_block(bm, blockIdx.x);
    const FrameDev& F = tab[f];
    if (!F.agr) return;  // uniform: the frame's scene has no refinement
    __shared__ __align__(16) float s_hid[4 * kAgrHidden * 8];  // per unit: W1[0:7], b1 + W1[7:27] gamma
    __shared__ __align__(16) float s_w2[kW2Floats];            // per unit: W2 column (padded)
    __shared__ float s_b2[36];
    __shared__ double s_gam[2 * kAgrK];
    const float* __restrict__ W = F.agr;
    const uint32_t tid = threadIdx.x;
    if (tid < 2 * kAgrK) {
        const double w = ldexp(3.14159265358979323846, (int)(tid >> 1)) * (double)F.t;
        s_gam[tid] = (tid & 1) ? cos(w) : sin(w);
    }
    if (tid < 35) {
        const int m = tid < 3 ? 0 : tid < 4 ? 1 : tid < 7 ? 2 : 3;
        const int o = tid - (m == 0 ? 0 : m == 1 ? 3 : m == 2 ? 4 : 7);
        s_b2[tid] = gload(W, agr_base(m) + kAgrHidden * kAgrIn + kAgrHidden + kAgrOut[m] * kAgrHidden + o);
    }
    __syncthreads();
    {
        // every weight the thread stages is loaded before its first LDS store
        const int m = tid / kAgrHidden, j = tid % kAgrHidden;  // 256 threads = 4 MLPs x 64 units
        const float* W1 = W + agr_base(m) + j * kAgrIn;
        const float* W2 = W + agr_base(m) + kAgrHidden * kAgrIn + kAgrHidden;
        float w1[kAgrIn], w2[28];
#pragma unroll
        for (int c = 0; c < kAgrIn; ++c) w1[c] = gload(W1, c);
        const float b1 = gload(W, agr_base(m) + kAgrHidden * kAgrIn + j);
#pragma unroll
        for (int o = 0; o < 28; ++o) w2[o] = o < kAgrOut[m] ? gload(W2, o * kAgrHidden + j) : 0.0f;
        double bias = (double)b1;
#pragma unroll
        for (int k = 0; k < 2 * kAgrK; ++k) bias = fma((double)w1[7 + k], s_gam[k], bias);
        float* hrow = s_hid + (m * kAgrHidden + j) * 8;
#pragma unroll
        for (int c = 0; c < 7; ++c) hrow[c] = w1[c];
        hrow[7] = (float)bias;
        float* w2row = s_w2 + kW2Off[m] + j * kW2Stride[m];
#pragma unroll
        for (int o = 0; o < 28; ++o)
            if (o < kAgrOut[m]) w2row[o] = w2[o];
    }
    __syncthreads();

    const uint32_t i = (blockIdx.x - bm.start[f]) * kBlock + tid;
    uint32_t flag = 0;
    if (i < F.n) {
        const uint32_t n = F.n;
        float x[7];
#pragma unroll
        for (int a = 0; a < 3; ++a) x[a] = gload(F.mu_p, (size_t)a * n + i);
        x[3] = gload(F.mu_t, i);
#pragma unroll
        for (int a = 0; a < 3; ++a) x[4 + a] = gload(F.mu_d, (size_t)a * n + i);
        float rp[3], rt[1], rd[3], rl[28];
#pragma unroll
        for (int o = 0; o < 3; ++o) rp[o] = s_b2[o];
        rt[0] = s_b2[3];
#pragma unroll
        for (int o = 0; o < 3; ++o) rd[o] = s_b2[4 + o];
#pragma unroll
        for (int o = 0; o < 28; ++o) rl[o] = s_b2[7 + o];
        mlp_layer2<3>(s_hid, s_w2, 0, x, rp);
        mlp_layer2<1>(s_hid, s_w2, 1, x, rt);
        mlp_layer2<3>(s_hid, s_w2, 2, x, rd);
        mlp_layer2<28>(s_hid, s_w2, 3, x, rl);
        // refined parameters (FP32), then the slice of k_slice
        double L[28];
#pragma unroll
        for (int k = 0; k < 28; ++k) L[k] = (double)(gload(F.L, (size_t)k * n + i) + rl[k]);
        SliceFixed S;
        slice_fixed(L, S, flag);
        float cv32[6];
        const bool cv_fin = slice_cov(S, cv32);
        float mu_p[3];
        double mu_d[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) mu_p[a] = x[a] + rp[a];
#pragma unroll
        for (int a = 0; a < 3; ++a) mu_d[a] = (double)(x[4 + a] + rd[a]);
        SliceView V;
        double d[3], rn;
        view_direction(F, mu_p, d, rn);
        slice_view<false>(S, (double)F.t, d, rn, (double)(x[3] + rt[0]), mu_d, F.lambda_t, F.lambda_d, V);
        float mc[3], cv[6], ac;
        slice_outputs(S, V, mu_p, cv32, cv_fin, gload(F.alpha, i), mc, cv, ac, flag);
        const size_t g0 = F.g0;
#pragma unroll
        for (int a = 0; a < 3; ++a) mu_c[3 * g0 + (size_t)a * n + i] = mc[a];
#pragma unroll
        for (int e = 0; e < 6; ++e) cov_c[6 * g0 + (size_t)e * n + i] = cv[e];
        alpha_c[g0 + i] = ac;
    }
    wave_flags(flag, counts, f);
}

}  // namespace sd7
