// Slice and projection fused over the frames of a call that share a scene
// (Sec. 4.2 then Sec. 4.4).  The conditional covariance, chol(Sigma_QQ),
// V = Sigma_PQ C^{-T} and chol(Sigma_DD) do not depend on the view (t, d):
// one lane per Gaussian forms them once, in FP64 registers, and then walks
// a run of the group's frames, doing only the view-dependent part of the
// slice (the residual r, mu_c = mu_p + V C^{-1} r, the modulations) and the
// projection of each.  The scene's parameters are read once per run instead
// of once per frame, and the sliced statistics go to projection in registers.
// The block's SH coefficients are staged in LDS once per run (48 x 256
// floats) and read from there by every frame.
// Each block takes an equal, contiguous share of the units (Gaussian block,
// frame), so a block's runs are the frames of one or a few Gaussian blocks;
// consecutive shares are laid out contiguously per XCD, so the scene reads of
// one Gaussian block split over two blocks meet in one L2.  The arithmetic is
// that of k_slice and k_project, so every output is bitwise the same as the
// two separate kernels'.
#include "common.h"
#include "gload.h"

namespace sd7 {

// SH coefficient j of the block's Gaussian t, staged in LDS (plane-major).
struct ShLds {
    const float* s;
    __device__ __forceinline__ float operator()(int j, uint32_t) const { return s[j * kBlock + threadIdx.x]; }
};

// Kept counts: with BLOCK_KEPT (calls whose scene groups have one frame each,
// so every run is one frame) the block sums its waves' counts in LDS and adds
// them to the frame's counter with one atomic per run; same-address atomics
// serialize in L2, and one per wave made up about half of a one-frame call
// (3,125 waves on one counter).  Runs of several frames keep one atomic per
// wave and frame: there each counter's atomics spread over the frames of the
// run and the launch, and the barriers of the block sums cost more (12 % at
// 25 frames of 200k Gaussians).
template <bool BLOCK_KEPT>
__global__ __launch_bounds__(kBlock, 3) void k_slice_project(const FrameDev* __restrict__ tab, SceneGroups sg,
                                                          float* __restrict__ mu_c, float* __restrict__ cov_c,
                                                          float* __restrict__ alpha_c, float4* __restrict__ splat,
                                                          uint4* __restrict__ rect, uint32_t* __restrict__ depth_key,
                                                          uint32_t* __restrict__ counts)
{
    const uint32_t lb = xcd_contiguous(blockIdx.x, gridDim.x);
    const uint32_t units = sg.start[sg.ng];
    uint32_t lo = (uint32_t)((uint64_t)lb * units / gridDim.x);
    uint32_t hi = (uint32_t)((uint64_t)(lb + 1) * units / gridDim.x);
    // Odd blocks take their runs last to first: a Gaussian block split
    // between the end of one share and the start of the next is then read by
    // both blocks at about the same time, while it is still in L2.
    const bool rev = lb & 1u;
    int gi = group_of_unit(sg, rev ? hi - 1u : lo);
    __shared__ float s_sh[48 * kBlock];
    __shared__ uint32_t s_kept[SD7_MAX_FRAMES];  // kept Gaussians of the block per frame of the run
    while (lo < hi) {  // one run: a Gaussian block and consecutive frames of its group
        uint32_t ua, ub;  // the run's units [ua, ub)
        uint32_t nq, gb;
        if (!rev) {
            ua = lo;
            while (ua >= sg.start[gi + 1]) ++gi;
            nq = sg.first[gi + 1] - sg.first[gi];
            gb = (ua - sg.start[gi]) / nq;
            ub = min(hi, sg.start[gi] + (gb + 1) * nq);
            lo = ub;
        } else {
            ub = hi;
            while (ub - 1u < sg.start[gi]) --gi;
            nq = sg.first[gi + 1] - sg.first[gi];
            gb = (ub - 1u - sg.start[gi]) / nq;
            ua = max(lo, sg.start[gi] + gb * nq);
            hi = ua;
        }
        const FrameDev& F0 = tab[sg.frame[sg.first[gi]]];
        const uint32_t n = F0.n;
        const uint32_t qa = ua - sg.start[gi] - gb * nq;
        const uint32_t run = ub - ua;
        // thread t < run zeroes, and after the frames adds out, the count of
        // the run's frame t (the previous run's reads were its own)
        if constexpr (BLOCK_KEPT) {
            if (threadIdx.x < run) s_kept[threadIdx.x] = 0;
            __syncthreads();
        }
        const uint32_t i = gb * kBlock + threadIdx.x;
        const bool valid = i < n;
        SliceFixed S;
        float mu_p[3] = {0.f, 0.f, 0.f}, mu_d[3] = {0.f, 0.f, 0.f}, cv32[6];
        float mu_t = 0.f, alpha = 0.f;
        bool cv_fin = false;
        uint32_t flag0 = 0;
        if (valid) {
            // every load of the Gaussian is issued before the first LDS store
            float sh[48];
#pragma unroll
            for (int j = 0; j < 48; ++j) sh[j] = gload(F0.sh, (size_t)j * n + i);
            double L[28];
            load_L(F0.L, n, i, L);
#pragma unroll
            for (int a = 0; a < 3; ++a) mu_p[a] = gload(F0.mu_p, (size_t)a * n + i);
            mu_t = gload(F0.mu_t, i);
#pragma unroll
            for (int k = 0; k < 3; ++k) mu_d[k] = gload(F0.mu_d, (size_t)k * n + i);
            alpha = gload(F0.alpha, i);
            // each lane reads back only what it wrote (this run's or the
            // previous run's column of its own): no barrier needed
#pragma unroll
            for (int j = 0; j < 48; ++j) s_sh[j * kBlock + threadIdx.x] = sh[j];
            slice_fixed(L, S, flag0);
            cv_fin = slice_cov(S, cv32);
        }
        const uint32_t qb = sg.first[gi] + qa, qe = qb + run;
        for (uint32_t q = qb; q < qe; ++q) {
            const int f = sg.frame[q];
            const FrameDev& F = tab[f];
            uint32_t flag = flag0;
            bool keep = false;
            if (valid) {
                SliceView W;
                const double md[3] = {(double)mu_d[0], (double)mu_d[1], (double)mu_d[2]};
                double d[3], rn;
                view_direction(F, mu_p, d, rn);
                slice_view<false>(S, (double)F.t, d, rn, (double)mu_t, md, F.lambda_t, F.lambda_d, W);
                float mc[3], cv[6], ac;
                slice_outputs(S, W, mu_p, cv32, cv_fin, alpha, mc, cv, ac, flag);
                const size_t g0 = F.g0;
                if (F.keep_sliced) {  // uniform over the block
#pragma unroll
                    for (int a = 0; a < 3; ++a) mu_c[3 * g0 + (size_t)a * n + i] = mc[a];
#pragma unroll
                    for (int e = 0; e < 6; ++e) cov_c[6 * g0 + (size_t)e * n + i] = cv[e];
                    alpha_c[g0 + i] = ac;
                }
                keep = project_emit(F, i, ac, mc, cv, ShLds{s_sh}, splat, rect, depth_key);
            }
            wave_flags(flag, counts, f);
            if constexpr (BLOCK_KEPT) {
                wave_kept(keep, &s_kept[q - qb]);
            } else {
                const uint64_t kept = __ballot(keep);
                if (__lane_id() == 0 && kept)
                    atomicAdd(&counts[f * SD7_CNT_WORDS + SD7_CNT_KEPT], (uint32_t)__popcll(kept));
            }
        }
        if constexpr (BLOCK_KEPT) {
            __syncthreads();
            if (threadIdx.x < run && s_kept[threadIdx.x])
                atomicAdd(&counts[sg.frame[qb + threadIdx.x] * SD7_CNT_WORDS + SD7_CNT_KEPT], s_kept[threadIdx.x]);
        }
    }
}

}  // namespace sd7
