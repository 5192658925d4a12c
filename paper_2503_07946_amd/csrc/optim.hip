// Training-side helpers (Sec. 4.4: the 3DGS optimizer and pruning with the
// raised opacity floor tau_min): a fused Adam step over every per-Gaussian
// parameter plane, and out-of-place compaction of the Gaussians whose
// opacity reaches tau.
#include "common.h"

namespace sd7 {

// The six parameter arrays (or their moments) of a scene, plane-major.
struct ArraySet {
    float* a[6];
};
constexpr int kGroupPlanes[6] = {3, 1, 3, 28, 1, 48};  // mu_p, mu_t, mu_d, L, alpha, sh

struct AdamArgs {
    float lr[6];
    float beta1, beta2, eps;
    float rbc1;        // 1 / (1 - beta1^step)
    float rsbc2;       // 1 / sqrt(1 - beta2^step)
    float alpha_lo, alpha_hi, diag_min;
};

// Values of one parameter plane a k_adam thread updates (kBlock apart).
constexpr uint32_t kAdamPerThread = 4;

// Block b updates values [chunk * kBlock * kAdamPerThread, ...) of plane
// b / chunks of the 84 per-Gaussian planes taken group by group (the group,
// its learning rate and clamps are uniform over the block).  Adam in the
// order PyTorch uses: m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
// p -= (lr / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t) + eps); then the
// opacity is clamped to [alpha_lo, alpha_hi] and L's diagonal to >= diag_min.
__global__ __launch_bounds__(kBlock) void k_adam(uint32_t n, uint32_t chunks, ArraySet p, ArraySet g, ArraySet m,
                                                 ArraySet v, AdamArgs c)
{
    const uint32_t plane = blockIdx.x / chunks, chunk = blockIdx.x - plane * chunks;
    int grp = 0;
    uint32_t pl = plane;  // plane within the group
#pragma unroll
    for (int k = 0; k < 5; ++k)
        if (pl >= (uint32_t)kGroupPlanes[grp]) { pl -= kGroupPlanes[grp]; ++grp; }
    const size_t base = (size_t)pl * n;
    float* __restrict__ pp = p.a[grp] + base;
    const float* __restrict__ gg = g.a[grp] + base;
    float* __restrict__ mp = m.a[grp] + base;
    float* __restrict__ vp = v.a[grp] + base;
    const float step = c.lr[grp] * c.rbc1;
    const bool clamp_alpha = grp == 4;
    const bool clamp_diag = grp == 3 && (pl == 0 || pl == 2 || pl == 5 || pl == 9 || pl == 14 || pl == 20 || pl == 27);
    const uint32_t i0 = chunk * kBlock * kAdamPerThread + threadIdx.x;
    float gr[kAdamPerThread], m0[kAdamPerThread], v0[kAdamPerThread], p0[kAdamPerThread];
#pragma unroll
    for (uint32_t k = 0; k < kAdamPerThread; ++k) {
        const uint32_t i = i0 + k * kBlock;
        if (i < n) {
            gr[k] = gg[i];
            m0[k] = mp[i];
            v0[k] = vp[i];
            p0[k] = pp[i];
        }
    }
#pragma unroll
    for (uint32_t k = 0; k < kAdamPerThread; ++k) {
        const uint32_t i = i0 + k * kBlock;
        if (i >= n) continue;
        const float mm = fmaf(c.beta1, m0[k], (1.0f - c.beta1) * gr[k]);
        const float vv = fmaf(c.beta2, v0[k], (1.0f - c.beta2) * gr[k] * gr[k]);
        mp[i] = mm;
        vp[i] = vv;
        const float denom = sqrtf(vv) * c.rsbc2 + c.eps;
        float x = p0[k] - step * (mm / denom);
        if (clamp_alpha) x = fminf(fmaxf(x, c.alpha_lo), c.alpha_hi);
        if (clamp_diag) x = fmaxf(x, c.diag_min);
        pp[i] = x;
    }
}

// keep[i] = alpha[i] >= tau, and the same flags into pos (scanned in place next)
__global__ __launch_bounds__(kBlock) void k_prune_flags(uint32_t n, const float* __restrict__ alpha, float tau,
                                                        uint32_t* __restrict__ keep, uint32_t* __restrict__ pos)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) keep[i] = pos[i] = alpha[i] >= tau ? 1u : 0u;
}

constexpr int kMaxPruneArrays = 32;
struct PruneArrays {
    const float* src[kMaxPruneArrays];
    float* dst[kMaxPruneArrays];
    uint32_t plane0[kMaxPruneArrays + 1];  // prefix of the arrays' plane counts
    int narrays;
};

// Block b: plane b / chunks (of all arrays' planes), values chunk * 256 ..
// The exclusive scan of the keep flags gives each kept Gaussian its index.
__global__ __launch_bounds__(kBlock) void k_prune_apply(uint32_t n, uint32_t n_kept, uint32_t chunks,
                                                        const uint32_t* __restrict__ keep,
                                                        const uint32_t* __restrict__ pos, PruneArrays pa)
{
    const uint32_t plane = blockIdx.x / chunks;
    const uint32_t i = (blockIdx.x - plane * chunks) * kBlock + threadIdx.x;
    if (i >= n || !keep[i]) return;
    int j = 0;
    while (j + 1 < pa.narrays && pa.plane0[j + 1] <= plane) ++j;
    const uint32_t k = plane - pa.plane0[j];
    pa.dst[j][(size_t)k * n_kept + pos[i]] = pa.src[j][(size_t)k * n + i];
}

__global__ void k_prune_total(uint32_t n, const uint32_t* __restrict__ keep, const uint32_t* __restrict__ pos,
                              uint32_t* __restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = n ? pos[n - 1] + keep[n - 1] : 0u;
}

}  // namespace sd7
