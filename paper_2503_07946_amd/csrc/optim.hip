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

// One lane per parameter value; block b covers values [256 b, 256 b + 256)
// of the 84 n values taken group by group.  Adam in the order PyTorch uses:
// m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
// p -= (lr / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t) + eps); then the
// opacity is clamped to [alpha_lo, alpha_hi] and L's diagonal to >= diag_min.
__global__ __launch_bounds__(kBlock) void k_adam(uint32_t n, ArraySet p, ArraySet g, ArraySet m, ArraySet v,
                                                 AdamArgs c)
{
    const uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    uint64_t off = e;
    int grp = 0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const uint64_t len = (uint64_t)kGroupPlanes[grp] * n;
        if (off >= len) { off -= len; ++grp; }
    }
    if (grp >= 6 || off >= (uint64_t)kGroupPlanes[grp] * n) return;
    const float gr = g.a[grp][off];
    const float mm = fmaf(c.beta1, m.a[grp][off], (1.0f - c.beta1) * gr);
    const float vv = fmaf(c.beta2, v.a[grp][off], (1.0f - c.beta2) * gr * gr);
    m.a[grp][off] = mm;
    v.a[grp][off] = vv;
    const float denom = sqrtf(vv) * c.rsbc2 + c.eps;
    float x = p.a[grp][off] - (c.lr[grp] * c.rbc1) * (mm / denom);
    if (grp == 4) x = fminf(fmaxf(x, c.alpha_lo), c.alpha_hi);
    if (grp == 3) {
        const uint32_t plane = (uint32_t)(off / n);
        const bool diag = plane == 0 || plane == 2 || plane == 5 || plane == 9 || plane == 14 || plane == 20 ||
                          plane == 27;
        if (diag) x = fmaxf(x, c.diag_min);
    }
    p.a[grp][off] = x;
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
