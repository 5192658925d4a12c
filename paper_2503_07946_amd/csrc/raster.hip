// Depth-aware, opacity-blended front-to-back compositing (Sec. 4.4) and its
// reverse.  One 256-lane block (4 wave64) per 16x16 tile, one lane per pixel.
// The tile list is streamed through LDS in batches of 256 splats (loaded by
// the 256 lanes in one coalesced step, gathered by Gaussian index); the block
// leaves as soon as every pixel is saturated.
//
// Per (pixel, splat):  q = a dx^2 + 2 b dx dy + c dy^2 (dx = u - px),
//   alpha = min(0.99, alpha_c exp(-q/2)); skip if alpha < 1/255;
//   stop before the splat if T (1 - alpha) < 1e-4; C += rgb alpha T.
// The exponent is evaluated as exp2 of -q/2 log2(e), with the conic scaled
// once per splat when it is staged in LDS.
#include "common.h"

namespace sd7 {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.69314718055994531f;

struct SplatLDS {
    float4 p0[256];  // u, v, A, B    (A = -a log2e / 2, B = -b log2e)
    float4 p1[256];  // C, opacity, r, g   (C = -c log2e / 2)
    float p2[256];   // b (blue)
};

__device__ __forceinline__ void stage_splat(SplatLDS& s, int slot, const float4* __restrict__ splat, size_t gi)
{
    const float4* r = splat + gi * 3;
    const float4 a = r[0], b = r[1];
    const float bb = r[2].x;
    s.p0[slot] = make_float4(a.x, a.y, -0.5f * kLog2e * a.z, -kLog2e * a.w);
    s.p1[slot] = make_float4(-0.5f * kLog2e * b.x, b.y, b.z, b.w);
    s.p2[slot] = bb;
}

__global__ __launch_bounds__(256) void k_raster(const FrameDev* __restrict__ tab, BlockMap bm,
                                                const uint2* __restrict__ ranges,
                                                const uint32_t* __restrict__ pair_g,
                                                const float4* __restrict__ splat)
{
    __shared__ SplatLDS s;
    const int f = frame_of_block(bm, blockIdx.x);
    const FrameDev& F = tab[f];
    const uint32_t tile = blockIdx.x - bm.start[f];
    const uint32_t tx = tile % F.tiles_x, ty = tile / F.tiles_x;
    const uint32_t px = tx * kTile + (threadIdx.x & 15), py = ty * kTile + (threadIdx.x >> 4);
    const bool inside = px < F.W && py < F.H;
    const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
    const uint2 rg = ranges[F.t0 + tile];
    const size_t g0 = F.g0;
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    uint32_t last = 0;
    bool done = !inside;
    for (uint32_t b = rg.x; b < rg.y; b += 256) {
        if (__syncthreads_count(done) == 256) break;
        const uint32_t e = b + threadIdx.x;
        if (e < rg.y) stage_splat(s, threadIdx.x, splat, g0 + min(pair_g[e], F.n - 1));
        __syncthreads();
        const int cnt = (int)min(256u, rg.y - b);
        if (!done) {
            for (int j = 0; j < cnt; ++j) {
                const float4 p0 = s.p0[j];
                const float4 p1 = s.p1[j];
                const float dx = p0.x - fpx, dy = p0.y - fpy;
                const float power = p0.z * dx * dx + p0.w * dx * dy + p1.x * dy * dy;
                const float alpha = fminf(kAlphaMax, p1.y * exp2f(power));
                if (alpha < kAlphaMin) continue;
                const float Tn = T * (1.0f - alpha);
                if (Tn < kTMin) {
                    done = true;
                    break;
                }
                const float wgt = alpha * T;
                C0 += p1.z * wgt;
                C1 += p1.w * wgt;
                C2 += s.p2[j] * wgt;
                T = Tn;
                last = b - rg.x + (uint32_t)j + 1;
            }
        }
    }
    if (inside) {
        const size_t pix = (size_t)py * F.W + px, plane = (size_t)F.W * F.H;
        F.image[pix] = C0 + T * F.bg[0];
        F.image[plane + pix] = C1 + T * F.bg[1];
        F.image[2 * plane + pix] = C2 + T * F.bg[2];
        F.final_T[pix] = T;
        F.last[pix] = last;
    }
}

// ---------------------------------------------------------------------------
// reverse
// ---------------------------------------------------------------------------

// Sum over the 64 lanes of a wave; the total lands in lane 63.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v)
{
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, true));
}

__device__ __forceinline__ float wave_sum_to_lane63(float v)
{
    v = dpp_add<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v = dpp_add<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v = dpp_add<0x141, 0xF>(v);  // row_half_mirror
    v = dpp_add<0x140, 0xF>(v);  // row_mirror: every lane of a row holds the row sum
    v = dpp_add<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

__global__ __launch_bounds__(256) void k_raster_bwd(const FrameDev* __restrict__ tab, BlockMap bm,
                                                    const uint2* __restrict__ ranges,
                                                    const uint32_t* __restrict__ pair_g,
                                                    const float4* __restrict__ splat,
                                                    float* __restrict__ d_splat)
{
    __shared__ SplatLDS s;
    __shared__ uint32_t s_g[256];
    __shared__ uint32_t s_maxlast;
    const int f = frame_of_block(bm, blockIdx.x);
    const FrameDev& F = tab[f];
    const uint32_t tile = blockIdx.x - bm.start[f];
    const uint32_t tx = tile % F.tiles_x, ty = tile / F.tiles_x;
    const uint32_t px = tx * kTile + (threadIdx.x & 15), py = ty * kTile + (threadIdx.x >> 4);
    const bool inside = px < F.W && py < F.H;
    const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
    const uint2 rg = ranges[F.t0 + tile];
    const size_t g0 = F.g0, n = F.n;
    const int lane = threadIdx.x & 63;

    float Cout[3] = {0.f, 0.f, 0.f}, gC[3] = {0.f, 0.f, 0.f};
    uint32_t last = 0;
    if (threadIdx.x == 0) s_maxlast = 0;
    __syncthreads();
    if (inside) {
        const size_t pix = (size_t)py * F.W + px, plane = (size_t)F.W * F.H;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            Cout[ch] = F.image[ch * plane + pix];
            gC[ch] = F.dL_dimage[ch * plane + pix];
        }
        last = F.last[pix];
        atomicMax(&s_maxlast, last);
    }
    __syncthreads();
    const uint32_t maxlast = s_maxlast;
    float T = 1.0f, acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
    for (uint32_t b = rg.x; b < rg.x + maxlast; b += 256) {
        const uint32_t e = b + threadIdx.x;
        if (e < rg.y) {
            const uint32_t g = min(pair_g[e], F.n - 1);  // in range for well-formed pairs
            s_g[threadIdx.x] = g;
            stage_splat(s, threadIdx.x, splat, g0 + g);
        }
        __syncthreads();
        const int cnt = (int)min(256u, rg.x + maxlast - b);
        for (int j = 0; j < cnt; ++j) {
            const float4 p0 = s.p0[j];
            const float4 p1 = s.p1[j];
            const float dx = p0.x - fpx, dy = p0.y - fpy;
            float g_u = 0.f, g_v = 0.f, g_A = 0.f, g_B = 0.f, g_C = 0.f, g_op = 0.f;
            float g_r = 0.f, g_g = 0.f, g_b = 0.f;
            bool contrib = false;
            if (b - rg.x + (uint32_t)j < last) {
                const float power = p0.z * dx * dx + p0.w * dx * dy + p1.x * dy * dy;
                const float G = exp2f(power);
                const float raw = p1.y * G;
                const float alpha = fminf(kAlphaMax, raw);
                if (alpha >= kAlphaMin) {
                    contrib = true;
                    const float rgb2 = s.p2[j];
                    const float wgt = alpha * T;
                    acc0 += p1.z * wgt;
                    acc1 += p1.w * wgt;
                    acc2 += rgb2 * wgt;
                    g_r = wgt * gC[0];
                    g_g = wgt * gC[1];
                    g_b = wgt * gC[2];
                    const float inv1m = 1.0f / (1.0f - alpha);
                    const float ga = gC[0] * (p1.z * T - (Cout[0] - acc0) * inv1m) +
                                     gC[1] * (p1.w * T - (Cout[1] - acc1) * inv1m) +
                                     gC[2] * (rgb2 * T - (Cout[2] - acc2) * inv1m);
                    if (raw < kAlphaMax) {
                        g_op = ga * G;
                        const float gp = ga * alpha * kLn2;  // dl/d power
                        g_u = gp * (2.f * p0.z * dx + p0.w * dy);
                        g_v = gp * (p0.w * dx + 2.f * p1.x * dy);
                        g_A = gp * dx * dx;
                        g_B = gp * dx * dy;
                        g_C = gp * dy * dy;
                    }
                    T = T * (1.0f - alpha);
                }
            }
            if (__ballot(contrib)) {
                float v[9] = {g_u, g_v, g_A, g_B, g_C, g_op, g_r, g_g, g_b};
                float mine = 0.f;
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    const float t = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_sum_to_lane63(v[k])), 63));
                    if (lane == k) mine = t;
                }
                // conic gradients back from the scaled (A, B, C) to (a, b, c)
                if (lane == 2 || lane == 4) mine *= -0.5f * kLog2e;
                if (lane == 3) mine *= -kLog2e;
                if (lane < 9) atomicAdd(&d_splat[9 * g0 + (size_t)lane * n + s_g[j]], mine);
            }
        }
        __syncthreads();
    }
}

}  // namespace sd7
