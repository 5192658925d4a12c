// Depth-aware, opacity-blended front-to-back compositing (Sec. 4.4) and its
// reverse.
//
// One wave64 per 16x16 tile.  Lane l owns one pixel in each of the tile's
// four 4-row bands: column l % 16, rows l / 16 + 4k (k = 0..3), so the column
// offset dx and its products are shared by the lane's four pixels, and band
// k is pixel k of every lane.  The wave walks the tile's list in order; a
// splat record is the same for every lane, so it is read with scalar loads
// through the scalar cache into SGPRs (no LDS staging, no barriers), a batch
// of two records ahead of the pair being blended, and the vector ALUs take
// it as scalar operands.  A band none of whose 64 pixels the splat reaches
// skips the blend; the wave leaves the list as soon as all 256 pixels have
// stopped.
//
// Per (pixel, splat), with the record's exponent coefficients
// (A, B, C) = -(a, 2b, c) log2(e) / 2 and lo = log2(alpha_c):
//   p = A dx^2 + B dx dy + C dy^2 + lo          (= log2 of alpha_c e^{-q/2})
//   the splat counts at the pixel iff p >= log2(1/255);
//   alpha = min(0.99, 2^p); w = T alpha; T' = T - T alpha;
//   stop before the splat if T' < 1e-4, else C += rgb w, T = T'.
// p is evaluated in full at the lane's first row only and carried down its
// four rows by forward differences of the quadratic (the record holds 16 C
// for that).  The forward and reverse kernels evaluate all of this with the
// same explicit fused operations, so they take the same decisions.
#include "common.h"

#include <type_traits>

namespace sd7 {

constexpr float kLog2AlphaMin = -7.99435343685886f;  // log2(1/255)
constexpr float kFar = 1e30f;                         // opacity threshold of a finished pixel

struct Splat {
    float u, v, A, B, C, lo, r, g, b, C16;
};

__device__ __forceinline__ Splat load_splat(const float4* __restrict__ rec, uint32_t g)
{
    const float4 p0 = rec[3 * (size_t)g];
    const float4 p1 = rec[3 * (size_t)g + 1];
    const float4 p2 = rec[3 * (size_t)g + 2];
    return Splat{p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w, p2.x, p2.y};
}

__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

// log2 of the splat's opacity at the lane's four pixels: sample column fx,
// sample rows fy0 + 4k.  With dy0 = v - fy0 the rows are dy0 - 4k, and
//   p_{k+1} - p_k = -4 (2 C dy0 + B dx) + 16 C (2k + 1).
// Also returns dx, B dx and dy0.
__device__ __forceinline__ void splat_exponents(const Splat& s, float fx, float fy0, float& dx,
                                                float& Bdx, float& dy0, float p[4])
{
    dx = s.u - fx;
    const float base = fmaf(s.A * dx, dx, s.lo);
    Bdx = s.B * dx;
    dy0 = s.v - fy0;
    const float in0 = fmaf(s.C, dy0, Bdx);
    p[0] = fmaf(dy0, in0, base);
    float D = fmaf(fmaf(s.C, dy0, in0), -4.0f, s.C16);
    p[1] = p[0] + D;
    D = fmaf(s.C16, 2.0f, D);
    p[2] = p[1] + D;
    D = fmaf(s.C16, 2.0f, D);
    p[3] = p[2] + D;
}

// List entries whose records one scalar-load batch brings in.
constexpr uint32_t kRasterBatch = 2;

// MASKED: a band's blend runs under an execution mask of the lanes the splat
// reaches (fewer vector instructions per entry, more scalar ones: faster
// where many waves share each SIMD); otherwise every lane of a band that some
// lane passes blends, with alpha 0 where it does not (fewer instructions on
// one wave's own chain: faster for calls of few tiles, where a tile's wave
// runs nearly alone).  Both give the same bits.
//
// The work of one wave: tile gt of the call (block gt of the one-block-per-tile
// map), bands K0 .. K1 - 1 of each lane (all four, or one band per wave where
// a call has so few tiles that their lists would otherwise be walked by a few
// waves alone).  A pixel's arithmetic is the same whichever wave blends it.
template <bool COUNT, bool WIDE, bool MASKED, int K0, int K1>
__device__ __forceinline__ void raster_tile(const FrameDev* __restrict__ tab, const BlockMap& bm, uint32_t gt,
                                            const uint2* __restrict__ ranges, const uint32_t* __restrict__ pair_g,
                                            const float4* __restrict__ splat)
{
    static_assert(0 <= K0 && K0 < K1 && K1 <= 4, "bands of a lane");
    const int f = frame_of_block(bm, gt);
    const FrameDev& F = tab[f];
    const uint32_t tile = gt - bm.start[f];
    const uint32_t tx = tile % F.tiles_x, ty = tile / F.tiles_x;
    const uint32_t lane = threadIdx.x;
    const uint32_t px = tx * kTile + (lane & 15);
    const uint32_t py0 = ty * kTile + (lane >> 4);  // band k: row py0 + 4k
    const float fx = (float)px + 0.5f, fy0 = (float)py0 + 0.5f;
    // th[k] is the pixel's opacity threshold, log2(1/255); a pixel that has
    // stopped (or lies outside the image) raises it to kFar, so it never
    // passes the opacity test again and needs no flag of its own.
    float th[4], T[4], C0[4], C1[4], C2[4];
    uint32_t last[4], ncon[4];
#pragma unroll
    for (int k = K0; k < K1; ++k) {
        const uint32_t py = py0 + 4 * k;
        th[k] = (px < F.W && py < F.H) ? kLog2AlphaMin : kFar;
        T[k] = 1.0f;
        C0[k] = C1[k] = C2[k] = 0.0f;
        last[k] = 0;
        ncon[k] = 0;
    }
    const uint2 rg = ranges[F.t0 + tile];
    const float4* __restrict__ rec = splat + (size_t)F.g0 * 3;
    const uint32_t gmax = __builtin_amdgcn_readfirstlane(F.n - 1);  // pairs exist only if n > 0
    // Blend one splat (list entry e) into the lane's pixels of bands K0 .. K1 - 1.
    auto blend = [&](const Splat& s, uint32_t e) {
        float dx, Bdx, dy0, p[4];
        splat_exponents(s, fx, fy0, dx, Bdx, dy0, p);
#pragma unroll
        for (int k = K0; k < K1; ++k) {
            const bool pass = p[k] >= th[k];
            // Only a passing pixel can stop (T >= 1e-4 before).  Once per
            // pixel: take this splat's blend back (T to at least 1e-4, so
            // the pixel cannot stop again) and retire the pixel, which has
            // consumed the entries before e.
            auto band = [&](float alpha) {
                const float w = T[k] * alpha;
                T[k] = fmaf(-T[k], alpha, T[k]);
                C0[k] = fmaf(s.r, w, C0[k]);
                C1[k] = fmaf(s.g, w, C1[k]);
                C2[k] = fmaf(s.b, w, C2[k]);
                if (COUNT) ncon[k] += pass ? 1u : 0u;
                const bool stop = T[k] < kTMin;
                if (__ballot(stop)) {
                    T[k] = stop ? fmaxf(T[k] + w, kTMin) : T[k];
                    C0[k] = stop ? fmaf(-s.r, w, C0[k]) : C0[k];
                    C1[k] = stop ? fmaf(-s.g, w, C1[k]) : C1[k];
                    C2[k] = stop ? fmaf(-s.b, w, C2[k]) : C2[k];
                    if (COUNT) ncon[k] -= stop ? 1u : 0u;
                    th[k] = stop ? kFar : th[k];
                    last[k] = stop ? e - rg.x : last[k];
                }
            };
            if constexpr (MASKED) {
                if (pass) band(fminf(kAlphaMax, exp2_fast(p[k])));  // skipped when no lane passes
            } else {
                if (__ballot(pass) == 0) continue;  // the splat reaches no pixel of band k
                band(pass ? fminf(kAlphaMax, exp2_fast(p[k])) : 0.0f);
            }
        }
    };
    // Splat records in scalar registers, two batches of kRasterBatch entries
    // (a, b): while one batch is blended the next is being loaded.  Scalar
    // loads complete out of order and are waited for all at once, so a
    // batch's loads are issued right after the wait for the batch the next
    // blends use; past the list's end the loads repeat its last entry (in
    // bounds, unused); indices are clamped where used.
    if (rg.x < rg.y) {
        constexpr uint32_t NB = kRasterBatch;
        // Entry rg.x + r of the list (r clamped to the list) and the record
        // of Gaussian g (clamped to the frame).  Unless WIDE, both are read
        // at 32-bit byte offsets from the list's start and the frame's first
        // record, which the scalar loads take as an offset register (the
        // caller sets WIDE where the frame's records span 4 GiB or more).
        const uint32_t lmax = rg.y - 1 - rg.x;
        auto idx = [&](uint32_t r) {
            if constexpr (WIDE) return pair_g[rg.x + min(r, lmax)];
            return *(const uint32_t*)((const char*)(pair_g + rg.x) + 4u * min(r, lmax));
        };
        auto rec_at = [&](uint32_t g) {
            if constexpr (WIDE) return load_splat(rec, min(g, gmax));
            const float4* q = (const float4*)((const char*)rec + 48u * min(g, gmax));
            const float4 p0 = q[0], p1 = q[1], p2 = q[2];
            return Splat{p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w, p2.x, p2.y};
        };
        Splat a[NB], b[NB];
        uint32_t ia[NB], ib[NB];  // list indices of a batch to come
        // One half step: wait for the batch `cur` (entries r ..) and the
        // indices `inxt` of the batch after it, start loading that batch
        // (`nxt`) and the indices `ifree` of the one after, then blend `cur`
        // (entry by entry up to the list's end when GUARD).
        auto half = [&](auto guard, Splat (&cur)[NB], Splat (&nxt)[NB], const uint32_t (&inxt)[NB],
                        uint32_t (&ifree)[NB], uint32_t r) {
            __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
#pragma unroll
            for (uint32_t j = 0; j < NB; ++j) nxt[j] = rec_at(inxt[j]);
#pragma unroll
            for (uint32_t j = 0; j < NB; ++j) ifree[j] = idx(r + 2 * NB + j);
            asm volatile("" ::: "memory");  // keep the loads ahead of the blends
#pragma unroll
            for (uint32_t j = 0; j < NB; ++j)
                if (!decltype(guard)::value || r + j <= lmax) blend(cur[j], rg.x + r + j);
        };
        using Full = std::false_type;
        using Guarded = std::true_type;
        auto all_stopped = [&]() {
            float m = th[K0];
#pragma unroll
            for (int k = K0 + 1; k < K1; ++k) m = fminf(m, th[k]);
            return __ballot(m < kFar) == 0;
        };
#pragma unroll
        for (uint32_t j = 0; j < NB; ++j) ia[j] = idx(j);
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
#pragma unroll
        for (uint32_t j = 0; j < NB; ++j) a[j] = rec_at(ia[j]);
#pragma unroll
        for (uint32_t j = 0; j < NB; ++j) ib[j] = idx(NB + j);
        // whole groups of 4 NB entries, then the rest with guards; the wave
        // checks every 4 NB entries whether all its pixels have stopped
        uint32_t r = 0;
        for (; r + 4 * NB <= lmax + 1; r += 4 * NB) {
            if (all_stopped()) break;
            half(Full{}, a, b, ib, ia, r);
            half(Full{}, b, a, ia, ib, r + NB);
            half(Full{}, a, b, ib, ia, r + 2 * NB);
            half(Full{}, b, a, ia, ib, r + 3 * NB);
        }
        for (; r <= lmax; r += 2 * NB) {
            if (all_stopped()) break;
            half(Guarded{}, a, b, ib, ia, r);
            if (r + NB > lmax) break;
            half(Guarded{}, b, a, ia, ib, r + NB);
        }
    }
    const size_t plane = (size_t)F.W * F.H;
#pragma unroll
    for (int k = K0; k < K1; ++k) {
        const uint32_t py = py0 + 4 * k;
        if (px < F.W && py < F.H) {
            const size_t pix = (size_t)py * F.W + px;
            F.image[pix] = C0[k] + T[k] * F.bg[0];
            F.image[plane + pix] = C1[k] + T[k] * F.bg[1];
            F.image[2 * plane + pix] = C2[k] + T[k] * F.bg[2];
            F.final_T[pix] = T[k];
            F.last[pix] = th[k] < kFar ? rg.y - rg.x : last[k];  // a pixel that never stopped used all
            if (COUNT && F.ncontrib) F.ncontrib[pix] = ncon[k];
        }
    }
}

template <bool COUNT, bool WIDE, bool MASKED>
__global__ __launch_bounds__(64) void k_raster(const FrameDev* __restrict__ tab, BlockMap bm,
                                               const uint2* __restrict__ ranges,
                                               const uint32_t* __restrict__ pair_g,
                                               const float4* __restrict__ splat)
{
    raster_tile<COUNT, WIDE, MASKED, 0, 4>(tab, bm, blockIdx.x, ranges, pair_g, splat);
}

// Calls of at most a few hundred tiles: wave 4 t + k takes band k of tile t,
// so each list is walked by four waves with a quarter of the vector work each
// (a call of 16 tiles would otherwise run 16 waves on a chip of 1,024 SIMDs).
template <bool WIDE>
__global__ __launch_bounds__(64) void k_raster_bands(const FrameDev* __restrict__ tab, BlockMap bm,
                                                     const uint2* __restrict__ ranges,
                                                     const uint32_t* __restrict__ pair_g,
                                                     const float4* __restrict__ splat)
{
    const uint32_t gt = blockIdx.x >> 2;
    switch (blockIdx.x & 3u) {
    case 0: raster_tile<false, WIDE, false, 0, 1>(tab, bm, gt, ranges, pair_g, splat); break;
    case 1: raster_tile<false, WIDE, false, 1, 2>(tab, bm, gt, ranges, pair_g, splat); break;
    case 2: raster_tile<false, WIDE, false, 2, 3>(tab, bm, gt, ranges, pair_g, splat); break;
    default: raster_tile<false, WIDE, false, 3, 4>(tab, bm, gt, ranges, pair_g, splat); break;
    }
}

// ---------------------------------------------------------------------------
// reverse
// ---------------------------------------------------------------------------

// v plus v of the lane that the DPP control selects (every lane has one for
// the controls used here).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v)
{
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, true));
}

// v + v of the partner lane lane ^ 4 (DPP row rotations by 12 and by 4, each
// on the two 4-lane banks of a row whose partner it reaches).
__device__ __forceinline__ float add_xor4(float keep, float send)
{
    int x = __builtin_amdgcn_update_dpp(0, __float_as_int(send), 0x12C, 0xF, 0x5, false);  // row_ror:12, banks 0, 2
    x = __builtin_amdgcn_update_dpp(x, __float_as_int(send), 0x124, 0xF, 0xA, false);      // row_ror:4, banks 1, 3
    return keep + __int_as_float(x);
}

// v + v of lane ^ 16 and then of lane ^ 32 (gfx950 lane-swap permutes, both
// operands the same value: the two results are the two halves' values).
__device__ __forceinline__ float add_xor16_xor32(float v)
{
    const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}

// Wave sums of nine values: returns in lane q < 8 the sum of v[q] over the 64
// lanes and in every other lane the sum of v[8].  A reduce-scatter: at each of
// the first three steps a lane and its partner (lane ^ 1, ^ 2, ^ 4) split the
// values they still hold, each keeping half and adding the partner's copy of
// it, so lane bits b0, b1, b2 end up selecting value 4 b2 + 2 b1 + b0; then
// the value is summed over the other lane bits.  v[8] is summed over every
// step alongside.  About 40 instructions against 72 for nine full reductions
// and the reads of their results.
__device__ __forceinline__ float wave_sums_scatter9(const float (&v)[9], uint32_t lane)
{
    const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;
    float r[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {  // lane ^ 1: keep v[2i + b0]
        const float keep = b0 ? v[2 * i + 1] : v[2 * i], send = b0 ? v[2 * i] : v[2 * i + 1];
        r[i] = keep + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), 0xB1, 0xF, 0xF, true));
    }
    float r8 = dpp_add<0xB1, 0xF>(v[8]);
    float t[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {  // lane ^ 2: keep r[2i + b1] = v[4i + 2 b1 + b0]
        const float keep = b1 ? r[2 * i + 1] : r[2 * i], send = b1 ? r[2 * i] : r[2 * i + 1];
        t[i] = keep + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), 0x4E, 0xF, 0xF, true));
    }
    r8 = dpp_add<0x4E, 0xF>(r8);
    // lane ^ 4: keep t[b2] = v[4 b2 + 2 b1 + b0]
    float u = add_xor4(b2 ? t[1] : t[0], b2 ? t[0] : t[1]);
    r8 = add_xor4(r8, r8);
    u = dpp_add<0x128, 0xF>(u);  // row_ror:8: lane ^ 8
    r8 = dpp_add<0x128, 0xF>(r8);
    u = add_xor16_xor32(u);
    r8 = add_xor16_xor32(r8);
    return lane < 8 ? u : r8;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off));
    return v;
}

// Back-to-front recomputation: each pixel starts from the forward's final
// transmittance T_final and walks the list entries it consumed (the first
// `last`) in reverse.  Behind entry i the colour still to come is
// S_i = T_final bg + sum_{j > i} rgb_j w_j, accumulated here from the back as
// a sum of non-negative terms (no cancellation however small T gets), and the
// transmittance in front of it is T_i = T_{i+1} / (1 - alpha_i).  Then
// dC/d rgb_i = w_i = T_i alpha_i and dC/d alpha_i = rgb_i T_i - S_i / (1 - alpha_i).
// Per lane the four pixels' terms are folded into sums (S0 = sum s,
// S1 = sum s dy, S2 = sum s dy^2 with s = dl/d alpha * alpha) from which the
// mean, conic and opacity derivatives follow; each of the nine splat
// derivatives is then summed over the wave and added with one atomic.
__global__ __launch_bounds__(64) void k_raster_bwd(const FrameDev* __restrict__ tab, BlockMap bm,
                                                   const uint2* __restrict__ ranges,
                                                   const uint32_t* __restrict__ pair_g,
                                                   const float4* __restrict__ splat,
                                                   float* __restrict__ d_splat)
{
    const int f = frame_of_block(bm, blockIdx.x);
    const FrameDev& F = tab[f];
    const uint32_t tile = blockIdx.x - bm.start[f];
    const uint32_t tx = tile % F.tiles_x, ty = tile / F.tiles_x;
    const uint32_t lane = threadIdx.x;
    const uint32_t px = tx * kTile + (lane & 15);
    const uint32_t py0 = ty * kTile + (lane >> 4);  // band k: row py0 + 4k
    const float fx = (float)px + 0.5f, fy0 = (float)py0 + 0.5f;
    const size_t plane = (size_t)F.W * F.H;
    float T[4], Sc[4][3], gC[4][3];
    uint32_t last[4];
    uint32_t lmax = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t py = py0 + 4 * k;
        T[k] = 1.0f;
        last[k] = 0;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) Sc[k][ch] = gC[k][ch] = 0.0f;
        if (px < F.W && py < F.H) {
            const size_t pix = (size_t)py * F.W + px;
            T[k] = F.final_T[pix];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                Sc[k][ch] = T[k] * F.bg[ch];
                gC[k][ch] = F.dL_dimage[ch * plane + pix];
            }
            last[k] = F.last[pix];
        }
        lmax = max(lmax, last[k]);
    }
    const uint32_t maxlast = wave_max(lmax);
    const uint2 rg = ranges[F.t0 + tile];
    const uint32_t e_end = min(rg.y, rg.x + maxlast);
    const float4* __restrict__ rec = splat + (size_t)F.g0 * 3;
    const uint32_t gmax = __builtin_amdgcn_readfirstlane(F.n - 1);  // pairs exist only if n > 0
    const size_t n = F.n, g0 = F.g0;
    for (uint32_t e = e_end; e-- > rg.x;) {
        const uint32_t g = min(pair_g[e], gmax);
        const Splat s = load_splat(rec, g);
        const uint32_t pos = e - rg.x;
        float dx, Bdx, dy0, p[4];
        splat_exponents(s, fx, fy0, dx, Bdx, dy0, p);
        bool pass[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) pass[k] = pos < last[k] && p[k] >= kLog2AlphaMin;
        if (__ballot(pass[0] || pass[1] || pass[2] || pass[3]) == 0) continue;
        float S0 = 0.f, S1 = 0.f, S2 = 0.f, Sr = 0.f, Sg = 0.f, Sb = 0.f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float raw = exp2_fast(p[k]);
            const float alpha = fminf(kAlphaMax, raw);
            const float inv = __builtin_amdgcn_rcpf(1.0f - alpha);  // 1 - alpha >= 0.01: the hardware reciprocal (1 ulp)
            const float Tb = pass[k] ? T[k] * inv : T[k];  // transmittance in front of the entry
            const float wc = pass[k] ? Tb * alpha : 0.0f;
            const float dot_rgb = gC[k][0] * s.r + gC[k][1] * s.g + gC[k][2] * s.b;
            const float dot_s = gC[k][0] * Sc[k][0] + gC[k][1] * Sc[k][1] + gC[k][2] * Sc[k][2];
            const float ga = Tb * dot_rgb - dot_s * inv;
            const float sk = (pass[k] && raw < kAlphaMax) ? ga * alpha : 0.0f;
            S0 += sk;
            const float dy = dy0 - 4.0f * k;
            const float sdy = sk * dy;
            S1 += sdy;
            S2 = fmaf(sdy, dy, S2);
            Sr = fmaf(wc, gC[k][0], Sr);
            Sg = fmaf(wc, gC[k][1], Sg);
            Sb = fmaf(wc, gC[k][2], Sb);
            Sc[k][0] = fmaf(s.r, wc, Sc[k][0]);
            Sc[k][1] = fmaf(s.g, wc, Sc[k][1]);
            Sc[k][2] = fmaf(s.b, wc, Sc[k][2]);
            T[k] = Tb;
        }
        // derivatives w.r.t. (u, v, a, b, c, opacity, r, g, b) of this lane's pixels
        float v9[9];
        v9[0] = kLn2 * (2.0f * s.A * dx * S0 + s.B * S1);
        v9[1] = kLn2 * (Bdx * S0 + 2.0f * s.C * S1);
        v9[2] = -0.5f * dx * dx * S0;
        v9[3] = -dx * S1;
        v9[4] = -0.5f * S2;
        v9[5] = S0;
        v9[6] = Sr;
        v9[7] = Sg;
        v9[8] = Sb;
        float sum = wave_sums_scatter9(v9, lane);  // lane q < 9: the sum of v9[q]
        if (lane == 5) sum *= exp2_fast(-s.lo);  // d alpha / d alpha_c = alpha / alpha_c
        if (lane < 9) atomicAdd(&d_splat[9 * g0 + (size_t)lane * n + g], sum);
    }
}

}  // namespace sd7
