// Perspective (EWA) projection of the conditional 3D Gaussians (Sec. 4.4),
// footprint, depth key and degree-3 SH colour (Sec. 3, eq. 2), and the
// reverse.  One lane per (frame, Gaussian), FP32.
//
// Footprint: the pixels where alpha_c exp(-q/2) >= 1/255 form the ellipse
// q <= k, k = 2 ln(alpha_c * 255); its exact bounding box has half-widths
// sqrt(k Sigma2D_xx), sqrt(k Sigma2D_yy).  Every 16x16 tile that box touches
// gets a (tile, Gaussian) pair, so tiles list every Gaussian that can reach
// alpha >= 1/255 at one of their pixel centres.
#include "common.h"
#include "footprint.h"
#include "gload.h"

namespace sd7 {

// Real SH basis of degree <= 3, k = l*l + l + m, (-1)^|m| sign convention.
__device__ __forceinline__ void sh_eval(float x, float y, float z, float Y[16])
{
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[0] = 0.28209479177387814f;
    Y[1] = -0.48860251190291992f * y;
    Y[2] = 0.48860251190291992f * z;
    Y[3] = -0.48860251190291992f * x;
    Y[4] = 1.0925484305920792f * x * y;
    Y[5] = -1.0925484305920792f * y * z;
    Y[6] = 0.31539156525252005f * (2.0f * zz - xx - yy);
    Y[7] = -1.0925484305920792f * x * z;
    Y[8] = 0.54627421529603959f * (xx - yy);
    Y[9] = -0.59004358992664352f * y * (3.0f * xx - yy);
    Y[10] = 2.8906114426405538f * x * y * z;
    Y[11] = -0.45704579946446572f * y * (4.0f * zz - xx - yy);
    Y[12] = 0.3731763325901154f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -0.45704579946446572f * x * (4.0f * zz - xx - yy);
    Y[14] = 1.4453057213202769f * z * (xx - yy);
    Y[15] = -0.59004358992664352f * x * (xx - 3.0f * yy);
}

// d(sum_k b_k Y_k)/d(x, y, z) for coefficient vector b (one channel).
__device__ __forceinline__ void sh_grad(float x, float y, float z, const float b[16], float g[3])
{
    const float xx = x * x, yy = y * y, zz = z * z;
    const float c1 = 0.48860251190291992f, c4 = 1.0925484305920792f, c6 = 0.31539156525252005f;
    const float c8 = 0.54627421529603959f, c9 = 0.59004358992664352f, c10 = 2.8906114426405538f;
    const float c11 = 0.45704579946446572f, c12 = 0.3731763325901154f, c14 = 1.4453057213202769f;
    float gx = 0.f, gy = 0.f, gz = 0.f;
    gy += b[1] * -c1;
    gz += b[2] * c1;
    gx += b[3] * -c1;
    gx += b[4] * c4 * y;            gy += b[4] * c4 * x;
    gy += b[5] * -c4 * z;           gz += b[5] * -c4 * y;
    gx += b[6] * c6 * -2.f * x;     gy += b[6] * c6 * -2.f * y;     gz += b[6] * c6 * 4.f * z;
    gx += b[7] * -c4 * z;           gz += b[7] * -c4 * x;
    gx += b[8] * c8 * 2.f * x;      gy += b[8] * c8 * -2.f * y;
    gx += b[9] * -c9 * 6.f * x * y; gy += b[9] * -c9 * (3.f * xx - 3.f * yy);
    gx += b[10] * c10 * y * z;      gy += b[10] * c10 * x * z;      gz += b[10] * c10 * x * y;
    gx += b[11] * -c11 * (-2.f * x * y);
    gy += b[11] * -c11 * (4.f * zz - xx - 3.f * yy);
    gz += b[11] * -c11 * (8.f * y * z);
    gx += b[12] * c12 * (-6.f * x * z);
    gy += b[12] * c12 * (-6.f * y * z);
    gz += b[12] * c12 * (6.f * zz - 3.f * xx - 3.f * yy);
    gx += b[13] * -c11 * (4.f * zz - 3.f * xx - yy);
    gy += b[13] * -c11 * (-2.f * x * y);
    gz += b[13] * -c11 * (8.f * x * z);
    gx += b[14] * c14 * 2.f * x * z; gy += b[14] * c14 * -2.f * y * z; gz += b[14] * c14 * (xx - yy);
    gx += b[15] * -c9 * (3.f * xx - 3.f * yy); gy += b[15] * -c9 * (-6.f * x * y);
    g[0] = gx; g[1] = gy; g[2] = gz;
}

// The projection of one conditional Gaussian, evaluated in FP64 from its FP32
// sliced statistics (the splat record and footprint are rounded to FP32 when
// written).  FP64 here keeps the 2D covariance's inverse accurate for
// elongated splats, whose 2D covariance is ill-conditioned: in FP32 its
// determinant cancels and the conic loses up to about 1e-3 of its value.
struct Proj {
    double x[3];      // camera coordinates
    double iz;        // 1 / z
    double u, v;      // mean2d
    double rx, ry;    // ratios used in J (clamped)
    bool clx, cly;    // ratio clamped
    double M[2][3];   // J R
    double s00, s01, s11, det;
    double a, b, c;   // conic
};

__device__ __forceinline__ bool project_one(const FrameDev& F, const float m[3], const float cv[6], Proj& p)
{
    const double dm0 = (double)m[0] - F.c[0], dm1 = (double)m[1] - F.c[1], dm2 = (double)m[2] - F.c[2];
#pragma unroll
    for (int r = 0; r < 3; ++r)
        p.x[r] = (double)F.R[3 * r] * dm0 + (double)F.R[3 * r + 1] * dm1 + (double)F.R[3 * r + 2] * dm2;
    const double z = p.x[2];
    if (!(z > (double)kZNear)) return false;
    const double fx = F.fx, fy = F.fy;
    p.iz = 1.0 / z;
    p.u = fx * p.x[0] * p.iz + (double)F.cx;
    p.v = fy * p.x[1] * p.iz + (double)F.cy;
    const double limx = F.limx, limy = F.limy;
    double rx = p.x[0] * p.iz, ry = p.x[1] * p.iz;
    p.clx = rx >= limx || rx <= -limx;
    p.cly = ry >= limy || ry <= -limy;
    rx = fmin(fmax(rx, -limx), limx);
    ry = fmin(fmax(ry, -limy), limy);
    p.rx = rx;
    p.ry = ry;
    const double j00 = fx * p.iz, j02 = -fx * rx * p.iz, j11 = fy * p.iz, j12 = -fy * ry * p.iz;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        p.M[0][k] = j00 * (double)F.R[k] + j02 * (double)F.R[6 + k];
        p.M[1][k] = j11 * (double)F.R[3 + k] + j12 * (double)F.R[6 + k];
    }
    const double S[3][3] = {{cv[0], cv[1], cv[2]}, {cv[1], cv[3], cv[4]}, {cv[2], cv[4], cv[5]}};
    double T[2][3];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) T[r][k] = p.M[r][0] * S[0][k] + p.M[r][1] * S[1][k] + p.M[r][2] * S[2][k];
    p.s00 = T[0][0] * p.M[0][0] + T[0][1] * p.M[0][1] + T[0][2] * p.M[0][2] + (double)kDilation;
    p.s01 = T[0][0] * p.M[1][0] + T[0][1] * p.M[1][1] + T[0][2] * p.M[1][2];
    p.s11 = T[1][0] * p.M[1][0] + T[1][1] * p.M[1][1] + T[1][2] * p.M[1][2] + (double)kDilation;
    p.det = p.s00 * p.s11 - p.s01 * p.s01;
    if (!(p.det > 0.0)) return false;
    const double idet = 1.0 / p.det;
    p.a = p.s11 * idet;
    p.b = -p.s01 * idet;
    p.c = p.s00 * idet;
    return true;
}

// Row trims of a footprint (the layout is described with Footprint): for the
// tile rows it stores, the tiles at either end of the row none of whose pixel
// centres the ellipse q <= k reaches.  The test runs on pixel centres: tile
// row ty's centres lie on the strip y in [16 ty + 1/2, 16 ty + 31/2], tile
// column tx's on x in [16 tx + 1/2, 16 tx + 31/2].  q is evaluated through
// the 2D covariance: at row offset dy the ellipse spans dx = dy s01 / s11 +-
// sqrt((k - dy^2 / s11) det / s11); on a strip of dy the left end is least at
// the clamp of the leftmost point's dy into the strip, the right end greatest
// at the clamp of the rightmost point's.  k is raised by 0.2 % plus 0.02 (in
// log2 of alpha, 3 % of headroom), well above the error of the hardware square
// root and reciprocal used here and of the rasterizer's FP32 exponent; a box
// one tile wide or high, or an ill-conditioned covariance, gets no trims.
__device__ __forceinline__ uint2 footprint_trims(const Proj& p, float k, uint32_t rx0, uint32_t ry0, uint32_t rx1,
                                                 uint32_t ry1)
{
    const uint32_t w = rx1 - rx0, h = ry1 - ry0;
    const float s00 = (float)p.s00, s01 = (float)p.s01, s11 = (float)p.s11, det = (float)p.det;
    const float pu = (float)p.u, pv = (float)p.v;
    const float tr = s00 + s11;
    if (w < 2 || h < 2 || !(tr * tr < 1e6f * det)) return make_uint2(0u, 0u);
    const uint32_t m = h > 8 ? h - 4 : 4;  // first of the bottom rows
    const uint32_t nrow = min(h, 8u);
    const float km = fmaf(k, 1.002f, 0.02f);
    const float r11 = __builtin_amdgcn_rcpf(s11);
    const float slope = s01 * r11, wsq = det * r11;
    const float dyx = s01 * __builtin_amdgcn_sqrtf(km * __builtin_amdgcn_rcpf(s00));  // rightmost point; leftmost at -dyx
    const float hy = __builtin_amdgcn_sqrtf(km * s11);
    const float inv_tile = 1.0f / (float)kTile;
    uint32_t word[2] = {0u, 0u};
    for (uint32_t q = 0; q < nrow; ++q) {
        const uint32_t r = q < 4 ? q : m + (q - 4);
        const float y = (float)((ry0 + r) * kTile) + 0.5f - pv;
        const float dya = fmaxf(y, -hy), dyb = fminf(y + (float)(kTile - 1), hy);
        const float yl = fminf(fmaxf(-dyx, dya), dyb), yr = fminf(fmaxf(dyx, dya), dyb);
        const float xl = fmaf(slope, yl, pu) - __builtin_amdgcn_sqrtf(fmaxf(fmaf(-yl * r11, yl, km), 0.0f) * wsq);
        const float xr = fmaf(slope, yr, pu) + __builtin_amdgcn_sqrtf(fmaxf(fmaf(-yr * r11, yr, km), 0.0f) * wsq);
        // tiles whose last centre column lies left of xl, or whose first lies
        // right of xr; a strip that misses the ellipse empties the row (as
        // far as 15 + 15 tiles go); NaN keeps the row whole (fmaxf returns the
        // other operand)
        float lt = fminf(fmaxf(ceilf((xl - (float)kTile + 0.5f) * inv_tile) - (float)rx0, 0.0f), 15.0f);
        float rt = fminf(fmaxf((float)(rx1 - 1) - floorf((xr - 0.5f) * inv_tile), 0.0f), 15.0f);
        if (!(dya <= dyb)) {
            lt = fminf((float)w, 15.0f);
            rt = fminf((float)w - lt, 15.0f);
        }
        word[q >> 2] |= ((uint32_t)lt | (uint32_t)rt << 4) << (8 * (q & 3));
    }
    return make_uint2(word[0], word[1]);
}

// SH coefficient j = 3k + ch of Gaussian i, read from the scene.
struct ShGlobal {
    const float* __restrict__ sh;
    uint32_t n;
    __device__ __forceinline__ float operator()(int j, uint32_t i) const { return gload(sh, (size_t)j * n + i); }
};

// Projection, footprint, colour and the splat record of Gaussian i of frame F
// from its FP32 slice outputs; returns whether the Gaussian is kept.  sh(j, i)
// gives SH coefficient j of the Gaussian.
template <class Sh>
__device__ __forceinline__ bool project_emit(const FrameDev& F, uint32_t i, float ac, const float m[3],
                                             const float cv[6], const Sh& sh, float4* __restrict__ splat,
                                             uint4* __restrict__ rect, uint32_t* __restrict__ depth_key)
{
    const size_t g0 = F.g0;
    Proj p;
    bool keep = ac >= kAlphaMin && project_one(F, m, cv, p);
    uint32_t rx0 = 0, ry0 = 0, rx1 = 0, ry1 = 0;
    uint2 trims = make_uint2(0u, 0u);
    if (keep) {
        const float k = 2.0f * logf(ac * 255.0f);
        const float pu = (float)p.u, pv = (float)p.v;
        const float hx = __builtin_amdgcn_sqrtf(k * (float)p.s00), hy = __builtin_amdgcn_sqrtf(k * (float)p.s11);
        float tx0 = floorf((pu - hx) / (float)kTile), tx1 = floorf((pu + hx) / (float)kTile);
        float ty0 = floorf((pv - hy) / (float)kTile), ty1 = floorf((pv + hy) / (float)kTile);
        tx0 = fmaxf(tx0, 0.0f);
        ty0 = fmaxf(ty0, 0.0f);
        tx1 = fminf(tx1, (float)F.tiles_x - 1.0f);
        ty1 = fminf(ty1, (float)F.tiles_y - 1.0f);
        keep = tx0 <= tx1 && ty0 <= ty1;  // false for NaN too
        if (keep) {
            rx0 = (uint32_t)tx0; ry0 = (uint32_t)ty0;
            rx1 = (uint32_t)tx1 + 1; ry1 = (uint32_t)ty1 + 1;
            trims = footprint_trims(p, k, rx0, ry0, rx1, ry1);
        }
    }
    float rgb[3] = {0.f, 0.f, 0.f};
    if (keep) {
        const float dx = m[0] - F.c[0], dy = m[1] - F.c[1], dz = m[2] - F.c[2];
        const float inv = __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
        float Y[16];
        sh_eval(dx * inv, dy * inv, dz * inv, Y);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float s = 0.5f;
#pragma unroll
            for (int k = 0; k < 16; ++k) s += sh(3 * k + ch, i) * Y[k];
            rgb[ch] = fmaxf(s, 0.0f);
        }
    }
    // a culled Gaussian gets only its depth key, which marks it: no later
    // stage reads its record or footprint
    if (keep) {
        float4* rec = splat + (g0 + i) * 3;
        // exponent of alpha in base 2: A dx^2 + B dx dy + C dy^2 + log2(alpha_c)
        const double nhl2e = -0.72134752044448170368;  // -log2(e) / 2
        const float C = (float)(nhl2e * p.c);
        rec[0] = make_float4((float)p.u, (float)p.v, (float)(nhl2e * p.a), (float)(2.0 * nhl2e * p.b));
        rec[1] = make_float4(C, log2f(ac), rgb[0], rgb[1]);
        rec[2] = make_float4(rgb[2], 16.0f * C, ac, (float)p.x[2]);
        rect[g0 + i] = make_uint4(rx0 | (ry0 << 16), rx1 | (ry1 << 16), trims.x, trims.y);
    }
    depth_key[g0 + i] = keep ? __float_as_uint((float)p.x[2]) : kCulled;
    return keep;
}

// Adds the wave's kept Gaussians to its block's count in LDS; the block then
// adds its count to the frame's counter with one atomic.  Same-address
// atomics serialize in L2: one per wave took more than half of a one-frame
// projection of 200k Gaussians (3,125 waves).
__device__ __forceinline__ void wave_kept(bool keep, uint32_t* s_count)
{
    const uint64_t kept = __ballot(keep);
    if (__lane_id() == 0 && kept) atomicAdd(s_count, (uint32_t)__popcll(kept));
}

__global__ __launch_bounds__(kBlock) void k_project(const FrameDev* __restrict__ tab, BlockMap bm,
                                                    const float* __restrict__ mu_c, const float* __restrict__ cov_c,
                                                    const float* __restrict__ alpha_c, float4* __restrict__ splat,
                                                    uint4* __restrict__ rect, uint32_t* __restrict__ depth_key,
                                                    uint32_t* __restrict__ counts)
{
    const int f = frame_of_block(bm, blockIdx.x);
    const FrameDev& F = tab[f];
    const uint32_t i = (blockIdx.x - bm.start[f]) * kBlock + threadIdx.x;
    __shared__ uint32_t s_kept;
    if (threadIdx.x == 0) s_kept = 0;
    __syncthreads();
    bool keep = false;
    if (i < F.n) {
        const uint32_t n = F.n;
        const size_t g0 = F.g0;
        float m[3], cv[6];
#pragma unroll
        for (int a = 0; a < 3; ++a) m[a] = mu_c[3 * g0 + (size_t)a * n + i];
#pragma unroll
        for (int e = 0; e < 6; ++e) cv[e] = cov_c[6 * g0 + (size_t)e * n + i];
        keep = project_emit(F, i, alpha_c[g0 + i], m, cv, ShGlobal{F.sh, n}, splat, rect, depth_key);
    }
    wave_kept(keep, &s_kept);
    __syncthreads();
    if (threadIdx.x == 0 && s_kept) atomicAdd(&counts[f * SD7_CNT_WORDS + SD7_CNT_KEPT], s_kept);
}

// Reverse of k_project.  d_splat planes per frame: (du, dv, da, db, dc, dop,
// dr, dg, db) where db is the derivative w.r.t. the conic b of
// q = a dx^2 + 2 b dx dy + c dy^2.
__global__ __launch_bounds__(kBlock) void k_project_bwd(const FrameDev* __restrict__ tab, BlockMap bm,
                                                        const float* __restrict__ mu_c,
                                                        const float* __restrict__ cov_c,
                                                        const float* __restrict__ alpha_c,
                                                        const uint32_t* __restrict__ depth_key,
                                                        const float* __restrict__ d_splat,
                                                        float* __restrict__ d_mu_c, float* __restrict__ d_cov_c,
                                                        float* __restrict__ d_alpha_c)
{
    const int f = frame_of_block(bm, blockIdx.x);
    const FrameDev& F = tab[f];
    const uint32_t i = (blockIdx.x - bm.start[f]) * kBlock + threadIdx.x;
    if (i >= F.n) return;
    const uint32_t n = F.n;
    const size_t g0 = F.g0;
    float gmu[3] = {0.f, 0.f, 0.f}, gcov[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, gac = 0.f;
    float gsh[48];
#pragma unroll
    for (int k = 0; k < 48; ++k) gsh[k] = 0.f;
    if (depth_key[g0 + i] != kCulled) {
        float ds[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) ds[k] = d_splat[9 * g0 + (size_t)k * n + i];
        float m[3], cv[6];
#pragma unroll
        for (int a = 0; a < 3; ++a) m[a] = mu_c[3 * g0 + (size_t)a * n + i];
#pragma unroll
        for (int e = 0; e < 6; ++e) cv[e] = cov_c[6 * g0 + (size_t)e * n + i];
        Proj p;
        project_one(F, m, cv, p);
        gac = ds[5];
        // colour
        const float dx = m[0] - F.c[0], dy = m[1] - F.c[1], dz = m[2] - F.c[2];
        const float len = sqrtf(dx * dx + dy * dy + dz * dz);
        const float inv = 1.0f / len;
        const float dir[3] = {dx * inv, dy * inv, dz * inv};
        float Y[16];
        sh_eval(dir[0], dir[1], dir[2], Y);
        float gdir[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float b[16];
            float s = 0.5f;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                b[k] = gload(F.sh, (size_t)(3 * k + ch) * n + i);
                s += b[k] * Y[k];
            }
            const float graw = s > 0.0f ? ds[6 + ch] : 0.0f;
            if (graw != 0.0f) {
#pragma unroll
                for (int k = 0; k < 16; ++k) gsh[3 * k + ch] = graw * Y[k];
                float g[3];
                sh_grad(dir[0], dir[1], dir[2], b, g);
#pragma unroll
                for (int a = 0; a < 3; ++a) gdir[a] += graw * g[a];
            }
        }
        const float dd = dir[0] * gdir[0] + dir[1] * gdir[1] + dir[2] * gdir[2];
#pragma unroll
        for (int a = 0; a < 3; ++a) gmu[a] += (gdir[a] - dir[a] * dd) * inv;

        // conic (a, b, c) = inverse of Sigma2D -> d(s00, s01, s11), FP64 like the forward
        const double ga = ds[2], gb = ds[3], gc = ds[4];
        const double A = p.a, B = p.b, C = p.c;
        const double g00 = -(ga * A * A + gb * A * B + gc * B * B);
        const double g11 = -(ga * B * B + gb * B * C + gc * C * C);
        const double g01 = -(2.0 * ga * A * B + gb * (A * C + B * B) + 2.0 * gc * B * C);
        // symmetric 2x2 gradient of Sigma2D (entries independent)
        const double G2[2][2] = {{g00, 0.5 * g01}, {0.5 * g01, g11}};
        // dSigma_c = M^T G2 M
        double GM[2][3];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k) GM[r][k] = G2[r][0] * p.M[0][k] + G2[r][1] * p.M[1][k];
        double Gs[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b2 = 0; b2 < 3; ++b2) Gs[a][b2] = p.M[0][a] * GM[0][b2] + p.M[1][a] * GM[1][b2];
        gcov[0] = (float)Gs[0][0];
        gcov[1] = (float)(Gs[0][1] + Gs[1][0]);
        gcov[2] = (float)(Gs[0][2] + Gs[2][0]);
        gcov[3] = (float)Gs[1][1];
        gcov[4] = (float)(Gs[1][2] + Gs[2][1]);
        gcov[5] = (float)Gs[2][2];
        // dM = 2 G2 M Sigma_c ; dJ = dM R^T
        const double S[3][3] = {{cv[0], cv[1], cv[2]}, {cv[1], cv[3], cv[4]}, {cv[2], cv[4], cv[5]}};
        double dM[2][3];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                dM[r][k] = 2.0 * (GM[r][0] * S[0][k] + GM[r][1] * S[1][k] + GM[r][2] * S[2][k]);
        double dJ[2][3];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int q = 0; q < 3; ++q)
                dJ[r][q] = dM[r][0] * F.R[3 * q] + dM[r][1] * F.R[3 * q + 1] + dM[r][2] * F.R[3 * q + 2];
        const double fx = F.fx, fy = F.fy;
        const double x = p.x[0], y = p.x[1];
        const double iz = p.iz, iz2 = iz * iz;
        double gx = 0.0, gy = 0.0, gz = 0.0;
        // J00 = fx/z, J02 = -fx rx/z, J11 = fy/z, J12 = -fy ry/z
        gz += dJ[0][0] * (-fx * iz2) + dJ[1][1] * (-fy * iz2);
        if (!p.clx) {
            gx += dJ[0][2] * (-fx * iz2);
            gz += dJ[0][2] * (2.0 * fx * x * iz2 * iz);
        } else {
            gz += dJ[0][2] * (fx * p.rx * iz2);
        }
        if (!p.cly) {
            gy += dJ[1][2] * (-fy * iz2);
            gz += dJ[1][2] * (2.0 * fy * y * iz2 * iz);
        } else {
            gz += dJ[1][2] * (fy * p.ry * iz2);
        }
        // mean2d
        gx += (double)ds[0] * fx * iz;
        gz += (double)ds[0] * (-fx * x * iz2);
        gy += (double)ds[1] * fy * iz;
        gz += (double)ds[1] * (-fy * y * iz2);
        // x_cam = R (mu - c)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            gmu[a] += (float)((double)F.R[a] * gx + (double)F.R[3 + a] * gy + (double)F.R[6 + a] * gz);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) d_mu_c[3 * g0 + (size_t)a * n + i] = gmu[a];
#pragma unroll
    for (int e = 0; e < 6; ++e) d_cov_c[6 * g0 + (size_t)e * n + i] = gcov[e];
    d_alpha_c[g0 + i] = gac;
#pragma unroll
    for (int k = 0; k < 48; ++k) F.g_sh[(size_t)k * n + i] = gsh[k];
}

}  // namespace sd7
