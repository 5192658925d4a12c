// Densification helpers (Sec. 4.4 "Optimization and Rendering Pipeline";
// Algorithm 1's optional last step): the scale and rotation of a sliced
// covariance, and the temporal split test.  One lane per Gaussian, FP64.
#include "common.h"

namespace sd7 {

// Sigma = R diag(S^2) R^T for a symmetric 3x3 Sigma (packed xx, xy, xz, yy,
// yz, zz): cyclic Jacobi rotations in FP64 until the off-diagonal part is
// below 2^-52 of the diagonal (at most kJacobiSweeps sweeps), eigenvalues in
// descending order, S = sqrt(max(eigenvalue, 0)), and the last column of R
// negated when det R < 0 so that R is a proper rotation.
constexpr int kJacobiSweeps = 12;

__device__ __forceinline__ void jacobi_rotate(double A[3][3], double V[3][3], int p, int q)
{
    const double apq = A[p][q];
    if (apq == 0.0) return;
    const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
    const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(fma(theta, theta, 1.0)));
    const double c = 1.0 / sqrt(fma(t, t, 1.0)), s = t * c;
    // A <- J^T A J with J the rotation in the (p, q) plane
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double akp = A[k][p], akq = A[k][q];
        A[k][p] = c * akp - s * akq;
        A[k][q] = s * akp + c * akq;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double apk = A[p][k], aqk = A[q][k];
        A[p][k] = c * apk - s * aqk;
        A[q][k] = s * apk + c * aqk;
    }
    A[p][q] = A[q][p] = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double vkp = V[k][p], vkq = V[k][q];
        V[k][p] = c * vkp - s * vkq;
        V[k][q] = s * vkp + c * vkq;
    }
}

__global__ __launch_bounds__(kBlock) void k_cov_decompose(uint32_t n, const float* __restrict__ cov,
                                                          float* __restrict__ scale, float* __restrict__ rot)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double A[3][3], V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    A[0][0] = cov[i];
    A[0][1] = A[1][0] = cov[(size_t)n + i];
    A[0][2] = A[2][0] = cov[2 * (size_t)n + i];
    A[1][1] = cov[3 * (size_t)n + i];
    A[1][2] = A[2][1] = cov[4 * (size_t)n + i];
    A[2][2] = cov[5 * (size_t)n + i];
    for (int sweep = 0; sweep < kJacobiSweeps; ++sweep) {
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (!(off > 0x1p-104 * dia)) break;  // also ends on a zero or non-finite matrix
        jacobi_rotate(A, V, 0, 1);
        jacobi_rotate(A, V, 0, 2);
        jacobi_rotate(A, V, 1, 2);
    }
    double ev[3] = {A[0][0], A[1][1], A[2][2]};
    int o[3] = {0, 1, 2};  // order of the eigenvalues, descending
    if (ev[o[0]] < ev[o[1]]) { const int t = o[0]; o[0] = o[1]; o[1] = t; }
    if (ev[o[1]] < ev[o[2]]) { const int t = o[1]; o[1] = o[2]; o[2] = t; }
    if (ev[o[0]] < ev[o[1]]) { const int t = o[0]; o[0] = o[1]; o[1] = t; }
    double R[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) R[r][c] = V[r][o[c]];
    const double det = R[0][0] * (R[1][1] * R[2][2] - R[1][2] * R[2][1]) -
                       R[0][1] * (R[1][0] * R[2][2] - R[1][2] * R[2][0]) +
                       R[0][2] * (R[1][0] * R[2][1] - R[1][1] * R[2][0]);
    if (det < 0.0) {
#pragma unroll
        for (int r = 0; r < 3; ++r) R[r][2] = -R[r][2];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) scale[(size_t)c * n + i] = (float)sqrt(fmax(ev[o[c]], 0.0));
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) rot[(size_t)(3 * r + c) * n + i] = (float)R[r][c];
}

// Split test: |Sigma_pt| = |(Sigma_xt, Sigma_yt, Sigma_zt)| > 0.05 extent and
// sqrt(Sigma_t) / time_span > 0.25, from Sigma = L L^T (FP64).
__global__ __launch_bounds__(kBlock) void k_split_test(uint32_t n, const float* __restrict__ Lp, float extent,
                                                       float time_span, uint8_t* __restrict__ out)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    auto l = [&](int a, int b) { return (double)Lp[(size_t)(a * (a + 1) / 2 + b) * n + i]; };
    double s2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;  // Sigma[a][t] = sum_k L[a][k] L[t][k], k <= a
#pragma unroll
        for (int k = 0; k <= a; ++k) s = fma(l(a, k), l(3, k), s);
        s2 = fma(s, s, s2);
    }
    double stt = 0.0;
#pragma unroll
    for (int k = 0; k <= 3; ++k) stt = fma(l(3, k), l(3, k), stt);
    const bool split = sqrt(s2) > 0.05 * (double)extent && sqrt(stt) / (double)time_span > 0.25;
    out[i] = split ? 1 : 0;
}

}  // namespace sd7
