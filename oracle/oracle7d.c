/*
 * oracle7d.c -- plain FP64 reference ("oracle") of the 7DGS render path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path (the
 * HIP library) shares no code, header, table or constant generator with it.
 *
 * What it computes, per view, for a scene of 7D Gaussians:
 *   slice    Sec. 4.2, eq. cond_mean / cond_cov (Schur complement of the 7x7
 *            covariance Sigma = L L^T of Sec. 4.1), the temporal and
 *            directional modulation eq. temp_mod / eq. dir_mod and the
 *            conditional opacity alpha_cond = alpha f_temp f_dir; Algorithm 1
 *            steps 3-6.
 *   agr      Sec. 4.3 (Algorithm 1 steps 1-2), optional: the feature vector
 *            f = mu_p (+) mu_t (+) mu_d (+) gamma(t) and four two-layer MLPs
 *            whose outputs are added to mu_p, mu_t, mu_d and the packed L
 *            before slicing.  Without it the path is the "w/o AGR" variant
 *            of Table 1.
 *   project  Sec. 4.4: standard perspective (EWA) projection of the
 *            conditional 3D Gaussian to a 2D Gaussian; colour from degree-3
 *            spherical harmonics (Sec. 3, eq. 2, reused unchanged per Sec. 4.1).
 *   render   Sec. 4.4: depth-aware, opacity-blended front-to-back compositing,
 *            done by brute force: every visible Gaussian is tested at every
 *            pixel, in (depth, index) order.  No tiles.
 *
 * The paper leaves the rasterizer constants unstated; the readings used here
 * are: ALPHA_MIN = (float)(1/255), ALPHA_MAX = 0.99f, T_MIN = 1e-4f,
 * Z_NEAR = 0.2f, DILATION = 0.3f px^2, J evaluated at view-ray ratios clamped
 * to 1.3x the half-fov tangent, depth = camera-space z, ties broken by
 * Gaussian index, colour = max(0, 0.5 + SH), SH evaluated at the unit vector
 * from the camera centre to the conditional mean.  Each constant is the FP32
 * value promoted to FP64.
 *
 * Inputs are FP64 arrays (structure of arrays, layouts in oracle7d.h); the
 * scene files are FP32 and are promoted exactly by the caller.  All
 * arithmetic is FP64.
 */
#include "oracle7d.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ALPHA_MIN ((double)(float)(1.0 / 255.0))
#define ALPHA_MAX ((double)0.99f)
#define T_MIN ((double)1e-4f)
#define Z_NEAR ((double)0.2f)
#define DILATION ((double)0.3f)
#define JCLAMP ((double)1.3f)
#define TILE 16
#define ORA_PI 3.14159265358979323846

static int tri(int i, int j) { return i * (i + 1) / 2 + j; }

/* ---------------------------------------------------------------------- */
/* small dense FP64 linear algebra                                         */
/* ---------------------------------------------------------------------- */

/* Cholesky A = C C^T of an SPD m x m matrix (row-major, stride m).
 * Returns 0 on success, -1 if A is not positive definite. */
static int cholesky(int m, const double* A, double* C)
{
    memset(C, 0, sizeof(double) * m * m);
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[i * m + j];
            for (int k = 0; k < j; ++k) s -= C[i * m + k] * C[j * m + k];
            if (i == j) {
                if (!(s > 0.0)) return -1;
                C[i * m + i] = sqrt(s);
            } else {
                C[i * m + j] = s / C[j * m + j];
            }
        }
    }
    return 0;
}

/* Solve (C C^T) x = b in place, C lower-triangular m x m. */
static void chol_solve(int m, const double* C, double* x)
{
    for (int i = 0; i < m; ++i) {          /* forward: C y = b */
        double s = x[i];
        for (int k = 0; k < i; ++k) s -= C[i * m + k] * x[k];
        x[i] = s / C[i * m + i];
    }
    for (int i = m - 1; i >= 0; --i) {     /* backward: C^T x = y */
        double s = x[i];
        for (int k = i + 1; k < m; ++k) s -= C[k * m + i] * x[k];
        x[i] = s / C[i * m + i];
    }
}

/* ---------------------------------------------------------------------- */
/* slice: Sec. 4.2                                                          */
/* ---------------------------------------------------------------------- */

int ora_slice(int64_t n, const double* mu_p, const double* mu_t, const double* mu_d,
              const double* Lp, const double* alpha, const ora_view* v,
              double* mu_c, double* cov_c, double* alpha_c, double* f_temp, double* f_dir,
              int32_t* status)
{
    const double t = v->t, lt = v->lambda_t, ld = v->lambda_d;
    const double d[3] = {v->d[0], v->d[1], v->d[2]};
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int64_t g = 0; g < n; ++g) {
        /* Sigma = L L^T (Sec. 4.1), dimensions (x, y, z, t, dx, dy, dz). */
        double L[7][7] = {{0}}, S[7][7];
        for (int i = 0; i < 7; ++i)
            for (int j = 0; j <= i; ++j) L[i][j] = Lp[(int64_t)tri(i, j) * n + g];
        for (int i = 0; i < 7; ++i)
            for (int j = 0; j < 7; ++j) {
                double s = 0.0;
                for (int k = 0; k < 7; ++k) s += L[i][k] * L[j][k];
                S[i][j] = s;
            }
        int st = 0;
        for (int i = 0; i < 7; ++i)
            if (!(L[i][i] > 0.0)) st = 1;

        /* Partition: P = {x, y, z}, Q = {t, dx, dy, dz}. */
        double SQQ[16], CQQ[16];
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) SQQ[i * 4 + j] = S[3 + i][3 + j];
        if (cholesky(4, SQQ, CQQ) != 0) st |= 2;

        /* r = (t - mu_t, d - mu_d); d is the view's, or unit(mu_p - c) */
        double dg[3] = {d[0], d[1], d[2]};
        if (v->d_mode) {
            double e[3], nn = 0.0;
            for (int k = 0; k < 3; ++k) {
                e[k] = mu_p[(int64_t)k * n + g] - (double)v->c[k];
                nn += e[k] * e[k];
            }
            nn = sqrt(nn);
            for (int k = 0; k < 3; ++k) dg[k] = e[k] / nn;
        }
        double r[4];
        r[0] = t - (double)mu_t[g];
        for (int k = 0; k < 3; ++k) r[1 + k] = dg[k] - (double)mu_d[(int64_t)k * n + g];

        /* eq. cond_mean: mu_cond = mu_p + Sigma_PQ Sigma_QQ^{-1} r */
        double w[4] = {r[0], r[1], r[2], r[3]};
        chol_solve(4, CQQ, w);
        double mc[3];
        for (int i = 0; i < 3; ++i) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += S[i][3 + k] * w[k];
            mc[i] = (double)mu_p[(int64_t)i * n + g] + s;
        }
        /* eq. cond_cov: Sigma_cond = Sigma_PP - Sigma_PQ Sigma_QQ^{-1} Sigma_QP */
        double Kt[3][4];   /* row i = Sigma_QQ^{-1} Sigma_Q,i  (i.e. K^T column) */
        for (int i = 0; i < 3; ++i) {
            for (int k = 0; k < 4; ++k) Kt[i][k] = S[3 + k][i];
            chol_solve(4, CQQ, Kt[i]);
        }
        double Sc[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s = 0.0;
                for (int k = 0; k < 4; ++k) s += S[i][3 + k] * Kt[j][k];
                Sc[i][j] = S[i][j] - s;
            }
        for (int i = 0; i < 3; ++i)           /* symmetrize */
            for (int j = i + 1; j < 3; ++j) {
                double m = 0.5 * (Sc[i][j] + Sc[j][i]);
                Sc[i][j] = Sc[j][i] = m;
            }

        /* eq. temp_mod with the marginal temporal variance Sigma_t = S[3][3] */
        double ft = exp(-0.5 * lt * r[0] * r[0] / S[3][3]);
        /* eq. dir_mod with the marginal directional covariance Sigma_d */
        double SDD[9], CDD[9], dd[3] = {r[1], r[2], r[3]};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) SDD[i * 3 + j] = S[4 + i][4 + j];
        double fd = 0.0;
        if (cholesky(3, SDD, CDD) == 0) {
            chol_solve(3, CDD, dd);
            double qd = r[1] * dd[0] + r[2] * dd[1] + r[3] * dd[2];
            fd = exp(-0.5 * ld * qd);
        } else {
            st |= 2;
        }
        double ac = (double)alpha[g] * ft * fd;

        for (int i = 0; i < 3; ++i) mu_c[(int64_t)i * n + g] = mc[i];
        cov_c[0 * n + g] = Sc[0][0];
        cov_c[1 * n + g] = Sc[0][1];
        cov_c[2 * n + g] = Sc[0][2];
        cov_c[3 * n + g] = Sc[1][1];
        cov_c[4 * n + g] = Sc[1][2];
        cov_c[5 * n + g] = Sc[2][2];
        alpha_c[g] = ac;
        if (f_temp) f_temp[g] = ft;
        if (f_dir) f_dir[g] = fd;
        if (status) status[g] = st;
        if (st) bad += 1;
    }
    return bad;
}

/* ---------------------------------------------------------------------- */
/* spherical harmonics, degree 3 (Sec. 3, eq. 2)                           */
/* ---------------------------------------------------------------------- */

/* Real SH basis Y_k, k = l*l + l + m, with the (-1)^|m| sign convention,
 * written out from the closed forms N_lm P_l^|m| (cos theta) trig(m phi). */
static void sh_basis(double x, double y, double z, double Y[16])
{
    const double pi = 3.14159265358979323846;
    Y[0] = 0.5 / sqrt(pi);
    Y[1] = -sqrt(3.0 / (4.0 * pi)) * y;
    Y[2] = sqrt(3.0 / (4.0 * pi)) * z;
    Y[3] = -sqrt(3.0 / (4.0 * pi)) * x;
    Y[4] = 0.5 * sqrt(15.0 / pi) * x * y;
    Y[5] = -0.5 * sqrt(15.0 / pi) * y * z;
    Y[6] = 0.25 * sqrt(5.0 / pi) * (2.0 * z * z - x * x - y * y);
    Y[7] = -0.5 * sqrt(15.0 / pi) * x * z;
    Y[8] = 0.25 * sqrt(15.0 / pi) * (x * x - y * y);
    Y[9] = -0.25 * sqrt(35.0 / (2.0 * pi)) * y * (3.0 * x * x - y * y);
    Y[10] = 0.5 * sqrt(105.0 / pi) * x * y * z;
    Y[11] = -0.25 * sqrt(21.0 / (2.0 * pi)) * y * (4.0 * z * z - x * x - y * y);
    Y[12] = 0.25 * sqrt(7.0 / pi) * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y);
    Y[13] = -0.25 * sqrt(21.0 / (2.0 * pi)) * x * (4.0 * z * z - x * x - y * y);
    Y[14] = 0.25 * sqrt(105.0 / pi) * z * (x * x - y * y);
    Y[15] = -0.25 * sqrt(35.0 / (2.0 * pi)) * x * (x * x - 3.0 * y * y);
}

void ora_sh_basis(double x, double y, double z, double* Y) { sh_basis(x, y, z, Y); }

/* ---------------------------------------------------------------------- */
/* project: Sec. 4.4 (perspective projection to 2D Gaussians)              */
/* ---------------------------------------------------------------------- */

int64_t ora_project(int64_t n, const double* mu_c, const double* cov_c, const double* alpha_c,
                    const double* sh, const ora_view* v, double* mean2d, double* conic,
                    double* depth, double* rgb, int32_t* rect, uint8_t* visible, double* box)
{
    double R[9], c[3];
    for (int k = 0; k < 9; ++k) R[k] = v->R[k];
    for (int k = 0; k < 3; ++k) c[k] = v->c[k];
    const double fx = v->fx, fy = v->fy, cx = v->cx, cy = v->cy;
    const int tiles_x = (v->W + TILE - 1) / TILE, tiles_y = (v->H + TILE - 1) / TILE;
    const double limx = JCLAMP * (0.5 * v->W) / fx, limy = JCLAMP * (0.5 * v->H) / fy;
    int64_t nvis = 0;
#pragma omp parallel for schedule(static) reduction(+ : nvis)
    for (int64_t g = 0; g < n; ++g) {
        int vis = 1;
        double m[3] = {mu_c[g], mu_c[n + g], mu_c[2 * n + g]};
        double ac = alpha_c[g];
        if (!(ac >= ALPHA_MIN)) vis = 0;
        /* camera coordinates x = R (mu - c) */
        double dm[3] = {m[0] - c[0], m[1] - c[1], m[2] - c[2]};
        double x[3];
        for (int i = 0; i < 3; ++i) x[i] = R[3 * i] * dm[0] + R[3 * i + 1] * dm[1] + R[3 * i + 2] * dm[2];
        if (!(x[2] > Z_NEAR)) vis = 0;
        double u = 0, vv = 0, a = 0, b = 0, cc = 0, S00 = 0, S11 = 0;
        if (vis) {
            u = fx * x[0] / x[2] + cx;
            vv = fy * x[1] / x[2] + cy;
            /* EWA: Sigma_2D = J R Sigma_c R^T J^T + DILATION I */
            double rx = x[0] / x[2], ry = x[1] / x[2];
            if (rx > limx) rx = limx;
            if (rx < -limx) rx = -limx;
            if (ry > limy) ry = limy;
            if (ry < -limy) ry = -limy;
            double J[2][3] = {{fx / x[2], 0.0, -fx * rx / x[2]}, {0.0, fy / x[2], -fy * ry / x[2]}};
            double Sc[3][3] = {{cov_c[g], cov_c[n + g], cov_c[2 * n + g]},
                               {cov_c[n + g], cov_c[3 * n + g], cov_c[4 * n + g]},
                               {cov_c[2 * n + g], cov_c[4 * n + g], cov_c[5 * n + g]}};
            double M[2][3];  /* M = J R */
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 3; ++j)
                    M[i][j] = J[i][0] * R[j] + J[i][1] * R[3 + j] + J[i][2] * R[6 + j];
            double S2[2][2];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) {
                    double s = 0.0;
                    for (int k = 0; k < 3; ++k)
                        for (int l = 0; l < 3; ++l) s += M[i][k] * Sc[k][l] * M[j][l];
                    S2[i][j] = s;
                }
            S2[0][0] += DILATION;
            S2[1][1] += DILATION;
            S00 = S2[0][0];
            S11 = S2[1][1];
            double det = S2[0][0] * S2[1][1] - S2[0][1] * S2[1][0];
            if (!(det > 0.0)) {
                vis = 0;
            } else {
                a = S2[1][1] / det;
                b = -S2[0][1] / det;
                cc = S2[0][0] / det;
            }
        }
        int32_t rc[4] = {0, 0, 0, 0};
        double bx[4] = {0, 0, 0, 0};
        if (vis) {
            /* exact bounding box of {alpha >= ALPHA_MIN}: q <= 2 ln(alpha_c / ALPHA_MIN) */
            double k = 2.0 * log(ac / ALPHA_MIN);
            double hx = sqrt(k * S00), hy = sqrt(k * S11);
            bx[0] = u - hx;
            bx[1] = vv - hy;
            bx[2] = u + hx;
            bx[3] = vv + hy;
            double tx0 = floor((u - hx) / TILE), tx1 = floor((u + hx) / TILE);
            double ty0 = floor((vv - hy) / TILE), ty1 = floor((vv + hy) / TILE);
            if (tx0 < 0) tx0 = 0;
            if (ty0 < 0) ty0 = 0;
            if (tx1 > tiles_x - 1) tx1 = tiles_x - 1;
            if (ty1 > tiles_y - 1) ty1 = tiles_y - 1;
            if (!(tx0 <= tx1 && ty0 <= ty1)) {
                vis = 0;
            } else {
                rc[0] = (int32_t)tx0;
                rc[1] = (int32_t)ty0;
                rc[2] = (int32_t)tx1 + 1;
                rc[3] = (int32_t)ty1 + 1;
            }
        }
        /* colour: SH at the world-space direction from the camera centre */
        double col[3] = {0, 0, 0};
        if (vis) {
            double len = sqrt(dm[0] * dm[0] + dm[1] * dm[1] + dm[2] * dm[2]);
            double Y[16];
            sh_basis(dm[0] / len, dm[1] / len, dm[2] / len, Y);
            for (int ch = 0; ch < 3; ++ch) {
                double s = 0.0;
                for (int k = 0; k < 16; ++k) s += (double)sh[(int64_t)(3 * k + ch) * n + g] * Y[k];
                s += 0.5;
                col[ch] = s > 0.0 ? s : 0.0;
            }
        }
        mean2d[g] = u;
        mean2d[n + g] = vv;
        conic[g] = a;
        conic[n + g] = b;
        conic[2 * n + g] = cc;
        depth[g] = x[2];
        for (int ch = 0; ch < 3; ++ch) rgb[(int64_t)ch * n + g] = col[ch];
        for (int k = 0; k < 4; ++k) rect[(int64_t)k * n + g] = rc[k];
        if (box)
            for (int k = 0; k < 4; ++k) box[(int64_t)k * n + g] = bx[k];
        visible[g] = (uint8_t)vis;
        nvis += vis;
    }
    return nvis;
}

/* ---------------------------------------------------------------------- */
/* render: brute-force front-to-back compositing (Sec. 4.4)               */
/* ---------------------------------------------------------------------- */

typedef struct {
    double z;
    int64_t g;
} zkey;

static int zkey_cmp(const void* pa, const void* pb)
{
    const zkey* a = (const zkey*)pa;
    const zkey* b = (const zkey*)pb;
    if (a->z < b->z) return -1;
    if (a->z > b->z) return 1;
    return (a->g > b->g) - (a->g < b->g);
}

int64_t ora_order(int64_t n, const double* depth, const uint8_t* visible, int64_t* order)
{
    int64_t m = 0;
    for (int64_t g = 0; g < n; ++g) m += visible[g] ? 1 : 0;
    zkey* keys = (zkey*)malloc(sizeof(zkey) * (m ? m : 1));
    int64_t j = 0;
    for (int64_t g = 0; g < n; ++g)
        if (visible[g]) {
            keys[j].z = depth[g];
            keys[j].g = g;
            ++j;
        }
    qsort(keys, (size_t)m, sizeof(zkey), zkey_cmp);
    for (j = 0; j < m; ++j) order[j] = keys[j].g;
    free(keys);
    return m;
}

/* ---------------------------------------------------------------------- */
/* FP32 decision bands of the parity protocol (not part of the method)     */
/* ---------------------------------------------------------------------- */

/* Per Gaussian, the scales of the error an FP32 evaluation of the path makes
 * in its splat (mean2d, conic, depth), given FP32-rounded sliced statistics:
 *   errpar[0] = max(fx, fy) / z * max_k |mu_c,k|  (mean2d error per unit of
 *               relative error of mu_c, in pixels)
 *   errpar[1..3] = (|M| |Sigma_c| |M|^T)_{00, 01, 11} with M = J R: a bound on
 *               the 2D covariance's change per unit of relative error of the
 *               entries of Sigma_c (no cancellation credited)
 *   errpar[4] = max_k |mu_c,k| + |z|  (depth error per unit relative error)
 * Culled Gaussians get zeros. */
void ora_fp32_model(int64_t n, const double* mu_c, const double* cov_c, const ora_view* v, double* errpar)
{
    double R[9], c[3];
    for (int k = 0; k < 9; ++k) R[k] = v->R[k];
    for (int k = 0; k < 3; ++k) c[k] = v->c[k];
    const double fx = v->fx, fy = v->fy;
    const double limx = JCLAMP * (0.5 * v->W) / fx, limy = JCLAMP * (0.5 * v->H) / fy;
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
        double m[3], x[3], mmax = 0.0;
        for (int k = 0; k < 3; ++k) {
            m[k] = mu_c[(int64_t)k * n + g] - c[k];
            const double a = fabs(mu_c[(int64_t)k * n + g]);
            if (a > mmax) mmax = a;
        }
        for (int i = 0; i < 3; ++i) x[i] = R[3 * i] * m[0] + R[3 * i + 1] * m[1] + R[3 * i + 2] * m[2];
        double e[5] = {0, 0, 0, 0, 0};
        if (x[2] > Z_NEAR) {
            double rx = x[0] / x[2], ry = x[1] / x[2];
            rx = rx > limx ? limx : (rx < -limx ? -limx : rx);
            ry = ry > limy ? limy : (ry < -limy ? -limy : ry);
            const double J[2][3] = {{fx / x[2], 0.0, -fx * rx / x[2]}, {0.0, fy / x[2], -fy * ry / x[2]}};
            double M[2][3];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 3; ++j) M[i][j] = fabs(J[i][0] * R[j] + J[i][1] * R[3 + j] + J[i][2] * R[6 + j]);
            const double S[3][3] = {{fabs(cov_c[g]), fabs(cov_c[n + g]), fabs(cov_c[2 * n + g])},
                                    {fabs(cov_c[n + g]), fabs(cov_c[3 * n + g]), fabs(cov_c[4 * n + g])},
                                    {fabs(cov_c[2 * n + g]), fabs(cov_c[4 * n + g]), fabs(cov_c[5 * n + g])}};
            double A[2][2];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) {
                    double s = 0.0;
                    for (int k = 0; k < 3; ++k)
                        for (int l = 0; l < 3; ++l) s += M[i][k] * S[k][l] * M[j][l];
                    A[i][j] = s;
                }
            e[0] = (fx > fy ? fx : fy) / x[2] * mmax;
            e[1] = A[0][0];
            e[2] = A[0][1];
            e[3] = A[1][1];
            e[4] = mmax + fabs(x[2]);
        }
        for (int k = 0; k < 5; ++k) errpar[(int64_t)k * n + g] = e[k];
    }
}

/* A decision the oracle takes within its FP32 band, for the per-pixel bound
 * on how much the image may change if an FP32 evaluation takes it the other
 * way.  kind: 0 skipped at ALPHA_MIN, 1 blended at ALPHA_MIN, 2 stopped at
 * T_MIN, 3 continued at T_MIN. */
typedef struct {
    int kind;
    double a, T, C[3], rgb[3];
} ora_event;
#define ORA_MAX_EVENTS 32

/* Band of ln alpha of Gaussian g at a pixel at offset (dx, dy) from its mean
 * (the model described with ora_flagcfg). */
static double band_lnalpha(int64_t n, int64_t g, const double* mean2d, const double* errpar,
                           const ora_flagcfg* fc, double ca, double cb, double cc, double dx, double dy)
{
    const double E = ldexp(1.0, -24);
    const double w0 = ca * dx + cb * dy, w1 = cb * dx + cc * dy;
    const double aw0 = fabs(w0), aw1 = fabs(w1);
    const double qabs = ca * dx * dx + 2.0 * fabs(cb * dx * dy) + cc * dy * dy;
    const double squad = aw0 * aw0 * errpar[n + g] + 2.0 * aw0 * aw1 * errpar[2 * n + g] +
                         aw1 * aw1 * errpar[3 * n + g];
    return E * (fc->k_mu * (aw0 + aw1) * errpar[g] + fc->k_uv * (aw0 * fabs(mean2d[g]) + aw1 * fabs(mean2d[n + g])) +
                fc->k_s * 0.5 * squad + fc->k_eval * (8.0 + 0.5 * qabs) + fc->k_ac);
}

int ora_composite(int64_t n, const double* mean2d, const double* conic, const double* alpha_c,
                  const double* depth, const double* rgb, const double* errpar, int64_t m,
                  const int64_t* order, const ora_view* v, int x0, int y0, int w, int h,
                  const ora_flagcfg* fc, double* image, double* final_T, int32_t* ncontrib,
                  uint64_t* chash, uint32_t* flags, double* fbound, int64_t* ntest, double* vbound)
{
    const double bg[3] = {v->bg[0], v->bg[1], v->bg[2]};
    const int64_t npx = (int64_t)w * h;
    const double E = ldexp(1.0, -24);
    const int banded = fc != NULL && errpar != NULL;
    /* largest colour any composite term can carry (for events beyond the
     * per-pixel record) */
    double cmax = 0.0;
    for (int ch = 0; ch < 3; ++ch) cmax = bg[ch] > cmax ? bg[ch] : cmax;
    for (int64_t j = 0; j < m; ++j)
        for (int ch = 0; ch < 3; ++ch) {
            const double x = rgb[(int64_t)ch * n + order[j]];
            cmax = x > cmax ? x : cmax;
        }
#pragma omp parallel for schedule(dynamic, 1)
    for (int py = 0; py < h; ++py) {
        for (int px = 0; px < w; ++px) {
            const double pxc = x0 + px + 0.5, pyc = y0 + py + 0.5;
            double T = 1.0, C[3] = {0, 0, 0};
            int32_t nc = 0;
            uint64_t hsh = 1469598103934665603ull;
            ora_event ev[ORA_MAX_EVENTS];
            int nev = 0;
            double fb = 0.0;     /* bound of events already settled */
            uint32_t fl = 0;
            double eT = 0.0;     /* band of ln T accumulated so far */
            int have_prev = 0;
            double prev_z = 0, prev_ez = 0, prev_a = 0, prev_rgb[3] = {0, 0, 0}, prev_T = 0;
            int64_t j = 0;
            for (; j < m; ++j) {
                const int64_t g = order[j];
                const double dx = mean2d[g] - pxc, dy = mean2d[n + g] - pyc;
                const double ca = conic[g], cb = conic[n + g], cc = conic[2 * n + g];
                const double q = ca * dx * dx + 2.0 * cb * dx * dy + cc * dy * dy;
                const double araw = alpha_c[g] * exp(-0.5 * q);
                const double a = araw < ALPHA_MAX ? araw : ALPHA_MAX;
                double ea = 0.0;   /* band of ln alpha at this (Gaussian, pixel) */
                if (banded) {
                    ea = band_lnalpha(n, g, mean2d, errpar, fc, ca, cb, cc, dx, dy);
                    if (fabs(log(araw / ALPHA_MIN)) < ea) {
                        ora_event e = {a < ALPHA_MIN ? 0 : 1, a < ALPHA_MIN ? ALPHA_MIN * exp(ea) : a, T,
                                       {C[0], C[1], C[2]}, {0, 0, 0}};
                        for (int ch = 0; ch < 3; ++ch) e.rgb[ch] = rgb[(int64_t)ch * n + g];
                        if (nev < ORA_MAX_EVENTS) ev[nev++] = e;
                        else fb += e.a * T * cmax;
                        fl |= ORA_FLAG_ALPHA;
                        /* taking it the other way rescales T by about (1 - alpha) */
                        eT += e.a;
                    }
                }
                if (a < ALPHA_MIN) continue;
                const double Tn = T * (1.0 - a);
                if (banded) {
                    eT += a / (1.0 - a) * ea + fc->k_T * E;
                    if (fabs(log(Tn / T_MIN)) < eT) {
                        ora_event e = {Tn < T_MIN ? 2 : 3, a, T, {C[0], C[1], C[2]}, {0, 0, 0}};
                        for (int ch = 0; ch < 3; ++ch) e.rgb[ch] = rgb[(int64_t)ch * n + g];
                        if (nev < ORA_MAX_EVENTS) ev[nev++] = e;
                        else fb += T * cmax;
                        fl |= ORA_FLAG_T;
                    }
                }
                if (Tn < T_MIN) break;
                const double ez = banded ? fc->k_z * E * errpar[4 * n + g] : 0.0;
                if (banded && have_prev && fabs(depth[g] - prev_z) < ez + prev_ez) {
                    double dc = 0.0;
                    for (int ch = 0; ch < 3; ++ch) {
                        const double e = fabs(rgb[(int64_t)ch * n + g] - prev_rgb[ch]);
                        if (e > dc) dc = e;
                    }
                    /* swapping two consecutive contributors changes C by
                     * T_prev a_prev a (rgb_prev - rgb) */
                    const double imp = prev_T * prev_a * a * dc;
                    fb += imp;
                    if (imp > fc->impact_min) fl |= ORA_FLAG_DEPTH;
                }
                for (int ch = 0; ch < 3; ++ch) C[ch] += rgb[(int64_t)ch * n + g] * a * T;
                have_prev = 1;
                prev_z = depth[g];
                prev_ez = ez;
                prev_a = a;
                prev_T = T;
                for (int ch = 0; ch < 3; ++ch) prev_rgb[ch] = rgb[(int64_t)ch * n + g];
                T = Tn;
                nc += 1;
                hsh = (hsh ^ (uint64_t)(g + 1)) * 1099511628211ull;
            }
            const int64_t p = (int64_t)py * w + px;
            double img[3];
            for (int ch = 0; ch < 3; ++ch) img[ch] = C[ch] + T * bg[ch];
            /* first-order change of the pixel if each recorded decision went
             * the other way (later decisions unchanged) */
            uint32_t fl_imp = fl & ORA_FLAG_DEPTH;
            for (int k = 0; k < nev; ++k) {
                const ora_event* e = &ev[k];
                double d = 0.0;
                for (int ch = 0; ch < 3; ++ch) {
                    double x;
                    if (e->kind == 0) {          /* blended instead: rest rescaled by (1 - a) */
                        x = e->a * (e->T * e->rgb[ch] - (img[ch] - e->C[ch]));
                    } else if (e->kind == 1) {   /* skipped instead */
                        const double rest = (img[ch] - e->C[ch] - e->a * e->T * e->rgb[ch]) / (1.0 - e->a);
                        x = e->a * (e->T * e->rgb[ch] - rest);
                    } else if (e->kind == 2) {   /* blended instead of stopping */
                        x = e->a * e->T * (e->rgb[ch] - bg[ch]);
                    } else {                     /* stopped instead */
                        x = img[ch] - e->C[ch] - e->T * bg[ch];
                    }
                    if (fabs(x) > d) d = fabs(x);
                }
                fb += d;
                if (d > fc->impact_min) fl_imp |= e->kind <= 1 ? ORA_FLAG_ALPHA : ORA_FLAG_T;
            }
            /* value band: first-order change of the pixel when each
             * contributor's ln alpha moves by its band (decisions kept):
             * d C / d ln a_i = a_i (T_i rgb_i - rest_i), rest_i the colour
             * behind it divided by (1 - a_i); a clamped alpha only moves
             * when its band reaches below the clamp */
            double vb = 0.0;
            if (banded && vbound) {
                double Tv = 1.0, Cv[3] = {0, 0, 0};
                for (int64_t jj = 0; jj < j && jj < m; ++jj) {
                    const int64_t g = order[jj];
                    const double dx = mean2d[g] - pxc, dy = mean2d[n + g] - pyc;
                    const double ca = conic[g], cb = conic[n + g], cc = conic[2 * n + g];
                    const double q = ca * dx * dx + 2.0 * cb * dx * dy + cc * dy * dy;
                    const double araw = alpha_c[g] * exp(-0.5 * q);
                    const double a = araw < ALPHA_MAX ? araw : ALPHA_MAX;
                    if (a < ALPHA_MIN) continue;
                    const double ea = band_lnalpha(n, g, mean2d, errpar, fc, ca, cb, cc, dx, dy);
                    if (araw < ALPHA_MAX * exp(ea)) {
                        double d = 0.0;
                        for (int ch = 0; ch < 3; ++ch) {
                            const double c = rgb[(int64_t)ch * n + g];
                            const double rest = (img[ch] - Cv[ch] - a * Tv * c) / (1.0 - a);
                            const double x = fabs(a * (Tv * c - rest));
                            if (x > d) d = x;
                        }
                        vb += ea * d;
                    }
                    for (int ch = 0; ch < 3; ++ch) Cv[ch] += rgb[(int64_t)ch * n + g] * a * Tv;
                    Tv *= 1.0 - a;
                }
            }
            for (int ch = 0; ch < 3; ++ch) image[ch * npx + p] = img[ch];
            if (vbound) vbound[p] = banded ? 1.01 * vb : 0.0;
            if (final_T) final_T[p] = T;
            if (ncontrib) ncontrib[p] = nc;
            if (chash) chash[p] = hsh;
            if (flags) flags[p] = banded ? fl_imp : 0u;
            if (fbound) fbound[p] = banded ? 1.01 * fb : 0.0;
            if (ntest) ntest[p] = j < m ? j + 1 : m;   /* Gaussians tested, the stopping one included */
        }
    }
    return 0;
}

/* ---- adaptive Gaussian refinement (Sec. 4.3) ------------------------------
 * gamma(t): for k = 0 .. K-1 the pair sin(2^k pi t), cos(2^k pi t), in that
 * order.  Each MLP maps f (27) to 64 hidden units, applies the activation
 * (ReLU: the paper does not name it) and maps to its output; the output is a
 * residual added to the parameter it refines. */
void ora_agr_encoding(double t, double* g)
{
    for (int k = 0; k < AGR_K; ++k) {
        const double w = ldexp(ORA_PI, k) * t;
        g[2 * k] = sin(w);
        g[2 * k + 1] = cos(w);
    }
}

void ora_agr(int64_t n, const double* mu_p, const double* mu_t, const double* mu_d, const double* L,
             double t, const double* wts, double* r_mu_p, double* r_mu_t, double* r_mu_d, double* r_L)
{
    static const int cout[4] = {3, 1, 3, 28};
    double gam[2 * AGR_K];
    ora_agr_encoding(t, gam);
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
        double f[AGR_IN];
        for (int a = 0; a < 3; ++a) f[a] = mu_p[a * n + g];
        f[3] = mu_t[g];
        for (int a = 0; a < 3; ++a) f[4 + a] = mu_d[a * n + g];
        for (int k = 0; k < 2 * AGR_K; ++k) f[7 + k] = gam[k];
        double* out[4] = {r_mu_p, r_mu_t, r_mu_d, r_L};
        const double* base[4] = {mu_p, mu_t, mu_d, L};
        const double* w = wts;
        for (int m = 0; m < 4; ++m) {
            const double* W1 = w;
            const double* b1 = W1 + AGR_HIDDEN * AGR_IN;
            const double* W2 = b1 + AGR_HIDDEN;
            const double* b2 = W2 + cout[m] * AGR_HIDDEN;
            double h[AGR_HIDDEN];
            for (int j = 0; j < AGR_HIDDEN; ++j) {
                double s = b1[j];
                for (int c = 0; c < AGR_IN; ++c) s += W1[j * AGR_IN + c] * f[c];
                h[j] = s > 0.0 ? s : 0.0;
            }
            for (int o = 0; o < cout[m]; ++o) {
                double s = b2[o];
                for (int j = 0; j < AGR_HIDDEN; ++j) s += W2[o * AGR_HIDDEN + j] * h[j];
                out[m][o * n + g] = base[m][o * n + g] + s;
            }
            w = b2 + cout[m];
        }
    }
}

int ora_render(int64_t n, const double* mu_p, const double* mu_t, const double* mu_d,
               const double* L, const double* alpha, const double* sh, const ora_view* v,
               int x0, int y0, int w, int h, const ora_flagcfg* fc,
               double* image, double* final_T, int32_t* ncontrib, uint64_t* chash,
               uint32_t* flags, double* fbound, int64_t* ntest, double* vbound)
{
    double* mu_c = (double*)malloc(sizeof(double) * 3 * n + 8);
    double* cov_c = (double*)malloc(sizeof(double) * 6 * n + 8);
    double* alpha_c = (double*)malloc(sizeof(double) * n + 8);
    double* mean2d = (double*)malloc(sizeof(double) * 2 * n + 8);
    double* conic = (double*)malloc(sizeof(double) * 3 * n + 8);
    double* depth = (double*)malloc(sizeof(double) * n + 8);
    double* rgb = (double*)malloc(sizeof(double) * 3 * n + 8);
    int32_t* rect = (int32_t*)malloc(sizeof(int32_t) * 4 * n + 8);
    uint8_t* vis = (uint8_t*)malloc((size_t)n + 8);
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * n + 8);
    double* errpar = fc ? (double*)malloc(sizeof(double) * 5 * n + 8) : NULL;
    int rc = 0;
    if (!mu_c || !cov_c || !alpha_c || !mean2d || !conic || !depth || !rgb || !rect || !vis || !order ||
        (fc && !errpar)) {
        rc = -1;
    } else {
        ora_slice(n, mu_p, mu_t, mu_d, L, alpha, v, mu_c, cov_c, alpha_c, NULL, NULL, NULL);
        ora_project(n, mu_c, cov_c, alpha_c, sh, v, mean2d, conic, depth, rgb, rect, vis, NULL);
        int64_t m = ora_order(n, depth, vis, order);
        if (errpar) ora_fp32_model(n, mu_c, cov_c, v, errpar);
        ora_composite(n, mean2d, conic, alpha_c, depth, rgb, errpar, m, order, v, x0, y0, w, h, fc,
                      image, final_T, ncontrib, chash, flags, fbound, ntest, vbound);
    }
    free(mu_c); free(cov_c); free(alpha_c); free(mean2d); free(conic);
    free(depth); free(rgb); free(rect); free(vis); free(order); free(errpar);
    return rc;
}

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_set_num_threads(int nt)
{
#ifdef _OPENMP
    if (nt > 0) omp_set_num_threads(nt);
#else
    (void)nt;
#endif
}
