/*
 * oracle7d.h -- FP64 reference of the 7DGS render path (test infrastructure).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * use this library.  It shares nothing with the HIP library.
 *
 * Array layouts (structure of arrays, n = number of Gaussians):
 *   inputs (FP64):  mu_p[3][n], mu_t[n], mu_d[3][n], L[28][n] (entry (i,j),
 *                   i >= j, at plane i*(i+1)/2+j; dims x,y,z,t,dx,dy,dz),
 *                   alpha[n], sh[48][n] (plane 3k+ch)
 *   outputs (FP64): mu_c[3][n], cov_c[6][n] (xx,xy,xz,yy,yz,zz), alpha_c[n],
 *                   mean2d[2][n], conic[3][n] (a,b,c with
 *                   q = a dx^2 + 2 b dx dy + c dy^2), depth[n], rgb[3][n],
 *                   rect[4][n] (tile x0, y0, x1, y1; x1, y1 exclusive)
 *   images:         image[3][h][w], final_T[h][w], ncontrib[h][w]
 */
#ifndef ORACLE7D_H
#define ORACLE7D_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A view exactly as the scene generator stores it (FP32). */
typedef struct {
    float R[9];        /* world -> camera rotation, row-major (rows: right, down, forward) */
    float c[3];        /* camera centre, world */
    float fx, fy, cx, cy;
    int32_t W, H;
    float t;           /* observed time */
    float d[3];        /* view direction the Gaussians are conditioned on */
    float lambda_t, lambda_d;
    float bg[3];
    int32_t d_mode;    /* 1: Gaussian g is conditioned on unit(mu_p,g - c) instead of d */
} ora_view;

/* The parity protocol's model of an FP32 evaluation of the path (not part of
 * the method).  For each (Gaussian, pixel) the band of ln alpha within which
 * an FP32 evaluation may take the opacity test the other way is
 *   2^-24 [k_mu (|w0| + |w1|) e_mu + k_uv (|w0| |u| + |w1| |v|)
 *          + k_s w^T Sabs w / 2 + k_eval (8 + qabs / 2) + k_ac]
 * with w = conic (u - p), qabs the quadratic form with |b|, e_mu and Sabs
 * from ora_fp32_model: the first-order effect on ln alpha of relative errors
 * 2^-24 k in mu_cond (through mean2d), in the stored mean2d, in Sigma_cond
 * (through the 2D covariance), of FP32 storage and evaluation of the
 * exponent's terms, and in alpha_cond.  The band of ln T grows along the pixel by
 * a/(1-a) times each contributor's band plus k_T 2^-24 per step (and by a
 * for each opacity decision in its band, which would rescale T by 1 - a).
 * Two consecutive contributors are a depth tie when their depths differ by
 * less than k_z 2^-24 (e_z,1 + e_z,2).  Pixel flags mark decisions in their
 * band whose first-order effect on the pixel exceeds impact_min. */
typedef struct {
    double k_mu, k_uv, k_s, k_eval, k_ac;  /* opacity-test band coefficients */
    double k_T;         /* transmittance rounding per step, units of 2^-24 */
    double k_z;         /* depth tie band coefficient */
    double impact_min;  /* events whose effect on the pixel is below this are not flagged */
} ora_flagcfg;

#define ORA_FLAG_ALPHA 1u
#define ORA_FLAG_T 2u
#define ORA_FLAG_DEPTH 4u

/* Returns the number of Gaussians with a non-positive L diagonal or a
 * non-SPD block; status[g] (optional) holds 1 (diagonal) | 2 (not SPD). */
int ora_slice(int64_t n, const double* mu_p, const double* mu_t, const double* mu_d,
              const double* L, const double* alpha, const ora_view* v,
              double* mu_c, double* cov_c, double* alpha_c, double* f_temp, double* f_dir,
              int32_t* status);

/* Returns the number of visible Gaussians.  box (optional) [4][n]: the
 * opacity footprint u -+ hx, v -+ hy in pixels (x0, y0, x1, y1), the exact
 * bounding box of {alpha_c e^{-q/2} >= ALPHA_MIN}; rect is its tile range
 * clipped to the grid.  Zeros for culled Gaussians. */
int64_t ora_project(int64_t n, const double* mu_c, const double* cov_c, const double* alpha_c,
                    const double* sh, const ora_view* v, double* mean2d, double* conic,
                    double* depth, double* rgb, int32_t* rect, uint8_t* visible, double* box);

/* Visible Gaussians ordered by (depth ascending, index ascending). */
int64_t ora_order(int64_t n, const double* depth, const uint8_t* visible, int64_t* order);

/* Error-model scales of each Gaussian for the FP32 bands (see ora_flagcfg):
 * errpar[5][n] = e_mu = max(fx, fy)/z max|mu_c|, Sabs_00, Sabs_01, Sabs_11
 * (= |J R| |Sigma_c| |J R|^T), e_z = max|mu_c| + |z|. */
void ora_fp32_model(int64_t n, const double* mu_c, const double* cov_c, const ora_view* v, double* errpar);

/* Brute-force compositing of the crop [x0, x0+w) x [y0, y0+h).  With fc and
 * errpar non-NULL it also flags pixels (ORA_FLAG_*) where a decision lies in
 * its FP32 band with an effect above fc->impact_min, and writes fbound[h][w]:
 * 1.01 x the sum over all in-band decisions of their first-order effect on the
 * pixel (max over channels) if taken the other way, 0 where there is none.
 * ntest (optional) [h][w]: the Gaussians the pixel's loop tested (the
 * stopping one included), the brute force's unit of work.  vbound (optional,
 * banded only) [h][w]: 1.01 x the sum over the pixel's contributors of
 * |d C / d ln alpha_i| (max over channels) times alpha_i's band, the
 * first-order change of the pixel when every contributor's opacity moves
 * within its FP32 band with every decision kept (0 without fc). */
int ora_composite(int64_t n, const double* mean2d, const double* conic, const double* alpha_c,
                  const double* depth, const double* rgb, const double* errpar, int64_t m,
                  const int64_t* order, const ora_view* v, int x0, int y0, int w, int h,
                  const ora_flagcfg* fc, double* image, double* final_T, int32_t* ncontrib,
                  uint64_t* chash, uint32_t* flags, double* fbound, int64_t* ntest, double* vbound);

/* slice + project + order + composite (fc NULL: no flags, fbound 0). */
int ora_render(int64_t n, const double* mu_p, const double* mu_t, const double* mu_d,
               const double* L, const double* alpha, const double* sh, const ora_view* v,
               int x0, int y0, int w, int h, const ora_flagcfg* fc,
               double* image, double* final_T, int32_t* ncontrib, uint64_t* chash,
               uint32_t* flags, double* fbound, int64_t* ntest, double* vbound);

/* Adaptive Gaussian refinement (Sec. 4.3).  wts: the four MLPs in the order
 * p, t, d, l, each as W1[64][27] (row-major), b1[64], W2[C_out][64], b2[C_out]
 * with C_out = 3, 1, 3, 28 (AGR_WEIGHTS values in all).  Writes the refined
 * mu_p[3][n], mu_t[n], mu_d[3][n], L[28][n]. */
#define AGR_K 10
#define AGR_IN 27
#define AGR_HIDDEN 64
#define AGR_WEIGHTS 9443
void ora_agr_encoding(double t, double* gamma20);
void ora_agr(int64_t n, const double* mu_p, const double* mu_t, const double* mu_d, const double* L,
             double t, const double* wts, double* r_mu_p, double* r_mu_t, double* r_mu_d, double* r_L);

void ora_sh_basis(double x, double y, double z, double* Y);
int ora_num_threads(void);
void ora_set_num_threads(int nt);

#ifdef __cplusplus
}
#endif
#endif
