/* Host sanitizer run of the FP64 oracle (test infrastructure): every entry
 * point of oracle7d.h on small seeded inputs, including culled Gaussians, a
 * Gaussian behind the camera, empty inputs, crops at the image border and
 * both direction modes.  Built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_sanitize_host.py; any report
 * aborts the run. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle7d.h"

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static double urand(void)
{
    rng = rng * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

static double* alloc(size_t count) { return (double*)calloc(count ? count : 1, sizeof(double)); }

int main(void)
{
    const int64_t n = 300;
    double *mu_p = alloc(3 * n), *mu_t = alloc(n), *mu_d = alloc(3 * n), *L = alloc(28 * n);
    double *alpha = alloc(n), *sh = alloc(48 * n);
    for (int64_t g = 0; g < n; ++g) {
        for (int k = 0; k < 3; ++k) mu_p[k * n + g] = 2.0 * urand() - 1.0;
        mu_t[g] = urand();
        for (int k = 0; k < 3; ++k) mu_d[k * n + g] = 2.0 * urand() - 1.0;
        for (int i = 0; i < 7; ++i)
            for (int j = 0; j <= i; ++j)
                L[(i * (i + 1) / 2 + j) * n + g] = i == j ? 0.05 + 0.2 * urand() : 0.05 * (urand() - 0.5);
        alpha[g] = 0.05 + 0.9 * urand();
        for (int k = 0; k < 48; ++k) sh[k * n + g] = 0.3 * (urand() - 0.5);
    }
    L[0 * n + 0] = -0.1;     /* non-positive diagonal: culled with status 1 */
    mu_p[2 * n + 1] = -10.0; /* behind the camera */

    ora_view v;
    memset(&v, 0, sizeof v);
    v.R[0] = v.R[4] = v.R[8] = 1.0f;
    v.c[2] = -3.0f;
    v.fx = v.fy = 60.0f;
    v.W = 48;
    v.H = 36;
    v.cx = 24.0f;
    v.cy = 18.0f;
    v.t = 0.5f;
    v.d[2] = 1.0f;
    v.lambda_t = v.lambda_d = 0.5f;
    v.bg[0] = 0.1f; v.bg[1] = 0.2f; v.bg[2] = 0.3f;

    double *mu_c = alloc(3 * n), *cov_c = alloc(6 * n), *alpha_c = alloc(n), *ft = alloc(n), *fd = alloc(n);
    int32_t* status = (int32_t*)calloc(n, sizeof(int32_t));
    const int bad = ora_slice(n, mu_p, mu_t, mu_d, L, alpha, &v, mu_c, cov_c, alpha_c, ft, fd, status);
    double *mean2d = alloc(2 * n), *conic = alloc(3 * n), *depth = alloc(n), *rgb = alloc(3 * n), *box = alloc(4 * n);
    int32_t* rect = (int32_t*)calloc(4 * n, sizeof(int32_t));
    uint8_t* vis = (uint8_t*)calloc(n, 1);
    const int64_t nv = ora_project(n, mu_c, cov_c, alpha_c, sh, &v, mean2d, conic, depth, rgb, rect, vis, box);
    int64_t* order = (int64_t*)calloc(n, sizeof(int64_t));
    const int64_t m = ora_order(n, depth, vis, order);
    double* errpar = alloc(5 * n);
    ora_fp32_model(n, mu_c, cov_c, &v, errpar);
    const ora_flagcfg fc = {1.0, 2.0, 1.0, 2.0, 2.0, 4.0, 2.0, 1e-5};
    const size_t px = (size_t)v.W * v.H;
    double *image = alloc(3 * px), *final_T = alloc(px), *fbound = alloc(px);
    int32_t* ncon = (int32_t*)calloc(px, sizeof(int32_t));
    uint64_t* chash = (uint64_t*)calloc(px, sizeof(uint64_t));
    uint32_t* flags = (uint32_t*)calloc(px, sizeof(uint32_t));
    int64_t* ntest = (int64_t*)calloc(px, sizeof(int64_t));
    double* vbound = alloc(px);
    int rc = ora_composite(n, mean2d, conic, alpha_c, depth, rgb, errpar, m, order, &v, 0, 0, v.W, v.H, &fc,
                           image, final_T, ncon, chash, flags, fbound, ntest, vbound);
    /* a crop at the bottom-right border, without flags */
    rc |= ora_composite(n, mean2d, conic, alpha_c, depth, rgb, NULL, m, order, &v, v.W - 7, v.H - 5, 7, 5, NULL,
                        image, final_T, ncon, chash, flags, fbound, ntest, NULL);
    /* the whole path per Gaussian direction, two threads then one */
    v.d_mode = 1;
    ora_set_num_threads(2);
    rc |= ora_render(n, mu_p, mu_t, mu_d, L, alpha, sh, &v, 3, 2, 20, 17, &fc, image, final_T, ncon, chash, flags,
                     fbound, ntest, vbound);
    ora_set_num_threads(1);
    rc |= ora_render(0, mu_p, mu_t, mu_d, L, alpha, sh, &v, 0, 0, v.W, v.H, NULL, image, final_T, ncon, NULL, NULL,
                     NULL, NULL, NULL);
    /* adaptive refinement with seeded weights */
    double* wts = alloc(AGR_WEIGHTS);
    for (int k = 0; k < AGR_WEIGHTS; ++k) wts[k] = 0.2 * (urand() - 0.5);
    double *r_mu_p = alloc(3 * n), *r_mu_t = alloc(n), *r_mu_d = alloc(3 * n), *r_L = alloc(28 * n);
    ora_agr(n, mu_p, mu_t, mu_d, L, 0.25, wts, r_mu_p, r_mu_t, r_mu_d, r_L);
    double gam[2 * AGR_K];
    ora_agr_encoding(0.75, gam);
    double Y[16];
    ora_sh_basis(0.0, 0.6, 0.8, Y);
    double chk = 0.0;
    for (size_t i = 0; i < 3 * px; ++i) chk += image[i];
    printf("oracle driver: culled %d, visible %lld, ordered %lld, rc %d, image sum %.6f, threads %d\n", bad,
           (long long)nv, (long long)m, rc, chk, ora_num_threads());
    free(mu_p); free(mu_t); free(mu_d); free(L); free(alpha); free(sh);
    free(mu_c); free(cov_c); free(alpha_c); free(ft); free(fd); free(status);
    free(mean2d); free(conic); free(depth); free(rgb); free(box); free(rect); free(vis); free(order); free(errpar);
    free(image); free(final_T); free(fbound); free(ncon); free(chash); free(flags); free(ntest); free(vbound);
    free(wts); free(r_mu_p); free(r_mu_t); free(r_mu_d); free(r_L);
    return (bad < 1 || nv < 1 || nv >= n || m != nv || rc != 0) ? 1 : 0;
}
