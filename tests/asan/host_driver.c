/* Host-only driver for the AddressSanitizer build of the library's host
 * math (filter polynomials, parameter rules, learned-form maps, dense
 * eigensolver).  Calls only entry points that touch no GPU; exits 0 when
 * every call returned its expected status. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "chebfd.h"

static int check(int rc, const char *what)
{
    if (rc != 0) {
        fprintf(stderr, "%s failed: %d %s\n", what, rc, chebfd_last_error());
        exit(2);
    }
    return rc;
}

int main(void)
{
    /* moments of a flat spectrum on [-1, 1] (exact, by the recurrence) */
    for (int n_mom = 4; n_mom <= 512; n_mom *= 2) {
        double *mu = (double *)calloc((size_t)n_mom, sizeof(double));
        const int D = 1000;
        for (int i = 1; i <= D; ++i) {
            const double x = -1.0 + 2.0 * i / (D + 1.0);
            double t0 = 1.0, t1 = x;
            mu[0] += t0 / D;
            if (n_mom > 1) mu[1] += t1 / D;
            for (int m = 2; m < n_mom; ++m) {
                const double t2 = 2.0 * x * t1 - t0;
                mu[m] += t2 / D;
                t0 = t1;
                t1 = t2;
            }
        }
        double nt, mg;
        int ns = 0, np = 0;
        check(chebfd_dos_params(mu, n_mom, D, -1.0, 1.0, -0.05, 0.05, 3.0, CHEBFD_KERNEL_LANCZOS,
                                2.0, 1024, &nt, &ns, &np, &mg),
              "chebfd_dos_params");
        float feat[514];
        check(chebfd_learned_features(mu, n_mom, -1.0, 1.0, -0.05, 0.05, feat),
              "chebfd_learned_features");
        free(mu);
    }
    double amp[16], sig;
    check(chebfd_fit_corrections(-1.0, 1.0, -0.02, 0.02, -0.04, 0.04, 120, CHEBFD_KERNEL_LANCZOS,
                                 2.0, 16, 0.5, 20, 1e-3, amp, &sig),
          "chebfd_fit_corrections");
    float out[18] = {0.1f, -0.2f, 0.0f};
    for (int j = 0; j < 16; ++j) out[2 + j] = (float)amp[j];
    double corr[121];
    int np, ns;
    check(chebfd_learned_decode(out, 120, 40, 16, 0.5, 1024, &np, &ns, corr, 121),
          "chebfd_learned_decode");
    double gam[301], s, e;
    check(chebfd_coeffs(-0.1, 0.1, -1.0, 1.0, 300, CHEBFD_KERNEL_JACKSON, 0.0, gam),
          "chebfd_coeffs");
    check(chebfd_filter_quality(gam, 300, -1.0, 1.0, -0.1, 0.1, -0.2, 0.2, &s, &e),
          "chebfd_filter_quality");
    /* division by a linear factor: n_p coefficients into an exact-size heap
       block, for the smallest and a large degree */
    for (int npd = 2; npd <= 300; npd += 298) {
        double *d = (double *)malloc(sizeof(double) * npd), pt;
        check(chebfd_coeffs_divided(gam, npd, -1.0, 1.0, 0.05, d, &pt), "chebfd_coeffs_divided");
        free(d);
    }
    int nopt;
    check(chebfd_optimal_np(-1.0, 1.0, -0.05, 0.05, -0.1, 0.1, CHEBFD_KERNEL_LANCZOS, 2.0, 8,
                            400, &nopt, &e),
          "chebfd_optimal_np");
    for (int n = 1; n <= 40; n += 13) {
        double *A = (double *)malloc(sizeof(double) * 2 * n * n);
        double *w = (double *)malloc(sizeof(double) * n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                A[2 * (i * n + j)] = 1.0 / (1.0 + i + j);
                A[2 * (i * n + j) + 1] = (i == j) ? 0.0 : 0.01 * (i - j);
            }
        check(chebfd_host_eigh(n, A, w), "chebfd_host_eigh");
        free(A);
        free(w);
    }
    printf("host driver ok\n");
    return 0;
}
