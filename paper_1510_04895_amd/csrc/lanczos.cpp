// Spectral bounds from the Lanczos process, an alternative to the Gershgorin
// interval for the scaling of Sec. 3.1 step 1 (the paper names Lanczos as the
// way to obtain [a, b]; the Gershgorin bound of Sec. 2 is rigorous but wide).
//
// k steps of Lanczos on H from a random start vector (stream 4 of the seed),
// without reorthogonalisation (only the extreme Ritz values are used).  The
// extreme Ritz values theta_1 <= ... <= theta_k of the tridiagonal matrix are
// widened by their residual bounds beta_k |s_k| (the last component of the
// Ritz vector times the last off-diagonal) and by a relative pad of the Ritz
// range, and clamped to the Gershgorin interval.  The solver checks every
// Rayleigh quotient against the interval it was given (a Rayleigh quotient
// outside [a, b] proves the interval too narrow) and restarts with the
// Gershgorin interval in that case.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace chebfd {

int lanczos_bounds(chebfd_ctx *ctx, const chebfd_matrix *H, int k, uint64_t seed, double pad,
                   void *V3, double *S_dev, double *T_dev, double *a_out, double *b_out)
{
    const int64_t n = H->n, ld = 3;
    auto col = [&](int j) { return (void *)((char *)V3 + (size_t)16 * j); };
    auto sync = [&]() -> int {
        CHEBFD_HIP(hipStreamSynchronize(ctx->stream));
        return CHEBFD_OK;
    };
    auto dot = [&](int x, int y, double &re) -> int {
        int rc = launch_gram(ctx, CHEBFD_PREC_C128, col(x), ld, 1, col(y), ld, 1, n, S_dev);
        if (rc) return rc;
        double s[2];
        CHEBFD_HIP(hipMemcpyAsync(s, S_dev, sizeof(s), hipMemcpyDeviceToHost, ctx->stream));
        if ((rc = sync())) return rc;
        re = s[0];
        return CHEBFD_OK;
    };
    // C <- C - t A (sub = 1) or C <- t A (sub = 0) for one column, t real
    auto scale = [&](int A, int Cc, double t, int sub) -> int {
        const double Tr[4] = {t, 0.0, 0.0, t};
        CHEBFD_HIP(hipMemcpyAsync(T_dev, Tr, sizeof(Tr), hipMemcpyHostToDevice, ctx->stream));
        int rc = launch_block_times(ctx, CHEBFD_PREC_C128, col(A), ld, n, 1, T_dev, 1,
                                    CHEBFD_PREC_C128, col(Cc), ld, sub);
        if (rc) return rc;
        return sync();   // Tr goes out of scope
    };
    int rc;
    // start vector, normalised
    int p = 0, v = 1, w = 2;
    if ((rc = launch_random(ctx, CHEBFD_PREC_C128, V3, n, 3, ld, 1, 1, seed, 4, 0))) return rc;
    double nv;
    if ((rc = dot(v, v, nv))) return rc;
    if (!(nv > 0.0)) return fail(CHEBFD_ERR_NONFINITE, "lanczos: zero start vector");
    if ((rc = scale(v, p, 1.0 / std::sqrt(nv), 0))) return rc;
    std::swap(p, v);   // v holds the unit start vector
    std::vector<double> alpha, beta;
    double beta_prev = 0.0;
    for (int j = 0; j < k; ++j) {
        StepArgs s{};
        s.mode = MODE_APPLY;
        s.precision = CHEBFD_PREC_C128;
        s.n = n;
        s.n_s = 1;
        s.ld = ld;
        s.u = col(v);
        s.wout = col(w);
        s.s_h = 1.0;
        s.s_u = 0.0;
        if ((rc = launch_step(ctx, H, s, nullptr))) return rc;   // w = H v
        double al;
        if ((rc = dot(v, w, al))) return rc;
        if ((rc = scale(v, w, al, 1))) return rc;                 // w -= alpha v
        if (j > 0 && (rc = scale(p, w, beta_prev, 1))) return rc; // w -= beta p
        double nw;
        if ((rc = dot(w, w, nw))) return rc;
        alpha.push_back(al);
        const double be = std::sqrt(std::max(nw, 0.0));
        beta.push_back(be);
        if (!std::isfinite(al) || !std::isfinite(be))
            return fail(CHEBFD_ERR_NONFINITE, "lanczos: non-finite recurrence");
        if (be <= 1e-14 * std::max(1.0, std::fabs(al))) break;   // invariant subspace
        // p <- v, v <- w / beta (into the old p column)
        if ((rc = scale(w, p, 1.0 / be, 0))) return rc;
        std::swap(p, v);
        beta_prev = be;
    }
    const int m = (int)alpha.size();
    std::vector<double> T((size_t)2 * m * m, 0.0), th;
    for (int i = 0; i < m; ++i) {
        T[2 * ((size_t)i * m + i)] = alpha[i];
        if (i + 1 < m) {
            T[2 * ((size_t)i * m + i + 1)] = beta[i];
            T[2 * ((size_t)(i + 1) * m + i)] = beta[i];
        }
    }
    if (herm_eig(m, T, th) != 0) return fail(CHEBFD_ERR_NONFINITE, "lanczos: tridiagonal eigensolver failed");
    // residual bound of Ritz pair j: beta_m |last component of its vector|
    auto resid = [&](int j) {
        const double re = T[2 * ((size_t)(m - 1) * m + j)], im = T[2 * ((size_t)(m - 1) * m + j) + 1];
        return beta[m - 1] * std::sqrt(re * re + im * im);
    };
    const double lo = th.front(), hi = th.back(), span = std::max(hi - lo, 1e-300);
    *a_out = std::max(H->g_lo, lo - resid(0) - pad * span);
    *b_out = std::min(H->g_hi, hi + resid(m - 1) + pad * span);
    return CHEBFD_OK;
}

}  // namespace chebfd

using namespace chebfd;

extern "C" int chebfd_lanczos_bounds(chebfd_ctx *ctx, const chebfd_matrix *H, int k,
                                     uint64_t seed, double pad, double *a, double *b)
{
    if (!ctx || !H || !a || !b || k < 2 || k > 1000 || !(pad >= 0.0))
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_lanczos_bounds: need 2 <= k <= 1000, pad >= 0");
    CHEBFD_HIP(hipSetDevice(ctx->device));
    char *buf = nullptr;
    const size_t vb = (size_t)H->n * 3 * 16;
    CHEBFD_HIP(hipMalloc((void **)&buf, vb + 256));
    int rc = lanczos_bounds(ctx, H, k, seed, pad, buf, (double *)(buf + vb),
                            (double *)(buf + vb + 64), a, b);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(buf);
    return rc;
}
