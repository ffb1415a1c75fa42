// Parameter selection from KPM moments (Sec. 3.1 steps 1-3, Sec. 2.4) and the
// maps between the learned network's inputs/outputs and solver parameters.
//
// KPM density of states in scaled units x = alpha lambda + beta:
//   rho(x) = [g_0 mu_0 + 2 sum_{m>=1} g_m mu_m T_m(x)] / (pi sqrt(1 - x^2)),
// with Jackson damping g_m (KPM with M moments: N -> M in Table
// tab:Kernel).  Its integral over a window is sum_m g_m mu_m c_m with c_m the
// window coefficients of Eq. (W1), so the target count is
//   N_T = N sum_m g_m c_m mu_m                       (Eq. DOS:target)
// and the search interval follows from N_S = N int_{I_S} rho (Eq. DOS:search).
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

namespace chebfd {
namespace {

double window_count(const double *mu, int n_mom, int64_t n, double a, double b, double lo,
                    double hi)
{
    // damping() fills n + 1 factors for degree n.  Table tab:Kernel with
    // N_p = n_mom is the Jackson kernel of n_mom - 1 moments: its factor
    // g_{n_mom-1} (like g_{n_mom}) is zero, so moment n_mom - 1 carries no
    // weight.
    std::vector<double> c(n_mom), g(n_mom + 1);
    window_coeffs(lo, hi, a, b, n_mom - 1, c.data());
    damping(CHEBFD_KERNEL_JACKSON, n_mom, 0.0, g.data());
    double s = 0.0;
    for (int m = 0; m < n_mom; ++m) s += g[m] * c[m] * mu[m];
    return (double)n * s;
}

// piecewise-linear hat functions on [0, 1] with n_hat equidistant nodes
inline double hat(int j, int n_hat, double t)
{
    const double x = t * (n_hat - 1) - j;
    return std::max(0.0, 1.0 - std::fabs(x));
}

}  // namespace
}  // namespace chebfd

using namespace chebfd;

extern "C" int chebfd_dos_params(const double *mu, int n_mom, int64_t n, double a, double b,
                                 double lam_lo, double lam_hi, double ns_over_nt, int kernel,
                                 double mu_k, int ns_max, double *n_t_est, int *n_s, int *n_p,
                                 double *margin)
{
    if (!mu || n_mom < 4 || n < 1 || !(a < b) || !(lam_lo < lam_hi) || !(ns_over_nt >= 1.0) ||
        ns_max < 2 || !n_t_est || !n_s || !n_p)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_dos_params: invalid arguments");
    const double nt = std::max(0.0, window_count(mu, n_mom, n, a, b, lam_lo, lam_hi));
    *n_t_est = nt;
    // N_S: ns_over_nt times the estimate, even, at least 16 (Sec. 3.1 step 2);
    // a positive *n_s on entry fixes N_S instead
    int s = *n_s > 0 ? *n_s : (int)std::ceil(ns_over_nt * std::max(nt, 1.0));
    if (*n_s <= 0) s = std::max(16, s + (s & 1));
    s = std::min(s, ns_max - (ns_max & 1));
    *n_s = s;
    // search interval: smallest margin delta' with N int_{I_S} rho >= N_S
    const double S = 0.5 * (b - a);
    double lo = 0.0, hi = S;
    if (window_count(mu, n_mom, n, a, b, lam_lo - hi, lam_hi + hi) < s) {
        lo = hi;
    } else {
        for (int it = 0; it < 60; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (window_count(mu, n_mom, n, a, b, lam_lo - mid, lam_hi + mid) >= s) hi = mid;
            else lo = mid;
        }
    }
    // the KPM resolution limits small margins: at least the kernel width
    const double dp = std::max(hi, 2.0 * S / n_mom);
    if (margin) *margin = dp;
    int np_best = 0;
    double eta = 0.0;
    const int np_min = std::max(8, (int)(0.5 * S / dp));
    const int np_max = std::max(np_min + 1, (int)(16.0 * S / dp) + 8);
    int rc = chebfd_optimal_np(a, b, lam_lo, lam_hi, lam_lo - dp, lam_hi + dp, kernel, mu_k,
                               np_min, std::min(np_max, 200000), &np_best, &eta);
    if (rc) return rc;
    *n_p = np_best;
    return CHEBFD_OK;
}

extern "C" int chebfd_learned_features(const double *mu, int n_mom, double a, double b,
                                       double lam_lo, double lam_hi, float *features)
{
    if (!mu || n_mom < 1 || !(a < b) || !features)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_learned_features: invalid arguments");
    const double alpha = 2.0 / (b - a), beta = (a + b) / (a - b);
    for (int m = 0; m < n_mom; ++m) features[m] = (float)mu[m];
    features[n_mom] = (float)(alpha * lam_lo + beta);
    features[n_mom + 1] = (float)(alpha * lam_hi + beta);
    return CHEBFD_OK;
}

extern "C" int chebfd_learned_decode(const float *out, int np_ref, int ns_ref, int n_hat,
                                     double c_max, int ns_max, int *n_p, int *n_s,
                                     double *gamma_corr, int corr_len)
{
    if (!out || np_ref < 2 || ns_ref < 1 || n_hat < 2 || !(c_max > 0.0) || ns_max < 2 || !n_p ||
        !n_s)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_learned_decode: invalid arguments");
    if (!std::isfinite(out[0]) || !std::isfinite(out[1]))
        return fail(CHEBFD_ERR_NONFINITE, "chebfd_learned_decode: non-finite output");
    // outputs 0 and 1 are log ratios to the rule-based choice, bounded to
    // a factor of 8 either way
    const double rp = std::exp(std::min(2.08, std::max(-2.08, (double)out[0])));
    const double rs = std::exp(std::min(2.08, std::max(-2.08, (double)out[1])));
    const int p = (int)std::lround(np_ref * rp);
    int s = (int)std::lround(ns_ref * rs);
    s = std::max(16, s + (s & 1));
    s = std::min(s, ns_max - (ns_max & 1));
    *n_p = std::max(8, p);
    *n_s = s;
    if (gamma_corr) {
        // corr_n = c_max tanh(sum_j a_j hat_j(n / n_p)), n = 0..corr_len-1
        for (int k = 0; k < corr_len; ++k) {
            const double t = corr_len > 1 ? (double)k / (corr_len - 1) : 0.0;
            double sacc = 0.0;
            for (int j = 0; j < n_hat; ++j) sacc += (double)out[2 + j] * hat(j, n_hat, t);
            gamma_corr[k] = c_max * std::tanh(sacc);
        }
    }
    return CHEBFD_OK;
}

// Fits the correction amplitudes a_j (j < n_hat) that minimise a smoothed
// log damping factor of the corrected filter
//   p(x) = sum_n gamma_n (1 + c_max tanh(sum_j a_j hat_j(n/n_p))) T_n(x),
//   L = smax_{x outside I_S} log|p(x)| - smin_{x in I_T} log|p(x)|
// (log-sum-exp with sharpness kappa over a theta-uniform grid) plus
// l2 * |a|^2, by Adam with the analytic gradient.  Writes a (n_hat values)
// and the smoothed sigma reached (without the penalty).
extern "C" int chebfd_fit_corrections(double a, double b, double t_lo, double t_hi, double s_lo,
                                      double s_hi, int n_p, int kernel, double mu_k, int n_hat,
                                      double c_max, int iters, double l2, double *amp,
                                      double *sigma_out)
{
    if (!amp || n_p < 2 || n_hat < 2 || !(a < b) || !(t_lo < t_hi) || s_lo > t_lo ||
        s_hi < t_hi || iters < 0)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_fit_corrections: invalid arguments");
    std::vector<double> gam(n_p + 1);
    int rc = chebfd_coeffs(t_lo, t_hi, a, b, n_p, kernel, mu_k, gam.data());
    if (rc) return rc;
    // grid: 8 points per period of T_{n_p}, inside I_T and outside I_S only,
    // plus the four interval edges (where the extrema usually sit)
    const int M = std::max(256, 4 * (n_p + 1));
    std::vector<double> xs;
    std::vector<char> inside;
    auto theta = [&](double x) { return std::acos(std::min(1.0, std::max(-1.0, (2.0 * x - a - b) / (b - a)))); };
    xs.push_back(theta(t_lo));
    inside.push_back(1);
    xs.push_back(theta(t_hi));
    inside.push_back(1);
    if (s_lo > a) { xs.push_back(theta(s_lo)); inside.push_back(0); }
    if (s_hi < b) { xs.push_back(theta(s_hi)); inside.push_back(0); }
    for (int k = 0; k <= M; ++k) {
        const double th = M_PI * k / M;
        const double x = 0.5 * (a + b) + 0.5 * (b - a) * std::cos(th);
        if (x >= t_lo && x <= t_hi) { xs.push_back(th); inside.push_back(1); }
        else if (x < s_lo || x > s_hi) { xs.push_back(th); inside.push_back(0); }
    }
    const int K = (int)xs.size();
    // hat basis per coefficient index
    std::vector<double> H((size_t)(n_p + 1) * n_hat);
    for (int n = 0; n <= n_p; ++n)
        for (int j = 0; j < n_hat; ++j) H[(size_t)n * n_hat + j] = hat(j, n_hat, (double)n / n_p);
    std::vector<double> m1(n_hat, 0.0), m2(n_hat, 0.0), grad(n_hat), s(n_p + 1), coef(n_p + 1),
        dcoef(n_p + 1), pv(K), w(K);
    const double kappa = 30.0, lr = 0.002;
    double best_L = INFINITY;
    std::vector<double> best(amp, amp + n_hat);
    for (int j = 0; j < n_hat; ++j) amp[j] = 0.0;
    for (int it = 0; it <= iters; ++it) {
        for (int n = 0; n <= n_p; ++n) {
            double acc = 0.0;
            for (int j = 0; j < n_hat; ++j) acc += amp[j] * H[(size_t)n * n_hat + j];
            s[n] = acc;
            coef[n] = gam[n] * (1.0 + c_max * std::tanh(acc));
        }
        // p at the grid points (x = cos th), Clenshaw
        for (int k = 0; k < K; ++k) {
            const double x = std::cos(xs[k]);
            double b1 = 0.0, b2 = 0.0;
            for (int n = n_p; n >= 1; --n) {
                const double t = coef[n] + 2.0 * x * b1 - b2;
                b2 = b1;
                b1 = t;
            }
            pv[k] = coef[0] + x * b1 - b2;
        }
        // smooth max over outside, smooth min over inside of log|p|
        double mo = -INFINITY, mi = INFINITY;
        for (int k = 0; k < K; ++k) {
            const double l = std::log(std::fabs(pv[k]) + 1e-300);
            if (inside[k]) mi = std::min(mi, l);
            else mo = std::max(mo, l);
        }
        double zo = 0.0, zi = 0.0;
        for (int k = 0; k < K; ++k) {
            const double l = std::log(std::fabs(pv[k]) + 1e-300);
            if (inside[k]) zi += std::exp(-kappa * (l - mi));
            else zo += std::exp(kappa * (l - mo));
        }
        double pen = 0.0;
        for (int j = 0; j < n_hat; ++j) pen += amp[j] * amp[j];
        const double L = (mo + std::log(zo) / kappa) - (mi - std::log(zi) / kappa) + l2 * pen;
        if (L < best_L) {
            best_L = L;
            std::copy(amp, amp + n_hat, best.begin());
        }
        if (it == iters) break;
        // dL/dp_k = w_k / p_k
        for (int k = 0; k < K; ++k) {
            const double l = std::log(std::fabs(pv[k]) + 1e-300);
            const double wk = inside[k] ? -std::exp(-kappa * (l - mi)) / zi
                                        : std::exp(kappa * (l - mo)) / zo;
            w[k] = wk / pv[k];
        }
        // acc[n] = sum_k w_k T_n(x_k) by the three-term recurrence
        std::fill(dcoef.begin(), dcoef.end(), 0.0);
        for (int k = 0; k < K; ++k) {
            const double x = std::cos(xs[k]);
            double t0 = 1.0, t1 = x;
            dcoef[0] += w[k];
            if (n_p >= 1) dcoef[1] += w[k] * x;
            for (int n = 2; n <= n_p; ++n) {
                const double t2 = 2.0 * x * t1 - t0;
                dcoef[n] += w[k] * t2;
                t0 = t1;
                t1 = t2;
            }
        }
        for (int n = 0; n <= n_p; ++n) {
            const double th = std::tanh(s[n]);
            dcoef[n] *= gam[n] * c_max * (1.0 - th * th);
        }
        for (int j = 0; j < n_hat; ++j) {
            double acc = 0.0;
            for (int n = 0; n <= n_p; ++n) acc += dcoef[n] * H[(size_t)n * n_hat + j];
            grad[j] = acc + 2.0 * l2 * amp[j];
        }
        const double b1 = 0.9, b2 = 0.999;
        for (int j = 0; j < n_hat; ++j) {
            m1[j] = b1 * m1[j] + (1 - b1) * grad[j];
            m2[j] = b2 * m2[j] + (1 - b2) * grad[j] * grad[j];
            const double mh = m1[j] / (1 - std::pow(b1, it + 1)), vh = m2[j] / (1 - std::pow(b2, it + 1));
            amp[j] -= lr * mh / (std::sqrt(vh) + 1e-12);
        }
    }
    std::copy(best.begin(), best.end(), amp);
    if (sigma_out) {
        double pen = 0.0;
        for (int j = 0; j < n_hat; ++j) pen += best[j] * best[j];
        *sigma_out = std::exp(best_L - l2 * pen);
    }
    return CHEBFD_OK;
}

// The learned form end to end (KPM moments -> network -> decode -> gate).
extern "C" int chebfd_learned_params(chebfd_ctx *ctx, const chebfd_matrix *H, chebfd_mlp *mlp,
                                     double a, double b, double lam_lo, double lam_hi, int n_vec,
                                     int n_mom, int n_mom_rule, uint64_t seed, double ns_over_nt,
                                     int n_hat,
                                     double c_max, int ns_max, int gate, int *n_p, int *n_s,
                                     double *gamma_corr, int corr_cap, int *corr_kept,
                                     int *np_rule, int *ns_rule)
{
    if (!ctx || !H || !mlp || !n_p || !n_s || !(a < b) || !(lam_lo < lam_hi) || n_vec < 1 ||
        n_mom < 4 || n_hat < 2 || ns_max < 16 || (gamma_corr && corr_cap < 1))
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_learned_params: invalid arguments");
    int ni = 0, no = 0;
    int rc = chebfd_mlp_dims(mlp, &ni, nullptr, &no);
    if (rc) return rc;
    if (ni != n_mom + 2 || no != 2 + n_hat)
        return fail(CHEBFD_ERR_INVALID_ARG,
                    "chebfd_learned_params: network needs n_mom + 2 inputs and 2 + n_hat outputs");
    // stochastic KPM moments in complex64 (Sec. 3.1 step 1); the network
    // reads the first n_mom, the rule all n_mom_rule of them (the moments of
    // a longer expansion begin with those of the shorter one)
    const int nm = std::max(n_mom, n_mom_rule + (n_mom_rule & 1));
    std::vector<double> mu(nm);
    if ((rc = chebfd_kpm_moments(ctx, H, CHEBFD_PREC_C64, n_vec + (n_vec & 1), nm, seed, a, b,
                                 mu.data())))
        return rc;
    // the rule (fallback and reference of the network's ratios); a positive
    // *n_s on entry fixes N_S
    const int ns_fixed = *n_s > 0 ? *n_s : 0;
    const int64_t n = H->n;
    double nt = 0.0;
    int ns0 = ns_fixed, np0 = 0;
    const int ns_cap = std::max(ns_max, ns_fixed);
    if ((rc = chebfd_dos_params(mu.data(), nm, n, a, b, lam_lo, lam_hi, ns_over_nt,
                                CHEBFD_KERNEL_LANCZOS, 2.0, ns_cap, &nt, &ns0, &np0, nullptr)))
        return rc;
    if (np_rule) *np_rule = np0;
    if (ns_rule) *ns_rule = ns0;
    // network on the device
    std::vector<float> feat(n_mom + 2), outv(no);
    if ((rc = chebfd_learned_features(mu.data(), n_mom, a, b, lam_lo, lam_hi, feat.data())))
        return rc;
    float *dev = nullptr;
    CHEBFD_HIP(hipMalloc((void **)&dev, (size_t)(ni + no) * sizeof(float)));
    rc = CHEBFD_OK;
    if (hipMemcpyAsync(dev, feat.data(), (size_t)ni * 4, hipMemcpyHostToDevice, ctx->stream) !=
        hipSuccess)
        rc = fail(CHEBFD_ERR_HIP, "chebfd_learned_params: upload failed");
    if (!rc) rc = chebfd_mlp_forward(ctx, mlp, dev, 1, dev + ni);
    if (!rc && hipMemcpyAsync(outv.data(), dev + ni, (size_t)no * 4, hipMemcpyDeviceToHost,
                              ctx->stream) != hipSuccess)
        rc = fail(CHEBFD_ERR_HIP, "chebfd_learned_params: download failed");
    if (!rc && hipStreamSynchronize(ctx->stream) != hipSuccess)
        rc = fail(CHEBFD_ERR_HIP, "chebfd_learned_params: synchronize failed");
    (void)hipFree(dev);
    if (rc) return rc;
    // decode; the corrections are evaluated for n = 0..n_p
    if (ns_fixed) outv[1] = 0.0f;
    int npl = 0, nsl = 0;
    if ((rc = chebfd_learned_decode(outv.data(), np0, ns0, n_hat, c_max, ns_cap, &npl, &nsl,
                                    nullptr, 0)))
        return rc;
    *n_p = npl;
    *n_s = nsl;
    if (corr_kept) *corr_kept = 0;
    if (!gamma_corr) return CHEBFD_OK;
    if (npl + 1 > corr_cap)
        return fail(CHEBFD_ERR_WORKSPACE,
                    "chebfd_learned_params: gamma_corr needs n_p + 1 = " + std::to_string(npl + 1) +
                        " entries");
    std::vector<double> corr(npl + 1, 0.0);
    if ((rc = chebfd_learned_decode(outv.data(), np0, ns0, n_hat, c_max, ns_cap, &npl, &nsl,
                                    corr.data(), npl + 1)))
        return rc;
    bool keep = false;
    for (double c : corr) keep = keep || c != 0.0;
    if (keep && gate) {
        // the plain expansion is the fallback: keep the corrections only if
        // they lower the damping factor sigma (Sec. 2.3) of the filter for
        // the rule's search interval at this (N_p, N_S)
        double nt2 = 0.0, margin = 0.0;
        int ns_fix = nsl, np_dummy = 0;
        if ((rc = chebfd_dos_params(mu.data(), nm, n, a, b, lam_lo, lam_hi, ns_over_nt,
                                    CHEBFD_KERNEL_LANCZOS, 2.0, std::max(ns_cap, nsl), &nt2,
                                    &ns_fix, &np_dummy, &margin)))
            return rc;
        std::vector<double> g(npl + 1), gc(npl + 1);
        if ((rc = chebfd_coeffs(lam_lo, lam_hi, a, b, npl, CHEBFD_KERNEL_LANCZOS, 2.0, g.data())))
            return rc;
        for (int k = 0; k <= npl; ++k) gc[k] = g[k] * (1.0 + corr[k]);
        double s_plain, s_corr, e;
        quality(g.data(), npl, a, b, lam_lo, lam_hi, lam_lo - margin, lam_hi + margin, &s_plain,
                &e);
        quality(gc.data(), npl, a, b, lam_lo, lam_hi, lam_lo - margin, lam_hi + margin, &s_corr,
                &e);
        keep = s_corr < s_plain;
    }
    for (int k = 0; k <= npl; ++k) gamma_corr[k] = keep ? corr[k] : 0.0;
    if (corr_kept) *corr_kept = keep ? 1 : 0;
    return CHEBFD_OK;
}
