// Host-side filter polynomial math (Sec. 2.1 and 2.3): window expansion
// coefficients, damping kernels, Clenshaw evaluation, filter quality and the
// eta-minimising polynomial degree.
#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <vector>

#include "internal.h"

namespace chebfd {

// c_n of the rectangular window W = 1 on [lo, hi] within [a, b] (Eq. (W1)).
// With x = cos(theta) the integral (2 - d_n0)/pi int W T_n (1-x^2)^{-1/2} dx
// becomes (2 - d_n0)/pi int_{theta_hi}^{theta_lo} cos(n theta) dtheta.
void window_coeffs(double lo, double hi, double a, double b, int n_p, double *c)
{
    const double alpha = 2.0 / (b - a), beta = (a + b) / (a - b);
    const double xl = std::min(1.0, std::max(-1.0, alpha * lo + beta));
    const double xh = std::min(1.0, std::max(-1.0, alpha * hi + beta));
    const double tl = std::acos(xl), th = std::acos(xh);
    c[0] = (tl - th) / M_PI;
    for (int n = 1; n <= n_p; ++n) c[n] = 2.0 * (std::sin(n * tl) - std::sin(n * th)) / (M_PI * n);
}

// Damping factors of Table tab:Kernel.
void damping(int kernel, int n_p, double mu, double *g)
{
    const double np = (double)n_p;
    for (int n = 0; n <= n_p; ++n) {
        switch (kernel) {
        case CHEBFD_KERNEL_FEJER:
            g[n] = (np - n + 1.0) / (np + 1.0);
            break;
        case CHEBFD_KERNEL_JACKSON: {
            const double q = M_PI / np;
            g[n] = ((np - n) * std::cos(q * n) + std::sin(q * n) / std::tan(q)) / np;
            break;
        }
        case CHEBFD_KERNEL_LANCZOS: {
            if (n == 0) {
                g[n] = 1.0;
            } else {
                const double s = M_PI * n / (np + 1.0);
                g[n] = std::pow(std::sin(s) / s, mu);
            }
            break;
        }
        default:
            g[n] = 1.0;
        }
    }
}

// p(x) = sum_n gamma_n T_n(alpha x + beta) by Clenshaw's backward recurrence.
double poly_value(const double *gamma, int n_p, double a, double b, double x)
{
    const double y = (2.0 * x - a - b) / (b - a);
    double b1 = 0.0, b2 = 0.0;
    for (int n = n_p; n >= 1; --n) {
        const double t = gamma[n] + 2.0 * y * b1 - b2;
        b2 = b1;
        b1 = t;
    }
    return gamma[0] + y * b1 - b2;
}

// Division by a linear factor in the Chebyshev basis.  For
// p(y) = sum_{n=0}^{N} c_n T_n(y) and a point t, q(y) = (p(y) - p(t)) / (y - t)
// = sum_{n=0}^{N-1} d_n T_n(y).  With y T_0 = T_1 and 2 y T_n = T_{n+1} +
// T_{n-1} (n >= 1), matching the T_m terms of (y - t) q = p - p(t) gives
// from the top d_{m-1} = 2 c_m + 2 t d_m - d_{m+1} (m = N .. 2, d_N = d_{N+1}
// = 0), then d_0 = c_1 + t d_1 - d_2 / 2, and the T_0 term leaves
// p(t) = c_0 + t d_0 - d_1 / 2 (Clenshaw's sum: d_{m-1} / 2 and d_0 are its
// intermediate values).  Writes d[0 .. N-1]; returns p(t).
double cheb_divide(const double *c, int N, double t, double *d)
{
    double d1 = 0.0, d2 = 0.0;   // d_m, d_{m+1}
    for (int m = N; m >= 2; --m) {
        const double v = 2.0 * c[m] + 2.0 * t * d1 - d2;
        d[m - 1] = v;
        d2 = d1;
        d1 = v;
    }
    const double d0 = c[1] + t * d1 - 0.5 * d2;
    d[0] = d0;
    return c[0] + t * d0 - 0.5 * d1;
}

// In-place iterative radix-2 complex FFT (length a power of two).
void fft(std::vector<std::complex<double>> &v)
{
    const size_t n = v.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(v[i], v[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        const double ang = -2.0 * M_PI / (double)len;
        const std::complex<double> wl(std::cos(ang), std::sin(ang));
        for (size_t i = 0; i < n; i += len) {
            std::complex<double> w(1.0, 0.0);
            for (size_t k = 0; k < len / 2; ++k) {
                const std::complex<double> x = v[i + k], y = v[i + k + len / 2] * w;
                v[i + k] = x + y;
                v[i + k + len / 2] = x - y;
                w *= wl;
            }
        }
    }
}

// sigma = max_{x in [a,b] \ [s_lo,s_hi]} |p| / min_{x in [t_lo,t_hi]} |p|,
// eta = -n_p / log10 sigma (Sec. 2.3).  |p| is sampled on the grid
// theta_k = pi k / M, k = 0..M, uniform in theta = acos((2x - a - b)/(b - a)),
// with M the smallest power of two giving at least 8 points per period of
// T_{n_p}, plus the four interval edges.  p(cos theta_k) = sum_n gamma_n
// cos(n theta_k) is a DCT-I, evaluated with one FFT of length 2M of the
// even extension of gamma: O(n_p log n_p) instead of a Clenshaw sum per point.
void quality(const double *gamma, int n_p, double a, double b, double t_lo, double t_hi,
             double s_lo, double s_hi, double *sigma, double *eta)
{
    size_t M = 64;
    while (M < (size_t)(4 * (n_p + 1))) M <<= 1;
    std::vector<std::complex<double>> v(2 * M, 0.0);
    for (int n = 0; n <= n_p; ++n) v[n] = gamma[n];
    for (int n = 1; n <= n_p; ++n) v[2 * M - n] = gamma[n];
    fft(v);
    double mx = 0.0, mn = INFINITY;
    for (size_t k = 0; k <= M; ++k) {
        const double th = M_PI * (double)k / (double)M;
        const double x = 0.5 * (a + b) + 0.5 * (b - a) * std::cos(th);
        const bool in_t = x >= t_lo && x <= t_hi;
        const bool out_s = x < s_lo || x > s_hi;
        if (!in_t && !out_s) continue;
        // FFT[k] = gamma_0 + 2 sum_{n>=1} gamma_n cos(n theta_k)
        const double p = std::fabs(0.5 * (v[k].real() + gamma[0]));
        if (in_t) mn = std::min(mn, p);
        if (out_s) mx = std::max(mx, p);
    }
    for (double x : {t_lo, t_hi}) mn = std::min(mn, std::fabs(poly_value(gamma, n_p, a, b, x)));
    for (double x : {s_lo, s_hi}) mx = std::max(mx, std::fabs(poly_value(gamma, n_p, a, b, x)));
    *sigma = mx / mn;
    *eta = (*sigma < 1.0) ? -n_p / std::log10(*sigma) : INFINITY;
}

}  // namespace chebfd

using namespace chebfd;

extern "C" int chebfd_coeffs(double lam_lo, double lam_hi, double a, double b, int n_p,
                             int kernel, double mu, double *gamma_out)
{
    if (!gamma_out) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_coeffs: gamma_out is NULL");
    if (!(lam_lo < lam_hi) || !(a < b) || n_p < 2 || kernel < 0 || kernel > 3 ||
        !std::isfinite(lam_lo) || !std::isfinite(lam_hi))
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_coeffs: need lam_lo < lam_hi, a < b, n_p >= 2, kernel 0..3");
    if (lam_hi <= a || lam_lo >= b)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_coeffs: window does not intersect [a, b]");
    std::vector<double> g(n_p + 1);
    window_coeffs(lam_lo, lam_hi, a, b, n_p, gamma_out);
    damping(kernel, n_p, mu, g.data());
    for (int n = 0; n <= n_p; ++n) gamma_out[n] *= g[n];
    return CHEBFD_OK;
}

extern "C" int chebfd_coeffs_divided(const double *gamma, int n_p, double a, double b,
                                     double lambda, double *d_out, double *p_out)
{
    if (!gamma || !d_out || n_p < 2 || !(a < b) || !std::isfinite(lambda))
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_coeffs_divided: invalid arguments");
    const double t = (2.0 * lambda - a - b) / (b - a);
    const double pt = cheb_divide(gamma, n_p, t, d_out);
    if (p_out) *p_out = pt;
    return CHEBFD_OK;
}

extern "C" int chebfd_filter_quality(const double *gamma, int n_p, double a, double b,
                                     double t_lo, double t_hi, double s_lo, double s_hi,
                                     double *sigma, double *eta)
{
    if (!gamma || !sigma || !eta || n_p < 1 || !(a < b) || !(t_lo < t_hi) || s_lo > t_lo ||
        s_hi < t_hi)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_filter_quality: invalid arguments");
    quality(gamma, n_p, a, b, t_lo, t_hi, s_lo, s_hi, sigma, eta);
    return CHEBFD_OK;
}

extern "C" int chebfd_optimal_np(double a, double b, double t_lo, double t_hi, double s_lo,
                                 double s_hi, int kernel, double mu, int np_min, int np_max,
                                 int *n_p, double *eta_out)
{
    if (!n_p || !eta_out || np_min < 2 || np_max < np_min || !(a < b) || !(t_lo < t_hi) ||
        s_lo > t_lo || s_hi < t_hi)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_optimal_np: invalid arguments");
    std::map<int, double> f;
    std::vector<double> gam, g;
    auto ev = [&](int k) {
        auto it = f.find(k);
        if (it != f.end()) return it->second;
        gam.resize(k + 1);
        g.resize(k + 1);
        window_coeffs(t_lo, t_hi, a, b, k, gam.data());
        damping(kernel, k, mu, g.data());
        for (int n = 0; n <= k; ++n) gam[n] *= g[n];
        double s, e;
        quality(gam.data(), k, a, b, t_lo, t_hi, s_lo, s_hi, &s, &e);
        f[k] = e;
        return e;
    };
    // eta(n_p) is jagged: scan a 2% geometric grid, refine the five best
    // points on a 0.25% grid within +-3%, then scan every integer within
    // +-max(2, 0.5%) of the three best points found so far.
    auto geometric = [](double lo, double hi, double step, std::vector<int> &out) {
        for (double x = lo; x <= hi * 1.0000001; x *= step) {
            const int k = (int)std::lround(x);
            if (out.empty() || out.back() != k) out.push_back(k);
        }
    };
    auto best_k = [&](size_t cnt) {
        std::vector<std::pair<double, int>> sc;
        for (auto &kv : f) sc.push_back({kv.second, kv.first});
        std::sort(sc.begin(), sc.end());
        std::vector<int> out;
        for (size_t i = 0; i < std::min(cnt, sc.size()); ++i) out.push_back(sc[i].second);
        return out;
    };
    std::vector<int> grid;
    geometric(np_min, np_max, 1.02, grid);
    if (grid.back() != np_max) grid.push_back(np_max);
    for (int k : grid) ev(k);
    for (int k : best_k(5)) {
        std::vector<int> fine;
        geometric(std::max<double>(np_min, 0.97 * k), std::min<double>(np_max, 1.03 * k), 1.0025,
                  fine);
        for (int j : fine) ev(j);
    }
    for (int k : best_k(3)) {
        const int w = std::max(2, (int)(0.005 * k));
        for (int j = std::max(np_min, k - w); j <= std::min(np_max, k + w); ++j) ev(j);
    }
    int best = np_min;
    double be = INFINITY;
    for (auto &kv : f)
        if (kv.second < be) {
            be = kv.second;
            best = kv.first;
        }
    *n_p = best;
    *eta_out = be;
    return CHEBFD_OK;
}
