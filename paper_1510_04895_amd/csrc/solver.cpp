// The ChebFD scheme (Sec. 3.1, steps 1-8) on one GPU.
//
// Per outer iteration: the polynomial filter on the active block (N_p fused
// launches, no host synchronisation), projection of the locked vectors out
// of the block, SVQB orthonormalisation with refill (step 6), Rayleigh-Ritz
// with Ritz vectors, H times Ritz vectors and FP64 residual norms (step 7),
// ghost/convergence classification and locking (step 8).  The dense
// contractions run on the FP64 matrix cores; the N_S x N_S eigenproblems on
// the host.
//
// Readings where the paper leaves a choice (shared with the CPU reference):
//  - an in-window Ritz pair is converged if r <= eps, converging if
//    eps < r <= sqrt(eps), a ghost candidate otherwise;
//  - exit after >= 2 iterations once no in-window pair is converging, the
//    converged count has not changed, and the smallest remaining in-window
//    residual fell by less than 10% while nothing has converged, or by less
//    than half once some pairs have (ghosts: a large residual that does not
//    decrease; a slowly converging search space gains more);
//  - the restart block is the set of Ritz vectors.
// Locking (a refinement the paper lists in Sec. 6): converged in-window
// pairs move to a locked set Q, later blocks are kept orthogonal to Q and
// only the remaining columns are filtered.
// Precision form (C64): the filter runs on complex64 blocks in FP32; Gram,
// Rayleigh-Ritz and residuals are FP64 on the FP64-converted block.  When the
// in-window residuals reach `polish_switch` (by default a few FP32 roundings
// of the spectral scale) or stop improving, the block is promoted to
// complex128, narrowed to the in-window Ritz vectors and their nearest
// neighbours, and the FP64 iteration (the polish) continues to eps.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.h"

struct chebfd_result {
    std::vector<double> evals, res, evecs;
    // precision form: the in-window Ritz pairs of the complex64 sweep whose
    // residual was below sqrt(eps), at its last iteration (before the polish)
    std::vector<double> sweep_evals, sweep_res;
    std::vector<chebfd_iter_info> history;   // one entry per outer iteration
    chebfd_stats stats{};
};

namespace chebfd {
namespace {

using clk = std::chrono::steady_clock;
static double secs(clk::time_point a, clk::time_point b)
{
    return std::chrono::duration<double>(b - a).count();
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t blk64 = 0, blk32 = 0;   // bytes of one c128 / c64 block
    size_t off_b[4] = {0, 0, 0, 0};
    size_t off_x32 = 0, off_q = 0, off_mom = 0, off_small = 0, total = 0;
    size_t small = 0;
};

Layout layout(int64_t n, const chebfd_params &p)
{
    Layout L;
    L.blk64 = align256((size_t)n * p.n_s * 16);
    L.blk32 = align256((size_t)n * p.n_s * 8);
    size_t off = 0;
    // three c128 blocks; in the C64 form the first one also hosts the two
    // c64 filter scratch blocks U32 (at 0) and W32 (at blk32), so it spans
    // at least 2 blk32 bytes (align256 can make 2 blk32 exceed blk64)
    for (int i = 0; i < 3; ++i) {
        L.off_b[i] = off;
        off += (i == 0 && p.precision == CHEBFD_PREC_C64) ? std::max(L.blk64, 2 * L.blk32)
                                                          : L.blk64;
    }
    if (p.precision == CHEBFD_PREC_C64) {
        L.off_x32 = off;
        off += L.blk32;
    }
    if (p.lock) {
        L.off_q = off;
        off += L.blk64;
    }
    if (p.adapt) {
        // Chebyshev moments of the first filter pass, (2 n_p + 1) x n_s
        L.off_mom = off;
        off += align256((size_t)(2 * p.n_p + 1) * p.n_s * 8);
    }
    // small device matrices: S (n_s^2 c128), Tr (4 n_s^2 doubles), theta,
    // residuals (n_s each), column index list (n_s int32)
    const size_t ns = (size_t)p.n_s;
    L.small = align256(ns * ns * 16) + align256(4 * ns * ns * 8) + 2 * align256(ns * 8) +
              align256(ns * 4) + align256(ns * ns * 16);
    L.off_small = off;
    off += L.small;
    L.total = off;
    return L;
}

// Harmonic Ritz extraction (Sec. 3.1 step 7 remarks, Sec. 6) for the
// target tau from G = X^H H X and Mu = (H X)^H (H X) of an orthonormal X:
// M = ((H - tau) X)^H ((H - tau) X) = Mu - tau (G + G^H) + tau^2 I, the
// Petrov-Galerkin pairs solve M s = (theta - tau) (G - tau I) s, i.e. the
// Hermitian problem T^H (G - tau I) T z = z / (theta - tau) with T = L^{-H}
// for M = L L^H, s = T z.  Returns the coefficient matrix S (k x k,
// interleaved, row-major) with unit columns ordered by their Rayleigh
// quotients rho_j = s_j^H G s_j (ascending), or -1 if M is not positive
// definite.
int harmonic_extract(int k, const std::vector<double> &G, const std::vector<double> &Mu, double tau,
                     std::vector<double> &Sout, std::vector<double> &rho)
{
    typedef std::complex<double> cd;
    auto at = [&](const std::vector<double> &A, int i, int j) {
        return cd(A[2 * ((size_t)i * k + j)], A[2 * ((size_t)i * k + j) + 1]);
    };
    std::vector<cd> Gh((size_t)k * k);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) Gh[(size_t)i * k + j] = 0.5 * (at(G, i, j) + std::conj(at(G, j, i)));
    std::vector<double> M((size_t)2 * k * k), T;
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            const cd gsym = Gh[(size_t)i * k + j] + std::conj(Gh[(size_t)j * k + i]);
            cd v = 0.5 * (at(Mu, i, j) + std::conj(at(Mu, j, i))) - tau * gsym;
            if (i == j) v += tau * tau;
            M[2 * ((size_t)i * k + j)] = v.real();
            M[2 * ((size_t)i * k + j) + 1] = v.imag();
        }
    if (chol_inv_factor(k, M, T) != 0) return -1;
    auto Tat = [&](int i, int j) { return cd(T[2 * ((size_t)i * k + j)], T[2 * ((size_t)i * k + j) + 1]); };
    // C = T^H (G - tau I) T
    std::vector<cd> AT((size_t)k * k, cd(0.0));
    for (int i = 0; i < k; ++i)
        for (int q = 0; q < k; ++q) {
            const cd a = Gh[(size_t)i * k + q] - (i == q ? tau : 0.0);
            if (a == cd(0.0)) continue;
            for (int j = q; j < k; ++j) AT[(size_t)i * k + j] += a * Tat(q, j);   // T upper
        }
    std::vector<double> Cm((size_t)2 * k * k), zeta;
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            cd v = 0.0;
            for (int p = 0; p <= i; ++p) v += std::conj(Tat(p, i)) * AT[(size_t)p * k + j];
            Cm[2 * ((size_t)i * k + j)] = v.real();
            Cm[2 * ((size_t)i * k + j) + 1] = v.imag();
        }
    if (herm_eig(k, Cm, zeta) != 0) return -1;
    // S = T Z, unit columns, Rayleigh quotients
    std::vector<cd> S((size_t)k * k, cd(0.0));
    for (int i = 0; i < k; ++i)
        for (int q = i; q < k; ++q) {
            const cd t = Tat(i, q);
            for (int j = 0; j < k; ++j) S[(size_t)i * k + j] += t * at(Cm, q, j);
        }
    std::vector<double> r(k);
    for (int j = 0; j < k; ++j) {
        double nrm = 0.0;
        for (int i = 0; i < k; ++i) nrm += std::norm(S[(size_t)i * k + j]);
        nrm = std::sqrt(nrm);
        for (int i = 0; i < k; ++i) S[(size_t)i * k + j] /= nrm;
        cd v = 0.0;
        for (int p = 0; p < k; ++p) {
            cd gs = 0.0;
            for (int q = 0; q < k; ++q) gs += Gh[(size_t)p * k + q] * S[(size_t)q * k + j];
            v += std::conj(S[(size_t)p * k + j]) * gs;
        }
        r[j] = v.real();
    }
    std::vector<int> ord(k);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return r[x] < r[y]; });
    Sout.assign((size_t)2 * k * k, 0.0);
    rho.resize(k);
    for (int j = 0; j < k; ++j) {
        rho[j] = r[ord[j]];
        for (int i = 0; i < k; ++i) {
            Sout[2 * ((size_t)i * k + j)] = S[(size_t)i * k + ord[j]].real();
            Sout[2 * ((size_t)i * k + j) + 1] = S[(size_t)i * k + ord[j]].imag();
        }
    }
    return 0;
}

struct Solver {
    chebfd_ctx *ctx;
    const chebfd_matrix *H;
    chebfd_params p;
    int64_t n;
    int ns;
    char *ws;
    Layout L;
    // device small buffers
    double *dS = nullptr, *dTr = nullptr, *dTheta = nullptr, *dRes = nullptr, *dS2 = nullptr;
    int32_t *dIdx = nullptr;
    std::vector<double> gamma;
    double a = 0, b = 0;
    chebfd_stats st{};
    uint64_t refill_ctr = 0;
    bool bounds_checked = false;   // [a, b] is an estimate: verify every Rayleigh quotient
    static constexpr int RESTART_WIDER = 1000;

    int sync() { CHEBFD_HIP(hipStreamSynchronize(ctx->stream)); return CHEBFD_OK; }

    int down(void *dst, const void *src, size_t bytes)
    {
        CHEBFD_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, ctx->stream));
        return sync();
    }
    int up(void *dst, const void *src, size_t bytes)
    {
        CHEBFD_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ctx->stream));
        return CHEBFD_OK;
    }

    // Uploads the real (2k x 2m) expansion of a complex k x m host matrix.
    int upload_T(const std::vector<double> &T, int k, int m)
    {
        std::vector<double> Tr((size_t)4 * k * m);
        const size_t mc = 2 * (size_t)m;
        for (int r = 0; r < k; ++r)
            for (int c = 0; c < m; ++c) {
                const double re = T[2 * ((size_t)r * m + c)], im = T[2 * ((size_t)r * m + c) + 1];
                Tr[(2 * r) * mc + 2 * c] = re;
                Tr[(2 * r) * mc + 2 * c + 1] = im;
                Tr[(2 * r + 1) * mc + 2 * c] = -im;
                Tr[(2 * r + 1) * mc + 2 * c + 1] = re;
            }
        int rc = up(dTr, Tr.data(), Tr.size() * 8);
        if (rc) return rc;
        return sync();   // the host vector goes out of scope
    }

    // S = A^H B on the device, copied to the host (k x m complex).
    int gram_host(int prec_a, const void *A, int k, int prec_b, const void *B, int m,
                  std::vector<double> &S)
    {
        int rc;
        if (prec_a != prec_b) return fail(CHEBFD_ERR_UNSUPPORTED, "mixed-precision Gram");
        if ((rc = launch_gram(ctx, prec_a, A, ns, k, B, ns, m, n, dS))) return rc;
        S.resize((size_t)2 * k * m);
        return down(S.data(), dS, S.size() * 8);
    }

    // X <- X - Q (Q^H X) for the nl locked columns (c128 Q).
    int project_locked(int prec, void *X, int k, int nl, void *Q)
    {
        if (nl == 0 || k == 0) return CHEBFD_OK;
        int rc;
        void *src = X;
        std::vector<double> S;
        if (prec == CHEBFD_PREC_C64) return fail(CHEBFD_ERR_UNSUPPORTED, "locking in c64 phase");
        if ((rc = gram_host(CHEBFD_PREC_C128, Q, nl, CHEBFD_PREC_C128, src, k, S))) return rc;
        if ((rc = upload_T(S, nl, k))) return rc;
        return launch_block_times(ctx, CHEBFD_PREC_C128, Q, ns, n, nl, dTr, k, prec, X, ns, 1);
    }

    // SVQB (Sec. 3.1 step 6): X (k columns) -> orthonormal, via scratch Y.
    // On return *X_out points at the buffer holding the result.
    int svqb(int prec, void **X, void **Y, int k, int nl, void *Q)
    {
        int clean = 0;
        std::vector<double> S, w, T;
        for (int pass = 0; pass < 8 && clean < 2; ++pass) {
            int rc;
            if ((rc = gram_host(prec, *X, k, prec, *X, k, S))) return rc;
            std::vector<double> d(k);
            for (int i = 0; i < k; ++i) {
                const double s = S[2 * ((size_t)i * k + i)];
                if (!std::isfinite(s)) {
                    // on an estimated interval the filter grows without
                    // bound outside [a, b] (T_n(x) for |x| > 1): an overflow
                    // proves the interval too narrow
                    if (bounds_checked) return RESTART_WIDER;
                    return fail(CHEBFD_ERR_NONFINITE, "non-finite Gram diagonal");
                }
                d[i] = s > 0.0 ? 1.0 / std::sqrt(s) : 0.0;
            }
            for (int i = 0; i < k; ++i)
                for (int j = 0; j < k; ++j) {
                    S[2 * ((size_t)i * k + j)] *= d[i] * d[j];
                    S[2 * ((size_t)i * k + j) + 1] *= d[i] * d[j];
                }
            // after a clean rank-revealing pass the block is close to
            // orthonormal: the second pass uses the Cholesky factor of the
            // scaled Gram (T = D L^{-H}), falling back to the eigenvalue
            // form if the factorisation breaks down
            int keep = k;
            bool done = false;
            if (clean >= 1 && chol_inv_factor(k, S, T) == 0) {
                for (int i = 0; i < k; ++i)
                    for (int j = 0; j < k; ++j) {
                        T[2 * ((size_t)i * k + j)] *= d[i];
                        T[2 * ((size_t)i * k + j) + 1] *= d[i];
                    }
                done = true;
            }
            if (!done) {
                if (herm_eig(k, S, w) != 0) {
                    if (bounds_checked) return RESTART_WIDER;
                    return fail(CHEBFD_ERR_NONFINITE, "SVQB eigensolver failed");
                }
                const double tmax = w[k - 1];
                // T = D U Theta^{-1/2}, kept directions, largest first
                T.assign((size_t)2 * k * k, 0.0);
                keep = 0;
                for (int j = k - 1; j >= 0; --j) {
                    if (!(w[j] > 1e-12 * tmax)) continue;
                    const double f = 1.0 / std::sqrt(w[j]);
                    for (int i = 0; i < k; ++i) {
                        T[2 * ((size_t)i * k + keep)] = d[i] * S[2 * ((size_t)i * k + j)] * f;
                        T[2 * ((size_t)i * k + keep) + 1] = d[i] * S[2 * ((size_t)i * k + j) + 1] * f;
                    }
                    ++keep;
                }
            }
            if ((rc = upload_T(T, k, k))) return rc;
            if ((rc = launch_block_times(ctx, prec, *X, ns, n, k, dTr, k, prec, *Y, ns, 0)))
                return rc;
            std::swap(*X, *Y);
            if (keep < k) {
                // refill the dropped directions with random vectors (stream 3)
                const uint64_t off = (uint64_t)(++refill_ctr) * (uint64_t)n * (uint64_t)ns;
                if ((rc = launch_random(ctx, prec, *X, n, ns, ns, keep, k - keep, p.seed, 3, off)))
                    return rc;
                st.refilled += k - keep;
                if ((rc = project_locked(prec, *X, k, nl, Q))) return rc;
                clean = 0;
            } else {
                ++clean;
            }
        }
        return CHEBFD_OK;
    }

    // Adaptive degree (the refinement of Sec. 6): the first pass filtered
    // the random start block, so its moments <x, T_m x> / <x, x>, averaged
    // over the k columns, estimate the normalised density of states (a
    // stochastic trace with k vectors).  N_T follows from Eq. DOS:target,
    // the search margin for N_S from Eq. DOS:search, and the degree that
    // minimises eta for that margin (Sec. 2.3-2.4) is used from now on.
    int reselect_degree(const double *dmom, int ld, int k)
    {
        const int M = 2 * p.n_p + 1;
        std::vector<double> m((size_t)M * ld), mu(M, 0.0);
        int rc = down(m.data(), dmom, m.size() * 8);
        if (rc) return rc;
        for (int c = 0; c < k; ++c) {
            const double m0 = m[c];
            if (!(m0 > 0.0)) continue;
            for (int j = 0; j < M; ++j) mu[j] += m[(size_t)j * ld + c] / m0;
        }
        for (int j = 0; j < M; ++j) mu[j] /= k;
        double nt = 0.0, margin = 0.0;
        int ns_fixed = p.n_s, np_new = 0;
        if ((rc = chebfd_dos_params(mu.data(), M, n, a, b, p.lam_lo, p.lam_hi, 1.0, p.kernel,
                                    p.mu, p.n_s, &nt, &ns_fixed, &np_new, &margin)))
            return rc;
        st.n_t_estimate = nt;
        if (p.verbose) {
            std::fprintf(stderr,
                         "chebfd: adaptive degree: N_T estimate %.1f, margin %.4g, n_p %d -> %d\n",
                         nt, margin, p.n_p, np_new);
            std::fflush(stderr);
        }
        if (np_new >= 2 && np_new != p.n_p) {
            p.n_p = np_new;
            gamma.assign(p.n_p + 1, 0.0);
            if ((rc = chebfd_coeffs(p.lam_lo, p.lam_hi, a, b, p.n_p, p.kernel, p.mu, gamma.data())))
                return rc;
        }
        return CHEBFD_OK;
    }

    std::vector<double> Gk, Sh;   // harmonic mode: X^H H X and the coefficients

    // Locks the converged harmonic Ritz vectors (columns conv of X, their H
    // images in W, coefficients Sh in the orthonormal basis of this
    // iteration, whose Rayleigh matrix is Gk): an orthonormal basis of them
    // by the Cholesky factor of their Gram Sc^H Sc, then the Ritz pairs of H
    // inside that space; the locked residuals are recomputed on the device.
    // U is scratch.
    int lock_harmonic(void *X, void *U, void *W, void *Q, int n_lock, const std::vector<int> &conv,
                      std::vector<double> &lock_vals, std::vector<double> &lock_res)
    {
        typedef std::complex<double> cd;
        const int k = (int)std::sqrt((double)(Sh.size() / 2) + 0.5), c = (int)conv.size();
        auto sh = [&](int i, int j) {
            return cd(Sh[2 * ((size_t)i * k + j)], Sh[2 * ((size_t)i * k + j) + 1]);
        };
        auto gk = [&](int i, int j) {
            return cd(Gk[2 * ((size_t)i * k + j)], Gk[2 * ((size_t)i * k + j) + 1]);
        };
        std::vector<double> Gc((size_t)2 * c * c), Tc;
        std::vector<cd> HcS((size_t)c * c, cd(0.0));
        for (int a = 0; a < c; ++a)
            for (int b = 0; b < c; ++b) {
                cd g = 0.0, h = 0.0;
                for (int i = 0; i < k; ++i) {
                    g += std::conj(sh(i, conv[a])) * sh(i, conv[b]);
                    cd gs = 0.0;
                    for (int q = 0; q < k; ++q) gs += gk(i, q) * sh(q, conv[b]);
                    h += std::conj(sh(i, conv[a])) * gs;
                }
                Gc[2 * ((size_t)a * c + b)] = g.real();
                Gc[2 * ((size_t)a * c + b) + 1] = g.imag();
                HcS[(size_t)a * c + b] = h;
            }
        if (chol_inv_factor(c, Gc, Tc) != 0)
            return fail(CHEBFD_ERR_NONFINITE, "harmonic locking: converged vectors are dependent");
        auto tc = [&](int i, int j) {
            return cd(Tc[2 * ((size_t)i * c + j)], Tc[2 * ((size_t)i * c + j) + 1]);
        };
        // Hc = Tc^H HcS Tc, Hermitian; its eigenvectors rotate the basis
        std::vector<double> Hc((size_t)2 * c * c), vals;
        for (int a = 0; a < c; ++a)
            for (int b = 0; b < c; ++b) {
                cd v = 0.0;
                for (int p = 0; p < c; ++p)
                    for (int q = 0; q < c; ++q) v += std::conj(tc(p, a)) * HcS[(size_t)p * c + q] * tc(q, b);
                Hc[2 * ((size_t)a * c + b)] = v.real();
                Hc[2 * ((size_t)a * c + b) + 1] = v.imag();
            }
        for (int a = 0; a < c; ++a)
            for (int b = a + 1; b < c; ++b) {   // exact Hermitian symmetry
                const double re = 0.5 * (Hc[2 * ((size_t)a * c + b)] + Hc[2 * ((size_t)b * c + a)]);
                const double im = 0.5 * (Hc[2 * ((size_t)a * c + b) + 1] - Hc[2 * ((size_t)b * c + a) + 1]);
                Hc[2 * ((size_t)a * c + b)] = re;
                Hc[2 * ((size_t)a * c + b) + 1] = im;
                Hc[2 * ((size_t)b * c + a)] = re;
                Hc[2 * ((size_t)b * c + a) + 1] = -im;
            }
        if (herm_eig(c, Hc, vals) != 0)
            return fail(CHEBFD_ERR_NONFINITE, "harmonic locking: eigensolver failed");
        // R = Tc Zc (c x c): locked = X_conv R, their images = W_conv R
        std::vector<double> R((size_t)2 * c * c, 0.0);
        for (int a = 0; a < c; ++a)
            for (int b = 0; b < c; ++b) {
                cd v = 0.0;
                for (int q = 0; q < c; ++q)
                    v += tc(a, q) * cd(Hc[2 * ((size_t)q * c + b)], Hc[2 * ((size_t)q * c + b) + 1]);
                R[2 * ((size_t)a * c + b)] = v.real();
                R[2 * ((size_t)a * c + b) + 1] = v.imag();
            }
        int rc;
        std::vector<int32_t> idx(conv.begin(), conv.end());
        if ((rc = up(dIdx, idx.data(), idx.size() * 4))) return rc;
        if ((rc = upload_T(R, c, c))) return rc;
        void *Qs = (char *)Q + (size_t)n_lock * 16;
        if ((rc = launch_gather_cols(ctx, CHEBFD_PREC_C128, X, ns, U, ns, 0, dIdx, n, c))) return rc;
        if ((rc = launch_block_times(ctx, CHEBFD_PREC_C128, U, ns, n, c, dTr, c, CHEBFD_PREC_C128,
                                     Qs, ns, 0)))
            return rc;
        if ((rc = launch_gather_cols(ctx, CHEBFD_PREC_C128, W, ns, U, ns, 0, dIdx, n, c))) return rc;
        if ((rc = launch_block_times(ctx, CHEBFD_PREC_C128, U, ns, n, c, dTr, c, CHEBFD_PREC_C128,
                                     W, ns, 0)))
            return rc;
        if ((rc = up(dTheta, vals.data(), (size_t)c * 8))) return rc;
        if ((rc = launch_residuals(ctx, CHEBFD_PREC_C128, Qs, W, n, c, ns, dTheta, dRes))) return rc;
        std::vector<double> r(c);
        if ((rc = down(r.data(), dRes, (size_t)c * 8))) return rc;
        for (int a = 0; a < c; ++a) {
            lock_vals.push_back(vals[a]);
            lock_res.push_back(r[a]);
        }
        return CHEBFD_OK;
    }

    // Correction pass of the precision form's polish: FP32 arithmetic with
    // FP64 accuracy.  With y = alpha x + beta, p(y) = p(t) + (y - t) q_t(y)
    // for every t (q_t of degree n_p - 1), so for a Ritz pair (theta, v) and
    // t = alpha theta + beta
    //     p(H~) v = p(t) v + q_t(H~) r,   r = (H~ - t) v,
    // exactly.  r is formed in FP64 and rounded to complex64, and only
    // q_t(H~) r is filtered in FP32: its rounding error scales with |r|
    // (the residual) instead of |v|, so a pass lowers the FP32 floor by
    // about that ratio (iterative refinement of the filter).  Column j is
    // filtered with the coefficients of its own q_t (cheb_divide), p(t) v is
    // added back in FP64.  In: X = the k active Ritz vectors (complex128),
    // th their Ritz values.  Out: X = p(H~) X; U, W the two other complex128
    // blocks.  The complex64 filter buffers U32, W32 live in B[0], so X is
    // moved out of B[0] first; the block that held H~ X carries the
    // coefficient table during the filter.
    int correction_pass(void *const B[3], void *&X, void *&U, void *&W, void *X32, void *U32,
                        void *W32, int k, const std::vector<double> &th)
    {
        int rc;
        const size_t bytes = (size_t)n * ns * 16;
        if (X == B[0]) {
            CHEBFD_HIP(hipMemcpyAsync(B[1], X, bytes, hipMemcpyDeviceToDevice, ctx->stream));
            X = B[1];
        }
        void *O = X == B[1] ? B[2] : B[1];
        const double alpha = 2.0 / (b - a), beta = (a + b) / (a - b);
        StepArgs s{};
        s.mode = MODE_APPLY;
        s.precision = CHEBFD_PREC_C128;
        s.u = X;
        s.wout = O;
        s.n = n;
        s.n_s = k;
        s.ld = ns;
        s.s_h = alpha;
        s.s_u = beta;
        if ((rc = launch_step(ctx, H, s, nullptr))) return rc;   // O = H~ X
        // per column: t_j, p(t_j) and the coefficients of q_{t_j}; the
        // filter runs degree max(2, n_p - 1) (zero padding) over kk columns
        // (even for complex64 packs; the padding column is zero)
        const int kk = k & 1 ? k + 1 : k;
        const int deg = std::max(2, p.n_p - 1);
        std::vector<double> t(k), pt(k), d(p.n_p), tab((size_t)(deg + 1) * kk, 0.0);
        for (int j = 0; j < k; ++j) {
            t[j] = std::min(1.0, std::max(-1.0, alpha * th[j] + beta));
            pt[j] = cheb_divide(gamma.data(), p.n_p, t[j], d.data());
            for (int m = 0; m < p.n_p; ++m) tab[(size_t)m * kk + j] = d[m];
        }
        if ((rc = up(dTheta, t.data(), (size_t)k * 8))) return rc;
        if ((rc = launch_defect(ctx, X, O, dTheta, X32, n, k, kk, ns, ns))) return rc;
        // the table replaces H~ X in O (stream order: after the defect kernel)
        if ((rc = up(O, tab.data(), tab.size() * 8))) return rc;
        if ((rc = up(dRes, pt.data(), (size_t)k * 8))) return rc;
        if ((rc = sync())) return rc;   // the host vectors go out of scope
        if ((rc = filter_apply(ctx, H, CHEBFD_PREC_C64, nullptr, deg, a, b, X32, U32, W32, kk, ns,
                               nullptr, p.verbose ? 1024 : 0, nullptr, (const double *)O, kk)))
            return rc;
        if ((rc = launch_combine(ctx, X, X32, dRes, n, k, ns, ns))) return rc;
        st.n_mvm += (int64_t)k * (deg + 1);
        U = O;
        W = B[0];
        return CHEBFD_OK;
    }

    int run(chebfd_result *out)
    {
        const auto t0 = clk::now();
        char *base = ws;
        const bool c64 = p.precision == CHEBFD_PREC_C64;
        void *B[3] = {base + L.off_b[0], base + L.off_b[1], base + L.off_b[2]};
        void *Q = p.lock ? (void *)(base + L.off_q) : nullptr;
        char *sm = base + L.off_small;
        const size_t nsz = (size_t)ns;
        dS = (double *)sm;
        sm += align256(nsz * nsz * 16);
        dTr = (double *)sm;
        sm += align256(4 * nsz * nsz * 8);
        dTheta = (double *)sm;
        sm += align256(nsz * 8);
        dRes = (double *)sm;
        sm += align256(nsz * 8);
        dIdx = (int32_t *)sm;
        sm += align256(nsz * 4);
        dS2 = (double *)sm;

        // filter buffers for each phase
        void *X32 = c64 ? (void *)(base + L.off_x32) : nullptr;
        void *U32 = B[0], *W32 = (char *)B[0] + L.blk32;
        // c128 roles: X, U, W rotate among B[0..2]
        void *X = B[1], *U = B[2], *W = B[0];
        int prec = c64 ? CHEBFD_PREC_C64 : CHEBFD_PREC_C128;
        int rc;
        if (c64) rc = launch_random(ctx, CHEBFD_PREC_C64, X32, n, ns, ns, 0, ns, p.seed, 1, 0);
        else rc = launch_random(ctx, CHEBFD_PREC_C128, X, n, ns, ns, 0, ns, p.seed, 1, 0);
        if (rc) return rc;

        int n_lock = 0, prev_conv = -1, status = CHEBFD_WARN_NOT_CONVERGED;
        double prev_rmin = INFINITY, prev_worst = INFINITY;
        int prev_good = 0;
        std::vector<double> lock_vals, lock_res;
        std::vector<double> theta, res, S, w;
        int last_active = ns;
        int ns_act = ns;   // search-space size (the FP64 polish may narrow it)
        // polish by FP32 correction passes: Ritz values of the active
        // columns, and the largest accepted residual of the last pass
        bool corr = false;
        std::vector<double> th_act;
        double corr_worst = INFINITY;
        int corr_conv = -1;
        std::vector<int> keep_idx, conv_idx;
        const double seps = std::sqrt(p.eps);
        int it;
        for (it = 1; it <= p.max_iter; ++it) {
            const int k = ns_act - n_lock;   // active columns
            last_active = k;
            if (k <= 0) break;
            // ---------------- step 5: filter
            auto ta = clk::now();
            // the first pass of an adaptive solve also returns the moments
            double *mom = (p.adapt && it == 1) ? (double *)(base + L.off_mom) : nullptr;
            if (corr) {
                rc = correction_pass(B, X, U, W, X32, U32, W32, k, th_act);
                ++st.iterations_corr;
            } else if (prec == CHEBFD_PREC_C64) {
                rc = filter_apply(ctx, H, CHEBFD_PREC_C64, gamma.data(), p.n_p, a, b, X32, U32,
                                  W32, k & 1 ? k + 1 : k, ns, mom, p.verbose ? 1024 : 0);
                ++st.iterations_c64;
            } else {
                rc = filter_apply(ctx, H, CHEBFD_PREC_C128, gamma.data(), p.n_p, a, b, X, U, W, k,
                                  ns, mom, p.verbose ? 1024 : 0);
            }
            if (rc) return rc;
            if (!corr) st.n_mvm += (int64_t)k * p.n_p;
            if ((rc = sync())) return rc;
            if (mom && (rc = reselect_degree(mom, k & 1 && prec == CHEBFD_PREC_C64 ? k + 1 : k,
                                             k)))
                return rc;
            auto tb = clk::now();
            st.t_filter += secs(ta, tb);
            // ---------------- step 6: orthogonalise (FP64 on the converted block)
            if (prec == CHEBFD_PREC_C64) {
                // X <- fp64(X32); orthogonalise in c128
                if ((rc = launch_convert(ctx, CHEBFD_PREC_C64, X32, CHEBFD_PREC_C128, X, n, k, ns, ns)))
                    return rc;
            }
            if ((rc = project_locked(CHEBFD_PREC_C128, X, k, n_lock, Q))) return rc;
            if ((rc = svqb(CHEBFD_PREC_C128, &X, &U, k, n_lock, Q))) return rc;
            auto tc = clk::now();
            st.t_ortho += secs(tb, tc);
            // ---------------- step 7: Rayleigh-Ritz
            StepArgs s{};
            s.mode = MODE_APPLY;
            s.precision = CHEBFD_PREC_C128;
            s.u = X;
            s.wout = U;
            s.n = n;
            s.n_s = k;
            s.ld = ns;
            s.s_h = 1.0;
            s.s_u = 0.0;
            if ((rc = launch_step(ctx, H, s, nullptr))) return rc;        // U = H X
            if ((rc = gram_host(CHEBFD_PREC_C128, X, k, CHEBFD_PREC_C128, U, k, S))) return rc;
            bool harm = false;
            if (p.harmonic) {
                // harmonic Ritz pairs for the window centre (one more Gram)
                std::vector<double> Mu;
                if ((rc = gram_host(CHEBFD_PREC_C128, U, k, CHEBFD_PREC_C128, U, k, Mu))) return rc;
                Gk = S;
                harm = harmonic_extract(k, S, Mu, 0.5 * (p.lam_lo + p.lam_hi), Sh, theta) == 0;
                if (harm) S = Sh;
            }
            if (!harm && herm_eig(k, S, theta) != 0) {
                if (bounds_checked) return RESTART_WIDER;
                return fail(CHEBFD_ERR_NONFINITE, "Rayleigh-Ritz eigensolver failed");
            }
            if ((rc = upload_T(S, k, k))) return rc;
            // W = X Ug (Ritz vectors), X = U Ug (H times Ritz vectors)
            if ((rc = launch_block_times(ctx, CHEBFD_PREC_C128, X, ns, n, k, dTr, k, CHEBFD_PREC_C128, W, ns, 0)))
                return rc;
            if ((rc = launch_block_times(ctx, CHEBFD_PREC_C128, U, ns, n, k, dTr, k, CHEBFD_PREC_C128, X, ns, 0)))
                return rc;
            if ((rc = up(dTheta, theta.data(), (size_t)k * 8))) return rc;
            if ((rc = launch_residuals(ctx, CHEBFD_PREC_C128, W, X, n, k, ns, dTheta, dRes))) return rc;
            res.resize(k);
            if ((rc = down(res.data(), dRes, (size_t)k * 8))) return rc;
            if (bounds_checked) {
                // a Rayleigh quotient lies in the convex hull of the
                // spectrum: one outside [a, b] (or an overflow of the filter)
                // proves the estimated interval too narrow
                const double tol = 1e-10 * std::max(std::fabs(a), std::fabs(b));
                for (int j = 0; j < k; ++j)
                    if (!std::isfinite(theta[j]) || !std::isfinite(res[j]) || theta[j] < a - tol ||
                        theta[j] > b + tol)
                        return RESTART_WIDER;
            }
            for (int j = 0; j < k; ++j)
                if (!std::isfinite(theta[j]) || !std::isfinite(res[j]))
                    return fail(CHEBFD_ERR_NONFINITE, "non-finite Ritz pair");
            auto td = clk::now();
            st.t_rr += secs(tc, td);
            // V now in W; new block = V
            std::swap(X, W);
            // ---------------- step 8: classify
            int nconv = 0, nconving = 0;
            double rmin = INFINITY, worst = 0.0;
            keep_idx.clear();
            conv_idx.clear();
            for (int j = 0; j < k; ++j) {
                const bool in = theta[j] >= p.lam_lo && theta[j] <= p.lam_hi;
                if (in && res[j] <= p.eps) {
                    ++nconv;
                    conv_idx.push_back(j);
                    continue;
                }
                keep_idx.push_back(j);
                if (!in) continue;
                if (res[j] <= seps) ++nconving;
                rmin = std::min(rmin, res[j]);
                if (res[j] <= seps) worst = std::max(worst, res[j]);
            }
            {
                // convergence history: residuals of the in-window Ritz pairs
                // of this iteration (and of the pairs locked before it)
                chebfd_iter_info h{};
                h.n_mvm = st.n_mvm;
                h.precision = corr ? CHEBFD_PREC_C64_CORRECTION : prec;
                h.n_locked = n_lock;
                h.n_converged = nconv;
                h.n_accepted = nconv + nconving;
                h.r_min = INFINITY;
                h.r_max_accepted = 0.0;
                for (int j = 0; j < k; ++j)
                    if (theta[j] >= p.lam_lo && theta[j] <= p.lam_hi) {
                        ++h.n_window;
                        h.r_min = std::min(h.r_min, res[j]);
                        if (res[j] <= seps) h.r_max_accepted = std::max(h.r_max_accepted, res[j]);
                    }
                for (double r : lock_res) {
                    h.r_min = std::min(h.r_min, r);
                    h.r_max_accepted = std::max(h.r_max_accepted, r);
                }
                if (h.n_accepted + n_lock == 0) h.r_max_accepted = NAN;
                if (!std::isfinite(h.r_min)) h.r_min = NAN;
                out->history.push_back(h);
            }
            if (p.verbose) {
                std::fprintf(stderr,
                             "chebfd: iteration %d (%s) active %d locked %d converged %d "
                             "converging %d min in-window residual %.3e filter %.2f s\n",
                             it, corr ? "c64 correction" : prec == CHEBFD_PREC_C64 ? "c64" : "c128",
                             k, n_lock, nconv,
                             nconving, rmin, secs(ta, tb));
                std::fflush(stderr);
            }
            if (prec == CHEBFD_PREC_C64) {
                // FP32 phase: switch to FP64 once the in-window residuals sit
                // below polish_switch or stop improving
                double mx = 0.0;
                std::vector<double> good_r;
                for (int j = 0; j < k; ++j)
                    if (theta[j] >= p.lam_lo && theta[j] <= p.lam_hi && res[j] <= seps) {
                        mx = std::max(mx, res[j]);
                        good_r.push_back(res[j]);
                    }
                double med = INFINITY;
                if (!good_r.empty()) {
                    std::nth_element(good_r.begin(), good_r.begin() + good_r.size() / 2, good_r.end());
                    med = good_r[good_r.size() / 2];
                }
                const int ngood = nconv + nconving;
                // default threshold: a few FP32 roundings of the spectral scale.
                // The sweep is done once every good residual is below it, or
                // once their median is below half of it: the typical pair
                // then sits at the FP32 rounding floor, where its residual is
                // rounding noise that one FP64 pass filters out, and the few
                // pairs above it converge in the same polish passes
                {
                    // record the sweep's result (ascending); the last
                    // iteration of the FP32 phase leaves it in the result
                    std::vector<std::pair<double, double>> sp;
                    for (int j = 0; j < k; ++j)
                        if (theta[j] >= p.lam_lo && theta[j] <= p.lam_hi && res[j] <= seps)
                            sp.push_back({theta[j], res[j]});
                    std::sort(sp.begin(), sp.end());
                    out->sweep_evals.clear();
                    out->sweep_res.clear();
                    for (const auto &q : sp) {
                        out->sweep_evals.push_back(q.first);
                        out->sweep_res.push_back(q.second);
                    }
                }
                const double sw = std::max(std::fabs(a), std::fabs(b));
                const double thr = std::isnan(p.polish_switch) ? 8.0 * 0x1p-23 * sw : p.polish_switch;
                const bool below = ngood > 0 && (mx <= thr || med <= 0.5 * thr);
                // stalled: the set of good pairs grew by at most 10% and their
                // median residual no longer halves (the FP32 floor; a few
                // slow pairs are left to the FP64 polish)
                const bool stalled = it >= 2 && ngood > 0 &&
                                     ngood <= prev_good + std::max(1, prev_good / 10) &&
                                     med > 0.5 * prev_worst;
                if (p.verbose) {
                    std::fprintf(stderr,
                                 "chebfd: FP32 phase: %d in-window pairs below sqrt(eps), median "
                                 "residual %.3e, largest %.3e, switch threshold %.3e%s\n",
                                 ngood, med, mx, thr,
                                 below ? " (below)" : stalled ? " (stalled)" : "");
                    std::fflush(stderr);
                }
                prev_worst = ngood > 0 ? med : INFINITY;
                prev_good = ngood;
                if (below || stalled) {
                    prec = CHEBFD_PREC_C128;   // X (c128 Ritz vectors) continues in FP64
                    void *others[2];
                    int q = 0;
                    for (void *bb : {B[0], B[1], B[2]})
                        if (bb != X && q < 2) others[q++] = bb;
                    U = others[0];
                    W = others[1];
                    // the FP64 polish filters the in-window Ritz vectors and
                    // their nearest neighbours outside the window only:
                    // max(n_in + 8, 5 n_in / 4) columns (the rest of the
                    // search space has done its work in the FP32 sweep)
                    std::vector<int> in_w, out_w;
                    for (int j = 0; j < k; ++j)
                        (theta[j] >= p.lam_lo && theta[j] <= p.lam_hi ? in_w : out_w).push_back(j);
                    const int n_in = (int)in_w.size();
                    const int m = std::min(k, std::max(n_in + 8, (5 * n_in + 3) / 4));
                    if (n_in > 0 && m < k) {
                        auto dist = [&](int j) {
                            return theta[j] < p.lam_lo ? p.lam_lo - theta[j] : theta[j] - p.lam_hi;
                        };
                        std::stable_sort(out_w.begin(), out_w.end(),
                                         [&](int x, int y) { return dist(x) < dist(y); });
                        std::vector<int32_t> sel(in_w.begin(), in_w.end());
                        sel.insert(sel.end(), out_w.begin(), out_w.begin() + (m - n_in));
                        std::sort(sel.begin(), sel.end());
                        if ((rc = up(dIdx, sel.data(), sel.size() * 4))) return rc;
                        if ((rc = launch_gather_cols(ctx, CHEBFD_PREC_C128, X, ns, U, ns, 0, dIdx,
                                                     n, (int64_t)m)))
                            return rc;
                        if ((rc = sync())) return rc;
                        std::swap(X, U);
                        ns_act = m;
                        th_act.clear();
                        for (int j : sel) th_act.push_back(theta[j]);
                    } else {
                        th_act.assign(theta.begin(), theta.begin() + k);
                    }
                    // the coefficient table ((n_p + 1) x n_s doubles at most)
                    // borrows a complex128 block during the correction pass
                    corr = p.polish == CHEBFD_POLISH_CORRECTION &&
                           (size_t)(p.n_p + 1) * ns * 8 <= L.blk64;
                    // the count to confirm is the number of in-window pairs
                    // the FP32 sweep brought below sqrt(eps)
                    prev_conv = ngood;
                    prev_rmin = rmin;
                } else {
                    // X32 <- Ritz vectors
                    if ((rc = launch_convert(ctx, CHEBFD_PREC_C128, X, CHEBFD_PREC_C64, X32, n, k, ns, ns)))
                        return rc;
                    if (k & 1) {
                        // keep the padding column of an odd block defined
                        if ((rc = launch_random(ctx, CHEBFD_PREC_C64, X32, n, ns, ns, k, 1, p.seed, 3, 0)))
                            return rc;
                    }
                }
                continue;
            }
            if (p.lock && !conv_idx.empty() && harm) {
                // harmonic Ritz vectors need not be orthogonal (inside a
                // cluster or degenerate pair): lock an orthonormal basis of
                // the converged ones, with the Ritz pairs of H inside it
                if ((rc = lock_harmonic(X, U, W, Q, n_lock, conv_idx, lock_vals, lock_res)))
                    return rc;
                n_lock += (int)conv_idx.size();
                if (!keep_idx.empty()) {
                    std::vector<int32_t> kid(keep_idx.begin(), keep_idx.end());
                    if ((rc = up(dIdx, kid.data(), kid.size() * 4))) return rc;
                    if ((rc = launch_gather_cols(ctx, CHEBFD_PREC_C128, X, ns, U, ns, 0, dIdx, n,
                                                 (int64_t)kid.size())))
                        return rc;
                    if ((rc = sync())) return rc;
                    std::swap(X, U);
                }
            } else if (p.lock && !conv_idx.empty()) {
                // Q[:, n_lock + j] = V[:, conv_j]; compact the rest into U
                std::vector<int32_t> idx(conv_idx.begin(), conv_idx.end());
                if ((rc = up(dIdx, idx.data(), idx.size() * 4))) return rc;
                if ((rc = launch_gather_cols(ctx, CHEBFD_PREC_C128, X, ns, Q, ns, n_lock, dIdx, n,
                                             (int64_t)idx.size())))
                    return rc;
                if ((rc = sync())) return rc;
                for (int j : conv_idx) {
                    lock_vals.push_back(theta[j]);
                    lock_res.push_back(res[j]);
                }
                n_lock += (int)conv_idx.size();
                if (!keep_idx.empty()) {
                    std::vector<int32_t> kid(keep_idx.begin(), keep_idx.end());
                    if ((rc = up(dIdx, kid.data(), kid.size() * 4))) return rc;
                    if ((rc = launch_gather_cols(ctx, CHEBFD_PREC_C128, X, ns, U, ns, 0, dIdx, n,
                                                 (int64_t)kid.size())))
                        return rc;
                    if ((rc = sync())) return rc;
                    std::swap(X, U);
                }
            }
            if (corr) {
                // Ritz values of the columns that stay active (in X's order)
                th_act.clear();
                if (p.lock && !conv_idx.empty())
                    for (int j : keep_idx) th_act.push_back(theta[j]);
                else
                    th_act.assign(theta.begin(), theta.begin() + k);
                // a pass that neither converges a pair nor halves the largest
                // accepted residual has met the correction's FP32 floor:
                // FP64 passes from now on
                const int cc = p.lock ? n_lock : nconv;
                if (nconving > 0 && worst >= 0.5 * corr_worst && cc <= corr_conv) corr = false;
                corr_worst = nconving > 0 ? worst : INFINITY;
                corr_conv = cc;
            }
            const int total_conv = p.lock ? n_lock : nconv;
            const bool stagnant =
                (rmin == INFINITY) || (rmin >= (total_conv > 0 ? 0.5 : 0.9) * prev_rmin);
            if (it >= 2 && nconving == 0 && total_conv == prev_conv && stagnant) {
                status = CHEBFD_OK;
                break;
            }
            prev_conv = total_conv;
            prev_rmin = rmin;
            if (p.lock && n_lock >= ns_act) {
                status = CHEBFD_WARN_SEARCH_SPACE_TOO_SMALL;
                break;
            }
        }
        st.iterations = std::min(it, p.max_iter);
        // ---------------- collect converged in-window pairs
        std::vector<std::pair<double, int>> order;   // (lambda, source)
        std::vector<double> vals, rs;
        std::vector<int> src_col;
        std::vector<char> from_q;
        if (p.lock) {
            for (int j = 0; j < n_lock; ++j) {
                vals.push_back(lock_vals[j]);
                rs.push_back(lock_res[j]);
                src_col.push_back(j);
                from_q.push_back(1);
            }
        }
        if (!p.lock || status != CHEBFD_OK) {
            // unlocked converged pairs of the last Rayleigh-Ritz (block X)
            for (size_t q = 0; q < (p.lock ? keep_idx.size() : (size_t)last_active); ++q) {
                const int j = p.lock ? keep_idx[q] : (int)q;
                if (j >= (int)theta.size()) break;
                if (theta[j] >= p.lam_lo && theta[j] <= p.lam_hi && res[j] <= p.eps &&
                    prec == CHEBFD_PREC_C128) {
                    vals.push_back(theta[j]);
                    rs.push_back(res[j]);
                    src_col.push_back(p.lock ? (int)q : j);
                    from_q.push_back(0);
                }
            }
        }
        std::vector<int> ord(vals.size());
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return vals[x] < vals[y]; });
        const int nf = (int)ord.size();
        out->evals.resize(nf);
        out->res.resize(nf);
        double maxr = 0.0;
        for (int i = 0; i < nf; ++i) {
            out->evals[i] = vals[ord[i]];
            out->res[i] = rs[ord[i]];
            maxr = std::max(maxr, out->res[i]);
        }
        if (p.vectors && nf > 0) {
            // gather the selected columns, in ascending order, into a
            // contiguous n x nf block in a free buffer and download it
            void *dst = nullptr;
            for (void *bb : {B[0], B[1], B[2]})
                if (bb != X) {
                    dst = bb;
                    break;
                }
            for (int i = 0; i < nf; ++i) {
                const int o = ord[i];
                int32_t one = src_col[o];
                if ((rc = up(dIdx, &one, 4))) return rc;
                if ((rc = launch_gather_cols(ctx, CHEBFD_PREC_C128, from_q[o] ? Q : X, ns, dst, nf,
                                             i, dIdx, n, 1)))
                    return rc;
                if ((rc = sync())) return rc;
            }
            out->evecs.resize((size_t)n * nf * 2);
            if ((rc = down(out->evecs.data(), dst, out->evecs.size() * 8))) return rc;
        }
        st.n_found = nf;
        st.n_locked = n_lock;
        st.n_p_used = p.n_p;
        st.a = a;
        st.b = b;
        st.max_residual = maxr;
        st.t_total = secs(t0, clk::now());
        out->stats = st;
        return status;
    }
};

}  // namespace
}  // namespace chebfd

using namespace chebfd;

extern "C" int chebfd_params_default(chebfd_params *p)
{
    if (!p) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_params_default: NULL");
    std::memset(p, 0, sizeof(*p));
    p->n_s = 32;
    p->n_p = 200;
    p->kernel = CHEBFD_KERNEL_LANCZOS;
    p->mu = 2.0;
    p->eps = 1e-9;
    p->max_iter = 50;
    p->precision = CHEBFD_PREC_C128;
    p->lock = 1;
    p->a = NAN;
    p->b = NAN;
    p->seed = 1;
    p->gamma_corr = nullptr;
    p->polish_switch = NAN;
    p->vectors = 1;
    p->verbose = 0;
    return CHEBFD_OK;
}

static int check_params(const chebfd_matrix *H, const chebfd_params *p)
{
    if (!H || !p) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_solve: NULL argument");
    if (!(p->lam_lo < p->lam_hi) || !std::isfinite(p->lam_lo) || !std::isfinite(p->lam_hi))
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_solve: need finite lam_lo < lam_hi");
    if (p->n_s < 1 || p->n_s > 1024 || p->n_s > H->n)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_solve: need 1 <= n_s <= min(1024, N)");
    if (p->n_p < 2) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_solve: n_p must be >= 2");
    if (p->kernel < 0 || p->kernel > 3) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_solve: unknown kernel");
    if (!(p->eps > 0.0)) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_solve: eps must be > 0");
    if (p->max_iter < 1) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_solve: max_iter must be >= 1");
    if (p->precision != CHEBFD_PREC_C128 && p->precision != CHEBFD_PREC_C64)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_solve: unknown precision");
    if (p->precision == CHEBFD_PREC_C64 && (p->n_s & 1))
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_solve: the c64 form needs an even n_s");
    if (p->bounds < 0 || p->bounds == 1 || p->bounds > 1000)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_solve: bounds must be 0 (Gershgorin) or 2..1000 Lanczos steps");
    if (p->adapt != 0 && p->adapt != 1)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_solve: adapt must be 0 or 1");
    if (p->harmonic != 0 && (p->harmonic != 1 || !p->lock))
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_solve: harmonic must be 0, or 1 with lock = 1");
    if (p->polish != CHEBFD_POLISH_CORRECTION && p->polish != CHEBFD_POLISH_FP64)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_solve: polish must be CORRECTION or FP64");
    return CHEBFD_OK;
}

extern "C" int chebfd_solve_workspace_size(const chebfd_matrix *H, const chebfd_params *p,
                                           int64_t *bytes)
{
    int rc = check_params(H, p);
    if (rc) return rc;
    if (!bytes) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_solve_workspace_size: NULL bytes");
    *bytes = (int64_t)layout(H->n, *p).total;
    return CHEBFD_OK;
}

extern "C" int chebfd_solve(chebfd_ctx *ctx, const chebfd_matrix *H, const chebfd_params *p,
                            void *workspace, int64_t workspace_bytes, chebfd_result **out)
{
    if (!ctx || !out) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_solve: NULL argument");
    *out = nullptr;
    int rc = check_params(H, p);
    if (rc) return rc;
    Solver S;
    S.ctx = ctx;
    S.H = H;
    S.p = *p;
    S.n = H->n;
    S.ns = p->n_s;
    S.L = layout(H->n, *p);
    if (!workspace || workspace_bytes < (int64_t)S.L.total || ((uintptr_t)workspace & 255))
        return fail(CHEBFD_ERR_WORKSPACE, "chebfd_solve: workspace missing, too small or not 256-byte aligned");
    S.ws = (char *)workspace;
    CHEBFD_HIP(hipSetDevice(ctx->device));
    S.a = std::isnan(p->a) ? H->g_lo : p->a;
    S.b = std::isnan(p->b) ? H->g_hi : p->b;
    if (std::isnan(p->a) && std::isnan(p->b) && p->bounds > 0 && p->n_s >= 3) {
        // Lanczos bounds, computed in the (still unused) workspace: the
        // first block as the three Lanczos vectors, the small area as scratch
        char *base = (char *)workspace;
        double lo, hi;
        if ((rc = lanczos_bounds(ctx, H, p->bounds, p->seed, 0.01, base + S.L.off_b[0],
                                 (double *)(base + S.L.off_small),
                                 (double *)(base + S.L.off_small + 256), &lo, &hi)))
            return rc;
        if (lo < hi && p->lam_lo > lo && p->lam_hi < hi) {
            S.a = lo;
            S.b = hi;
            S.bounds_checked = true;
        }
    }
    if (!(S.a < S.b)) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_solve: empty spectral interval");
    if (p->lam_hi <= S.a || p->lam_lo >= S.b)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_solve: window outside the spectral interval");
    auto coeffs = [&]() -> int {
        S.gamma.assign(p->n_p + 1, 0.0);
        int r = chebfd_coeffs(p->lam_lo, p->lam_hi, S.a, S.b, p->n_p, p->kernel, p->mu,
                              S.gamma.data());
        if (r) return r;
        if (p->gamma_corr)
            for (int k = 0; k <= p->n_p; ++k) {
                if (!std::isfinite(p->gamma_corr[k]))
                    return fail(CHEBFD_ERR_NONFINITE, "chebfd_solve: non-finite coefficient correction");
                S.gamma[k] *= 1.0 + p->gamma_corr[k];
            }
        return CHEBFD_OK;
    };
    if ((rc = coeffs())) return rc;
    auto *res = new chebfd_result();
    rc = S.run(res);
    if (rc == Solver::RESTART_WIDER) {
        // the estimated interval was too narrow: start again on Gershgorin's
        const chebfd_stats first = S.st;
        S.p = *p;   // the adaptive degree of the first run does not carry over
        S.a = H->g_lo;
        S.b = H->g_hi;
        S.bounds_checked = false;
        S.st = chebfd_stats{};
        S.refill_ctr = 0;
        if ((rc = coeffs())) {
            delete res;
            return rc;
        }
        *res = chebfd_result();
        rc = S.run(res);
        res->stats.iterations += first.iterations;
        res->stats.n_mvm += first.n_mvm;
    }
    if (rc < 0) {
        delete res;
        return rc;
    }
    *out = res;
    return rc;
}

extern "C" int chebfd_result_get(const chebfd_result *r, int64_t *n_found, const double **evals,
                                 const double **residuals, const double **evecs,
                                 chebfd_stats *stats)
{
    if (!r) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_result_get: NULL result");
    if (n_found) *n_found = (int64_t)r->evals.size();
    if (evals) *evals = r->evals.data();
    if (residuals) *residuals = r->res.data();
    if (evecs) *evecs = r->evecs.empty() ? nullptr : r->evecs.data();
    if (stats) *stats = r->stats;
    return CHEBFD_OK;
}

extern "C" int chebfd_result_sweep(const chebfd_result *r, int64_t *n, const double **evals,
                                   const double **residuals)
{
    if (!r) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_result_sweep: NULL result");
    if (n) *n = (int64_t)r->sweep_evals.size();
    if (evals) *evals = r->sweep_evals.data();
    if (residuals) *residuals = r->sweep_res.data();
    return CHEBFD_OK;
}

extern "C" int chebfd_result_history(const chebfd_result *r, int64_t *n,
                                     const chebfd_iter_info **history)
{
    if (!r) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_result_history: NULL result");
    if (n) *n = (int64_t)r->history.size();
    if (history) *history = r->history.data();
    return CHEBFD_OK;
}

extern "C" int chebfd_result_destroy(chebfd_result *r)
{
    delete r;
    return CHEBFD_OK;
}
