// Small dense Hermitian eigenproblem on the host (the N_S x N_S matrices of
// orthogonalisation and Rayleigh-Ritz, Sec. 3.1 steps 6-7).
//
// Method: Householder reduction A = Q T Q^H to Hermitian tridiagonal form,
// a diagonal unitary D making the subdiagonal real (T = D Tr D^H), the
// implicit QL iteration with Wilkinson shifts on the real tridiagonal Tr
// (Bowdler, Martin, Reinsch and Wilkinson, Numer. Math. 11, 1968), and the
// eigenvectors Q D Z, with Q applied as its stored reflectors.  O(n^3).  The
// complex matrices are kept as separate real and imaginary planes so the
// inner loops are plain FMA streams.
#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>
#include <vector>

#include "internal.h"

namespace chebfd {

using cd = std::complex<double>;

namespace {

// Householder tridiagonalisation in place on split real/imaginary planes
// (Ar, Ai row-major n x n).  Step k maps column k below the diagonal onto
// alpha e_1 with H_k = I - tau_k v_k v_k^H; v_k (m = n - k - 1 entries) goes
// to row k of (Vr, Vi) from column k + 1 on, tau_k to tau[k] (0: no
// reflection).  A = Q T Q^H with Q = H_0 H_1 ... H_{n-3}.  Only the lower
// triangle of the trailing block is read and updated (A is Hermitian); the
// tridiagonal is left in the diagonal and the first subdiagonal.
void tridiagonalise(int n, std::vector<double> &Ar, std::vector<double> &Ai,
                    std::vector<double> &Vr, std::vector<double> &Vi, std::vector<double> &tau)
{
    Vr.assign((size_t)n * n, 0.0);
    Vi.assign((size_t)n * n, 0.0);
    tau.assign(n, 0.0);
    std::vector<double> pr(n), pi(n), qr(n), qi(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        double *__restrict__ vr = &Vr[(size_t)k * n + k + 1];
        double *__restrict__ vi = &Vi[(size_t)k * n + k + 1];
        double xn = 0.0;
        for (int i = 0; i < m; ++i) {
            vr[i] = Ar[(size_t)(k + 1 + i) * n + k];
            vi[i] = Ai[(size_t)(k + 1 + i) * n + k];
            xn += vr[i] * vr[i] + vi[i] * vi[i];
        }
        xn = std::sqrt(xn);
        if (xn == 0.0) continue;
        const double ax = std::hypot(vr[0], vi[0]);
        const double phr = ax > 0.0 ? vr[0] / ax : 1.0, phi = ax > 0.0 ? vi[0] / ax : 0.0;
        const double alr = -phr * xn, ali = -phi * xn;   // H x = alpha e_1
        vr[0] -= alr;
        vi[0] -= ali;
        double vn2 = 0.0;
        for (int i = 0; i < m; ++i) vn2 += vr[i] * vr[i] + vi[i] * vi[i];
        if (vn2 == 0.0) continue;
        const double t = 2.0 / vn2;
        tau[k] = t;
        // p = tau A22 v ; K = tau/2 v^H p (real) ; q = p - K v ;
        // A22 -= v q^H + q v^H
        // p = A22 v from the lower triangle: row i gives A_ij v_j (j < i) to
        // p_i and conj(A_ij) v_i to p_j; the diagonal is real
        std::fill(pr.begin(), pr.begin() + m, 0.0);
        std::fill(pi.begin(), pi.begin() + m, 0.0);
        double *__restrict__ p_r = pr.data();
        double *__restrict__ p_i = pi.data();
        for (int i = 0; i < m; ++i) {
            const double *__restrict__ rr = &Ar[(size_t)(k + 1 + i) * n + k + 1];
            const double *__restrict__ ri = &Ai[(size_t)(k + 1 + i) * n + k + 1];
            const double a = vr[i], b = vi[i];
            double sr = 0.0, si = 0.0;
            for (int j = 0; j < i; ++j) {
                sr += rr[j] * vr[j] - ri[j] * vi[j];
                si += rr[j] * vi[j] + ri[j] * vr[j];
                p_r[j] += rr[j] * a + ri[j] * b;
                p_i[j] += rr[j] * b - ri[j] * a;
            }
            p_r[i] += sr + rr[i] * a;
            p_i[i] += si + rr[i] * b;
        }
        for (int i = 0; i < m; ++i) {
            pr[i] *= t;
            pi[i] *= t;
        }
        double K = 0.0;
        for (int i = 0; i < m; ++i) K += vr[i] * pr[i] + vi[i] * pi[i];
        K *= 0.5 * t;
        for (int i = 0; i < m; ++i) {
            qr[i] = pr[i] - K * vr[i];
            qi[i] = pi[i] - K * vi[i];
        }
        for (int i = 0; i < m; ++i) {
            double *__restrict__ rr = &Ar[(size_t)(k + 1 + i) * n + k + 1];
            double *__restrict__ ri = &Ai[(size_t)(k + 1 + i) * n + k + 1];
            const double a = vr[i], b = vi[i], c = qr[i], d = qi[i];
            for (int j = 0; j <= i; ++j) {
                // v_i conj(q_j) + q_i conj(v_j)
                rr[j] -= a * qr[j] + b * qi[j] + c * vr[j] + d * vi[j];
                ri[j] -= b * qr[j] - a * qi[j] + d * vr[j] - c * vi[j];
            }
        }
        Ar[(size_t)(k + 1) * n + k] = alr;
        Ai[(size_t)(k + 1) * n + k] = ali;
        Ar[(size_t)k * n + k + 1] = alr;
        Ai[(size_t)k * n + k + 1] = -ali;
        for (int i = 1; i < m; ++i) {
            Ar[(size_t)(k + 1 + i) * n + k] = Ai[(size_t)(k + 1 + i) * n + k] = 0.0;
            Ar[(size_t)k * n + k + 1 + i] = Ai[(size_t)k * n + k + 1 + i] = 0.0;
        }
    }
}

// Implicit QL on the real symmetric tridiagonal (d, e), e[i] coupling i and
// i+1.  The rotations are accumulated into Zt, the transpose of the
// eigenvector matrix (row i of Zt = eigenvector column i).  One sweep's
// rotations act on rows (i, i+1) for i = m-1 down to lo in turn; they are
// recorded and then applied chunk of columns by chunk, the row carried from
// one rotation to the next kept in registers.
// Applies the rotations i = m-1 .. lo of one sweep to rows lo .. m of Zt:
// rows (i, i+1) <- (c z_i - s z_{i+1}, s z_i + c z_{i+1}).  Row i+1 is final
// after rotation i; the new row i is carried into rotation i-1.
void apply_sweep(int n, int lo, int m, const double *rc, const double *rs, double *Zt)
{
    if (lo >= m) return;
    constexpr int CB = 16;
    for (int k0 = 0; k0 < n; k0 += CB) {
        const int w = std::min(CB, n - k0);
        double carry[CB];
        const double *zm = Zt + (size_t)m * n + k0;
        for (int k = 0; k < w; ++k) carry[k] = zm[k];
        for (int i = m - 1; i >= lo; --i) {
            const double s = rs[i], c = rc[i];
            const double *zi = Zt + (size_t)i * n + k0;
            double *zo = Zt + (size_t)(i + 1) * n + k0;
            if (w == CB) {
#pragma unroll
                for (int k = 0; k < CB; ++k) {
                    const double a = zi[k], cj = carry[k];
                    zo[k] = s * a + c * cj;
                    carry[k] = c * a - s * cj;
                }
            } else {
                for (int k = 0; k < w; ++k) {
                    const double a = zi[k], cj = carry[k];
                    zo[k] = s * a + c * cj;
                    carry[k] = c * a - s * cj;
                }
            }
        }
        double *zl = Zt + (size_t)lo * n + k0;
        for (int k = 0; k < w; ++k) zl[k] = carry[k];
    }
}

int tridiagonal_ql(int n, std::vector<double> &d, std::vector<double> &e, std::vector<double> &Zt)
{
    const double eps = 2.220446049250313e-16;
    std::vector<double> rc(n), rs(n);
    e.resize(n);
    e[n - 1] = 0.0;
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        for (;;) {
            int m = l;
            for (; m < n - 1; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= eps * dd) break;
            }
            if (m == l) break;
            if (++iter > 80) return -1;
            // Wilkinson-type shift from the leading 2x2 block
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            bool split = false;
            int lo = m;   // rows lo .. m were rotated in this sweep
            for (int i = m - 1; i >= l; --i) {
                const double f = s * e[i], bb = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    split = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * bb;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - bb;
                rs[i] = s;
                rc[i] = c;
                lo = i;
            }
            apply_sweep(n, lo, m, rc.data(), rs.data(), Zt.data());
            if (split) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    return 0;
}

}  // namespace

int herm_eig(int n, std::vector<double> &Ain, std::vector<double> &w)
{
    w.assign(n, 0.0);
    if (n == 0) return 0;
    const size_t nn = (size_t)n * n;
    std::vector<double> Ar(nn), Ai(nn), Vr, Vi, tau;
    // split planes with exact Hermitian symmetry of the input
    for (int i = 0; i < n; ++i) {
        Ar[(size_t)i * n + i] = Ain[2 * ((size_t)i * n + i)];
        Ai[(size_t)i * n + i] = 0.0;
        for (int j = i + 1; j < n; ++j) {
            const size_t ij = (size_t)i * n + j, ji = (size_t)j * n + i;
            const double re = 0.5 * (Ain[2 * ij] + Ain[2 * ji]);
            const double im = 0.5 * (Ain[2 * ij + 1] - Ain[2 * ji + 1]);
            Ar[ij] = re;
            Ai[ij] = im;
            Ar[ji] = re;
            Ai[ji] = -im;
        }
    }
    tridiagonalise(n, Ar, Ai, Vr, Vi, tau);
    std::vector<double> d(n), e(n, 0.0), dr(n, 1.0), di(n, 0.0);
    for (int i = 0; i < n; ++i) d[i] = Ar[(size_t)i * n + i];
    for (int i = 0; i + 1 < n; ++i) {
        const double sr = Ar[(size_t)(i + 1) * n + i], si = Ai[(size_t)(i + 1) * n + i];
        const double a = std::hypot(sr, si);
        e[i] = a;
        // delta_{i+1} = delta_i * sub / |sub|
        if (a > 0.0) {
            dr[i + 1] = (dr[i] * sr - di[i] * si) / a;
            di[i + 1] = (dr[i] * si + di[i] * sr) / a;
        } else {
            dr[i + 1] = dr[i];
            di[i + 1] = di[i];
        }
    }
    std::vector<double> Zt(nn, 0.0);
    for (int i = 0; i < n; ++i) Zt[(size_t)i * n + i] = 1.0;
    if (tridiagonal_ql(n, d, e, Zt) != 0) return -1;
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return d[x] < d[y]; });
    for (int j = 0; j < n; ++j) w[j] = d[ord[j]];
    // W = D Z with the columns in ascending eigenvalue order (Ar, Ai reused)
    std::vector<double> &Wr = Ar, &Wi = Ai;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const double z = Zt[(size_t)ord[j] * n + i];
            Wr[(size_t)i * n + j] = dr[i] * z;
            Wi[(size_t)i * n + j] = di[i] * z;
        }
    // V = H_0 H_1 ... H_{n-3} W, the reflectors applied last first to rows
    // k+1 .. n-1: W <- W - tau v (v^H W)
    std::vector<double> sr(n), si(n);
    for (int k = n - 3; k >= 0; --k) {
        const double t = tau[k];
        if (t == 0.0) continue;
        const int m = n - k - 1;
        const double *vr = &Vr[(size_t)k * n + k + 1], *vi = &Vi[(size_t)k * n + k + 1];
        std::fill(sr.begin(), sr.end(), 0.0);
        std::fill(si.begin(), si.end(), 0.0);
        double *__restrict__ s_r = sr.data();
        double *__restrict__ s_i = si.data();
        for (int i = 0; i < m; ++i) {
            const double *__restrict__ wr = &Wr[(size_t)(k + 1 + i) * n];
            const double *__restrict__ wi = &Wi[(size_t)(k + 1 + i) * n];
            const double a = vr[i], b = vi[i];
            for (int j = 0; j < n; ++j) {
                s_r[j] += a * wr[j] + b * wi[j];   // conj(v_i) W_ij
                s_i[j] += a * wi[j] - b * wr[j];
            }
        }
        for (int i = 0; i < m; ++i) {
            double *__restrict__ wr = &Wr[(size_t)(k + 1 + i) * n];
            double *__restrict__ wi = &Wi[(size_t)(k + 1 + i) * n];
            const double a = t * vr[i], b = t * vi[i];
            for (int j = 0; j < n; ++j) {
                wr[j] -= a * s_r[j] - b * s_i[j];
                wi[j] -= a * s_i[j] + b * s_r[j];
            }
        }
    }
    for (size_t q = 0; q < nn; ++q) {
        Ain[2 * q] = Wr[q];
        Ain[2 * q + 1] = Wi[q];
    }
    return 0;
}

// T = L^{-H} for the Cholesky factor S = L L^H of a Hermitian positive
// definite S (n x n, interleaved complex, row-major); T is upper
// triangular, so that (Y T)^H (Y T) = I for S = Y^H Y.  Returns -1 when S is
// not numerically positive definite.
int chol_inv_factor(int n, const std::vector<double> &Sin, std::vector<double> &Tout)
{
    std::vector<cd> L((size_t)n * n, cd(0.0));
    for (int j = 0; j < n; ++j) {
        double djj = Sin[2 * ((size_t)j * n + j)];
        for (int k = 0; k < j; ++k) djj -= std::norm(L[(size_t)j * n + k]);
        if (!(djj > 0.0)) return -1;
        const double ljj = std::sqrt(djj);
        L[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            cd sij(Sin[2 * ((size_t)i * n + j)], Sin[2 * ((size_t)i * n + j) + 1]);
            for (int k = 0; k < j; ++k) sij -= L[(size_t)i * n + k] * std::conj(L[(size_t)j * n + k]);
            L[(size_t)i * n + j] = sij / ljj;
        }
    }
    // M = L^{-1} (lower) by forward substitution, column by column
    std::vector<cd> M((size_t)n * n, cd(0.0));
    for (int c = 0; c < n; ++c) {
        M[(size_t)c * n + c] = 1.0 / L[(size_t)c * n + c];
        for (int i = c + 1; i < n; ++i) {
            cd s = 0.0;
            for (int k = c; k < i; ++k) s += L[(size_t)i * n + k] * M[(size_t)k * n + c];
            M[(size_t)i * n + c] = -s / L[(size_t)i * n + i];
        }
    }
    Tout.assign((size_t)2 * n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const cd t = std::conj(M[(size_t)j * n + i]);   // (L^{-1})^H
            Tout[2 * ((size_t)i * n + j)] = t.real();
            Tout[2 * ((size_t)i * n + j) + 1] = t.imag();
        }
    return 0;
}

}  // namespace chebfd

extern "C" int chebfd_host_eigh(int n, double *A, double *w)
{
    if (n < 0 || (n > 0 && (!A || !w)))
        return chebfd::fail(CHEBFD_ERR_INVALID_ARG, "chebfd_host_eigh: invalid arguments");
    std::vector<double> a(A, A + 2 * (size_t)n * n), ww;
    for (double x : a)
        if (!std::isfinite(x)) return chebfd::fail(CHEBFD_ERR_NONFINITE, "chebfd_host_eigh: non-finite input");
    if (chebfd::herm_eig(n, a, ww) != 0)
        return chebfd::fail(CHEBFD_ERR_NONFINITE, "chebfd_host_eigh: QL iteration did not converge");
    std::copy(a.begin(), a.end(), A);
    std::copy(ww.begin(), ww.end(), w);
    return CHEBFD_OK;
}
