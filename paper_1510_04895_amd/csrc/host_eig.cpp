// Small dense Hermitian eigenproblem on the host (the N_S x N_S matrices of
// orthogonalisation and Rayleigh-Ritz, Sec. 3.1 steps 6-7).
//
// Method: Householder reduction A = Q T Q^H to Hermitian tridiagonal form,
// a diagonal unitary D making the subdiagonal real (T = D Tr D^H), the
// implicit QL iteration with Wilkinson shifts on the real tridiagonal Tr
// (Bowdler, Martin, Reinsch and Wilkinson, Numer. Math. 11, 1968), and the
// eigenvectors Q D Z.  O(n^3), about 10 n^3 flops.
#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>
#include <vector>

#include "internal.h"

namespace chebfd {

using cd = std::complex<double>;

namespace {

// Householder tridiagonalisation in place; Q accumulates the reflectors.
void tridiagonalise(int n, std::vector<cd> &A, std::vector<cd> &Q)
{
    Q.assign((size_t)n * n, cd(0.0));
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
    std::vector<cd> v(n), p(n), q(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        double xn = 0.0;
        for (int i = 0; i < m; ++i) xn += std::norm(A[(size_t)(k + 1 + i) * n + k]);
        xn = std::sqrt(xn);
        if (xn == 0.0) continue;
        const cd x0 = A[(size_t)(k + 1) * n + k];
        const cd ph = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : cd(1.0);
        const cd alpha = -ph * xn;            // H x = alpha e_1
        for (int i = 0; i < m; ++i) v[i] = A[(size_t)(k + 1 + i) * n + k];
        v[0] -= alpha;
        double vn2 = 0.0;
        for (int i = 0; i < m; ++i) vn2 += std::norm(v[i]);
        if (vn2 == 0.0) continue;
        const double tau = 2.0 / vn2;         // H = I - tau v v^H
        // p = tau A22 v ; K = tau/2 v^H p ; q = p - K v ; A22 -= v q^H + q v^H
        for (int i = 0; i < m; ++i) {
            cd s = 0.0;
            const cd *row = &A[(size_t)(k + 1 + i) * n + k + 1];
            for (int j = 0; j < m; ++j) s += row[j] * v[j];
            p[i] = tau * s;
        }
        cd K = 0.0;
        for (int i = 0; i < m; ++i) K += std::conj(v[i]) * p[i];
        K *= 0.5 * tau;
        for (int i = 0; i < m; ++i) q[i] = p[i] - K.real() * v[i];
        for (int i = 0; i < m; ++i) {
            cd *row = &A[(size_t)(k + 1 + i) * n + k + 1];
            for (int j = 0; j < m; ++j) row[j] -= v[i] * std::conj(q[j]) + q[i] * std::conj(v[j]);
        }
        A[(size_t)(k + 1) * n + k] = alpha;
        A[(size_t)k * n + k + 1] = std::conj(alpha);
        for (int i = 1; i < m; ++i) {
            A[(size_t)(k + 1 + i) * n + k] = 0.0;
            A[(size_t)k * n + k + 1 + i] = 0.0;
        }
        // Q <- Q H
        for (int r = 0; r < n; ++r) {
            cd *row = &Q[(size_t)r * n + k + 1];
            cd s = 0.0;
            for (int j = 0; j < m; ++j) s += row[j] * v[j];
            s *= tau;
            for (int j = 0; j < m; ++j) row[j] -= s * std::conj(v[j]);
        }
    }
}

// Implicit QL on the real symmetric tridiagonal (d, e), e[i] coupling i and
// i+1.  The rotations are accumulated into Zt, the transpose of the
// eigenvector matrix (row i of Zt = eigenvector column i), so each rotation
// updates two contiguous rows.
int tridiagonal_ql(int n, std::vector<double> &d, std::vector<double> &e, std::vector<double> &Zt)
{
    const double eps = 2.220446049250313e-16;
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
                double *zi = &Zt[(size_t)i * n], *zj = &Zt[(size_t)(i + 1) * n];
                for (int k = 0; k < n; ++k) {
                    const double zf = zj[k];
                    zj[k] = s * zi[k] + c * zf;
                    zi[k] = c * zi[k] - s * zf;
                }
            }
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
    std::vector<cd> A((size_t)n * n), Q;
    for (size_t i = 0; i < (size_t)n * n; ++i) A[i] = cd(Ain[2 * i], Ain[2 * i + 1]);
    // enforce exact Hermitian symmetry of the input
    for (int i = 0; i < n; ++i) {
        A[(size_t)i * n + i] = A[(size_t)i * n + i].real();
        for (int j = i + 1; j < n; ++j) {
            const cd v = 0.5 * (A[(size_t)i * n + j] + std::conj(A[(size_t)j * n + i]));
            A[(size_t)i * n + j] = v;
            A[(size_t)j * n + i] = std::conj(v);
        }
    }
    tridiagonalise(n, A, Q);
    std::vector<double> d(n), e(n, 0.0);
    std::vector<cd> delta(n, cd(1.0));
    for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i].real();
    for (int i = 0; i + 1 < n; ++i) {
        const cd sub = A[(size_t)(i + 1) * n + i];
        const double a = std::abs(sub);
        e[i] = a;
        delta[i + 1] = a > 0.0 ? delta[i] * (sub / a) : delta[i];
    }
    std::vector<double> Zt((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Zt[(size_t)i * n + i] = 1.0;
    if (tridiagonal_ql(n, d, e, Zt) != 0) return -1;
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return d[x] < d[y]; });
    // V = Q D Z, columns in ascending eigenvalue order:
    // V[r][j] = sum_i (Q D)[r][i] Zt[ord j][i]
    std::vector<cd> QD((size_t)n * n);
    for (int r = 0; r < n; ++r)
        for (int i = 0; i < n; ++i) QD[(size_t)r * n + i] = Q[(size_t)r * n + i] * delta[i];
    for (int j = 0; j < n; ++j) w[j] = d[ord[j]];
    for (int r = 0; r < n; ++r) {
        const cd *qr = &QD[(size_t)r * n];
        for (int j = 0; j < n; ++j) {
            const double *z = &Zt[(size_t)ord[j] * n];
            double sr = 0.0, si = 0.0;
            for (int i = 0; i < n; ++i) {
                sr += qr[i].real() * z[i];
                si += qr[i].imag() * z[i];
            }
            Ain[2 * ((size_t)r * n + j)] = sr;
            Ain[2 * ((size_t)r * n + j) + 1] = si;
        }
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
