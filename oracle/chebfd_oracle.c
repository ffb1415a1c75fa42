/*
 * Plain CPU FP64 oracle for Chebyshev filter diagonalisation (ChebFD).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  The GPU library never
 * links, includes or calls anything in this directory, and this file shares no
 * code with it.
 *
 * Everything is complex128 (C99 `double complex`), row-major blocks of
 * N rows x n_s columns with leading dimension n_s, CSR matrices with 0-based
 * int64 row pointers and int32 column indices.  Loops are written in the order
 * the paper states the operations; OpenMP "static" schedules parallelise the
 * row loops (the schedule the paper chose for its production runs, Sec. 4.2).
 * The file is compiled with -ffp-contract=off so every product and sum is
 * rounded separately.
 *
 * Paper: Pieper et al., "High-performance implementation of Chebyshev filter
 * diagonalization for interior eigenvalue computations" (arXiv:1510.04895).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers.                                             */
/* The mixing function is the 64-bit finaliser of SplitMix64 (Steele, Lea,   */
/* Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014).    */
/* A value is addressed by (seed, stream, index):                            */
/*   k = mix(seed + G*(stream+1)),  h = mix(k + G*(index+1)),                */
/*   u = (h >> 11) * 2^-53  in [0, 1),   G = 0x9E3779B97F4A7C15.             */
/* Streams: 0 on-site disorder, 1 initial block, 2 KPM phases, 3 refill.     */
/* ------------------------------------------------------------------------ */
static uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t orc_mix64_public(uint64_t z) { return orc_mix64(z); }

uint64_t orc_hash(uint64_t seed, uint64_t stream, uint64_t index)
{
    const uint64_t G = 0x9E3779B97F4A7C15ULL;
    uint64_t k = orc_mix64(seed + G * (stream + 1u));
    return orc_mix64(k + G * (index + 1u));
}

double orc_u01(uint64_t seed, uint64_t stream, uint64_t index)
{
    return (double)(orc_hash(seed, stream, index) >> 11) * 0x1.0p-53;
}

/* Random search block (Sec. 3.1, step 4): X_ik = (2u-1) + i(2u'-1). */
void orc_random_block(int64_t n, int64_t n_s, uint64_t seed, uint64_t stream,
                      uint64_t offset, cplx *X)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = 0; k < n_s; ++k) {
            uint64_t e = offset + (uint64_t)(i * n_s + k);
            double re = 2.0 * orc_u01(seed, stream, 2 * e) - 1.0;
            double im = 2.0 * orc_u01(seed, stream, 2 * e + 1) - 1.0;
            X[i * n_s + k] = re + I * im;
        }
}

/* ------------------------------------------------------------------------ */
/* Topological-insulator Hamiltonian, Sec. 5.1, Eq. (Ham).                   */
/* Sites n = x + Lx*(y + Ly*z); rows 4n + o with orbital o = 2*tau + s.      */
/* G0 = tau_z (x) s_0,  Gj = tau_x (x) s_j (j = x,y,z).                      */
/* On-site block m*G0 + V_n*1 (the paper writes m = 2).                      */
/* Hop from n to n+e_j: H[n+e_j, n] = -t (G0 - i Gj)/2, plus its adjoint     */
/* H[n, n+e_j] = -t (G0 + i Gj)/2.                                           */
/* V_n = V*(u - 1/2) with u from stream 0 at index n (box distribution of   */
/* width V, Sec. 5.1).  pbc bit j set = periodic along direction j.          */
/* ------------------------------------------------------------------------ */
static double g0_entry(int o) { return (o >> 1) == 0 ? 1.0 : -1.0; }

/* Gj[o][o'] for j = 0 (x), 1 (y), 2 (z). */
static cplx gj_entry(int j, int o, int op)
{
    int ta = o >> 1, sa = o & 1, tb = op >> 1, sb = op & 1;
    if (ta == tb) return 0.0;              /* tau_x is off-diagonal */
    if (j == 0) return (sa != sb) ? 1.0 : 0.0;                    /* s_x */
    if (j == 1) return (sa != sb) ? (sa == 0 ? -I : I) : 0.0;     /* s_y */
    return (sa == sb) ? (sa == 0 ? 1.0 : -1.0) : 0.0;             /* s_z */
}

typedef struct { int32_t c; cplx v; } orc_entry;

static int cmp_entry(const void *a, const void *b)
{
    const orc_entry *x = (const orc_entry *)a, *y = (const orc_entry *)b;
    return (x->c > y->c) - (x->c < y->c);
}

/* Upper bound on stored entries: 13 per row. */
int64_t orc_ti_max_nnz(int Lx, int Ly, int Lz) { return (int64_t)13 * 4 * Lx * Ly * Lz; }

/* Fills rowptr (n+1), col, val; duplicate columns (lattices of extent 1 or
 * 2 along a periodic direction) are summed and exact zeros dropped.
 * Returns nnz. */
int64_t orc_ti_csr(int Lx, int Ly, int Lz, int pbc, double t, double m, double V,
                   uint64_t seed, int64_t *rowptr, int32_t *col, cplx *val)
{
    const int L[3] = {Lx, Ly, Lz};
    int64_t nnz = 0;
    rowptr[0] = 0;
    for (int z = 0; z < Lz; ++z)
        for (int y = 0; y < Ly; ++y)
            for (int x = 0; x < Lx; ++x) {
                int64_t site = x + (int64_t)Lx * (y + (int64_t)Ly * z);
                double vn = V * (orc_u01(seed, 0, (uint64_t)site) - 0.5);
                int r[3] = {x, y, z};
                for (int o = 0; o < 4; ++o) {
                    orc_entry e[32];
                    int ne = 0;
                    e[ne].c = (int32_t)(4 * site + o);
                    e[ne].v = m * g0_entry(o) + vn;
                    ++ne;
                    for (int j = 0; j < 3; ++j)
                        for (int dir = -1; dir <= 1; dir += 2) {
                            int q[3] = {r[0], r[1], r[2]};
                            q[j] += dir;
                            if (q[j] < 0 || q[j] >= L[j]) {
                                if (!((pbc >> j) & 1)) continue;
                                q[j] = (q[j] + L[j]) % L[j];
                            }
                            int64_t nb = q[0] + (int64_t)Lx * (q[1] + (int64_t)Ly * q[2]);
                            /* dir=+1: neighbour is n+e_j, entry H[n, n+e_j] = -t(G0 + iGj)/2.
                             * dir=-1: neighbour is n-e_j, entry H[n, n-e_j] = -t(G0 - iGj)/2. */
                            for (int op = 0; op < 4; ++op) {
                                cplx g = (o == op ? g0_entry(o) : 0.0)
                                         + (dir > 0 ? I : -I) * gj_entry(j, o, op);
                                if (g == 0.0) continue;
                                e[ne].c = (int32_t)(4 * nb + op);
                                e[ne].v = -0.5 * t * g;
                                ++ne;
                            }
                        }
                    qsort(e, (size_t)ne, sizeof(orc_entry), cmp_entry);
                    int64_t row = 4 * site + o;
                    int64_t start = nnz;
                    for (int k = 0; k < ne; ++k) {
                        if (nnz > start && col[nnz - 1] == e[k].c) val[nnz - 1] += e[k].v;
                        else { col[nnz] = e[k].c; val[nnz] = e[k].v; ++nnz; }
                    }
                    /* drop entries that cancelled exactly */
                    int64_t w = start;
                    for (int64_t k = start; k < nnz; ++k)
                        if (val[k] != 0.0) { col[w] = col[k]; val[w] = val[k]; ++w; }
                    nnz = w;
                    rowptr[row + 1] = nnz;
                }
            }
    return nnz;
}

/* Gershgorin interval enclosing the spectrum (Sec. 3.1, step 1). */
void orc_gershgorin(int64_t n, const int64_t *rowptr, const int32_t *col, const cplx *val,
                    double *a, double *b)
{
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0, r = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            if (col[p] == i) d += creal(val[p]);
            else r += cabs(val[p]);
        }
        if (d - r < lo) lo = d - r;
        if (d + r > hi) hi = d + r;
    }
    *a = lo; *b = hi;
}

/* Y = H X (plain sparse matrix times block). */
void orc_spmm(int64_t n, const int64_t *rowptr, const int32_t *col, const cplx *val,
              const cplx *X, cplx *Y, int64_t n_s)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t k = 0; k < n_s; ++k) Y[i * n_s + k] = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            const cplx h = val[p];
            const cplx *x = X + (int64_t)col[p] * n_s;
            for (int64_t k = 0; k < n_s; ++k) Y[i * n_s + k] += h * x[k];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Chebyshev window expansion (Sec. 2.1, Eqs. (W1), (W2), Table tab:Kernel).  */
/* ------------------------------------------------------------------------ */

/* c_n of the rectangular window on [lam_lo, lam_hi] inside [a, b].
 * From the integral definition with x = cos(theta):
 *   c_0 = (acos(x_lo) - acos(x_hi))/pi,
 *   c_n = 2/(pi n) (sin(n acos(x_lo)) - sin(n acos(x_hi))),
 * x = alpha*lambda + beta, alpha = 2/(b-a), beta = (a+b)/(a-b).  The closed
 * form printed in Sec. 2.1 has the two arguments exchanged (an overall sign);
 * this is the sign the integral gives.  Arguments are clamped to [-1, 1]. */
void orc_window_coeffs(double lam_lo, double lam_hi, double a, double b, int n_p, double *c)
{
    double alpha = 2.0 / (b - a), beta = (a + b) / (a - b);
    double xl = alpha * lam_lo + beta, xh = alpha * lam_hi + beta;
    if (xl < -1.0) xl = -1.0;
    if (xl > 1.0) xl = 1.0;
    if (xh < -1.0) xh = -1.0;
    if (xh > 1.0) xh = 1.0;
    double tl = acos(xl), th = acos(xh);
    c[0] = (tl - th) / M_PI;
    for (int n = 1; n <= n_p; ++n)
        c[n] = 2.0 / (M_PI * n) * (sin(n * tl) - sin(n * th));
}

/* Kernel damping factors g_n, n = 0..n_p (Table tab:Kernel).
 * kind: 0 none, 1 Fejer, 2 Jackson (as printed: N_p in the denominators),
 *       3 Lanczos with exponent mu (g_0 = 1, the sinc limit). */
void orc_kernel(int kind, int n_p, double mu, double *g)
{
    for (int n = 0; n <= n_p; ++n) {
        double v = 1.0;
        if (kind == 1) {
            v = (double)(n_p - n + 1) / (double)(n_p + 1);
        } else if (kind == 2) {
            double q = M_PI / n_p;
            v = ((n_p - n) * cos(q * n) + sin(q * n) * cos(q) / sin(q)) / n_p;
        } else if (kind == 3) {
            if (n == 0) v = 1.0;
            else {
                double s = M_PI * n / (n_p + 1.0);
                v = pow(sin(s) / s, mu);
            }
        }
        g[n] = v;
    }
}

/* p(lambda) = sum_n gamma_n T_n(alpha*lambda + beta) by the three-term
 * recurrence of Sec. 2.1 (evaluated point by point). */
double orc_poly_eval(const double *gamma, int n_p, double a, double b, double lam)
{
    double x = (2.0 / (b - a)) * lam + (a + b) / (a - b);
    double t0 = 1.0, t1 = x, s = gamma[0];
    if (n_p >= 1) s += gamma[1] * x;
    for (int n = 2; n <= n_p; ++n) {
        double t2 = 2.0 * x * t1 - t0;
        s += gamma[n] * t2;
        t0 = t1; t1 = t2;
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Polynomial filter, Sec. 3.1 step 5 and Fig. fig:ChebFD.                   */
/* X <- p(H) X with p(x) = sum_{n=0}^{n_p} gamma_n T_n(alpha x + beta),       */
/* gamma_n = g_n c_n.  U, W are two scratch blocks of the same shape.        */
/* If mom != NULL it receives per-column Chebyshev moments                   */
/* mu_m = <x, T_m(alpha H + beta) x>, m = 0..2 n_p (layout mom[m*n_s + k]),   */
/* from the dot products of the two vectors present at each step:            */
/* mu_{2n} = 2<T_n x, T_n x> - mu_0,  mu_{2n-1} = 2<T_{n-1} x, T_n x> - mu_1. */
/* ------------------------------------------------------------------------ */
static void scaled_apply(int64_t n, const int64_t *rowptr, const int32_t *col, const cplx *val,
                         double alpha, double beta, double s, const cplx *u,
                         const cplx *sub, cplx *out, int64_t n_s)
{
    /* out = s*(alpha H + beta) u - sub   (sub may be NULL) */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t k = 0; k < n_s; ++k) {
            cplx acc = 0.0;
            for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
                acc += val[p] * u[(int64_t)col[p] * n_s + k];
            cplx v = s * (alpha * acc + beta * u[i * n_s + k]);
            if (sub) v -= sub[i * n_s + k];
            out[i * n_s + k] = v;
        }
    }
}

static double re_dot_col(int64_t n, int64_t n_s, int64_t k, const cplx *x, const cplx *y)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += creal(conj(x[i * n_s + k]) * y[i * n_s + k]);
    return s;
}

static void step_moments(int64_t n, int64_t n_s, const cplx *u, const cplx *w,
                         double *mom, int m_uw, int m_ww)
{
    for (int64_t k = 0; k < n_s; ++k) {
        mom[(int64_t)m_uw * n_s + k] = 2.0 * re_dot_col(n, n_s, k, u, w) - mom[n_s + k];
        mom[(int64_t)m_ww * n_s + k] = 2.0 * re_dot_col(n, n_s, k, w, w) - mom[k];
    }
}

int orc_filter(int64_t n, const int64_t *rowptr, const int32_t *col, const cplx *val,
               double a, double b, const double *gamma, int n_p,
               cplx *X, cplx *U, cplx *W, int64_t n_s, double *mom)
{
    if (n_p < 2) return -1;
    double alpha = 2.0 / (b - a), beta = (a + b) / (a - b);
    /* first two recurrence steps */
    scaled_apply(n, rowptr, col, val, alpha, beta, 1.0, X, NULL, U, n_s);      /* u = A x */
    if (mom) {
        for (int64_t k = 0; k < n_s; ++k) {
            mom[k] = re_dot_col(n, n_s, k, X, X);                                /* mu_0 */
            mom[n_s + k] = re_dot_col(n, n_s, k, X, U);                          /* mu_1 */
            mom[2 * n_s + k] = 2.0 * re_dot_col(n, n_s, k, U, U) - mom[k];       /* mu_2 */
        }
    }
    scaled_apply(n, rowptr, col, val, alpha, beta, 2.0, U, X, W, n_s);          /* w = 2Au - x */
    if (mom) step_moments(n, n_s, U, W, mom, 3, 4);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n * n_s; ++e)
        X[e] = gamma[0] * X[e] + gamma[1] * U[e] + gamma[2] * W[e];
    /* remaining recurrence steps */
    cplx *u = U, *w = W;
    for (int s = 3; s <= n_p; ++s) {
        cplx *t = u; u = w; w = t;                                               /* swap */
        scaled_apply(n, rowptr, col, val, alpha, beta, 2.0, u, w, w, n_s);      /* w = 2Au - w */
        if (mom) step_moments(n, n_s, u, w, mom, 2 * s - 1, 2 * s);
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < n * n_s; ++e) X[e] = X[e] + gamma[s] * w[e];
    }
    return 0;
}

/* Direct moments mu_m = <x, T_m(alpha H + beta) x>, m = 0..n_mom-1, per
 * column, from an explicit recurrence on a separate block (no doubling). */
void orc_moments_direct(int64_t n, const int64_t *rowptr, const int32_t *col, const cplx *val,
                        double a, double b, const cplx *X, int64_t n_s, int n_mom, double *mom)
{
    double alpha = 2.0 / (b - a), beta = (a + b) / (a - b);
    size_t sz = (size_t)(n * n_s) * sizeof(cplx);
    cplx *t0 = (cplx *)malloc(sz), *t1 = (cplx *)malloc(sz), *t2 = (cplx *)malloc(sz);
    memcpy(t0, X, sz);
    for (int64_t k = 0; k < n_s; ++k) mom[k] = re_dot_col(n, n_s, k, X, t0);
    if (n_mom > 1) {
        scaled_apply(n, rowptr, col, val, alpha, beta, 1.0, t0, NULL, t1, n_s);
        for (int64_t k = 0; k < n_s; ++k) mom[n_s + k] = re_dot_col(n, n_s, k, X, t1);
    }
    for (int m = 2; m < n_mom; ++m) {
        scaled_apply(n, rowptr, col, val, alpha, beta, 2.0, t1, t0, t2, n_s);
        for (int64_t k = 0; k < n_s; ++k) mom[(int64_t)m * n_s + k] = re_dot_col(n, n_s, k, X, t2);
        cplx *t = t0; t0 = t1; t1 = t2; t2 = t;
    }
    free(t0); free(t1); free(t2);
}

/* ------------------------------------------------------------------------ */
/* Dense linear algebra.                                                     */
/* ------------------------------------------------------------------------ */

/* S = A^H B (n_a x n_b) with Kahan-compensated sums over the n rows
 * (Sec. 3.1, step 6 remarks). A: n x n_a, B: n x n_b, row-major.
 * The paper fixes the compensation, not the association of the sums: the
 * rows are split into one contiguous range per thread, each range is summed
 * in row order with compensation (s - c is the range sum), and the range
 * sums are then added in range order, again with compensation.  Each thread
 * reads every row of its range once (row-major blocks). */
void orc_gram_kahan(int64_t n, const cplx *A, int64_t n_a, const cplx *B, int64_t n_b, cplx *S)
{
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    const int64_t m = n_a * n_b;
    double *acc = (double *)calloc((size_t)nt * (size_t)m * 4, sizeof(double));
#pragma omp parallel num_threads(nt)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        const int64_t i0 = n * t / nt, i1 = n * (t + 1) / nt;
        double *sr = acc + (size_t)t * m * 4, *cr = sr + m, *si = cr + m, *ci = si + m;
        for (int64_t i = i0; i < i1; ++i)
            for (int64_t k = 0; k < n_a; ++k) {
                const cplx a = conj(A[i * n_a + k]);
                for (int64_t l = 0; l < n_b; ++l) {
                    const cplx p = a * B[i * n_b + l];
                    const int64_t q = k * n_b + l;
                    double y = creal(p) - cr[q], tt = sr[q] + y;
                    cr[q] = (tt - sr[q]) - y; sr[q] = tt;
                    y = cimag(p) - ci[q]; tt = si[q] + y;
                    ci[q] = (tt - si[q]) - y; si[q] = tt;
                }
            }
    }
    for (int64_t q = 0; q < m; ++q) {
        double sre = 0.0, cre = 0.0, sim = 0.0, cim = 0.0;
        for (int t = 0; t < nt; ++t) {
            const double *sr = acc + (size_t)t * m * 4, *cr = sr + m, *si = cr + m, *ci = si + m;
            double y = (sr[q] - cr[q]) - cre, tt = sre + y;
            cre = (tt - sre) - y; sre = tt;
            y = (si[q] - ci[q]) - cim; tt = sim + y;
            cim = (tt - sim) - y; sim = tt;
        }
        S[q] = sre + I * sim;
    }
    free(acc);
}

/* C = A T with A: n x k (row-major), T: k x m, C: n x m. */
void orc_block_times_small(int64_t n, const cplx *A, int64_t k, const cplx *T, int64_t m, cplx *C)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < m; ++j) {
            cplx s = 0.0;
            for (int64_t q = 0; q < k; ++q) s += A[i * k + q] * T[q * m + j];
            C[i * m + j] = s;
        }
}

/* Cyclic Jacobi eigen-decomposition of a complex Hermitian matrix A (n x n,
 * row-major, overwritten).  evals ascending; evecs (n x n, row-major) holds
 * the eigenvectors as columns.  Each rotation J = Phi R first removes the
 * phase of a_pq (Phi = diag(1 at p, e^{-i phi} at q)) and then applies the
 * real 2x2 Jacobi rotation that annihilates the now real entry. */
int orc_jacobi_herm(int n, cplx *A, double *evals, cplx *V)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;
    double fro = 0.0;
    for (int i = 0; i < n * n; ++i) fro += creal(A[i] * conj(A[i]));
    fro = sqrt(fro);
    int sweep;
    for (sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += creal(A[p * n + q] * conj(A[p * n + q]));
        if (sqrt(2.0 * off) <= 1e-15 * fro || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                cplx apq = A[p * n + q];
                double r = cabs(apq);
                if (r == 0.0) continue;
                double app = creal(A[p * n + p]), aqq = creal(A[q * n + q]);
                if (sweep > 3 && r <= 1e-18 * (fabs(app) + fabs(aqq))) {
                    A[p * n + q] = 0.0; A[q * n + p] = 0.0; continue;
                }
                cplx ph = apq / r;                       /* e^{i phi} */
                double zeta = (aqq - app) / (2.0 * r);
                double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                /* J entries */
                cplx jpp = c, jpq = s, jqp = -s * conj(ph), jqq = c * conj(ph);
                /* A <- A J (columns p, q) */
                for (int i = 0; i < n; ++i) {
                    cplx aip = A[i * n + p], aiq = A[i * n + q];
                    A[i * n + p] = aip * jpp + aiq * jqp;
                    A[i * n + q] = aip * jpq + aiq * jqq;
                }
                /* A <- J^H A (rows p, q) */
                for (int j = 0; j < n; ++j) {
                    cplx apj = A[p * n + j], aqj = A[q * n + j];
                    A[p * n + j] = conj(jpp) * apj + conj(jqp) * aqj;
                    A[q * n + j] = conj(jpq) * apj + conj(jqq) * aqj;
                }
                A[p * n + q] = 0.0; A[q * n + p] = 0.0;
                A[p * n + p] = creal(A[p * n + p]);
                A[q * n + q] = creal(A[q * n + q]);
                /* V <- V J */
                for (int i = 0; i < n; ++i) {
                    cplx vip = V[i * n + p], viq = V[i * n + q];
                    V[i * n + p] = vip * jpp + viq * jqp;
                    V[i * n + q] = vip * jpq + viq * jqq;
                }
            }
    }
    /* sort ascending (selection sort: plain) */
    for (int i = 0; i < n; ++i) evals[i] = creal(A[i * n + i]);
    for (int i = 0; i < n; ++i) {
        int mi = i;
        for (int j = i + 1; j < n; ++j) if (evals[j] < evals[mi]) mi = j;
        if (mi != i) {
            double tv = evals[i]; evals[i] = evals[mi]; evals[mi] = tv;
            for (int r = 0; r < n; ++r) {
                cplx tc = V[r * n + i]; V[r * n + i] = V[r * n + mi]; V[r * n + mi] = tc;
            }
        }
    }
    return sweep;
}

/* SVQB orthonormalisation (Sec. 3.1, step 6; Stathopoulos & Wu):
 * S = Y^H Y, D = diag(S)^{-1/2}, D S D = U Theta U^H, keep Theta_j > tau*max,
 * Y <- Y D U Theta^{-1/2}.  Dropped directions are replaced by random
 * vectors (stream 3, index offset from `refill_offset`) and the pass is
 * repeated; two clean passes are made.  Y is n x n_s, T a scratch block of
 * the same size.  Returns the number of columns refilled in total. */
int orc_svqb(int64_t n, cplx *Y, cplx *Tmp, int64_t n_s, double tau,
             uint64_t seed, uint64_t refill_offset)
{
    int ns = (int)n_s, refilled = 0, clean = 0;
    cplx *S = (cplx *)malloc(sizeof(cplx) * ns * ns);
    cplx *Uv = (cplx *)malloc(sizeof(cplx) * ns * ns);
    cplx *Tm = (cplx *)malloc(sizeof(cplx) * ns * ns);
    double *th = (double *)malloc(sizeof(double) * ns);
    double *d = (double *)malloc(sizeof(double) * ns);
    for (int pass = 0; pass < 8 && clean < 2; ++pass) {
        orc_gram_kahan(n, Y, n_s, Y, n_s, S);
        for (int k = 0; k < ns; ++k) {
            double s = creal(S[k * ns + k]);
            d[k] = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
        }
        for (int k = 0; k < ns; ++k)
            for (int l = 0; l < ns; ++l) S[k * ns + l] *= d[k] * d[l];
        orc_jacobi_herm(ns, S, th, Uv);
        double tmax = th[ns - 1];
        int keep = 0;
        /* columns of T = D U Theta^{-1/2} for kept eigenvalues, largest first */
        for (int j = ns - 1; j >= 0; --j) {
            if (!(th[j] > tau * tmax)) continue;
            double f = 1.0 / sqrt(th[j]);
            for (int k = 0; k < ns; ++k) Tm[k * ns + keep] = d[k] * Uv[k * ns + j] * f;
            ++keep;
        }
        for (int j = keep; j < ns; ++j)
            for (int k = 0; k < ns; ++k) Tm[k * ns + j] = 0.0;
        orc_block_times_small(n, Y, n_s, Tm, n_s, Tmp);
        memcpy(Y, Tmp, sizeof(cplx) * (size_t)(n * n_s));
        if (keep < ns) {
            for (int64_t i = 0; i < n; ++i)
                for (int k = keep; k < ns; ++k) {
                    uint64_t e = refill_offset + (uint64_t)(i * n_s + k);
                    double re = 2.0 * orc_u01(seed, 3, 2 * e) - 1.0;
                    double im = 2.0 * orc_u01(seed, 3, 2 * e + 1) - 1.0;
                    Y[i * n_s + k] = re + I * im;
                }
            refilled += ns - keep;
            refill_offset += (uint64_t)(n * n_s);
            clean = 0;
        } else {
            ++clean;
        }
    }
    free(S); free(Uv); free(Tm); free(th); free(d);
    return refilled;
}

/* Rayleigh-Ritz (Sec. 3.1, step 7) on an orthonormal block Y (n x n_s):
 * W = H Y, G = Y^H W, G = U Theta U^H, V = Y U, HV = W U,
 * r_k = || HV_k - theta_k V_k ||_2.  Y is overwritten by V, W by HV. */
void orc_rayleigh_ritz(int64_t n, const int64_t *rowptr, const int32_t *col, const cplx *val,
                       cplx *Y, cplx *W, cplx *Tmp, int64_t n_s, double *theta, double *res)
{
    int ns = (int)n_s;
    cplx *G = (cplx *)malloc(sizeof(cplx) * ns * ns);
    cplx *Uv = (cplx *)malloc(sizeof(cplx) * ns * ns);
    orc_spmm(n, rowptr, col, val, Y, W, n_s);
    orc_gram_kahan(n, Y, n_s, W, n_s, G);
    /* symmetrise the rounding noise away: G <- (G + G^H)/2 */
    for (int k = 0; k < ns; ++k)
        for (int l = k; l < ns; ++l) {
            cplx v = 0.5 * (G[k * ns + l] + conj(G[l * ns + k]));
            G[k * ns + l] = v; G[l * ns + k] = conj(v);
        }
    orc_jacobi_herm(ns, G, theta, Uv);
    orc_block_times_small(n, Y, n_s, Uv, n_s, Tmp);
    memcpy(Y, Tmp, sizeof(cplx) * (size_t)(n * n_s));
    orc_block_times_small(n, W, n_s, Uv, n_s, Tmp);
    memcpy(W, Tmp, sizeof(cplx) * (size_t)(n * n_s));
#pragma omp parallel for schedule(static)
    for (int k = 0; k < ns; ++k) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            cplx r = W[i * n_s + k] - theta[k] * Y[i * n_s + k];
            s += creal(r * conj(r));
        }
        res[k] = sqrt(s);
    }
    free(G); free(Uv);
}

/* Harmonic Ritz extraction (Sec. 3.1 step 7 remarks, Sec. 6: the cleaner
 * alternative to Ritz values for interior eigenvalues; Morgan 1991, Paige,
 * Parlett and van der Vorst 1995).  For the orthonormal block Y and the
 * target tau, a harmonic Ritz pair (theta, Y s) satisfies the Petrov-Galerkin
 * condition
 *     (H - tau) Y s - (theta - tau) Y s  orthogonal to  (H - tau) Y,
 * i.e. M s = (theta - tau) A s with A = Y^H (H - tau) Y (Hermitian) and
 * M = ((H - tau) Y)^H ((H - tau) Y) (positive definite).  With the Cholesky
 * factor M = L L^H and z = L^H s this is the Hermitian problem
 *     L^{-1} A L^{-H} z = z / (theta - tau),
 * solved by the cyclic Jacobi method; s = L^{-H} z.  The vectors y = Y s /
 * |s| (|Y s| = |s|) carry the eigenvalue estimate rho = y^H H y (the Rayleigh
 * quotient), by which the pairs are returned in ascending order, with the
 * residuals |H y - rho y|.  Y and W (W = H Y on return) are overwritten by
 * the vectors and their images.  Returns -1 if M is not numerically
 * positive definite (tau an eigenvalue with its vector in span Y). */
int orc_harmonic_ritz(int64_t n, const int64_t *rowptr, const int32_t *col, const cplx *val,
                      cplx *Y, cplx *W, cplx *Tmp, int64_t n_s, double tau, double *rho,
                      double *res)
{
    int ns = (int)n_s, rc = 0;
    size_t blk = (size_t)(n * n_s);
    cplx *G = (cplx *)malloc(sizeof(cplx) * ns * ns);
    cplx *M = (cplx *)malloc(sizeof(cplx) * ns * ns);
    cplx *L = (cplx *)calloc((size_t)ns * ns, sizeof(cplx));
    cplx *Li = (cplx *)calloc((size_t)ns * ns, sizeof(cplx));
    cplx *Cm = (cplx *)malloc(sizeof(cplx) * ns * ns);
    cplx *Z = (cplx *)malloc(sizeof(cplx) * ns * ns);
    cplx *S = (cplx *)malloc(sizeof(cplx) * ns * ns);
    double *zeta = (double *)malloc(sizeof(double) * ns);
    int *ord = (int *)malloc(sizeof(int) * ns);
    orc_spmm(n, rowptr, col, val, Y, W, n_s);
    /* G = Y^H H Y, Hermitian part; M from the block (H - tau) Y */
    orc_gram_kahan(n, Y, n_s, W, n_s, G);
    for (int k = 0; k < ns; ++k)
        for (int l = k; l < ns; ++l) {
            cplx v = 0.5 * (G[k * ns + l] + conj(G[l * ns + k]));
            G[k * ns + l] = v; G[l * ns + k] = conj(v);
        }
    for (size_t i = 0; i < blk; ++i) Tmp[i] = W[i] - tau * Y[i];
    orc_gram_kahan(n, Tmp, n_s, Tmp, n_s, M);
    /* Cholesky M = L L^H (lower) */
    for (int j = 0; j < ns && rc == 0; ++j) {
        double d = creal(M[j * ns + j]);
        for (int q = 0; q < j; ++q) d -= creal(L[j * ns + q] * conj(L[j * ns + q]));
        if (!(d > 0.0)) { rc = -1; break; }
        L[j * ns + j] = sqrt(d);
        for (int i = j + 1; i < ns; ++i) {
            cplx v = M[i * ns + j];
            for (int q = 0; q < j; ++q) v -= L[i * ns + q] * conj(L[j * ns + q]);
            L[i * ns + j] = v / L[j * ns + j];
        }
    }
    if (rc == 0) {
        /* Li = L^{-1} by forward substitution */
        for (int c = 0; c < ns; ++c) {
            Li[c * ns + c] = 1.0 / L[c * ns + c];
            for (int i = c + 1; i < ns; ++i) {
                cplx v = 0.0;
                for (int q = c; q < i; ++q) v += L[i * ns + q] * Li[q * ns + c];
                Li[i * ns + c] = -v / L[i * ns + i];
            }
        }
        /* C = Li (G - tau I) Li^H */
        for (int i = 0; i < ns; ++i)
            for (int j = 0; j < ns; ++j) {
                cplx v = 0.0;
                for (int p = 0; p < ns; ++p)
                    for (int q = 0; q < ns; ++q) {
                        cplx a = G[p * ns + q] - (p == q ? tau : 0.0);
                        v += Li[i * ns + p] * a * conj(Li[j * ns + q]);
                    }
                Cm[i * ns + j] = v;
            }
        orc_jacobi_herm(ns, Cm, zeta, Z);
        /* S = Li^H Z, unit columns; rho_j = s_j^H G s_j */
        for (int i = 0; i < ns; ++i)
            for (int j = 0; j < ns; ++j) {
                cplx v = 0.0;
                for (int q = 0; q < ns; ++q) v += conj(Li[q * ns + i]) * Z[q * ns + j];
                S[i * ns + j] = v;
            }
        for (int j = 0; j < ns; ++j) {
            double nrm = 0.0;
            for (int i = 0; i < ns; ++i) nrm += creal(S[i * ns + j] * conj(S[i * ns + j]));
            nrm = sqrt(nrm);
            for (int i = 0; i < ns; ++i) S[i * ns + j] /= nrm;
            cplx r = 0.0;
            for (int p = 0; p < ns; ++p)
                for (int q = 0; q < ns; ++q) r += conj(S[p * ns + j]) * G[p * ns + q] * S[q * ns + j];
            zeta[j] = creal(r);
        }
        /* ascending rho: a permutation of the columns of S */
        for (int j = 0; j < ns; ++j) ord[j] = j;
        for (int j = 1; j < ns; ++j) {
            int o = ord[j], q = j - 1;
            while (q >= 0 && zeta[ord[q]] > zeta[o]) { ord[q + 1] = ord[q]; --q; }
            ord[q + 1] = o;
        }
        for (int j = 0; j < ns; ++j) {
            rho[j] = zeta[ord[j]];
            for (int i = 0; i < ns; ++i) Z[i * ns + j] = S[i * ns + ord[j]];
        }
        orc_block_times_small(n, Y, n_s, Z, n_s, Tmp);
        memcpy(Y, Tmp, sizeof(cplx) * blk);
        orc_block_times_small(n, W, n_s, Z, n_s, Tmp);
        memcpy(W, Tmp, sizeof(cplx) * blk);
#pragma omp parallel for schedule(static)
        for (int k = 0; k < ns; ++k) {
            double s2 = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                cplx r = W[i * n_s + k] - rho[k] * Y[i * n_s + k];
                s2 += creal(r * conj(r));
            }
            res[k] = sqrt(s2);
        }
    }
    free(G); free(M); free(L); free(Li); free(Cm); free(Z); free(S); free(zeta); free(ord);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* The ChebFD scheme, Sec. 3.1 steps 1-8.                                     */
/* Readings where the paper leaves a choice:                                 */
/*  - a Ritz pair with value in [lam_lo, lam_hi] is converged if r <= eps,   */
/*    converging if eps < r <= sqrt(eps), a ghost candidate otherwise       */
/*    (step 7 remarks: pairs whose residual stays above sqrt(eps) are       */
/*    discarded as ghosts);                                                 */
/*  - exit (step 8a, with those ghosts discarded) once, after at least two  */
/*    iterations, no in-window pair is converging, the converged count      */
/*    equals that of the previous iteration, and the ghost candidates       */
/*    "remain" large: the smallest of their residuals did not decrease      */
/*    from the previous iteration (a ghost's residual is large and does     */
/*    not decrease, step 7 remarks).  No tolerance factor is applied;       */
/*  - the restart block is the full set of n_s Ritz vectors (step 8b).      */
/* With harmonic != 0 step 7 extracts harmonic Ritz pairs for the target at */
/* the window centre (orc_harmonic_ritz) instead of Ritz pairs.             */
/* Outputs the converged in-window pairs in ascending order.                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    int iterations;
    int n_found;
    int64_t n_mvm;          /* iterations * n_s * n_p */
    int refilled;
    double a, b;
} orc_solve_stats;

int orc_chebfd_solve(int64_t n, const int64_t *rowptr, const int32_t *col, const cplx *val,
                     double lam_lo, double lam_hi, int64_t n_s, int n_p, int kernel, double mu,
                     double eps, int max_iter, uint64_t seed, double a, double b,
                     double *evals_out, double *res_out, cplx *evecs_out /* n x n_s, nullable */,
                     orc_solve_stats *st, int harmonic)
{
    if (!(lam_lo < lam_hi) || n_p < 2 || n_s < 1) return -1;
    if (isnan(a) || isnan(b)) orc_gershgorin(n, rowptr, col, val, &a, &b);
    double *gam = (double *)malloc(sizeof(double) * (n_p + 1));
    double *g = (double *)malloc(sizeof(double) * (n_p + 1));
    orc_window_coeffs(lam_lo, lam_hi, a, b, n_p, gam);
    orc_kernel(kernel, n_p, mu, g);
    for (int k = 0; k <= n_p; ++k) gam[k] *= g[k];
    size_t blk = (size_t)(n * n_s);
    cplx *X = (cplx *)malloc(sizeof(cplx) * blk);
    cplx *U = (cplx *)malloc(sizeof(cplx) * blk);
    cplx *W = (cplx *)malloc(sizeof(cplx) * blk);
    double *theta = (double *)malloc(sizeof(double) * n_s);
    double *res = (double *)malloc(sizeof(double) * n_s);
    orc_random_block(n, n_s, seed, 1, 0, X);
    int it, prev_conv = -1, nconv = 0, refilled = 0, status = 1;
    double seps = sqrt(eps), prev_rmin = INFINITY;
    for (it = 1; it <= max_iter; ++it) {
        orc_filter(n, rowptr, col, val, a, b, gam, n_p, X, U, W, n_s, NULL);
        refilled += orc_svqb(n, X, U, n_s, 1e-12, seed, (uint64_t)it * 64u * (uint64_t)blk);
        if (!harmonic ||
            orc_harmonic_ritz(n, rowptr, col, val, X, W, U, n_s, 0.5 * (lam_lo + lam_hi), theta,
                              res) != 0)
            orc_rayleigh_ritz(n, rowptr, col, val, X, W, U, n_s, theta, res);
        int nconving = 0;
        double rmin = INFINITY;
        nconv = 0;
        for (int k = 0; k < n_s; ++k) {
            if (theta[k] < lam_lo || theta[k] > lam_hi) continue;
            if (res[k] <= eps) ++nconv;
            else {
                if (res[k] <= seps) ++nconving;
                if (res[k] < rmin) rmin = res[k];
            }
        }
        int stagnant = (rmin == INFINITY) || (rmin >= prev_rmin);
        if (it >= 2 && nconving == 0 && nconv == prev_conv && stagnant) { status = 0; break; }
        prev_conv = nconv;
        prev_rmin = rmin;
    }
    if (it > max_iter) it = max_iter;
    int f = 0;
    for (int k = 0; k < n_s; ++k) {
        if (theta[k] < lam_lo || theta[k] > lam_hi || res[k] > eps) continue;
        evals_out[f] = theta[k];
        res_out[f] = res[k];
        if (evecs_out)
            for (int64_t i = 0; i < n; ++i) evecs_out[i * n_s + f] = X[i * n_s + k];
        ++f;
    }
    if (st) {
        st->iterations = it; st->n_found = f; st->n_mvm = (int64_t)it * n_s * n_p;
        st->refilled = refilled; st->a = a; st->b = b;
    }
    free(gam); free(g); free(X); free(U); free(W); free(theta); free(res);
    return status;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
