/*
 * chebfd.h -- C ABI of the MI355X (gfx950) Chebyshev filter diagonalisation
 * library.
 *
 * The library computes the eigenpairs (lambda_i, v_i) of a sparse Hermitian
 * matrix H that lie in a target window [lam_lo, lam_hi], each with residual
 * ||H v_i - lambda_i v_i|| <= eps (problem statement of Sec. 2 of Pieper et
 * al., arXiv:1510.04895), by the ChebFD scheme of Sec. 3.1: a Chebyshev
 * window-filter polynomial p(H) of degree N_p applied to a block of N_S search
 * vectors (Fig. fig:ChebFD), followed by orthogonalisation, Rayleigh-Ritz and
 * a residual check.
 *
 * Conventions for every entry point
 *  - Return value: 0 = success; negative = error (nothing was written to the
 *    outputs unless stated); positive = warning, outputs are valid.
 *    chebfd_last_error() gives a message for the calling thread.
 *  - Complex numbers are stored interleaved (re, im): "c128" = two doubles,
 *    "c64" = two floats.
 *  - Blocks of vectors are row-major: element (row i, column k) at
 *    base[i * ld + k] (in complex elements), ld >= n_s.  Row i is the i-th
 *    component of every search vector (Sec. 4: row-major block vectors).
 *  - "device" pointers are HIP device memory owned by the caller; the library
 *    never frees them.  "host" pointers are ordinary memory.
 *  - Work is enqueued on the stream given to chebfd_create(); the low-level
 *    calls return without synchronising unless stated.
 *  - One context per host thread.  Handles (matrix, result) are owned by the
 *    library until the matching *_destroy.
 */
#ifndef CHEBFD_H
#define CHEBFD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct chebfd_ctx chebfd_ctx;
typedef struct chebfd_matrix chebfd_matrix;
typedef struct chebfd_result chebfd_result;

/* status codes */
#define CHEBFD_OK 0
#define CHEBFD_ERR_INVALID_ARG (-1)
#define CHEBFD_ERR_OOM (-2)
#define CHEBFD_ERR_HIP (-3)
#define CHEBFD_ERR_NONFINITE (-4)
#define CHEBFD_ERR_UNSUPPORTED (-5)
#define CHEBFD_ERR_WORKSPACE (-6)
#define CHEBFD_WARN_NOT_CONVERGED 1
#define CHEBFD_WARN_SEARCH_SPACE_TOO_SMALL 2

/* damping kernels g_n (Table tab:Kernel) */
#define CHEBFD_KERNEL_NONE 0
#define CHEBFD_KERNEL_FEJER 1
#define CHEBFD_KERNEL_JACKSON 2
#define CHEBFD_KERNEL_LANCZOS 3

/* arithmetic of the filter sweep */
#define CHEBFD_PREC_C128 0   /* complex128 storage, FP64 recurrence */
#define CHEBFD_PREC_C64 1    /* complex64 storage, FP32 recurrence */
/* history only: an FP32 correction pass of the precision form's polish */
#define CHEBFD_PREC_C64_CORRECTION 2

/* polish of the precision form (chebfd_params.polish) */
#define CHEBFD_POLISH_CORRECTION 0   /* FP32 correction passes (default) */
#define CHEBFD_POLISH_FP64 1         /* FP64 filter passes */

/* matrix storage */
#define CHEBFD_STORAGE_SELL 0     /* SELL-C-sigma, values and column indices */
#define CHEBFD_STORAGE_STENCIL 1  /* topological-insulator stencil, no index stream */

/* ------------------------------------------------------------------ */
/* context                                                             */
/* ------------------------------------------------------------------ */

/* Creates a context on HIP device `device`; `hip_stream` is a hipStream_t
 * (NULL = the null stream) on which all work is enqueued.  Fails with
 * CHEBFD_ERR_HIP when no device is present. */
int chebfd_create(chebfd_ctx **out, int device, void *hip_stream);
int chebfd_destroy(chebfd_ctx *ctx);
/* Blocks until all work enqueued by the context has finished. */
int chebfd_synchronize(chebfd_ctx *ctx);
const char *chebfd_strerror(int code);
const char *chebfd_last_error(void);
/* Library version string (host only). */
const char *chebfd_version(void);

/* ------------------------------------------------------------------ */
/* sparse matrices                                                     */
/* ------------------------------------------------------------------ */

/* Uploads a Hermitian matrix given in CSR (0-based; rowptr has n+1 int64
 * entries, col int32, val n_nz interleaved complex doubles; host memory, only
 * read) into SELL-C-sigma storage (Sec. 4.2): rows are sorted by length
 * within windows of `sell_sigma` rows, grouped into chunks of `sell_C` rows
 * and padded to the chunk's longest row.  Both a c128 and a c64 copy of the
 * values are kept so either precision can run.  The Gershgorin interval of
 * the rows (Sec. 3.1 step 1) is computed on the way.  Hermiticity is not
 * checked.  Errors: INVALID_ARG (n < 1, sell_C not in {1,2,4,...,64},
 * sell_sigma < 1 or not a multiple of sell_C, a column out of range, a
 * decreasing rowptr), OOM. */
int chebfd_matrix_from_csr(chebfd_ctx *ctx, int64_t n, const int64_t *rowptr,
                           const int32_t *col, const double *val, int sell_C,
                           int sell_sigma, chebfd_matrix **out);

/* Builds the topological-insulator Hamiltonian of Sec. 5.1, Eq. (Ham), on an
 * Lx x Ly x Lz lattice with 4 orbitals per site (N = 4 Lx Ly Lz):
 *   site n = x + Lx (y + Ly z), row 4n + o, orbital o = 2 tau + s,
 *   G0 = tau_z (x) s_0, Gj = tau_x (x) s_j,
 *   on-site block m G0 + V_n 1,  V_n = V (u_n - 1/2),
 *   H[n, n+e_j] = -t (G0 + i Gj)/2 and H[n+e_j, n] = -t (G0 - i Gj)/2,
 * with u_n the counter-based uniform number of stream 0 at index n for
 * `seed` (SplitMix64 finaliser; see chebfd_random_block).  Bit j of
 * pbc_mask makes direction j periodic.  storage = SELL builds SELL-C-sigma
 * (sell_C, sell_sigma as above); storage = STENCIL keeps only the per-site
 * potential and generates the hopping blocks inside the kernel.
 * Errors: INVALID_ARG (an extent < 1, N >= 2^31), OOM. */
int chebfd_matrix_ti(chebfd_ctx *ctx, int Lx, int Ly, int Lz, int pbc_mask, double t,
                     double m, double V, uint64_t seed, int storage, int sell_C,
                     int sell_sigma, chebfd_matrix **out);

/* Properties of a matrix handle (host outputs, any may be NULL):
 * n rows, nnz stored entries without padding, padded entries, Gershgorin
 * interval [g_lo, g_hi], and the bytes one filter step reads of the matrix
 * in c128 and in c64 storage (0 for STENCIL). */
int chebfd_matrix_info(const chebfd_matrix *H, int64_t *n, int64_t *nnz, int64_t *padded,
                       double *g_lo, double *g_hi, int64_t *matrix_bytes_c128,
                       int64_t *matrix_bytes_c64);
int chebfd_matrix_destroy(chebfd_matrix *H);

/* ------------------------------------------------------------------ */
/* filter polynomials (host only)                                      */
/* ------------------------------------------------------------------ */

/* gamma_n = g_n c_n, n = 0..n_p (Sec. 2.1, Eqs. (W1)-(W2), Table
 * tab:Kernel): c_n are the Chebyshev coefficients of the rectangular window
 * on [lam_lo, lam_hi] in the spectral interval [a, b]
 *   c_0 = (acos x_lo - acos x_hi)/pi,
 *   c_n = 2/(pi n) (sin(n acos x_lo) - sin(n acos x_hi)),  x = alpha l + beta,
 * (the sign the integral definition gives; arguments clamped to [-1,1]) and
 * g_n the damping factors of `kernel` (Lanczos exponent `mu`; Jackson as
 * printed, so g_{N_p-1} = g_{N_p} = 0).  `gamma_out` holds n_p + 1 doubles.
 * Errors: INVALID_ARG (lam_lo >= lam_hi, a >= b, n_p < 2, unknown kernel,
 * window not intersecting [a, b]). */
int chebfd_coeffs(double lam_lo, double lam_hi, double a, double b, int n_p, int kernel,
                  double mu, double *gamma_out);

/* Division of the filter polynomial by a linear factor (host only): for
 * p(y) = sum_{n=0}^{n_p} gamma_n T_n(y) in the scaled variable
 * y = (2x - a - b) / (b - a) and t = (2 lambda - a - b) / (b - a), writes the
 * n_p coefficients d_0 .. d_{n_p - 1} of q(y) = (p(y) - p(t)) / (y - t) to
 * d_out and p(t) to *p_out (may be NULL).  Then for any vector v,
 * p(H~) v = p(t) v + q(H~) (H~ - t) v, H~ = alpha H + beta -- the identity
 * behind the precision form's correction passes.  Backward recurrence from
 * the top coefficient (the intermediate values of Clenshaw's sum). */
int chebfd_coeffs_divided(const double *gamma, int n_p, double a, double b, double lambda,
                          double *d_out, double *p_out);

/* Damping factor sigma and quality eta = -n_p / log10(sigma) of a filter
 * polynomial (Sec. 2.3): sigma = max |p| outside the search interval
 * [s_lo, s_hi] over [a, b] divided by min |p| inside [t_lo, t_hi]. */
int chebfd_filter_quality(const double *gamma, int n_p, double a, double b, double t_lo,
                          double t_hi, double s_lo, double s_hi, double *sigma, double *eta);

/* Polynomial degree minimising eta for the target window [t_lo, t_hi] and
 * search interval [s_lo, s_hi] (Sec. 2.3, Sec. 3.1 step 3); searches
 * n_p in [np_min, np_max] exhaustively (eta(n_p) has many local minima). */
int chebfd_optimal_np(double a, double b, double t_lo, double t_hi, double s_lo, double s_hi,
                      int kernel, double mu, int np_min, int np_max, int *n_p, double *eta);

/* ------------------------------------------------------------------ */
/* low-level device operations (caller-owned device buffers)           */
/* ------------------------------------------------------------------ */

/* The polynomial filter of Fig. fig:ChebFD, in place:
 *   X <- p(H) X,  p(x) = sum_{n=0}^{n_p} gamma_n T_n(alpha x + beta),
 *   alpha = 2/(b-a), beta = (a+b)/(a-b).
 * gamma: host array of n_p + 1 doubles.  X, U, W: device blocks of n rows
 * and n_s columns with leading dimension ld, element type per `precision`
 * (c128 or c64); U and W are scratch and are overwritten.  The first step
 * forms u = (alpha H + beta) x, w = 2 (alpha H + beta) u - x and
 * x = gamma_0 x + gamma_1 u + gamma_2 w; every later step swaps u and w,
 * forms w = 2 (alpha H + beta) u - w and adds gamma_n w to x, each step one
 * fused kernel.  If moments_dev != NULL (device, (2 n_p + 1) x n_s doubles,
 * row-major) it receives the Chebyshev moments mu_m = <x, T_m x> of the
 * input columns, m = 0..2 n_p, obtained from mu_{2n} = 2<T_n x,T_n x> - mu_0
 * and mu_{2n-1} = 2<T_{n-1} x,T_n x> - mu_1 (Sec. 4, moments during the
 * filter).  Requirements: n_p >= 2, 1 <= n_s <= ld, a < b; for c64 ld and n_s
 * even and the buffers 16-byte aligned.  Errors: INVALID_ARG, HIP. */
int chebfd_filter_apply(chebfd_ctx *ctx, const chebfd_matrix *H, int precision,
                        const double *gamma, int n_p, double a, double b, void *X, void *U,
                        void *W, int64_t n_s, int64_t ld, double *moments_dev);

/* The filter with a coefficient sequence of its own for every column (the
 * correction pass of the precision form, where column j carries the
 * coefficients of (p(y) - p(t_j)) / (y - t_j) from chebfd_coeffs_divided):
 *   X[:, j] <- sum_{n=0}^{n_p} gcol[n * ldg + j] T_n(alpha H + beta) X[:, j].
 * gcol: DEVICE array of n_p + 1 rows of ldg >= n_s doubles (read only).
 * complex64 only (UNSUPPORTED otherwise); no moments.  Buffers, layout and
 * errors as chebfd_filter_apply (the coefficients are not checked for
 * finiteness: they are on the device). */
int chebfd_filter_apply_columns(chebfd_ctx *ctx, const chebfd_matrix *H, int precision,
                                const double *gcol, int64_t ldg, int n_p, double a, double b,
                                void *X, void *U, void *W, int64_t n_s, int64_t ld);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * filter as chebfd_filter_apply, same arguments and results (the same
 * kernels in the same order, so bitwise equal output), but it allocates
 * nothing.  With moments_dev != NULL the moment partial sums live in a fixed
 * 64 MiB device array that the library holds on every GPU it runs on until
 * the process ends (located by chebfd_create); the partials need
 * 24 * n_s * (row blocks of one launch) bytes, e.g. 12.6 MB for 8 columns of
 * a 524,288-row SELL-32 matrix.  Calls on one GPU share that array: calls
 * that overlap in time on one GPU (two streams, two threads) race and give
 * wrong moments.  Errors: as chebfd_filter_apply, and INVALID_ARG when the
 * partial sums exceed the array. */
int chebfd_filter_apply_noalloc(chebfd_ctx *ctx, const chebfd_matrix *H, int precision,
                                const double *gamma, int n_p, double a, double b, void *X,
                                void *U, void *W, int64_t n_s, int64_t ld, double *moments_dev);

/* Y = (s_h H + s_u) X for a block (the plain spMMVM, Sec. 4), same layout
 * rules as chebfd_filter_apply; X and Y must not overlap. */
int chebfd_spmm(chebfd_ctx *ctx, const chebfd_matrix *H, int precision, const void *X, void *Y,
                int64_t n_s, int64_t ld, double s_h, double s_u);

/* S = A^H B (n_a x n_b, complex128, row-major, device) for blocks A (n x n_a,
 * lda) and B (n x n_b, ldb) of element type `precision`, accumulated in FP64
 * on the matrix cores with a fixed-order split over rows (bitwise
 * reproducible).  Errors: INVALID_ARG, HIP. */
int chebfd_gram(chebfd_ctx *ctx, int precision, const void *A, int64_t lda, int64_t n_a,
                const void *B, int64_t ldb, int64_t n_b, int64_t n, double *S_dev);

/* C = A T (c_beta = 0) or C = C - A T (c_beta = 1) with A (n x k, lda,
 * element type prec_a), T (k x m complex128 row-major, device) and C (n x m,
 * ldc, element type prec_c); FP64 accumulation on the matrix cores.  C must
 * not overlap A. */
int chebfd_block_times(chebfd_ctx *ctx, int prec_a, const void *A, int64_t lda, int64_t n,
                       int64_t k, const double *T_dev, int64_t m, int prec_c, void *C,
                       int64_t ldc, int c_beta);

/* res[j] = || HV_j - theta_j V_j ||_2 for j < m (FP64; V, HV n x m with ld;
 * theta host, res host).  Synchronises. */
int chebfd_residual_norms(chebfd_ctx *ctx, int precision, const void *V, const void *HV,
                          int64_t n, int64_t m, int64_t ld, const double *theta, double *res);

/* Fills columns [k0, k0 + m) of a block with counter-based random numbers:
 * element (i, k) = (2u - 1) + i (2u' - 1), u = U(seed, stream, 2e),
 * u' = U(seed, stream, 2e + 1), e = offset + i * n_s + k, where
 * U(s, st, j) = (h >> 11) 2^-53, h = f(f(s + G (st + 1)) + G (j + 1)),
 * G = 0x9E3779B97F4A7C15 and f is the SplitMix64 finaliser (Steele, Lea and
 * Flood 2014).  Streams: 1 initial block, 3 refill. */
int chebfd_random_block(chebfd_ctx *ctx, int precision, void *X, int64_t n, int64_t n_s,
                        int64_t ld, int64_t k0, int64_t m, uint64_t seed, uint64_t stream,
                        uint64_t offset);

/* Converts a block between c128 and c64 (round to nearest). */
int chebfd_convert(chebfd_ctx *ctx, int prec_in, const void *X, int prec_out, void *Y,
                   int64_t n, int64_t n_s, int64_t ld_in, int64_t ld_out);

/* Stochastic KPM moments of the density of states (Sec. 3.1 steps 1-2):
 * mu_m = (1/(N R)) sum_r <x_r, T_m(alpha H + beta) x_r>, m = 0..n_mom-1,
 * with R = n_vec random-phase vectors x_r (entries e^{2 pi i u}, u from
 * stream 2), computed in `precision` with n_mom/2 fused steps (doubling).
 * out: host, n_mom doubles.  a, b: spectral interval.  Synchronises. */
int chebfd_kpm_moments(chebfd_ctx *ctx, const chebfd_matrix *H, int precision, int n_vec,
                       int n_mom, uint64_t seed, double a, double b, double *out);

/* Launch configuration of the fused filter step for this context:
 *   "lanes"       lanes sharing one row (SELL) or site (stencil): 16, 32, 64,
 *                 0 = default (32; 16 for blocks of at most 16 packs; 64,
 *                 a whole wave per site, for the matrix-free step in
 *                 complex64 with more than 32 packs);
 *   "nontemporal" 1 (default) = streamed blocks w, x bypass cache retention;
 *   "order"       matrix-free lattice only: -1 (default) = automatic: the
 *                 tiled lattice order when, column-slab major, the bytes
 *                 moved between a site's gather as a z-neighbour from above
 *                 and from below (two lattice planes of the five block
 *                 streams over one slab) exceed the 256 MB memory-side
 *                 cache, column-slab major otherwise; 0 = column-slab major
 *                 with sites in lattice order; 1 = tiled lattice order
 *                 (strips of "tile" x-columns, z fastest inside a column,
 *                 one strip per XCD group);
 *   "tile"        strip width of the tiled lattice order, in sites along x:
 *                 -1 (default) = 4 for the matrix-free step, 2 for SELL,
 *                 used where the tiled order pays (above);
 *                 a positive value also makes every SELL matrix built by
 *                 chebfd_matrix_ti on this context take the tiled row order
 *                 (the chunk composition of SELL-C-sigma); 0 = never tiled;
 *   "pair_rows"   SELL matrices built on this context: 1 (default) = inside
 *                 each chunk, rows whose entries gather the same columns at
 *                 the same positions are placed in adjacent slots (one wave
 *                 instruction), 0 = length-sorted order only;
 *   "slabs"       SELL only: column slabs (32 lanes x 16 bytes) a workgroup
 *                 runs on one staging of its row block's index and value
 *                 stream; 0 (default) = all slabs of the block, so the
 *                 matrix is read from memory once per launch;
 *   "row_group"   SELL matrices built on this context: -1 (default) = the
 *                 row-group layout where it saves at least a quarter of the
 *                 gathers, trying groups of 4 rows, then 2 (each group of
 *                 consecutive slots stores the union of its rows' columns
 *                 once with one value per row and entry, and one lane
 *                 applies every gathered row to all rows of its group);
 *                 2 or 4 = that group size whenever every union fits the
 *                 32-entry LDS stage; 1 = one row per slot (plain
 *                 SELL-C-sigma);
 *   "xcd_group"   consecutive workgroups placed on one of the 8 XCDs (each
 *                 with its own L2): 1 = hardware round-robin order, a power
 *                 of two up to 2^20, 0 = default (the workgroups of one SELL
 *                 chunk, or of one strip in a tiled order; stencil otherwise 1).
 * The filtered blocks are bitwise identical for every setting (each element
 * is computed by the same operations in the same order); moment sums may
 * differ in rounding; only speed changes.
 * Errors: INVALID_ARG for an unknown key or value. */
int chebfd_set_tuning(chebfd_ctx *ctx, const char *key, int value);

/* Spectral interval [a, b] of H from k steps of the Lanczos process, the
 * alternative to the Gershgorin bound for the scaling of Sec. 3.1 step 1.
 * Random start vector (stream 4 of `seed`), no reorthogonalisation; the
 * extreme Ritz values are widened by their residual bounds beta_k |s_k| and
 * by `pad` times the Ritz range, and clamped to the Gershgorin interval.
 * Not a rigorous enclosure: chebfd_solve checks its Rayleigh quotients
 * against the interval and falls back to Gershgorin if one lies outside.
 * Allocates 3 N complex128 of device memory for the call.  Synchronises.
 * Errors: INVALID_ARG (k outside [2, 1000], pad < 0), NONFINITE. */
int chebfd_lanczos_bounds(chebfd_ctx *ctx, const chebfd_matrix *H, int k, uint64_t seed,
                          double pad, double *a, double *b);

/* Attainable HBM bandwidth: gbs[0] the read-only reduction benchmark of
 * Sec. 4.1, gbs[1] a plain copy (bytes read + written), gbs[2] the fused
 * step's streams without the gather (read three blocks, write two:
 * w = 2u - w, x = x + w/2).  Each runs `reps` times over the caller-owned
 * device buffer `buf` (`bytes` long, 16-byte aligned, contents overwritten).
 * GB/s = 10^9 bytes/s.  Synchronises. */
int chebfd_bandwidth_probe(chebfd_ctx *ctx, void *buf, int64_t bytes, int reps, double *gbs);

/* Hermitian eigen-decomposition of a small dense matrix on the host
 * (Householder tridiagonalisation + implicit QL): A (n x n complex128,
 * row-major, host) is overwritten by the eigenvectors (columns), w receives
 * the eigenvalues in ascending order. */
int chebfd_host_eigh(int n, double *A, double *w);

/* ------------------------------------------------------------------ */
/* parameter choice from KPM moments, and the learned form            */
/* ------------------------------------------------------------------ */

/* Rule-based parameters from n_mom KPM moments mu (host, as returned by
 * chebfd_kpm_moments, normalised by N R) of an N x N matrix with spectral
 * interval [a, b] (Sec. 3.1 steps 1-3): the target count
 * N_T = N sum_m g_m c_m mu_m (Eq. DOS:target; Jackson damping, window
 * coefficients c_m of Eq. (W1)); N_S = max(16, ceil(ns_over_nt N_T)) rounded
 * to even and capped at ns_max; the search margin delta' from
 * N_S = N int_{I_S} rho (Eq. DOS:search), at least the KPM resolution
 * (b - a)/n_mom; and N_p minimising eta (Sec. 2.3) for that configuration
 * with the given kernel.  A positive *n_s on entry fixes N_S (the margin and
 * N_p then follow from it).  *margin (may be NULL) receives delta'.  This is
 * the fallback of the learned form. */
int chebfd_dos_params(const double *mu, int n_mom, int64_t n, double a, double b, double lam_lo,
                      double lam_hi, double ns_over_nt, int kernel, double mu_k, int ns_max,
                      double *n_t_est, int *n_s, int *n_p, double *margin);

/* Network inputs (n_mom + 2 floats, host): the moments followed by the window
 * edges in scaled units alpha lambda + beta. */
int chebfd_learned_features(const double *mu, int n_mom, double a, double b, double lam_lo,
                            double lam_hi, float *features);

/* Decodes network outputs (host, 2 + n_hat floats: log(N_p / np_ref),
 * log(N_S / ns_ref), hat amplitudes a_j; the ratios are bounded to 8 either
 * way and np_ref, ns_ref are the rule-based choice) into n_p, an even n_s in
 * [16, ns_max], and, if gamma_corr is not NULL, corr_len multiplicative
 * coefficient corrections corr_n = c_max tanh(sum_j a_j hat_j(n /
 * (corr_len - 1))) with n_hat equidistant piecewise-linear hats on [0, 1] (a
 * zero output reproduces the rule-based filter exactly). */
int chebfd_learned_decode(const float *out, int np_ref, int ns_ref, int n_hat, double c_max,
                          int ns_max, int *n_p, int *n_s, double *gamma_corr, int corr_len);

/* Fits hat amplitudes (amp: n_hat doubles, host) that minimise a smoothed
 * damping factor sigma (Sec. 2.3) of the corrected filter
 * sum_n gamma_n (1 + c_max tanh(sum_j a_j hat_j(n/n_p))) T_n for target
 * [t_lo, t_hi] and search interval [s_lo, s_hi] plus l2 |a|^2, by `iters`
 * Adam steps with the analytic gradient; sigma_out receives the smoothed
 * sigma reached.  Produces the correction targets the network is trained on. */
int chebfd_fit_corrections(double a, double b, double t_lo, double t_hi, double s_lo, double s_hi,
                           int n_p, int kernel, double mu_k, int n_hat, double c_max, int iters,
                           double l2, double *amp, double *sigma_out);

typedef struct chebfd_mlp chebfd_mlp;

/* Fully connected network n_in -> n_hidden (tanh) -> n_hidden (tanh) -> n_out
 * (linear) in FP32 on the device, Glorot-uniform weights from the counter
 * generator (stream 5 of `seed`), zero biases, output map y = raw scale +
 * shift (initially identity).  Parameters are one flat array: W1 [n_in][h],
 * b1, W2 [h][h], b2, W3 [h][n_out], b3. */
int chebfd_mlp_create(chebfd_ctx *ctx, int n_in, int n_hidden, int n_out, uint64_t seed,
                      chebfd_mlp **out);
int chebfd_mlp_destroy(chebfd_mlp *mlp);
int chebfd_mlp_num_params(const chebfd_mlp *mlp, int64_t *n);
/* Layer widths of a network (host outputs, any may be NULL). */
int chebfd_mlp_dims(const chebfd_mlp *mlp, int *n_in, int *n_hidden, int *n_out);
/* Copies parameters / output shift and scale (n_out each) to or from the host;
 * any pointer may be NULL.  Synchronises. */
int chebfd_mlp_get_params(chebfd_ctx *ctx, const chebfd_mlp *mlp, float *params, float *shift,
                          float *scale);
int chebfd_mlp_set_params(chebfd_ctx *ctx, chebfd_mlp *mlp, const float *params,
                          const float *shift, const float *scale);
/* Input standardisation x -> (x - shift)/scale applied before the first
 * layer (n_in floats each, host; identity at creation).  get = 1 copies the
 * current values out instead.  Synchronises. */
int chebfd_mlp_input_scaling(chebfd_ctx *ctx, chebfd_mlp *mlp, float *shift, float *scale,
                             int get);
/* Y = network(X) for `batch` rows (X: batch x n_in, Y: batch x n_out, device,
 * row-major). */
int chebfd_mlp_forward(chebfd_ctx *ctx, chebfd_mlp *mlp, const float *X_dev, int batch,
                       float *Y_dev);
/* Mean-squared error between the raw outputs and the standardised targets
 * (T - shift)/scale, and its gradient w.r.t. every parameter (host, may be
 * NULL).  Synchronises. */
int chebfd_mlp_loss_grad(chebfd_ctx *ctx, chebfd_mlp *mlp, const float *X_dev,
                         const float *T_dev, int batch, float *loss, float *grad);
/* One Adam step (beta 0.9/0.999, eps 1e-8, decoupled weight decay) on the
 * loss above; `loss` (host, may be NULL) receives the pre-step loss. */
int chebfd_mlp_train_step(chebfd_ctx *ctx, chebfd_mlp *mlp, const float *X_dev,
                          const float *T_dev, int batch, float lr, float weight_decay,
                          float *loss);

/* The learned parameter choice for the window [lam_lo, lam_hi] of H in
 * the spectral interval [a, b], end to end on the device and the host
 * (Sec. 3.1 steps 1-3 with the network in place of the rule):
 *   1. max(n_mom, n_mom_rule) stochastic KPM moments from n_vec
 *      random-phase vectors (chebfd_kpm_moments, complex64, stream 2 of
 *      `seed`; n_vec rounded up to even);
 *   2. the rule-based choice from all of them (chebfd_dos_params with
 *      ns_over_nt, Lanczos kernel mu = 2, ns_max), returned in *np_rule,
 *      *ns_rule (may be NULL); a positive *n_s on entry fixes N_S (the rule
 *      then gives N_p for it and the network's N_S output is ignored);
 *   3. the network `mlp` (n_mom + 2 inputs from chebfd_learned_features
 *      on the first n_mom moments, 2 + n_hat outputs) on the context's
 *      stream;
 *   4. chebfd_learned_decode into *n_p, *n_s and the corrections corr_n,
 *      n = 0..n_p (amplitude c_max);
 *   5. with gate != 0 the corrections are kept only if they lower the
 *      damping factor sigma (Sec. 2.3) of the Lanczos-kernel filter of
 *      degree *n_p for the search interval the rule gives at *n_s; else (or
 *      for a zero network output) gamma_corr is all zero, which is exactly
 *      the plain method (the fallback).  *corr_kept (may be NULL) says which.
 * gamma_corr (host, may be NULL) receives *n_p + 1 doubles, to pass as
 * chebfd_params.gamma_corr; if corr_cap < *n_p + 1 the call returns
 * CHEBFD_ERR_WORKSPACE with *n_p and *n_s already set.  Allocates a few
 * hundred bytes of device memory and the moment blocks (3 N n_vec complex64)
 * for the call.  Synchronises.  Errors: INVALID_ARG (network shape, sizes),
 * WORKSPACE, HIP. */
int chebfd_learned_params(chebfd_ctx *ctx, const chebfd_matrix *H, chebfd_mlp *mlp, double a,
                          double b, double lam_lo, double lam_hi, int n_vec, int n_mom,
                          int n_mom_rule, uint64_t seed, double ns_over_nt, int n_hat,
                          double c_max, int ns_max,
                          int gate, int *n_p, int *n_s, double *gamma_corr, int corr_cap,
                          int *corr_kept, int *np_rule, int *ns_rule);

/* ------------------------------------------------------------------ */
/* the ChebFD solver (Sec. 3.1 steps 1-8)                              */
/* ------------------------------------------------------------------ */

typedef struct {
    double lam_lo, lam_hi;   /* target window I_T */
    int n_s;                 /* search vectors N_S */
    int n_p;                 /* filter degree N_p (>= 2) */
    int kernel;              /* CHEBFD_KERNEL_* */
    double mu;               /* Lanczos exponent */
    double eps;              /* residual goal */
    int max_iter;            /* outer iterations */
    int precision;           /* CHEBFD_PREC_C128, or C64 (FP32 sweep + FP64 polish) */
    int lock;                /* lock converged pairs (1) or not (0) */
    double a, b;             /* spectral interval; NaN = Gershgorin of H */
    uint64_t seed;           /* initial block: stream 1 of this seed */
    const double *gamma_corr; /* NULL or host array of n_p + 1 multiplicative
                                 corrections: gamma_n <- gamma_n (1 + corr_n) */
    double polish_switch;    /* C64 only: go to FP64 once every in-window
                                residual below sqrt(eps) is below this, or
                                their median is below half of it, or their
                                median stops halving with no new pair below
                                sqrt(eps); NaN = 8 * 2^-23 * S_w
                                (S_w = max(|a|, |b|)).  The FP64 polish then
                                filters only the in-window Ritz vectors and
                                the nearest ones outside the window
                                (max(n_in + 8, 5 n_in / 4) columns). */
    int vectors;             /* 1: copy the eigenvectors to the host result */
    int verbose;             /* 1: progress on stderr: one line per outer
                                iteration and per 1024 filter steps */
    int bounds;              /* with a = b = NaN: 0 Gershgorin interval, k > 0
                                Lanczos bounds with k steps (pad 0.01, start
                                vector from `seed`), checked against every
                                Rayleigh quotient with a fallback to
                                Gershgorin */
    int adapt;               /* 1: re-select the degree after the first filter
                                pass from the density of states that pass
                                measures (the 2 n_p + 1 Chebyshev moments of
                                the random start block, Sec. 4): N_T by Eq.
                                DOS:target, the search margin for n_s by Eq.
                                DOS:search, then the eta-minimising n_p
                                (Sec. 2.3-2.4) for the remaining iterations
                                (gamma_corr is then dropped).  0 (default):
                                keep n_p.  The moment partial sums use the
                                context's scratch memory. */
    int harmonic;            /* 1 (with lock = 1): step 7 extracts harmonic
                                Ritz pairs for the target at the window centre
                                (the refinement of the step 7 remarks and
                                Sec. 6) instead of Ritz pairs: the Petrov-
                                Galerkin pairs of (H - tau) against
                                (H - tau) X, ranked by their Rayleigh
                                quotients; converged ones are locked as an
                                orthonormal basis with the Ritz pairs of H
                                inside it.  One more Gram (of H X) per
                                iteration.  0 (default): Ritz pairs. */
    int polish;              /* C64 only, after the sweep:
                                CHEBFD_POLISH_CORRECTION (default) filters in
                                FP32 with FP64 accuracy: for a Ritz pair
                                (theta, v), with y = alpha x + beta and
                                t = alpha theta + beta, p(y) = p(t) + (y - t)
                                q_t(y) gives p(H~) v = p(t) v + q_t(H~) r,
                                r = (H~ - t) v (formed in FP64), and only
                                q_t(H~) r -- of the size of the residual --
                                is filtered in complex64, column j with the
                                coefficients of its own q_t
                                (chebfd_coeffs_divided); a pass that stops
                                reducing the residuals hands over to FP64
                                passes.  CHEBFD_POLISH_FP64: FP64 filter
                                passes throughout the polish. */
} chebfd_params;

typedef struct {
    int iterations;          /* outer iterations (all phases) */
    int iterations_c64;      /* of which in the FP32 sweep */
    int n_found;
    int n_locked;
    int refilled;            /* random columns added by orthogonalisation */
    int64_t n_mvm;           /* sum over iterations of active columns * n_p */
    double a, b;
    double t_total, t_filter, t_ortho, t_rr;   /* seconds */
    double max_residual;
    int n_p_used;            /* filter degree of the last iteration */
    double n_t_estimate;     /* adapt = 1: KPM count of the window (Eq.
                                DOS:target) from the first pass; else 0 */
    int iterations_corr;     /* FP32 correction passes of the polish */
} chebfd_stats;

/* Fills `p` with defaults: Lanczos kernel mu = 2, eps 1e-9, max_iter 50, C128,
 * lock 1, a = b = NaN, seed 1, polish_switch NaN, vectors 1, verbose 0,
 * bounds 0, n_s 32, n_p 200. */
int chebfd_params_default(chebfd_params *p);

/* Device workspace (bytes) chebfd_solve needs for this matrix and params. */
int chebfd_solve_workspace_size(const chebfd_matrix *H, const chebfd_params *p, int64_t *bytes);

/* Runs the ChebFD scheme on H with a caller-provided device workspace of at
 * least chebfd_solve_workspace_size bytes (256-byte aligned).  Converged
 * in-window pairs (residual <= eps on H in FP64) are returned in a result
 * handle, ascending in lambda.  Returns 0, NOT_CONVERGED (max_iter reached;
 * the pairs converged so far are returned), SEARCH_SPACE_TOO_SMALL (every
 * search vector ended up converged in the window, so the window may hold
 * more), or an error (INVALID_ARG, WORKSPACE, HIP, NONFINITE). */
int chebfd_solve(chebfd_ctx *ctx, const chebfd_matrix *H, const chebfd_params *p,
                 void *workspace, int64_t workspace_bytes, chebfd_result **out);

/* Pointers into the result (host memory owned by the result): n_found
 * eigenvalues, residuals, and eigenvectors as an N x n_found row-major c128
 * block.  Any output may be NULL. */
int chebfd_result_get(const chebfd_result *r, int64_t *n_found, const double **evals,
                      const double **residuals, const double **evecs, chebfd_stats *stats);
int chebfd_result_destroy(chebfd_result *r);

/* Convergence history, one entry per outer iteration (Sec. 3.1 step 8):
 * the matrix-vector products so far (sum of active columns times n_p), the
 * phase's precision, the pairs locked before the iteration, the in-window
 * Ritz pairs with residual <= eps (converged) and <= sqrt(eps) (accepted,
 * i.e. not ghosts) and all in-window pairs of the block, the smallest residual of an in-window Ritz pair and the
 * largest residual of an accepted or locked one (NaN if none).  After a
 * restart on the Gershgorin interval the history is the restarted run's. */
typedef struct {
    int64_t n_mvm;
    int precision;           /* CHEBFD_PREC_C128 (FP64 pass), C64 (FP32
                                sweep) or C64_CORRECTION (FP32 correction
                                pass of the polish) */
    int n_locked;
    int n_converged;
    int n_accepted;
    int n_window;            /* in-window Ritz pairs of the block (accepted
                                ones and ghosts) */
    double r_min;
    double r_max_accepted;
} chebfd_iter_info;

int chebfd_result_history(const chebfd_result *r, int64_t *n, const chebfd_iter_info **history);

/* Precision form (CHEBFD_PREC_C64): the result of the complex64 sweep
 * before the FP64 polish -- the in-window Ritz values of its last iteration
 * (Rayleigh-Ritz in FP64 on the FP32-filtered block) whose residual
 * ||Hv - theta v|| was at most sqrt(eps), ascending, with those residuals.
 * n = 0 for complex128 solves.  Pointers into the result, owned by it. */
int chebfd_result_sweep(const chebfd_result *r, int64_t *n, const double **evals,
                        const double **residuals);

#ifdef __cplusplus
}
#endif
#endif
