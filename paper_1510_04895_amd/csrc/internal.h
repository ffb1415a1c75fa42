// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/chebfd.h"

namespace chebfd {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

#define CHEBFD_HIP(call)                                                              \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return ::chebfd::fail(CHEBFD_ERR_HIP, std::string(#call ": ") +            \
                                                      hipGetErrorString(e_));         \
    } while (0)

#define CHEBFD_CHECK_LAUNCH()                                                         \
    do {                                                                              \
        hipError_t e_ = hipGetLastError();                                            \
        if (e_ != hipSuccess)                                                         \
            return ::chebfd::fail(CHEBFD_ERR_HIP, std::string("kernel launch: ") +     \
                                                      hipGetErrorString(e_));         \
    } while (0)

// ---------------------------------------------------------------- handles
// Entries per row (or row pair) the SELL kernels stage in LDS; longer rows
// read the index stream directly (single rows) or keep the plain layout
// (pairs).
constexpr int kStageLen = 32;

struct Sell {
    int64_t n = 0;           // rows
    int C = 32;              // chunk height
    int sigma = 256;         // sorting window
    int64_t nchunks = 0;
    int64_t nnz = 0;         // stored entries without padding
    int64_t stored = 0;      // stored entries with padding
    int max_len = 0;         // longest row
    // device arrays
    int64_t *chunk_ptr = nullptr;   // nchunks + 1, offset of chunk c's first slot
    int32_t *chunk_len = nullptr;   // nchunks, padded width of chunk c
    int32_t *perm = nullptr;        // nchunks*C: original row of slot (or -1)
    int32_t *col = nullptr;         // stored
    double *val64 = nullptr;        // stored complex128 (interleaved)
    float *val32 = nullptr;         // stored complex64
    // Row groups (group = G > 1): slots G q .. G q + G - 1 of a chunk form
    // group q (C/G groups per chunk); a group stores the union of its rows'
    // columns once, with G values per entry (zero where a row has no
    // entry), entry j of group q at chunk_ptr[c] + j*C/G + q; val64/val32
    // then hold G complex values per stored entry and chunk_len is the
    // widest union of the chunk.  group = 1: plain SELL-C-sigma.
    int group = 1;
    // rows per locality group of the chunk order (one strip of a tiled
    // lattice numbering; 0 = none): the workgroups of one group share an XCD
    int64_t group_rows = 0;
};

struct Stencil {
    int L[3] = {0, 0, 0};
    int pbc = 0;
    double t = 1.0, m = 2.0;
    double *pot64 = nullptr;  // per-site potential V_n (device)
    float *pot32 = nullptr;
};

}  // namespace chebfd

struct chebfd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // persistent small device scratch (partial sums, small matrices)
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    double *pinned = nullptr;       // host pinned staging for small results
    size_t pinned_bytes = 0;
    int num_cu = 256;
    // launch configuration of the fused step (chebfd_set_tuning)
    int tune_lpr = 0;     // lanes per row/site: 0 = default (32), 16, 32, 64
    int tune_nt = 1;      // non-temporal hint on the streamed blocks w, x
    int tune_order = -1;  // matrix-free step: -1 automatic, 0 slab-major, 1 tiled lattice order
    int tune_pair_rows = 1; // SELL build: pair rows with equal gather columns in a chunk
    int tune_slabs = 0;     // SELL: column slabs per workgroup (0 = default)
    int tune_row_group = -1; // SELL build: row-group layout, -1 where it pays, 2/4 whenever it fits, 1 never
    int tune_xcd_group = 0; // consecutive workgroups per XCD: 0 = default, 1 = hardware order
    int tune_tile = -1;     // strip width (sites along x) of the tiled lattice order: -1 default, 0 off
};

struct chebfd_matrix {
    int storage = CHEBFD_STORAGE_SELL;
    int64_t n = 0;
    double g_lo = 0.0, g_hi = 0.0;  // Gershgorin interval
    chebfd::Sell sell;
    chebfd::Stencil st;
    int device = 0;
};

namespace chebfd {

// scratch management (grows on demand; synchronises the stream before growing)
int default_tile(const chebfd_ctx *ctx, bool sell);
bool tiled_order_pays(const int L[3], int64_t slab_row);
int ensure_scratch(chebfd_ctx *ctx, size_t bytes);
int ensure_pinned(chebfd_ctx *ctx, size_t bytes);

// ---------------------------------------------------------------- kernels
// Step modes of the fused kernel.
enum StepMode { MODE_APPLY = 0, MODE_SECOND = 1, MODE_STEP = 2 };

struct StepArgs {
    int mode;
    int precision;
    const void *u;     // gathered block
    const void *wold;  // subtracted block (MODE_SECOND: x, MODE_STEP: w)
    void *wout;        // written block
    void *y;           // accumulated block (MODE_SECOND: x, MODE_STEP: x)
    int64_t n, n_s, ld;
    double s_h, s_u;   // w = s_h H u + s_u u (- wold)
    double g0, g1, g2; // MODE_SECOND: y = g0 x + g1 u + g2 w; MODE_STEP: y += g0 w
    double *partials;  // moment partial sums, or nullptr
    // per-column coefficients in place of g0..g2, or nullptr: row r of the
    // device table at gcol + r * ldg holds one coefficient per column
    // (MODE_SECOND reads rows 0..2, MODE_STEP row 0)
    const double *gcol;
    int64_t ldg;
};

// Launch shape of the matrix-free step (order 0 column-slab major, 1 tiled
// with strips of tile x-columns; nblk workgroups per slab).
struct TiShape {
    int order = 0, tile = 1;
    int64_t bpr = 0, nblk = 0;
};
TiShape ti_shape(const chebfd_ctx *ctx, const Stencil &S, int64_t n_s, int elem, int nb, int lps);
int pick_lpr(const chebfd_ctx *ctx, int64_t n_s, int nb, bool stencil);

// Launches one fused step; returns number of partial-sum rows written
// (per column triples) in *n_part when partials != nullptr.
int launch_step(chebfd_ctx *ctx, const chebfd_matrix *H, const StepArgs &a, int64_t *n_part);
// Number of per-workgroup moment partial rows one step launch writes.
int64_t step_partial_blocks(const chebfd_ctx *ctx, const chebfd_matrix *H, int precision,
                            int64_t n_s);

// Sums the moment partials of one step into the moment array.
int launch_moment_finalize(chebfd_ctx *ctx, const double *partials, int64_t n_part,
                           int64_t n_s, int mode, int step, double *mom);

int launch_gram(chebfd_ctx *ctx, int prec, const void *A, int64_t lda, int64_t n_a,
                const void *B, int64_t ldb, int64_t n_b, int64_t n, double *S_dev);
int launch_block_times(chebfd_ctx *ctx, int prec_a, const void *A, int64_t lda, int64_t n,
                       int64_t k, const double *T_dev, int64_t m, int prec_c, void *C,
                       int64_t ldc, int c_beta);
int launch_residuals(chebfd_ctx *ctx, int prec, const void *V, const void *HV, int64_t n,
                     int64_t m, int64_t ld, const double *theta_dev, double *res_dev);
int launch_random(chebfd_ctx *ctx, int prec, void *X, int64_t n, int64_t n_s, int64_t ld,
                  int64_t k0, int64_t m, uint64_t seed, uint64_t stream, uint64_t offset);
int launch_convert(chebfd_ctx *ctx, int prec_in, const void *X, int prec_out, void *Y,
                   int64_t n, int64_t n_s, int64_t ld_in, int64_t ld_out);
// Correction pass of the precision form: R = f32(HV - V diag(t)) with zero
// columns k .. kk-1 (V, HV complex128, ld_v; R complex64, ld_r), and
// V = V diag(p) + f64(D) (D complex64, ld_d).
int launch_defect(chebfd_ctx *ctx, const void *V, const void *HV, const double *t_dev, void *R,
                  int64_t n, int64_t k, int64_t kk, int64_t ld_v, int64_t ld_r);
int launch_combine(chebfd_ctx *ctx, void *V, const void *D, const double *p_dev, int64_t n,
                   int64_t k, int64_t ld_v, int64_t ld_d);
int launch_phase_block(chebfd_ctx *ctx, int prec, void *X, int64_t n, int64_t n_s,
                       int64_t ld, uint64_t seed, uint64_t stream);
int launch_bandwidth_probe(chebfd_ctx *ctx, void *buf, int64_t bytes, int reps, double *gbs);
int launch_expand_T(chebfd_ctx *ctx, const double *T, int64_t k, int64_t m, double *Tr);
int launch_gather_cols(chebfd_ctx *ctx, int prec, const void *src, int64_t lds, void *dst,
                       int64_t ldd, int64_t d0, const int32_t *idx_dev, int64_t n, int64_t m);
// The filter of Fig. fig:ChebFD; with mom != nullptr the moment partial sums
// go to `partials` (moment_partial_bytes long) or, if that is nullptr, to the
// context's grow-only scratch.
// With gcol != nullptr column j is filtered with its own coefficients
// gcol[n * ldg + j], n = 0..n_p (a device table), and gamma is not read.
int filter_apply(chebfd_ctx *ctx, const chebfd_matrix *H, int prec, const double *gamma, int n_p,
                 double a, double b, void *X, void *U, void *W, int64_t n_s, int64_t ld,
                 double *mom, int progress = 0, double *partials = nullptr,
                 const double *gcol = nullptr, int64_t ldg = 0);
size_t moment_partial_bytes(const chebfd_ctx *ctx, const chebfd_matrix *H, int prec, int64_t n_s);
int check_filter_args(const char *who, chebfd_ctx *ctx, const chebfd_matrix *H, int precision,
                      const double *gamma, int n_p, double a, double b, void *X, void *U,
                      void *W, int64_t n_s, int64_t ld);
// Locates the allocation-free entry point's device array on `device` (the
// current device); called once per device by chebfd_create.
int noalloc_setup(int device);
int check_block(const char *who, int precision, const void *p, int64_t n, int64_t n_s,
                int64_t ld, bool packed);
// Lanczos spectral bounds (lanczos.cpp); V3 = n x 3 c128 scratch (ld 3),
// S_dev 2 doubles, T_dev 4 doubles of device scratch.
int lanczos_bounds(chebfd_ctx *ctx, const chebfd_matrix *H, int k, uint64_t seed, double pad,
                   void *V3, double *S_dev, double *T_dev, double *a_out, double *b_out);

// ---------------------------------------------------------------- host math
void window_coeffs(double lo, double hi, double a, double b, int n_p, double *c);
void damping(int kernel, int n_p, double mu, double *g);
double poly_value(const double *gamma, int n_p, double a, double b, double x);
// coefficients d[0 .. N-1] of (p(y) - p(t)) / (y - t) for p = sum c_n T_n
// (degree N, scaled variable); returns p(t)
double cheb_divide(const double *c, int N, double t, double *d);
void quality(const double *gamma, int n_p, double a, double b, double t_lo, double t_hi,
             double s_lo, double s_hi, double *sigma, double *eta);
int herm_eig(int n, std::vector<double> &A /* 2*n*n, overwritten by vectors */,
             std::vector<double> &w);
int chol_inv_factor(int n, const std::vector<double> &S, std::vector<double> &T);

// host-side random numbers (same definition as the device kernels)
uint64_t mix64(uint64_t z);
double u01(uint64_t seed, uint64_t stream, uint64_t index);

}  // namespace chebfd
