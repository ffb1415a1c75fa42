// C ABI: contexts, errors, and the low-level device entry points.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace chebfd {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg)
{
    set_error(msg);
    return code;
}

int ensure_scratch(chebfd_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->scratch_bytes) return CHEBFD_OK;
    if (ctx->scratch) {
        CHEBFD_HIP(hipStreamSynchronize(ctx->stream));
        CHEBFD_HIP(hipFree(ctx->scratch));
        ctx->scratch = nullptr;
        ctx->scratch_bytes = 0;
    }
    size_t sz = bytes + bytes / 4 + 4096;
    if (hipMalloc(&ctx->scratch, sz) != hipSuccess) {
        ctx->scratch = nullptr;
        return fail(CHEBFD_ERR_OOM, "device scratch allocation failed");
    }
    ctx->scratch_bytes = sz;
    return CHEBFD_OK;
}

int ensure_pinned(chebfd_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->pinned_bytes) return CHEBFD_OK;
    if (ctx->pinned) {
        CHEBFD_HIP(hipStreamSynchronize(ctx->stream));
        CHEBFD_HIP(hipHostFree(ctx->pinned));
        ctx->pinned = nullptr;
        ctx->pinned_bytes = 0;
    }
    size_t sz = bytes + 4096;
    if (hipHostMalloc((void **)&ctx->pinned, sz, hipHostMallocDefault) != hipSuccess) {
        ctx->pinned = nullptr;
        return fail(CHEBFD_ERR_OOM, "pinned host allocation failed");
    }
    ctx->pinned_bytes = sz;
    return CHEBFD_OK;
}

uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

double u01(uint64_t seed, uint64_t stream, uint64_t index)
{
    const uint64_t G = 0x9E3779B97F4A7C15ULL;
    const uint64_t key = mix64(seed + G * (stream + 1u));
    return (double)(mix64(key + G * (index + 1u)) >> 11) * 0x1.0p-53;
}

// Validation shared by the block entry points.
int check_block(const char *who, int precision, const void *p, int64_t n, int64_t n_s,
                int64_t ld, bool packed)
{
    if (precision != CHEBFD_PREC_C128 && precision != CHEBFD_PREC_C64)
        return fail(CHEBFD_ERR_INVALID_ARG, std::string(who) + ": unknown precision");
    if (!p) return fail(CHEBFD_ERR_INVALID_ARG, std::string(who) + ": NULL block");
    if (n < 1 || n_s < 1 || ld < n_s)
        return fail(CHEBFD_ERR_INVALID_ARG, std::string(who) + ": need n >= 1, 1 <= n_s <= ld");
    if (packed && precision == CHEBFD_PREC_C64 &&
        ((ld & 1) || (n_s & 1) || ((uintptr_t)p & 15)))
        return fail(CHEBFD_ERR_INVALID_ARG,
                    std::string(who) + ": c64 blocks need even ld and n_s and 16-byte alignment");
    if (packed && precision == CHEBFD_PREC_C128 && ((uintptr_t)p & 15))
        return fail(CHEBFD_ERR_INVALID_ARG, std::string(who) + ": c128 blocks need 16-byte alignment");
    if ((uintptr_t)p & 7)
        return fail(CHEBFD_ERR_INVALID_ARG, std::string(who) + ": blocks need 8-byte alignment");
    return CHEBFD_OK;
}

size_t moment_partial_bytes(const chebfd_ctx *ctx, const chebfd_matrix *H, int prec, int64_t n_s)
{
    return (size_t)step_partial_blocks(ctx, H, prec, n_s) * (size_t)n_s * 3 * sizeof(double);
}

// Argument checks of chebfd_filter_apply (shared with its allocation-free
// variant).
int check_filter_args(const char *who, chebfd_ctx *ctx, const chebfd_matrix *H, int precision,
                      const double *gamma, int n_p, double a, double b, void *X, void *U,
                      void *W, int64_t n_s, int64_t ld)
{
    if (!ctx || !H || !gamma) return fail(CHEBFD_ERR_INVALID_ARG, std::string(who) + ": NULL argument");
    if (n_p < 2) return fail(CHEBFD_ERR_INVALID_ARG, std::string(who) + ": n_p must be >= 2");
    if (!(a < b) || !std::isfinite(a) || !std::isfinite(b))
        return fail(CHEBFD_ERR_INVALID_ARG, std::string(who) + ": need finite a < b");
    int rc;
    if ((rc = check_block(who, precision, X, H->n, n_s, ld, true)) ||
        (rc = check_block(who, precision, U, H->n, n_s, ld, true)) ||
        (rc = check_block(who, precision, W, H->n, n_s, ld, true)))
        return rc;
    if (X == U || X == W || U == W)
        return fail(CHEBFD_ERR_INVALID_ARG, std::string(who) + ": X, U, W must be distinct");
    for (int k = 0; k <= n_p; ++k)
        if (!std::isfinite(gamma[k]))
            return fail(CHEBFD_ERR_NONFINITE, std::string(who) + ": non-finite coefficient");
    return CHEBFD_OK;
}

// The polynomial filter (Fig. fig:ChebFD) on caller buffers.
int filter_apply(chebfd_ctx *ctx, const chebfd_matrix *H, int prec, const double *gamma, int n_p,
                 double a, double b, void *X, void *U, void *W, int64_t n_s, int64_t ld,
                 double *mom, int progress, double *partials, const double *gcol, int64_t ldg)
{
    const double alpha = 2.0 / (b - a), beta = (a + b) / (a - b);
    double *part = partials;
    int64_t n_part = 0;
    if (mom && !part) {
        // partial sums: one row of 3 per column per workgroup row block
        int rc = ensure_scratch(ctx, moment_partial_bytes(ctx, H, prec, n_s));
        if (rc) return rc;
        part = (double *)ctx->scratch;
    }
    StepArgs s{};
    s.precision = prec;
    s.n = H->n;
    s.n_s = n_s;
    s.ld = ld;
    s.partials = part;
    // u = (alpha H + beta) x
    s.mode = MODE_APPLY;
    s.u = X;
    s.wold = nullptr;
    s.wout = U;
    s.y = nullptr;
    s.s_h = alpha;
    s.s_u = beta;
    int rc = launch_step(ctx, H, s, &n_part);
    if (rc) return rc;
    if (mom && (rc = launch_moment_finalize(ctx, part, n_part, n_s, MODE_APPLY, 1, mom))) return rc;
    // w = 2 (alpha H + beta) u - x ;  x = g0 x + g1 u + g2 w
    s.mode = MODE_SECOND;
    s.u = U;
    s.wold = X;
    s.wout = W;
    s.y = X;
    s.s_h = 2.0 * alpha;
    s.s_u = 2.0 * beta;
    if (gcol) {
        s.gcol = gcol;
        s.ldg = ldg;
    } else {
        s.g0 = gamma[0];
        s.g1 = gamma[1];
        s.g2 = gamma[2];
    }
    if ((rc = launch_step(ctx, H, s, &n_part))) return rc;
    if (mom && (rc = launch_moment_finalize(ctx, part, n_part, n_s, MODE_SECOND, 2, mom))) return rc;
    void *u = U, *w = W;
    for (int k = 3; k <= n_p; ++k) {
        std::swap(u, w);
        s.mode = MODE_STEP;
        s.u = u;
        s.wold = w;
        s.wout = w;
        s.y = X;
        if (gcol) s.gcol = gcol + (int64_t)k * ldg;
        else s.g0 = gamma[k];
        if ((rc = launch_step(ctx, H, s, &n_part))) return rc;
        if (mom && (rc = launch_moment_finalize(ctx, part, n_part, n_s, MODE_STEP, k, mom)))
            return rc;
        if (progress > 0 && k % progress == 0 && k < n_p) {
            // progress of a long filter pass: the steps up to k have run
            CHEBFD_HIP(hipStreamSynchronize(ctx->stream));
            std::fprintf(stderr, "chebfd: filter step %d of %d done\n", k, n_p);
            std::fflush(stderr);
        }
    }
    return CHEBFD_OK;
}

}  // namespace chebfd

using namespace chebfd;

extern "C" {

const char *chebfd_version(void) { return "chebfd-gfx950 0.1"; }

const char *chebfd_last_error(void) { return g_last_error.c_str(); }

const char *chebfd_strerror(int code)
{
    switch (code) {
    case CHEBFD_OK: return "ok";
    case CHEBFD_ERR_INVALID_ARG: return "invalid argument";
    case CHEBFD_ERR_OOM: return "out of memory";
    case CHEBFD_ERR_HIP: return "HIP runtime error";
    case CHEBFD_ERR_NONFINITE: return "non-finite value";
    case CHEBFD_ERR_UNSUPPORTED: return "unsupported";
    case CHEBFD_ERR_WORKSPACE: return "workspace too small";
    case CHEBFD_WARN_NOT_CONVERGED: return "not converged (max_iter reached)";
    case CHEBFD_WARN_SEARCH_SPACE_TOO_SMALL: return "search space may be too small";
    default: return "unknown status";
    }
}

int chebfd_create(chebfd_ctx **out, int device, void *hip_stream)
{
    if (!out) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_create: out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
        return fail(CHEBFD_ERR_HIP, "chebfd_create: no HIP device");
    if (device < 0 || device >= count)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_create: device index out of range");
    CHEBFD_HIP(hipSetDevice(device));
    // the allocation-free entry point's device array, located once per device
    if (int rc = noalloc_setup(device)) return rc;
    auto *c = new chebfd_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->num_cu = prop.multiProcessorCount;
    *out = c;
    return CHEBFD_OK;
}

int chebfd_destroy(chebfd_ctx *ctx)
{
    if (!ctx) return CHEBFD_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
    return CHEBFD_OK;
}

int chebfd_synchronize(chebfd_ctx *ctx)
{
    if (!ctx) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_synchronize: NULL context");
    CHEBFD_HIP(hipStreamSynchronize(ctx->stream));
    return CHEBFD_OK;
}

int chebfd_filter_apply(chebfd_ctx *ctx, const chebfd_matrix *H, int precision,
                        const double *gamma, int n_p, double a, double b, void *X, void *U,
                        void *W, int64_t n_s, int64_t ld, double *moments_dev)
{
    int rc = check_filter_args("chebfd_filter_apply", ctx, H, precision, gamma, n_p, a, b, X, U,
                               W, n_s, ld);
    if (rc) return rc;
    CHEBFD_HIP(hipSetDevice(ctx->device));
    return filter_apply(ctx, H, precision, gamma, n_p, a, b, X, U, W, n_s, ld, moments_dev);
}

int chebfd_filter_apply_columns(chebfd_ctx *ctx, const chebfd_matrix *H, int precision,
                                const double *gcol, int64_t ldg, int n_p, double a, double b,
                                void *X, void *U, void *W, int64_t n_s, int64_t ld)
{
    static const char *who = "chebfd_filter_apply_columns";
    if (!ctx || !H || !gcol) return fail(CHEBFD_ERR_INVALID_ARG, std::string(who) + ": NULL argument");
    if (precision != CHEBFD_PREC_C64)
        return fail(CHEBFD_ERR_UNSUPPORTED, std::string(who) + ": complex64 only");
    if (n_p < 2) return fail(CHEBFD_ERR_INVALID_ARG, std::string(who) + ": n_p must be >= 2");
    if (ldg < n_s) return fail(CHEBFD_ERR_INVALID_ARG, std::string(who) + ": ldg < n_s");
    if (!(a < b) || !std::isfinite(a) || !std::isfinite(b))
        return fail(CHEBFD_ERR_INVALID_ARG, std::string(who) + ": need finite a < b");
    int rc;
    if ((rc = check_block(who, precision, X, H->n, n_s, ld, true)) ||
        (rc = check_block(who, precision, U, H->n, n_s, ld, true)) ||
        (rc = check_block(who, precision, W, H->n, n_s, ld, true)))
        return rc;
    if (X == U || X == W || U == W)
        return fail(CHEBFD_ERR_INVALID_ARG, std::string(who) + ": X, U, W must be distinct");
    CHEBFD_HIP(hipSetDevice(ctx->device));
    return filter_apply(ctx, H, precision, nullptr, n_p, a, b, X, U, W, n_s, ld, nullptr, 0,
                        nullptr, gcol, ldg);
}

int chebfd_spmm(chebfd_ctx *ctx, const chebfd_matrix *H, int precision, const void *X, void *Y,
                int64_t n_s, int64_t ld, double s_h, double s_u)
{
    if (!ctx || !H) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_spmm: NULL argument");
    int rc;
    if ((rc = check_block("chebfd_spmm", precision, X, H->n, n_s, ld, true)) ||
        (rc = check_block("chebfd_spmm", precision, Y, H->n, n_s, ld, true)))
        return rc;
    if (X == Y) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_spmm: X and Y must differ");
    CHEBFD_HIP(hipSetDevice(ctx->device));
    StepArgs s{};
    s.mode = MODE_APPLY;
    s.precision = precision;
    s.u = X;
    s.wout = Y;
    s.n = H->n;
    s.n_s = n_s;
    s.ld = ld;
    s.s_h = s_h;
    s.s_u = s_u;
    return launch_step(ctx, H, s, nullptr);
}

int chebfd_gram(chebfd_ctx *ctx, int precision, const void *A, int64_t lda, int64_t n_a,
                const void *B, int64_t ldb, int64_t n_b, int64_t n, double *S_dev)
{
    if (!ctx || !S_dev) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_gram: NULL argument");
    int rc;
    if ((rc = check_block("chebfd_gram", precision, A, n, n_a, lda, false)) ||
        (rc = check_block("chebfd_gram", precision, B, n, n_b, ldb, false)))
        return rc;
    CHEBFD_HIP(hipSetDevice(ctx->device));
    return launch_gram(ctx, precision, A, lda, n_a, B, ldb, n_b, n, S_dev);
}

int chebfd_block_times(chebfd_ctx *ctx, int prec_a, const void *A, int64_t lda, int64_t n,
                       int64_t k, const double *T_dev, int64_t m, int prec_c, void *C,
                       int64_t ldc, int c_beta)
{
    if (!ctx || !T_dev) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_block_times: NULL argument");
    int rc;
    if ((rc = check_block("chebfd_block_times", prec_a, A, n, k, lda, false)) ||
        (rc = check_block("chebfd_block_times", prec_c, C, n, m, ldc, false)))
        return rc;
    if (A == C) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_block_times: C must not overlap A");
    CHEBFD_HIP(hipSetDevice(ctx->device));
    // real expansion of T in the scratch area
    if ((rc = ensure_scratch(ctx, (size_t)4 * k * m * sizeof(double)))) return rc;
    double *Tr = (double *)ctx->scratch;
    if ((rc = launch_expand_T(ctx, T_dev, k, m, Tr))) return rc;
    return launch_block_times(ctx, prec_a, A, lda, n, k, Tr, m, prec_c, C, ldc, c_beta);
}

int chebfd_residual_norms(chebfd_ctx *ctx, int precision, const void *V, const void *HV,
                          int64_t n, int64_t m, int64_t ld, const double *theta, double *res)
{
    if (!ctx || !theta || !res) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_residual_norms: NULL argument");
    int rc;
    if ((rc = check_block("chebfd_residual_norms", precision, V, n, m, ld, false)) ||
        (rc = check_block("chebfd_residual_norms", precision, HV, n, m, ld, false)))
        return rc;
    CHEBFD_HIP(hipSetDevice(ctx->device));
    double *dev = nullptr;
    CHEBFD_HIP(hipMalloc((void **)&dev, 2 * m * sizeof(double)));
    rc = CHEBFD_OK;
    if (hipMemcpyAsync(dev, theta, m * sizeof(double), hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
        rc = fail(CHEBFD_ERR_HIP, "chebfd_residual_norms: upload failed");
    if (!rc) rc = launch_residuals(ctx, precision, V, HV, n, m, ld, dev, dev + m);
    if (!rc && hipMemcpyAsync(res, dev + m, m * sizeof(double), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess)
        rc = fail(CHEBFD_ERR_HIP, "chebfd_residual_norms: download failed");
    if (!rc && hipStreamSynchronize(ctx->stream) != hipSuccess)
        rc = fail(CHEBFD_ERR_HIP, "chebfd_residual_norms: synchronize failed");
    (void)hipFree(dev);
    return rc;
}

int chebfd_random_block(chebfd_ctx *ctx, int precision, void *X, int64_t n, int64_t n_s,
                        int64_t ld, int64_t k0, int64_t m, uint64_t seed, uint64_t stream,
                        uint64_t offset)
{
    if (!ctx) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_random_block: NULL context");
    int rc = check_block("chebfd_random_block", precision, X, n, n_s, ld, false);
    if (rc) return rc;
    if (k0 < 0 || m < 0 || k0 + m > n_s)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_random_block: columns out of range");
    CHEBFD_HIP(hipSetDevice(ctx->device));
    return launch_random(ctx, precision, X, n, n_s, ld, k0, m, seed, stream, offset);
}

int chebfd_convert(chebfd_ctx *ctx, int prec_in, const void *X, int prec_out, void *Y, int64_t n,
                   int64_t n_s, int64_t ld_in, int64_t ld_out)
{
    if (!ctx) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_convert: NULL context");
    int rc;
    if ((rc = check_block("chebfd_convert", prec_in, X, n, n_s, ld_in, false)) ||
        (rc = check_block("chebfd_convert", prec_out, Y, n, n_s, ld_out, false)))
        return rc;
    if (X == Y) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_convert: X and Y must differ");
    CHEBFD_HIP(hipSetDevice(ctx->device));
    return launch_convert(ctx, prec_in, X, prec_out, Y, n, n_s, ld_in, ld_out);
}

int chebfd_set_tuning(chebfd_ctx *ctx, const char *key, int value)
{
    if (!ctx || !key) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_set_tuning: NULL argument");
    const std::string k(key);
    if (k == "lanes" && (value == 0 || value == 16 || value == 32 || value == 64)) ctx->tune_lpr = value;
    else if (k == "nontemporal" && (value == 0 || value == 1)) ctx->tune_nt = value;
    else if (k == "order" && value >= -1 && value <= 1) ctx->tune_order = value;
    else if (k == "tile" && value >= -1 && value <= 256) ctx->tune_tile = value;
    else if (k == "pair_rows" && (value == 0 || value == 1)) ctx->tune_pair_rows = value;
    else if (k == "slabs" && value >= 0 && value <= 64) ctx->tune_slabs = value;
    else if (k == "row_group" && (value == -1 || value == 1 || value == 2 || value == 4))
        ctx->tune_row_group = value;
    else if (k == "xcd_group" && value >= 0 && value <= (1 << 20) && !(value & (value - 1)))
        ctx->tune_xcd_group = value;
    else return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_set_tuning: unknown key or value");
    return CHEBFD_OK;
}

int chebfd_bandwidth_probe(chebfd_ctx *ctx, void *buf, int64_t bytes, int reps, double *gbs)
{
    if (!ctx || !buf || !gbs || bytes < 4096 || reps < 1 || ((uintptr_t)buf & 15))
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_bandwidth_probe: invalid arguments");
    CHEBFD_HIP(hipSetDevice(ctx->device));
    return launch_bandwidth_probe(ctx, buf, bytes, reps, gbs);
}

int chebfd_kpm_moments(chebfd_ctx *ctx, const chebfd_matrix *H, int precision, int n_vec,
                       int n_mom, uint64_t seed, double a, double b, double *out)
{
    if (!ctx || !H || !out) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_kpm_moments: NULL argument");
    if (n_vec < 1 || n_mom < 4 || (n_mom & 1) || !(a < b) ||
        (precision == CHEBFD_PREC_C64 && (n_vec & 1)) ||
        (precision != CHEBFD_PREC_C64 && precision != CHEBFD_PREC_C128))
        return fail(CHEBFD_ERR_INVALID_ARG,
                    "chebfd_kpm_moments: need n_vec >= 1 (even for c64), even n_mom >= 4, a < b");
    CHEBFD_HIP(hipSetDevice(ctx->device));
    const int64_t n = H->n, es = precision == CHEBFD_PREC_C128 ? 16 : 8;
    const int n_p = n_mom / 2;
    const size_t blk = (size_t)n * n_vec * es;
    const size_t mom_bytes = (size_t)(2 * n_p + 1) * n_vec * sizeof(double);
    char *buf = nullptr;
    CHEBFD_HIP(hipMalloc((void **)&buf, 3 * blk + mom_bytes + 1024));
    void *X = buf, *U = buf + blk, *W = buf + 2 * blk;
    double *mom = (double *)(buf + 3 * blk);
    std::vector<double> gam(n_p + 1, 0.0);
    int rc = launch_phase_block(ctx, precision, X, n, n_vec, n_vec, seed, 2);
    if (!rc) rc = filter_apply(ctx, H, precision, gam.data(), n_p, a, b, X, U, W, n_vec, n_vec, mom);
    std::vector<double> h((size_t)(2 * n_p + 1) * n_vec);
    if (!rc && hipMemcpyAsync(h.data(), mom, mom_bytes, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess)
        rc = fail(CHEBFD_ERR_HIP, "chebfd_kpm_moments: download failed");
    if (!rc && hipStreamSynchronize(ctx->stream) != hipSuccess)
        rc = fail(CHEBFD_ERR_HIP, "chebfd_kpm_moments: synchronize failed");
    (void)hipFree(buf);
    if (rc) return rc;
    for (int m = 0; m < n_mom; ++m) {
        double s = 0.0;
        for (int r = 0; r < n_vec; ++r) s += h[(size_t)m * n_vec + r];
        out[m] = s / ((double)n * n_vec);
    }
    return CHEBFD_OK;
}

}  // extern "C"
