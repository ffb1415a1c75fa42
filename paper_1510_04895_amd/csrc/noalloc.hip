// Allocation-free form of chebfd_filter_apply for callers that cannot
// allocate device memory (code under HIP graph capture, serving loops).
//
// The only device memory chebfd_filter_apply allocates is the moment
// partial-sum buffer (one row of three doubles per column and per workgroup
// row block of a launch), which it keeps in the context's grow-only scratch.
// Here that buffer is a fixed file-scope device array.  Its device address is
// looked up once per device, when chebfd_create runs on that device; host code
// uses only that address (the array's name is a host-side stand-in that no
// kernel may receive).
#include <mutex>

#include "internal.h"

namespace chebfd {
namespace {

constexpr size_t kNoallocBytes = (size_t)64 << 20;

// Moment partial sums of chebfd_filter_apply_noalloc; every launch writes
// every partial row it later sums, so nothing needs clearing between calls.
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

}  // namespace

int noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(CHEBFD_ERR_UNSUPPORTED, "chebfd_create: device index beyond 63");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return CHEBFD_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(CHEBFD_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                        hipGetErrorString(e));
    g_scratch[device] = p;
    return CHEBFD_OK;
}

}  // namespace chebfd

using namespace chebfd;

extern "C" int chebfd_filter_apply_noalloc(chebfd_ctx *ctx, const chebfd_matrix *H,
                                           int precision, const double *gamma, int n_p, double a,
                                           double b, void *X, void *U, void *W, int64_t n_s,
                                           int64_t ld, double *moments_dev)
{
    int rc = check_filter_args("chebfd_filter_apply_noalloc", ctx, H, precision, gamma, n_p, a, b,
                               X, U, W, n_s, ld);
    if (rc) return rc;
    double *part = nullptr;
    if (moments_dev) {
        const size_t need = moment_partial_bytes(ctx, H, precision, n_s);
        if (need > kNoallocBytes)
            return fail(CHEBFD_ERR_INVALID_ARG,
                        "chebfd_filter_apply_noalloc: the moment partial sums need " +
                            std::to_string(need) + " bytes, more than the fixed " +
                            std::to_string(kNoallocBytes) + "-byte device buffer");
        void *p;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            p = (ctx->device >= 0 && ctx->device < kMaxDevices) ? g_scratch[ctx->device] : nullptr;
        }
        if (!p)
            return fail(CHEBFD_ERR_HIP,
                        "chebfd_filter_apply_noalloc: device buffer not located (chebfd_create)");
        part = static_cast<double *>(p);
    }
    CHEBFD_HIP(hipSetDevice(ctx->device));
    return filter_apply(ctx, H, precision, gamma, n_p, a, b, X, U, W, n_s, ld, moments_dev, 0,
                        part);
}
