// Small fully connected network (FP32) for the learned parameter choice:
// standardised inputs (x - in_shift)/in_scale ->
// n_in -> n_hidden (tanh) -> n_hidden (tanh) -> n_out (linear), trained with
// a mean-squared error on standardised targets and Adam.  Forward, backward
// and the optimiser step are the kernels below; every reduction (over the
// batch for weight gradients, over outputs for the loss) runs in a fixed
// order, so training is bitwise reproducible.
//
// Parameter layout (one flat float array): W1 [n_in][h], b1 [h],
// W2 [h][h], b2 [h], W3 [h][n_out], b3 [n_out]; row-major, y = x W + b.
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

struct chebfd_mlp {
    int n_in = 0, h = 0, n_out = 0;
    int64_t n_params = 0;
    int device = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;   // params, grads, Adam moments
    float *shift = nullptr, *scale = nullptr;                        // output affine map
    float *in_shift = nullptr, *in_scale = nullptr;                  // input standardisation
    float *xn = nullptr;                                             // standardised inputs
    // activations for up to cap_batch rows
    int cap_batch = 0;
    float *a1 = nullptr, *a2 = nullptr, *a3 = nullptr;   // layer outputs
    float *d1 = nullptr, *d2 = nullptr, *d3 = nullptr;   // gradients w.r.t. layer outputs
    float *loss = nullptr;
    int64_t step = 0;
};

namespace chebfd {
namespace {

struct Offsets {
    int64_t W1, b1, W2, b2, W3, b3, total;
};

Offsets offsets(int n_in, int h, int n_out)
{
    Offsets o;
    o.W1 = 0;
    o.b1 = o.W1 + (int64_t)n_in * h;
    o.W2 = o.b1 + h;
    o.b2 = o.W2 + (int64_t)h * h;
    o.W3 = o.b2 + h;
    o.b3 = o.W3 + (int64_t)h * n_out;
    o.total = o.b3 + n_out;
    return o;
}

// out[b][j] = act(sum_k in[b][k] W[k][j] + bias[j]); act: 0 identity, 1 tanh
__global__ void k_dense_fwd(const float *__restrict__ in, const float *__restrict__ W,
                            const float *__restrict__ bias, float *__restrict__ out, int B, int K,
                            int N, int act)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (j >= N || b >= B) return;
    float s = bias[j];
    const float *x = in + (int64_t)b * K;
    for (int k = 0; k < K; ++k) s = fmaf(x[k], W[(int64_t)k * N + j], s);
    out[(int64_t)b * N + j] = act ? tanhf(s) : s;
}

// din[b][k] = (sum_j dz[b][j] W[k][j]) * (1 - in[b][k]^2 if the input came
// from a tanh layer); dz is the gradient w.r.t. the pre-activation
__global__ void k_dense_bwd_in(const float *__restrict__ dz, const float *__restrict__ W,
                               const float *__restrict__ in, float *__restrict__ din, int B, int K,
                               int N, int in_is_tanh)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (k >= K || b >= B) return;
    float s = 0.0f;
    const float *d = dz + (int64_t)b * N;
    const float *w = W + (int64_t)k * N;
    for (int j = 0; j < N; ++j) s = fmaf(d[j], w[j], s);
    if (in_is_tanh) {
        const float a = in[(int64_t)b * K + k];
        s *= 1.0f - a * a;
    }
    din[(int64_t)b * K + k] = s;
}

// gW[k][j] = sum_b in[b][k] dz[b][j], gb[j] = sum_b dz[b][j] (fixed order)
__global__ void k_dense_bwd_w(const float *__restrict__ in, const float *__restrict__ dz,
                              float *__restrict__ gW, float *__restrict__ gb, int B, int K, int N)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;   // k == K: the bias row
    if (j >= N || k > K) return;
    float s = 0.0f;
    if (k < K) {
        for (int b = 0; b < B; ++b) s = fmaf(in[(int64_t)b * K + k], dz[(int64_t)b * N + j], s);
        gW[(int64_t)k * N + j] = s;
    } else {
        for (int b = 0; b < B; ++b) s += dz[(int64_t)b * N + j];
        gb[j] = s;
    }
}

// Standardised mean-squared error: loss = mean over (b, j) of
// (y - (t - shift_j)/scale_j)^2 ; dy = 2 (y - t_std) / (B N).  One block.
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ y, const float *__restrict__ t,
                                             const float *__restrict__ shift,
                                             const float *__restrict__ scale,
                                             float *__restrict__ dy, float *__restrict__ loss, int B,
                                             int N)
{
    __shared__ float red[256];
    const int tid = threadIdx.x;
    const int64_t total = (int64_t)B * N;
    const float inv = 1.0f / (float)total;
    float s = 0.0f;
    for (int64_t i = tid; i < total; i += 256) {
        const int j = (int)(i % N);
        const float ts = (t[i] - shift[j]) / scale[j];
        const float r = y[i] - ts;
        dy[i] = 2.0f * r * inv;
        s = fmaf(r, r, s);
    }
    red[tid] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) *loss = red[0] * inv;
}

// Adam with decoupled weight decay (on weights and biases alike).
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float wd, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    p[i] -= lr * (mh / (sqrtf(vh) + eps) + wd * p[i]);
}

// xn = (x - shift) / scale per input column
__global__ void k_standardise(const float *__restrict__ x, const float *__restrict__ shift,
                              const float *__restrict__ scale, float *__restrict__ xn, int B, int K)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)B * K) return;
    const int k = (int)(i % K);
    xn[i] = (x[i] - shift[k]) / scale[k];
}

// y = raw * scale + shift (inference outputs in target units)
__global__ void k_affine(float *__restrict__ y, const float *__restrict__ shift,
                         const float *__restrict__ scale, int B, int N)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)B * N) return;
    const int j = (int)(i % N);
    y[i] = y[i] * scale[j] + shift[j];
}

inline unsigned nb(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

int ensure_batch(chebfd_mlp *M, int B)
{
    if (B <= M->cap_batch) return CHEBFD_OK;
    for (float *q : {M->a1, M->a2, M->a3, M->d1, M->d2, M->d3, M->xn})
        if (q) (void)hipFree(q);
    const int cap = B;
    CHEBFD_HIP(hipMalloc((void **)&M->xn, (size_t)cap * M->n_in * 4));
    CHEBFD_HIP(hipMalloc((void **)&M->a1, (size_t)cap * M->h * 4));
    CHEBFD_HIP(hipMalloc((void **)&M->a2, (size_t)cap * M->h * 4));
    CHEBFD_HIP(hipMalloc((void **)&M->a3, (size_t)cap * M->n_out * 4));
    CHEBFD_HIP(hipMalloc((void **)&M->d1, (size_t)cap * M->h * 4));
    CHEBFD_HIP(hipMalloc((void **)&M->d2, (size_t)cap * M->h * 4));
    CHEBFD_HIP(hipMalloc((void **)&M->d3, (size_t)cap * M->n_out * 4));
    M->cap_batch = cap;
    return CHEBFD_OK;
}

int forward(chebfd_ctx *ctx, chebfd_mlp *M, const float *X, int B)
{
    const Offsets o = offsets(M->n_in, M->h, M->n_out);
    const int h = M->h, no = M->n_out;
    hipLaunchKernelGGL(k_standardise, dim3(nb((int64_t)B * M->n_in, 256)), dim3(256), 0,
                       ctx->stream, X, M->in_shift, M->in_scale, M->xn, B, M->n_in);
    hipLaunchKernelGGL(k_dense_fwd, dim3(nb(h, 64), B), dim3(64), 0, ctx->stream, M->xn, M->p + o.W1,
                       M->p + o.b1, M->a1, B, M->n_in, h, 1);
    hipLaunchKernelGGL(k_dense_fwd, dim3(nb(h, 64), B), dim3(64), 0, ctx->stream, M->a1,
                       M->p + o.W2, M->p + o.b2, M->a2, B, h, h, 1);
    hipLaunchKernelGGL(k_dense_fwd, dim3(nb(no, 64), B), dim3(64), 0, ctx->stream, M->a2,
                       M->p + o.W3, M->p + o.b3, M->a3, B, h, no, 0);
    CHEBFD_CHECK_LAUNCH();
    return CHEBFD_OK;
}

// loss and parameter gradients (into M->g) for one batch
int backward(chebfd_ctx *ctx, chebfd_mlp *M, const float *X, const float *T, int B)
{
    const Offsets o = offsets(M->n_in, M->h, M->n_out);
    const int h = M->h, no = M->n_out, ni = M->n_in;
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, ctx->stream, M->a3, T, M->shift, M->scale,
                       M->d3, M->loss, B, no);
    // layer 3 (linear): dz3 = d3
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(nb(no, 64), h + 1), dim3(64), 0, ctx->stream, M->a2,
                       M->d3, M->g + o.W3, M->g + o.b3, B, h, no);
    hipLaunchKernelGGL(k_dense_bwd_in, dim3(nb(h, 64), B), dim3(64), 0, ctx->stream, M->d3,
                       M->p + o.W3, M->a2, M->d2, B, h, no, 1);   // d2 = dz2 (tanh')
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(nb(h, 64), h + 1), dim3(64), 0, ctx->stream, M->a1,
                       M->d2, M->g + o.W2, M->g + o.b2, B, h, h);
    hipLaunchKernelGGL(k_dense_bwd_in, dim3(nb(h, 64), B), dim3(64), 0, ctx->stream, M->d2,
                       M->p + o.W2, M->a1, M->d1, B, h, h, 1);    // d1 = dz1
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(nb(h, 64), ni + 1), dim3(64), 0, ctx->stream, M->xn,
                       M->d1, M->g + o.W1, M->g + o.b1, B, ni, h);
    CHEBFD_CHECK_LAUNCH();
    return CHEBFD_OK;
}

}  // namespace
}  // namespace chebfd

using namespace chebfd;

extern "C" {

int chebfd_mlp_create(chebfd_ctx *ctx, int n_in, int n_hidden, int n_out, uint64_t seed,
                      chebfd_mlp **out)
{
    if (!ctx || !out || n_in < 1 || n_hidden < 1 || n_out < 1)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_mlp_create: invalid arguments");
    *out = nullptr;
    CHEBFD_HIP(hipSetDevice(ctx->device));
    auto *M = new chebfd_mlp();
    M->n_in = n_in;
    M->h = n_hidden;
    M->n_out = n_out;
    M->device = ctx->device;
    const Offsets o = offsets(n_in, n_hidden, n_out);
    M->n_params = o.total;
    // Glorot-uniform weights from the counter generator (stream 5), zero biases
    std::vector<float> p(o.total, 0.0f);
    uint64_t idx = 0;
    auto fill = [&](int64_t off, int fan_in, int fan_out) {
        const double lim = std::sqrt(6.0 / (fan_in + fan_out));
        for (int64_t i = 0; i < (int64_t)fan_in * fan_out; ++i)
            p[off + i] = (float)(lim * (2.0 * u01(seed, 5, idx++) - 1.0));
    };
    fill(o.W1, n_in, n_hidden);
    fill(o.W2, n_hidden, n_hidden);
    fill(o.W3, n_hidden, n_out);
    std::vector<float> zero(o.total, 0.0f), sh(n_out, 0.0f), sc(n_out, 1.0f),
        ish(n_in, 0.0f), isc(n_in, 1.0f);
    hipError_t e = hipSuccess;
    for (float **q : {&M->p, &M->g, &M->m, &M->v})
        if (e == hipSuccess) e = hipMalloc((void **)q, o.total * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&M->shift, n_out * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&M->scale, n_out * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&M->loss, 4 * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&M->in_shift, n_in * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&M->in_scale, n_in * 4);
    if (e == hipSuccess) e = hipMemcpy(M->in_shift, ish.data(), n_in * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(M->in_scale, isc.data(), n_in * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(M->p, p.data(), o.total * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(M->g, zero.data(), o.total * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(M->m, zero.data(), o.total * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(M->v, zero.data(), o.total * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(M->shift, sh.data(), n_out * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(M->scale, sc.data(), n_out * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        chebfd_mlp_destroy(M);
        return fail(CHEBFD_ERR_HIP, std::string("chebfd_mlp_create: ") + hipGetErrorString(e));
    }
    *out = M;
    return CHEBFD_OK;
}

int chebfd_mlp_destroy(chebfd_mlp *M)
{
    if (!M) return CHEBFD_OK;
    (void)hipSetDevice(M->device);
    for (float *q : {M->p, M->g, M->m, M->v, M->shift, M->scale, M->a1, M->a2, M->a3, M->d1, M->d2,
                     M->d3, M->loss, M->in_shift, M->in_scale, M->xn})
        if (q) (void)hipFree(q);
    delete M;
    return CHEBFD_OK;
}

int chebfd_mlp_dims(const chebfd_mlp *M, int *n_in, int *n_hidden, int *n_out)
{
    if (!M) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_mlp_dims: NULL network");
    if (n_in) *n_in = M->n_in;
    if (n_hidden) *n_hidden = M->h;
    if (n_out) *n_out = M->n_out;
    return CHEBFD_OK;
}

int chebfd_mlp_num_params(const chebfd_mlp *M, int64_t *n)
{
    if (!M || !n) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_mlp_num_params: NULL argument");
    *n = M->n_params;
    return CHEBFD_OK;
}

int chebfd_mlp_get_params(chebfd_ctx *ctx, const chebfd_mlp *M, float *host, float *shift,
                          float *scale)
{
    if (!ctx || !M) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_mlp_get_params: NULL argument");
    CHEBFD_HIP(hipStreamSynchronize(ctx->stream));
    if (host) CHEBFD_HIP(hipMemcpy(host, M->p, M->n_params * 4, hipMemcpyDeviceToHost));
    if (shift) CHEBFD_HIP(hipMemcpy(shift, M->shift, M->n_out * 4, hipMemcpyDeviceToHost));
    if (scale) CHEBFD_HIP(hipMemcpy(scale, M->scale, M->n_out * 4, hipMemcpyDeviceToHost));
    return CHEBFD_OK;
}

int chebfd_mlp_set_params(chebfd_ctx *ctx, chebfd_mlp *M, const float *host, const float *shift,
                          const float *scale)
{
    if (!ctx || !M) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_mlp_set_params: NULL argument");
    CHEBFD_HIP(hipStreamSynchronize(ctx->stream));
    if (host) {
        for (int64_t i = 0; i < M->n_params; ++i)
            if (!std::isfinite(host[i]))
                return fail(CHEBFD_ERR_NONFINITE, "chebfd_mlp_set_params: non-finite parameter");
        CHEBFD_HIP(hipMemcpy(M->p, host, M->n_params * 4, hipMemcpyHostToDevice));
    }
    if (scale)
        for (int j = 0; j < M->n_out; ++j)
            if (!(scale[j] > 0.0f)) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_mlp_set_params: scale must be > 0");
    if (shift) CHEBFD_HIP(hipMemcpy(M->shift, shift, M->n_out * 4, hipMemcpyHostToDevice));
    if (scale) CHEBFD_HIP(hipMemcpy(M->scale, scale, M->n_out * 4, hipMemcpyHostToDevice));
    return CHEBFD_OK;
}

int chebfd_mlp_input_scaling(chebfd_ctx *ctx, chebfd_mlp *M, float *shift, float *scale,
                             int get)
{
    if (!ctx || !M || !shift || !scale)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_mlp_input_scaling: NULL argument");
    CHEBFD_HIP(hipStreamSynchronize(ctx->stream));
    if (get) {
        CHEBFD_HIP(hipMemcpy(shift, M->in_shift, M->n_in * 4, hipMemcpyDeviceToHost));
        CHEBFD_HIP(hipMemcpy(scale, M->in_scale, M->n_in * 4, hipMemcpyDeviceToHost));
        return CHEBFD_OK;
    }
    for (int k = 0; k < M->n_in; ++k)
        if (!(scale[k] > 0.0f) || !std::isfinite(shift[k]))
            return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_mlp_input_scaling: need finite shift, scale > 0");
    CHEBFD_HIP(hipMemcpy(M->in_shift, shift, M->n_in * 4, hipMemcpyHostToDevice));
    CHEBFD_HIP(hipMemcpy(M->in_scale, scale, M->n_in * 4, hipMemcpyHostToDevice));
    return CHEBFD_OK;
}

int chebfd_mlp_forward(chebfd_ctx *ctx, chebfd_mlp *M, const float *X_dev, int batch, float *Y_dev)
{
    if (!ctx || !M || !X_dev || !Y_dev || batch < 1)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_mlp_forward: invalid arguments");
    CHEBFD_HIP(hipSetDevice(ctx->device));
    int rc = ensure_batch(M, batch);
    if (!rc) rc = forward(ctx, M, X_dev, batch);
    if (rc) return rc;
    CHEBFD_HIP(hipMemcpyAsync(Y_dev, M->a3, (size_t)batch * M->n_out * 4, hipMemcpyDeviceToDevice,
                              ctx->stream));
    hipLaunchKernelGGL(k_affine, dim3(nb((int64_t)batch * M->n_out, 256)), dim3(256), 0,
                       ctx->stream, Y_dev, M->shift, M->scale, batch, M->n_out);
    CHEBFD_CHECK_LAUNCH();
    return CHEBFD_OK;
}

int chebfd_mlp_loss_grad(chebfd_ctx *ctx, chebfd_mlp *M, const float *X_dev, const float *T_dev,
                         int batch, float *loss_host, float *grad_host)
{
    if (!ctx || !M || !X_dev || !T_dev || batch < 1 || !loss_host)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_mlp_loss_grad: invalid arguments");
    CHEBFD_HIP(hipSetDevice(ctx->device));
    int rc = ensure_batch(M, batch);
    if (!rc) rc = forward(ctx, M, X_dev, batch);
    if (!rc) rc = backward(ctx, M, X_dev, T_dev, batch);
    if (rc) return rc;
    CHEBFD_HIP(hipMemcpyAsync(loss_host, M->loss, 4, hipMemcpyDeviceToHost, ctx->stream));
    if (grad_host)
        CHEBFD_HIP(hipMemcpyAsync(grad_host, M->g, M->n_params * 4, hipMemcpyDeviceToHost,
                                  ctx->stream));
    CHEBFD_HIP(hipStreamSynchronize(ctx->stream));
    return CHEBFD_OK;
}

int chebfd_mlp_train_step(chebfd_ctx *ctx, chebfd_mlp *M, const float *X_dev, const float *T_dev,
                          int batch, float lr, float weight_decay, float *loss_host)
{
    if (!ctx || !M || !X_dev || !T_dev || batch < 1 || !(lr > 0.0f) || weight_decay < 0.0f)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_mlp_train_step: invalid arguments");
    CHEBFD_HIP(hipSetDevice(ctx->device));
    int rc = ensure_batch(M, batch);
    if (!rc) rc = forward(ctx, M, X_dev, batch);
    if (!rc) rc = backward(ctx, M, X_dev, T_dev, batch);
    if (rc) return rc;
    M->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)M->step), c2 = 1.0f - std::pow(b2, (float)M->step);
    hipLaunchKernelGGL(k_adam, dim3(nb(M->n_params, 256)), dim3(256), 0, ctx->stream, M->p, M->g,
                       M->m, M->v, M->n_params, lr, b1, b2, 1e-8f, weight_decay, c1, c2);
    CHEBFD_CHECK_LAUNCH();
    if (loss_host) {
        CHEBFD_HIP(hipMemcpyAsync(loss_host, M->loss, 4, hipMemcpyDeviceToHost, ctx->stream));
        CHEBFD_HIP(hipStreamSynchronize(ctx->stream));
    }
    return CHEBFD_OK;
}

}  // extern "C"
