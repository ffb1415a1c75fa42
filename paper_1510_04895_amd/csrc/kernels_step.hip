// Fused Chebyshev filter step on SELL-C-sigma storage (gfx950).
//
// One launch performs one step of the polynomial filter (Fig. fig:ChebFD,
// Sec. 3.1) on a row-major block of search vectors, fusing the sparse
// matrix-multiple-vector product, the three-term recurrence and the filter
// accumulation (the augmented spMMVM of Sec. 4), plus optional per-column dot
// products for the Chebyshev moments:
//   MODE_APPLY : w = s_h H u + s_u u
//   MODE_SECOND: w = s_h H u + s_u u - x ;  x = g0 x + g1 u + g2 w
//   MODE_STEP  : w = s_h H u + s_u u - w ;  x = x + g0 w
// Work decomposition: a workgroup of 256 lanes owns one SELL chunk (C <= 64
// rows) and one column slab of LPR*NB complex columns.  LPR lanes share a row, so a
// wave covers 64/LPR rows; each lane owns NB consecutive complex columns and
// moves them with one 16-byte access.  The gathered block u is only read;
// w and x are read and written only at the workgroup's own rows, so the
// in-place updates are race-free.  Workgroups are ordered slab-major (all
// chunks of slab 0, then slab 1, ...) so the cache working set of u is one
// slab wide.
#include <type_traits>

#include "internal.h"
#include "pack.h"

namespace chebfd {
namespace {

// Accumulates one row of the sparse product from (index, value) pairs
// served by `src(j)`, GB gathers in flight at a time.
template <typename T, int NB, int GB, typename Src>
__device__ __forceinline__ void row_product(const T *__restrict__ u, int64_t ld, int64_t c0,
                                            int cnt, int len, Src src, T (&ar)[NB], T (&ai)[NB])
{
#pragma unroll
    for (int e = 0; e < NB; ++e) ar[e] = ai[e] = T(0);
    for (int j = 0; j < len; j += GB) {
        Pack<T, NB> g[GB];
        T hr[GB], hi[GB];
#pragma unroll
        for (int i = 0; i < GB; ++i) {
            if (j + i < len) {
                int ci;
                src(j + i, ci, hr[i], hi[i]);
                g[i] = load_pack_n<T, NB>(u + 2 * ((int64_t)ci * ld + c0), cnt);
            }
        }
#pragma unroll
        for (int i = 0; i < GB; ++i) {
            if (j + i < len) {
#pragma unroll
                for (int e = 0; e < NB; ++e) {
                    ar[e] += hr[i] * g[i].re[e] - hi[i] * g[i].im[e];
                    ai[e] += hr[i] * g[i].im[e] + hi[i] * g[i].re[e];
                }
            }
        }
    }
}

constexpr int LDS_ENTRIES = 1024;   // index/value pairs of one chunk staged in LDS

template <typename T, int LPR, int NB, int MODE, bool MOM, bool NT, bool STAGED, int GB>
__global__ __launch_bounds__(256) void k_step_sell(
    const int64_t *__restrict__ chunk_ptr, const int32_t *__restrict__ chunk_len,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ col,
    const T *__restrict__ val, int C, int64_t nchunks, const T *__restrict__ u,
    const T *wold, T *wout, T *y, int64_t n_s, int64_t ld, T s_h, T s_u, T g0, T g1, T g2,
    double *__restrict__ partials, int order, int64_t nslab)
{
    constexpr int RPW = 64 / LPR;        // rows per wave
    constexpr int RPP = 4 * RPW;         // rows per pass of the workgroup
    constexpr int SW = LPR * NB;         // slab width in complex columns
    __shared__ int32_t s_col[LDS_ENTRIES];
    __shared__ T s_val[2 * LDS_ENTRIES];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int rsub = lane / LPR, cl = lane % LPR;
    const int64_t b = blockIdx.x;
    // order 0: slab-major (all chunks of a column slab, then the next slab);
    // order 1: chunk-major (all slabs of a chunk adjacent)
    int64_t slab, chunk;
    if (order == 0) {
        slab = b / nchunks;
        chunk = b - slab * nchunks;
    } else {
        chunk = b / nslab;
        slab = b - chunk * nslab;
    }
    const int64_t c0 = slab * SW + (int64_t)cl * NB;
    const int cnt = (int)((n_s - c0) < NB ? (n_s - c0) : NB);   // valid columns of the pack
    const bool active = c0 < n_s;
    const int len = chunk_len[chunk];
    const int64_t base = chunk_ptr[chunk];
    // chunks that fit are staged in LDS with coalesced loads, so the gathers
    // of a row never wait on an index load; wider chunks read the stream
    // directly
    constexpr bool staged = STAGED;
    if (staged) {
        for (int t = tid; t < len * C; t += 256) {
            s_col[t] = col[base + t];
            s_val[2 * t] = val[2 * (base + t)];
            s_val[2 * t + 1] = val[2 * (base + t) + 1];
        }
        __syncthreads();
    }

    double m0[NB], m1[NB], m2[NB];
#pragma unroll
    for (int e = 0; e < NB; ++e) m0[e] = m1[e] = m2[e] = 0.0;

    for (int r = wave * RPW + rsub; r < C; r += RPP) {
        const int row = perm[chunk * C + r];
        if (row < 0 || !active) continue;
        // the row's own operands first: they do not depend on the product
        const int64_t off = 2 * ((int64_t)row * ld + c0);
        const Pack<T, NB> uo = load_pack_n<T, NB>(u + off, cnt);
        Pack<T, NB> wo, yv;
        if (MODE == MODE_SECOND || MODE == MODE_STEP) wo = load_pack_n<T, NB, NT>(wold + off, cnt);
        if (MODE == MODE_STEP) yv = load_pack_n<T, NB, NT>(y + off, cnt);
        T ar[NB], ai[NB];
        if (staged) {
            row_product<T, NB, GB>(u, ld, c0, cnt, len,
                                   [&](int j, int &ci, T &hr, T &hi) {
                                       const int t = j * C + r;
                                       ci = s_col[t];
                                       hr = s_val[2 * t];
                                       hi = s_val[2 * t + 1];
                                   },
                                   ar, ai);
        } else {
            const int64_t eb = base + r;
            row_product<T, NB, GB>(u, ld, c0, cnt, len,
                                   [&](int j, int &ci, T &hr, T &hi) {
                                       const int64_t e = eb + (int64_t)j * C;
                                       ci = col[e];
                                       hr = val[2 * e];
                                       hi = val[2 * e + 1];
                                   },
                                   ar, ai);
        }
        Pack<T, NB> w;
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            w.re[e] = s_h * ar[e] + s_u * uo.re[e];
            w.im[e] = s_h * ai[e] + s_u * uo.im[e];
        }
        if (MODE == MODE_APPLY) {
            store_pack_n<T, NB, NT>(wout + off, w, cnt);
            if (MOM) {
#pragma unroll
                for (int e = 0; e < NB; ++e) {
                    const double xr = uo.re[e], xi = uo.im[e], wr = w.re[e], wi = w.im[e];
                    m0[e] += xr * xr + xi * xi;
                    m1[e] += xr * wr + xi * wi;
                    m2[e] += wr * wr + wi * wi;
                }
            }
        } else if (MODE == MODE_SECOND) {
            const Pack<T, NB> xo = wo;
            Pack<T, NB> xn;
#pragma unroll
            for (int e = 0; e < NB; ++e) {
                w.re[e] -= xo.re[e];
                w.im[e] -= xo.im[e];
                xn.re[e] = g0 * xo.re[e] + g1 * uo.re[e] + g2 * w.re[e];
                xn.im[e] = g0 * xo.im[e] + g1 * uo.im[e] + g2 * w.im[e];
            }
            store_pack_n<T, NB, NT>(wout + off, w, cnt);
            store_pack_n<T, NB, NT>(y + off, xn, cnt);
            if (MOM) {
#pragma unroll
                for (int e = 0; e < NB; ++e) {
                    m1[e] += (double)uo.re[e] * w.re[e] + (double)uo.im[e] * w.im[e];
                    m2[e] += (double)w.re[e] * w.re[e] + (double)w.im[e] * w.im[e];
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < NB; ++e) {
                w.re[e] -= wo.re[e];
                w.im[e] -= wo.im[e];
                yv.re[e] += g0 * w.re[e];
                yv.im[e] += g0 * w.im[e];
            }
            store_pack_n<T, NB, NT>(wout + off, w, cnt);
            store_pack_n<T, NB, NT>(y + off, yv, cnt);
            if (MOM) {
#pragma unroll
                for (int e = 0; e < NB; ++e) {
                    m1[e] += (double)uo.re[e] * w.re[e] + (double)uo.im[e] * w.im[e];
                    m2[e] += (double)w.re[e] * w.re[e] + (double)w.im[e] * w.im[e];
                }
            }
        }
    }

    if (MOM) {
        // reduce over the rows of the wave (lanes with the same column), then
        // over the four waves through LDS, in a fixed order
        __shared__ double red[4][64][3 * NB];
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            for (int off = LPR; off < 64; off <<= 1) {
                m0[e] += __shfl_xor(m0[e], off);
                m1[e] += __shfl_xor(m1[e], off);
                m2[e] += __shfl_xor(m2[e], off);
            }
            red[wave][lane][3 * e + 0] = m0[e];
            red[wave][lane][3 * e + 1] = m1[e];
            red[wave][lane][3 * e + 2] = m2[e];
        }
        __syncthreads();
        if (wave == 0 && lane < LPR && active) {
#pragma unroll
            for (int e = 0; e < NB; ++e) {
                if (e >= cnt) continue;
                double sq[3];
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    sq[q] = red[0][lane][3 * e + q] + red[1][lane][3 * e + q] +
                            red[2][lane][3 * e + q] + red[3][lane][3 * e + q];
                double *p = partials + 3 * (chunk * n_s + c0 + e);
                p[0] = sq[0];
                p[1] = sq[1];
                p[2] = sq[2];
            }
        }
    }
}

// Moment finalisation: one workgroup per (column, quantity) sums the
// per-chunk partials in a fixed order (strided per lane, then a tree).
__global__ __launch_bounds__(256) void k_moment_finalize(const double *__restrict__ part,
                                                         int64_t n_part, int64_t n_s, int mode,
                                                         int step, double *__restrict__ mom)
{
    const int64_t k = blockIdx.x;
    const int tid = threadIdx.x;
    __shared__ double red[3][256];
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t c = tid; c < n_part; c += 256) {
        const double *p = part + 3 * (c * n_s + k);
        s[0] += p[0];
        s[1] += p[1];
        s[2] += p[2];
    }
    for (int q = 0; q < 3; ++q) red[q][tid] = s[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w)
            for (int q = 0; q < 3; ++q) red[q][tid] += red[q][tid + w];
        __syncthreads();
    }
    if (tid == 0) {
        if (mode == MODE_APPLY) {
            // step 1: x -> u = T_1 x
            const double mu0 = red[0][0];
            mom[0 * n_s + k] = mu0;
            mom[1 * n_s + k] = red[1][0];
            mom[2 * n_s + k] = 2.0 * red[2][0] - mu0;
        } else {
            // step n: u = T_{n-1} x, w = T_n x
            const double mu0 = mom[k], mu1 = mom[n_s + k];
            mom[(int64_t)(2 * step - 1) * n_s + k] = 2.0 * red[1][0] - mu1;
            mom[(int64_t)(2 * step) * n_s + k] = 2.0 * red[2][0] - mu0;
        }
    }
}

template <typename T, int LPR, int NB, int MODE, bool MOM, bool NT>
int launch_sell_t(chebfd_ctx *ctx, const Sell &S, const StepArgs &a)
{
    constexpr int SW = LPR * NB;
    const int64_t nslab = (a.n_s + SW - 1) / SW;
    const int64_t grid = S.nchunks * nslab;
    const T *val = std::is_same<T, double>::value ? (const T *)S.val64 : (const T *)S.val32;
    // every chunk fits in LDS -> staged variant, else direct index stream
    if ((int64_t)S.max_len * S.C <= LDS_ENTRIES && ctx->tune_gathers == 16)
        hipLaunchKernelGGL((k_step_sell<T, LPR, NB, MODE, MOM, NT, true, 16>), dim3((unsigned)grid),
                           dim3(256), 0, ctx->stream, S.chunk_ptr, S.chunk_len, S.perm, S.col,
                           val, S.C, S.nchunks, (const T *)a.u, (const T *)a.wold, (T *)a.wout,
                           (T *)a.y, a.n_s, a.ld, (T)a.s_h, (T)a.s_u, (T)a.g0, (T)a.g1, (T)a.g2,
                           a.partials, ctx->tune_order, nslab);
    else if ((int64_t)S.max_len * S.C <= LDS_ENTRIES)
        hipLaunchKernelGGL((k_step_sell<T, LPR, NB, MODE, MOM, NT, true, 8>), dim3((unsigned)grid),
                           dim3(256), 0, ctx->stream, S.chunk_ptr, S.chunk_len, S.perm, S.col,
                           val, S.C, S.nchunks, (const T *)a.u, (const T *)a.wold, (T *)a.wout,
                           (T *)a.y, a.n_s, a.ld, (T)a.s_h, (T)a.s_u, (T)a.g0, (T)a.g1, (T)a.g2,
                           a.partials, ctx->tune_order, nslab);
    else
        hipLaunchKernelGGL((k_step_sell<T, LPR, NB, MODE, MOM, NT, false, 8>), dim3((unsigned)grid),
                           dim3(256), 0, ctx->stream, S.chunk_ptr, S.chunk_len, S.perm, S.col,
                           val, S.C, S.nchunks, (const T *)a.u, (const T *)a.wold, (T *)a.wout,
                           (T *)a.y, a.n_s, a.ld, (T)a.s_h, (T)a.s_u, (T)a.g0, (T)a.g1, (T)a.g2,
                           a.partials, ctx->tune_order, nslab);
    CHEBFD_CHECK_LAUNCH();
    return CHEBFD_OK;
}

template <typename T, int LPR, int NB, bool NT>
int launch_sell_mode(chebfd_ctx *ctx, const Sell &S, const StepArgs &a)
{
    const bool mom = a.partials != nullptr;
    switch (a.mode) {
    case MODE_APPLY:
        return mom ? launch_sell_t<T, LPR, NB, MODE_APPLY, true, NT>(ctx, S, a)
                   : launch_sell_t<T, LPR, NB, MODE_APPLY, false, NT>(ctx, S, a);
    case MODE_SECOND:
        return mom ? launch_sell_t<T, LPR, NB, MODE_SECOND, true, NT>(ctx, S, a)
                   : launch_sell_t<T, LPR, NB, MODE_SECOND, false, NT>(ctx, S, a);
    default:
        return mom ? launch_sell_t<T, LPR, NB, MODE_STEP, true, NT>(ctx, S, a)
                   : launch_sell_t<T, LPR, NB, MODE_STEP, false, NT>(ctx, S, a);
    }
}

template <typename T, int NB>
int launch_sell_lpr(chebfd_ctx *ctx, const Sell &S, const StepArgs &a, int lpr)
{
    const bool nt = ctx->tune_nt != 0;
    switch (lpr) {
    case 16:
        return nt ? launch_sell_mode<T, 16, NB, true>(ctx, S, a)
                  : launch_sell_mode<T, 16, NB, false>(ctx, S, a);
    case 64:
        return nt ? launch_sell_mode<T, 64, NB, true>(ctx, S, a)
                  : launch_sell_mode<T, 64, NB, false>(ctx, S, a);
    default:
        return nt ? launch_sell_mode<T, 32, NB, true>(ctx, S, a)
                  : launch_sell_mode<T, 32, NB, false>(ctx, S, a);
    }
}

}  // namespace

int launch_stencil_step(chebfd_ctx *ctx, const chebfd_matrix *H, const StepArgs &a,
                        int64_t *n_part);

// Lanes per row: the narrowest slab that still covers the block (fewer idle
// lanes for thin blocks such as the KPM vectors), else the tuned width
// (default 32 lanes = 512-byte row segments in c128).
int pick_lpr(const chebfd_ctx *ctx, int64_t n_s, int nb)
{
    const int64_t packs = (n_s + nb - 1) / nb;
    if (packs <= 16) return 16;
    if (ctx->tune_lpr == 16 || ctx->tune_lpr == 32 || ctx->tune_lpr == 64) return ctx->tune_lpr;
    return 32;
}

int launch_step(chebfd_ctx *ctx, const chebfd_matrix *H, const StepArgs &a, int64_t *n_part)
{
    if (H->storage == CHEBFD_STORAGE_STENCIL) return launch_stencil_step(ctx, H, a, n_part);
    const Sell &S = H->sell;
    if (n_part) *n_part = S.nchunks;
    if (a.precision == CHEBFD_PREC_C128)
        return launch_sell_lpr<double, 1>(ctx, S, a, pick_lpr(ctx, a.n_s, 1));
    return launch_sell_lpr<float, 2>(ctx, S, a, pick_lpr(ctx, a.n_s, 2));
}

int launch_moment_finalize(chebfd_ctx *ctx, const double *partials, int64_t n_part,
                           int64_t n_s, int mode, int step, double *mom)
{
    hipLaunchKernelGGL(k_moment_finalize, dim3((unsigned)n_s), dim3(256), 0, ctx->stream,
                       partials, n_part, n_s, mode, step, mom);
    CHEBFD_CHECK_LAUNCH();
    return CHEBFD_OK;
}

}  // namespace chebfd
