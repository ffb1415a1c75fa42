// Dense kernels around the filter (gfx950):
//  - Gram matrices S = A^H B of tall blocks (orthogonalisation, Sec. 3.1 step
//    6, and the Rayleigh-Ritz matrix, step 7) on the FP64 matrix cores;
//  - block times small matrix C = A T (basis updates, Ritz vectors);
//  - residual norms, counter-based random blocks, precision conversion.
//
// A complex block with interleaved storage is a real matrix with twice the
// columns.  For A = Ar + i Ai, B = Br + i Bi the real Gram G = Z_A^T Z_B of the
// interleaved real matrices holds every product needed:
//   (A^H B)[k][l] = G[2k][2l] + G[2k+1][2l+1] + i (G[2k][2l+1] - G[2k+1][2l]).
// Likewise A T (complex T) equals Z_A Treal with Treal[2k][2l] = Re T,
// Treal[2k][2l+1] = Im T, Treal[2k+1][2l] = -Im T, Treal[2k+1][2l+1] = Re T.
// Both are therefore plain real FP64 contractions on v_mfma_f64_16x16x4_f64.
#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace chebfd {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ double ld_real(const T *p)
{
    return (double)(*p);
}

// ------------------------------------------------------------------ Gram
// Real G_part[ks] = Z_A^T Z_B over rows [ks*rows, (ks+1)*rows).
// Workgroup tile 64 (m) x 64 (n); four waves of 32 x 32, each 2 x 2 MFMA
// blocks of 16 x 16; K (the row index of the tall blocks) staged 16 at a time
// through LDS, the next stage's global loads issued into registers before the
// current stage's MFMAs (their latency overlaps the matrix work; the
// accumulation order is unchanged; a register budget for 4 waves per SIMD
// keeps the occupancy the version without prefetch had).  MFMA f64 16x16x4
// operand layout (measured on gfx950): lane l
// holds A[m = l%16][k = l/16] and B[k = l/16][n = l%16]; result register r
// of lane l is D[m = l/16 + 4r][n = l%16].
constexpr int GT = 64;   // tile
constexpr int GK = 16;   // rows per LDS stage

template <typename T>
__global__ __launch_bounds__(256, 4) void k_gram(const T *__restrict__ A, int64_t lda2, int64_t ma,
                                              const T *__restrict__ B, int64_t ldb2, int64_t mb,
                                              int64_t n, int64_t rows_per_split,
                                              double *__restrict__ part)
{
    __shared__ double As[GK][GT];
    __shared__ double Bs[GK][GT];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t m0 = (int64_t)blockIdx.x * GT, n0 = (int64_t)blockIdx.y * GT;
    const int64_t ks = blockIdx.z;
    const int64_t r0 = ks * rows_per_split;
    int64_t r1 = r0 + rows_per_split;
    if (r1 > n) r1 = n;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    v4d acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    constexpr int PER = (GK * GT) / 256;
    double pa[PER], pb[PER];
    auto fetch = [&](int64_t s0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = tid + 256 * q;
            const int kk = idx / GT, mm = idx % GT;
            const int64_t row = s0 + kk;
            const bool rv = row < r1;
            pa[q] = (rv && m0 + mm < ma) ? ld_real(A + row * lda2 + m0 + mm) : 0.0;
            pb[q] = (rv && n0 + mm < mb) ? ld_real(B + row * ldb2 + n0 + mm) : 0.0;
        }
    };
    if (r0 < r1) fetch(r0);
    for (int64_t rb = r0; rb < r1; rb += GK) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = tid + 256 * q;
            As[idx / GT][idx % GT] = pa[q];
            Bs[idx / GT][idx % GT] = pb[q];
        }
        __syncthreads();
        if (rb + GK < r1) fetch(rb + GK);
#pragma unroll
        for (int k4 = 0; k4 < GK; k4 += 4) {
            const int kk = k4 + (lane >> 4);
            double av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = As[kk][wm + 16 * i + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = Bs[kk][wn + 16 * j + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // write the partial tile (ks, m, n) of the (ma x mb) real Gram
    double *P = part + ks * ma * mb;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t m = m0 + wm + 16 * i + (lane >> 4) + 4 * r;
                const int64_t nn = n0 + wn + 16 * j + (lane & 15);
                if (m < ma && nn < mb) P[m * mb + nn] = acc[i][j][r];
            }
}

// Sums the split partials in fixed order and assembles the complex Gram.
__global__ void k_gram_reduce(const double *__restrict__ part, int64_t ks_count, int64_t ma,
                              int64_t mb, int64_t na, int64_t nb, double *__restrict__ S)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= na * nb) return;
    const int64_t k = idx / nb, l = idx - k * nb;
    double rr = 0, ii = 0, ri = 0, ir = 0;
    for (int64_t s = 0; s < ks_count; ++s) {
        const double *P = part + s * ma * mb;
        rr += P[(2 * k) * mb + 2 * l];
        ii += P[(2 * k + 1) * mb + 2 * l + 1];
        ri += P[(2 * k) * mb + 2 * l + 1];
        ir += P[(2 * k + 1) * mb + 2 * l];
    }
    S[2 * idx] = rr + ii;
    S[2 * idx + 1] = ri - ir;
}

// ------------------------------------------------------------ block times
// C (n x mc real) = Z_A (n x ka real) Treal (ka x mc), or C -= Z_A Treal.
// Workgroup tile 64 rows x 64 columns; waves 32 x 32 as in the Gram.
template <typename TA, typename TC, bool SUB>
__global__ __launch_bounds__(256, 4) void k_block_times(const TA *__restrict__ A, int64_t lda2,
                                                     int64_t n, int64_t ka,
                                                     const double *__restrict__ Tr, int64_t mc,
                                                     TC *C, int64_t ldc2, int64_t ntile_c)
{
    __shared__ double As[GT][GK + 1];
    __shared__ double Ts[GK][GT];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    // column tile fastest: consecutive workgroups share the same rows of A
    const int64_t tc = blockIdx.x % ntile_c, tr = blockIdx.x / ntile_c;
    const int64_t i0 = tr * GT, c0 = tc * GT;
    const int wi = (wave >> 1) * 32, wc = (wave & 1) * 32;
    v4d acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    constexpr int PER = (GK * GT) / 256;
    double pa[PER], pt[PER];
    // next stage into registers, issued before the current stage's MFMAs
    auto fetch = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = tid + 256 * q;
            // A tile: 64 rows x 16 k, read 16 consecutive doubles per row
            const int ii = idx / GK, kk = idx % GK;
            const int64_t row = i0 + ii, kc = k0 + kk;
            pa[q] = (row < n && kc < ka) ? (double)A[row * lda2 + kc] : 0.0;
            // T tile: 16 k x 64 columns
            const int tk = idx / GT, tm = idx % GT;
            const int64_t kr = k0 + tk, cc = c0 + tm;
            pt[q] = (kr < ka && cc < mc) ? Tr[kr * mc + cc] : 0.0;
        }
    };
    if (ka > 0) fetch(0);
    for (int64_t kb = 0; kb < ka; kb += GK) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = tid + 256 * q;
            As[idx / GK][idx % GK] = pa[q];
            Ts[idx / GT][idx % GT] = pt[q];
        }
        __syncthreads();
        if (kb + GK < ka) fetch(kb + GK);
#pragma unroll
        for (int k4 = 0; k4 < GK; k4 += 4) {
            const int kk = k4 + (lane >> 4);
            double av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = As[wi + 16 * i + (lane & 15)][kk];
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = Ts[kk][wc + 16 * j + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = i0 + wi + 16 * i + (lane >> 4) + 4 * r;
                const int64_t cc = c0 + wc + 16 * j + (lane & 15);
                if (row < n && cc < mc) {
                    TC *p = C + row * ldc2 + cc;
                    if (SUB) *p = (TC)((double)*p - acc[i][j][r]);
                    else *p = (TC)acc[i][j][r];
                }
            }
}

// -------------------------------------------------------------- residuals
// part[blk][j] = sum over the workgroup's rows of |HV_ij - theta_j V_ij|^2.
template <typename T>
__global__ __launch_bounds__(256) void k_residual(const T *__restrict__ V,
                                                  const T *__restrict__ HV, int64_t n, int64_t m,
                                                  int64_t ld, const double *__restrict__ theta,
                                                  int64_t rows_per_blk, double *__restrict__ part)
{
    const int64_t j = (int64_t)blockIdx.y * 256 + threadIdx.x;
    if (j >= m) return;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
    int64_t r1 = r0 + rows_per_blk;
    if (r1 > n) r1 = n;
    const double th = theta[j];
    double s = 0.0;
    for (int64_t i = r0; i < r1; ++i) {
        const int64_t o = 2 * (i * ld + j);
        const double dr = (double)HV[o] - th * (double)V[o];
        const double di = (double)HV[o + 1] - th * (double)V[o + 1];
        s += dr * dr + di * di;
    }
    part[(int64_t)blockIdx.x * m + j] = s;
}

__global__ void k_residual_reduce(const double *__restrict__ part, int64_t nblk, int64_t m,
                                  double *__restrict__ res)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    double s = 0.0;
    for (int64_t b = 0; b < nblk; ++b) s += part[b * m + j];
    res[j] = sqrt(s);
}

// ------------------------------------------------------------------ random
__device__ __forceinline__ uint64_t dmix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double du01(uint64_t key, uint64_t index)
{
    const uint64_t G = 0x9E3779B97F4A7C15ULL;
    return (double)(dmix(key + G * (index + 1u)) >> 11) * 0x1.0p-53;
}

template <typename T>
__global__ void k_random(T *X, int64_t n, int64_t n_s, int64_t ld, int64_t k0, int64_t m,
                         uint64_t key, uint64_t offset)
{
    const int64_t total = n * m, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += stride) {
        const int64_t i = idx / m, k = k0 + (idx - (idx / m) * m);
        const uint64_t e = offset + (uint64_t)(i * n_s + k);
        const double re = 2.0 * du01(key, 2 * e) - 1.0;
        const double im = 2.0 * du01(key, 2 * e + 1) - 1.0;
        X[2 * (i * ld + k)] = (T)re;
        X[2 * (i * ld + k) + 1] = (T)im;
    }
}

template <typename T>
__global__ void k_phase(T *X, int64_t n, int64_t n_s, int64_t ld, uint64_t key)
{
    const int64_t total = n * n_s, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += stride) {
        const int64_t i = idx / n_s, k = idx - (idx / n_s) * n_s;
        const double u = du01(key, (uint64_t)idx);
        double s, c;
        sincospi(2.0 * u, &s, &c);
        X[2 * (i * ld + k)] = (T)c;
        X[2 * (i * ld + k) + 1] = (T)s;
    }
}

template <typename TI, typename TO>
__global__ void k_convert(const TI *__restrict__ X, TO *__restrict__ Y, int64_t n, int64_t n_s,
                          int64_t ld_in, int64_t ld_out)
{
    const int64_t total = n * n_s, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += stride) {
        const int64_t i = idx / n_s, k = idx - (idx / n_s) * n_s;
        Y[2 * (i * ld_out + k)] = (TO)X[2 * (i * ld_in + k)];
        Y[2 * (i * ld_out + k) + 1] = (TO)X[2 * (i * ld_in + k) + 1];
    }
}

inline unsigned nblocks(int64_t total, int per) { return (unsigned)((total + per - 1) / per); }

// Grid of the element-wise kernels (one element per lane, grid-stride): a
// dispatch holds fewer than 2^32 work-items, and a block of N x N_S
// elements can hold more (N = 2^24 rows, N_S = 256), so the grid is capped
// at 2^20 workgroups of 256 lanes and each lane strides over the rest.
inline unsigned elem_grid(int64_t total)
{
    return (unsigned)std::min<int64_t>((total + 255) / 256, (int64_t)1 << 20);
}

// Scaled residual block of the correction pass, rounded to complex64:
// R[:, j] = HV[:, j] - t_j V[:, j] for j < k (HV the scaled product
// (alpha H + beta) V, t_j the scaled Ritz value), zero for k <= j < kk.
__global__ void k_defect(const double *__restrict__ V, const double *__restrict__ HV,
                         const double *__restrict__ t, float *__restrict__ R, int64_t n,
                         int64_t k, int64_t kk, int64_t ld_v, int64_t ld_r)
{
    const int64_t total = n * kk, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += stride) {
        const int64_t i = idx / kk, j = idx - (idx / kk) * kk;
        float re = 0.0f, im = 0.0f;
        if (j < k) {
            const double *v = V + 2 * (i * ld_v + j), *h = HV + 2 * (i * ld_v + j);
            re = (float)__builtin_fma(-t[j], v[0], h[0]);
            im = (float)__builtin_fma(-t[j], v[1], h[1]);
        }
        R[2 * (i * ld_r + j)] = re;
        R[2 * (i * ld_r + j) + 1] = im;
    }
}

// V[:, j] = p_j V[:, j] + D[:, j] (D complex64), j < k.
__global__ void k_combine(double *__restrict__ V, const float *__restrict__ D,
                          const double *__restrict__ pt, int64_t n, int64_t k, int64_t ld_v,
                          int64_t ld_d)
{
    const int64_t total = n * k, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += stride) {
        const int64_t i = idx / k, j = idx - (idx / k) * k;
        double *v = V + 2 * (i * ld_v + j);
        const float *d = D + 2 * (i * ld_d + j);
        v[0] = __builtin_fma(pt[j], v[0], (double)d[0]);
        v[1] = __builtin_fma(pt[j], v[1], (double)d[1]);
    }
}

// Attainable-bandwidth probes (the read-only reduction of Sec. 4.1, a copy,
// and the fused step's five streams without the gather).  A workgroup owns
// one contiguous tile of 256 x PU 16-byte elements and issues all PU
// accesses of a lane before the first use, so every lane keeps PU requests
// in flight; streamed data carries the non-temporal hint, as in the step.
typedef double pd2 __attribute__((ext_vector_type(2)));
constexpr int PU = 4;

__global__ __launch_bounds__(256) void k_read_reduce(const pd2 *__restrict__ p, int64_t n16,
                                                     double *__restrict__ out)
{
    const int64_t base = (int64_t)blockIdx.x * (256 * PU) + threadIdx.x;
    pd2 v[PU];
#pragma unroll
    for (int k = 0; k < PU; ++k) {
        const int64_t i = base + 256 * k;
        v[k] = i < n16 ? __builtin_nontemporal_load(p + i) : pd2{0.0, 0.0};
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < PU; ++k) s += v[k].x + v[k].y;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void k_copy16(const pd2 *__restrict__ src, pd2 *__restrict__ dst,
                                                int64_t n16)
{
    const int64_t base = (int64_t)blockIdx.x * (256 * PU) + threadIdx.x;
    pd2 v[PU];
#pragma unroll
    for (int k = 0; k < PU; ++k) {
        const int64_t i = base + 256 * k;
        if (i < n16) v[k] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int k = 0; k < PU; ++k) {
        const int64_t i = base + 256 * k;
        if (i < n16) __builtin_nontemporal_store(v[k], dst + i);
    }
}

// The fused step's streams without the gather: read u, w, x; write
// w = 2u - w and x = x + w/2 (three reads, two writes per element).
__global__ __launch_bounds__(256) void k_stream_3r2w(const pd2 *__restrict__ u, pd2 *w, pd2 *x,
                                                     int64_t n16)
{
    const int64_t base = (int64_t)blockIdx.x * (256 * PU) + threadIdx.x;
    pd2 a[PU], b[PU], c[PU];
#pragma unroll
    for (int k = 0; k < PU; ++k) {
        const int64_t i = base + 256 * k;
        if (i < n16) {
            a[k] = u[i];
            b[k] = __builtin_nontemporal_load(w + i);
            c[k] = __builtin_nontemporal_load(x + i);
        }
    }
#pragma unroll
    for (int k = 0; k < PU; ++k) {
        const int64_t i = base + 256 * k;
        if (i < n16) {
            const pd2 wn = 2.0 * a[k] - b[k];
            __builtin_nontemporal_store(wn, w + i);
            __builtin_nontemporal_store(c[k] + 0.5 * wn, x + i);
        }
    }
}

// Real (2k x 2m) expansion of a complex (k x m) matrix for A T products.
__global__ void k_expand_T(const double *__restrict__ T, int64_t k, int64_t m,
                           double *__restrict__ Tr)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= k * m) return;
    const int64_t r = idx / m, c = idx - (idx / m) * m;
    const double re = T[2 * idx], im = T[2 * idx + 1];
    const int64_t mc = 2 * m;
    Tr[(2 * r) * mc + 2 * c] = re;
    Tr[(2 * r) * mc + 2 * c + 1] = im;
    Tr[(2 * r + 1) * mc + 2 * c] = -im;
    Tr[(2 * r + 1) * mc + 2 * c + 1] = re;
}

// Copies selected columns: dst[:, d0 + j] = src[:, idx[j]], j < m.
template <typename T>
__global__ void k_gather_cols(const T *__restrict__ src, int64_t lds, T *__restrict__ dst,
                              int64_t ldd, int64_t d0, const int32_t *__restrict__ idx, int64_t n,
                              int64_t m)
{
    const int64_t total = n * m, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        const int64_t i = t / m, j = t - (t / m) * m;
        const int64_t s = 2 * (i * lds + idx[j]), d = 2 * (i * ldd + d0 + j);
        dst[d] = src[s];
        dst[d + 1] = src[s + 1];
    }
}

}  // namespace

// ---------------------------------------------------------------- launchers
int launch_gram(chebfd_ctx *ctx, int prec, const void *A, int64_t lda, int64_t n_a, const void *B,
                int64_t ldb, int64_t n_b, int64_t n, double *S_dev)
{
    const int64_t ma = 2 * n_a, mb = 2 * n_b;
    const int64_t tm = (ma + GT - 1) / GT, tn = (mb + GT - 1) / GT;
    // split the rows so that about 2048 workgroups run; whole 16-row stages
    int64_t ks = (2048 + tm * tn - 1) / (tm * tn);
    int64_t maxks = (n + 4 * GK - 1) / (4 * GK);
    if (ks > maxks) ks = maxks;
    if (ks < 1) ks = 1;
    int64_t rows = (n + ks - 1) / ks;
    rows = (rows + GK - 1) / GK * GK;
    ks = (n + rows - 1) / rows;
    const size_t need = (size_t)ks * ma * mb * sizeof(double);
    int rc = ensure_scratch(ctx, need);
    if (rc) return rc;
    double *part = (double *)ctx->scratch;
    dim3 grid((unsigned)tm, (unsigned)tn, (unsigned)ks);
    if (prec == CHEBFD_PREC_C128)
        hipLaunchKernelGGL(k_gram<double>, grid, dim3(256), 0, ctx->stream, (const double *)A,
                           2 * lda, ma, (const double *)B, 2 * ldb, mb, n, rows, part);
    else
        hipLaunchKernelGGL(k_gram<float>, grid, dim3(256), 0, ctx->stream, (const float *)A,
                           2 * lda, ma, (const float *)B, 2 * ldb, mb, n, rows, part);
    CHEBFD_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_gram_reduce, dim3(nblocks(n_a * n_b, 256)), dim3(256), 0, ctx->stream,
                       part, ks, ma, mb, n_a, n_b, S_dev);
    CHEBFD_CHECK_LAUNCH();
    return CHEBFD_OK;
}

int launch_block_times(chebfd_ctx *ctx, int prec_a, const void *A, int64_t lda, int64_t n,
                       int64_t k, const double *Tr_dev, int64_t m, int prec_c, void *C,
                       int64_t ldc, int c_beta)
{
    // Tr_dev is the real (2k x 2m) expansion of T
    const int64_t ka = 2 * k, mc = 2 * m;
    const int64_t ntc = (mc + GT - 1) / GT, ntr = (n + GT - 1) / GT;
    dim3 grid((unsigned)(ntc * ntr));
#define CHEBFD_BT(TA, TC, SUB)                                                               \
    hipLaunchKernelGGL((k_block_times<TA, TC, SUB>), grid, dim3(256), 0, ctx->stream,          \
                       (const TA *)A, 2 * lda, n, ka, Tr_dev, mc, (TC *)C, 2 * ldc, ntc)
    const bool a64 = prec_a == CHEBFD_PREC_C128, c64o = prec_c == CHEBFD_PREC_C128;
    if (a64 && c64o) {
        if (c_beta) CHEBFD_BT(double, double, true); else CHEBFD_BT(double, double, false);
    } else if (a64 && !c64o) {
        if (c_beta) CHEBFD_BT(double, float, true); else CHEBFD_BT(double, float, false);
    } else if (!a64 && c64o) {
        if (c_beta) CHEBFD_BT(float, double, true); else CHEBFD_BT(float, double, false);
    } else {
        if (c_beta) CHEBFD_BT(float, float, true); else CHEBFD_BT(float, float, false);
    }
#undef CHEBFD_BT
    CHEBFD_CHECK_LAUNCH();
    return CHEBFD_OK;
}

int launch_residuals(chebfd_ctx *ctx, int prec, const void *V, const void *HV, int64_t n,
                     int64_t m, int64_t ld, const double *theta_dev, double *res_dev)
{
    const int64_t rows = 2048;
    const int64_t nblk = (n + rows - 1) / rows;
    const size_t need = (size_t)nblk * m * sizeof(double);
    int rc = ensure_scratch(ctx, need);
    if (rc) return rc;
    double *part = (double *)ctx->scratch;
    dim3 grid((unsigned)nblk, (unsigned)((m + 255) / 256));
    if (prec == CHEBFD_PREC_C128)
        hipLaunchKernelGGL(k_residual<double>, grid, dim3(256), 0, ctx->stream,
                           (const double *)V, (const double *)HV, n, m, ld, theta_dev, rows, part);
    else
        hipLaunchKernelGGL(k_residual<float>, grid, dim3(256), 0, ctx->stream, (const float *)V,
                           (const float *)HV, n, m, ld, theta_dev, rows, part);
    CHEBFD_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_residual_reduce, dim3(nblocks(m, 256)), dim3(256), 0, ctx->stream, part,
                       nblk, m, res_dev);
    CHEBFD_CHECK_LAUNCH();
    return CHEBFD_OK;
}

int launch_random(chebfd_ctx *ctx, int prec, void *X, int64_t n, int64_t n_s, int64_t ld,
                  int64_t k0, int64_t m, uint64_t seed, uint64_t stream, uint64_t offset)
{
    const uint64_t key = mix64(seed + 0x9E3779B97F4A7C15ULL * (stream + 1u));
    if (n * m == 0) return CHEBFD_OK;
    if (prec == CHEBFD_PREC_C128)
        hipLaunchKernelGGL(k_random<double>, dim3(elem_grid(n * m)), dim3(256), 0,
                           ctx->stream, (double *)X, n, n_s, ld, k0, m, key, offset);
    else
        hipLaunchKernelGGL(k_random<float>, dim3(elem_grid(n * m)), dim3(256), 0, ctx->stream,
                           (float *)X, n, n_s, ld, k0, m, key, offset);
    CHEBFD_CHECK_LAUNCH();
    return CHEBFD_OK;
}

int launch_expand_T(chebfd_ctx *ctx, const double *T, int64_t k, int64_t m, double *Tr)
{
    if (k * m == 0) return CHEBFD_OK;
    hipLaunchKernelGGL(k_expand_T, dim3(nblocks(k * m, 256)), dim3(256), 0, ctx->stream, T, k, m,
                       Tr);
    CHEBFD_CHECK_LAUNCH();
    return CHEBFD_OK;
}

int launch_gather_cols(chebfd_ctx *ctx, int prec, const void *src, int64_t lds, void *dst,
                       int64_t ldd, int64_t d0, const int32_t *idx_dev, int64_t n, int64_t m)
{
    if (n * m == 0) return CHEBFD_OK;
    if (prec == CHEBFD_PREC_C128)
        hipLaunchKernelGGL(k_gather_cols<double>, dim3(elem_grid(n * m)), dim3(256), 0,
                           ctx->stream, (const double *)src, lds, (double *)dst, ldd, d0, idx_dev,
                           n, m);
    else
        hipLaunchKernelGGL(k_gather_cols<float>, dim3(elem_grid(n * m)), dim3(256), 0,
                           ctx->stream, (const float *)src, lds, (float *)dst, ldd, d0, idx_dev,
                           n, m);
    CHEBFD_CHECK_LAUNCH();
    return CHEBFD_OK;
}

int launch_bandwidth_probe(chebfd_ctx *ctx, void *buf, int64_t bytes, int reps, double *gbs)
{
    const int64_t n16 = bytes / 16;
    const int64_t half = n16 / 2, third = n16 / 3;
    auto tiles = [](int64_t m) { return (unsigned)((m + 256 * PU - 1) / (256 * PU)); };
    int rc = ensure_scratch(ctx, (size_t)tiles(n16) * sizeof(double));
    if (rc) return rc;
    double *part = (double *)ctx->scratch;
    pd2 *p = (pd2 *)buf;
    hipEvent_t e0, e1;
    CHEBFD_HIP(hipEventCreate(&e0));
    CHEBFD_HIP(hipEventCreate(&e1));
    for (int which = 0; which < 3; ++which) {
        float ms = 0.0f;
        for (int r = -1; r < reps; ++r) {   // r = -1: warm-up
            if (r == 0) CHEBFD_HIP(hipEventRecord(e0, ctx->stream));
            if (which == 0)
                hipLaunchKernelGGL(k_read_reduce, dim3(tiles(n16)), dim3(256), 0, ctx->stream, p,
                                   n16, part);
            else if (which == 1)
                hipLaunchKernelGGL(k_copy16, dim3(tiles(half)), dim3(256), 0, ctx->stream, p,
                                   p + half, half);
            else
                hipLaunchKernelGGL(k_stream_3r2w, dim3(tiles(third)), dim3(256), 0, ctx->stream,
                                   p, p + third, p + 2 * third, third);
        }
        CHEBFD_HIP(hipEventRecord(e1, ctx->stream));
        CHEBFD_HIP(hipEventSynchronize(e1));
        CHEBFD_HIP(hipEventElapsedTime(&ms, e0, e1));
        const double moved = which == 0 ? n16 * 16.0 : (which == 1 ? half * 32.0 : third * 80.0);
        gbs[which] = moved * reps / (ms * 1e-3) / 1e9;
    }
    CHEBFD_HIP(hipEventDestroy(e0));
    CHEBFD_HIP(hipEventDestroy(e1));
    CHEBFD_CHECK_LAUNCH();
    return CHEBFD_OK;
}

int launch_phase_block(chebfd_ctx *ctx, int prec, void *X, int64_t n, int64_t n_s, int64_t ld,
                       uint64_t seed, uint64_t stream)
{
    const uint64_t key = mix64(seed + 0x9E3779B97F4A7C15ULL * (stream + 1u));
    if (n * n_s == 0) return CHEBFD_OK;
    if (prec == CHEBFD_PREC_C128)
        hipLaunchKernelGGL(k_phase<double>, dim3(elem_grid(n * n_s)), dim3(256), 0,
                           ctx->stream, (double *)X, n, n_s, ld, key);
    else
        hipLaunchKernelGGL(k_phase<float>, dim3(elem_grid(n * n_s)), dim3(256), 0,
                           ctx->stream, (float *)X, n, n_s, ld, key);
    CHEBFD_CHECK_LAUNCH();
    return CHEBFD_OK;
}

int launch_defect(chebfd_ctx *ctx, const void *V, const void *HV, const double *t_dev, void *R,
                  int64_t n, int64_t k, int64_t kk, int64_t ld_v, int64_t ld_r)
{
    if (n * kk == 0) return CHEBFD_OK;
    hipLaunchKernelGGL(k_defect, dim3(elem_grid(n * kk)), dim3(256), 0, ctx->stream,
                       (const double *)V, (const double *)HV, t_dev, (float *)R, n, k, kk, ld_v,
                       ld_r);
    CHEBFD_CHECK_LAUNCH();
    return CHEBFD_OK;
}

int launch_combine(chebfd_ctx *ctx, void *V, const void *D, const double *p_dev, int64_t n,
                   int64_t k, int64_t ld_v, int64_t ld_d)
{
    if (n * k == 0) return CHEBFD_OK;
    hipLaunchKernelGGL(k_combine, dim3(elem_grid(n * k)), dim3(256), 0, ctx->stream,
                       (double *)V, (const float *)D, p_dev, n, k, ld_v, ld_d);
    CHEBFD_CHECK_LAUNCH();
    return CHEBFD_OK;
}

int launch_convert(chebfd_ctx *ctx, int prec_in, const void *X, int prec_out, void *Y, int64_t n,
                   int64_t n_s, int64_t ld_in, int64_t ld_out)
{
    if (n * n_s == 0) return CHEBFD_OK;
    const unsigned g = elem_grid(n * n_s);
    if (prec_in == CHEBFD_PREC_C128 && prec_out == CHEBFD_PREC_C64)
        hipLaunchKernelGGL((k_convert<double, float>), dim3(g), dim3(256), 0, ctx->stream,
                           (const double *)X, (float *)Y, n, n_s, ld_in, ld_out);
    else if (prec_in == CHEBFD_PREC_C64 && prec_out == CHEBFD_PREC_C128)
        hipLaunchKernelGGL((k_convert<float, double>), dim3(g), dim3(256), 0, ctx->stream,
                           (const float *)X, (double *)Y, n, n_s, ld_in, ld_out);
    else if (prec_in == CHEBFD_PREC_C128)
        hipLaunchKernelGGL((k_convert<double, double>), dim3(g), dim3(256), 0, ctx->stream,
                           (const double *)X, (double *)Y, n, n_s, ld_in, ld_out);
    else
        hipLaunchKernelGGL((k_convert<float, float>), dim3(g), dim3(256), 0, ctx->stream,
                           (const float *)X, (float *)Y, n, n_s, ld_in, ld_out);
    CHEBFD_CHECK_LAUNCH();
    return CHEBFD_OK;
}

}  // namespace chebfd
