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
// slab wide; the chunk order itself is the matrix's row order (for large
// lattices a tiled order, built with the matrix).
#include <algorithm>
#include <type_traits>

#include "dispatch.h"
#include "internal.h"
#include "pack.h"

namespace chebfd {
namespace {

// Complex matrix value j of a SELL stream as (re, im), one vector load, and
// its LDS counterpart.
template <typename T>
struct CVal;
template <>
struct CVal<double> {
    typedef d2v V;
};
template <>
struct CVal<float> {
    typedef float V __attribute__((ext_vector_type(2)));
};

template <typename T>
__device__ __forceinline__ void load_value(const T *val, int64_t j, T &re, T &im)
{
    const typename CVal<T>::V v = *reinterpret_cast<const typename CVal<T>::V *>(val + 2 * j);
    re = v.x;
    im = v.y;
}

template <typename T>
__device__ __forceinline__ void store_value(T *p, T re, T im)
{
    typename CVal<T>::V v;
    v.x = re;
    v.y = im;
    *reinterpret_cast<typename CVal<T>::V *>(p) = v;
}

// acc += h * g for complex h, g, as four fused multiply-adds in a fixed
// order, so that every SELL layout computes each row's sum with the same
// operations (an entry with h = 0 leaves acc unchanged).
template <typename T>
__device__ __forceinline__ T fmadd(T a, T b, T c)
{
    if constexpr (std::is_same<T, double>::value) return __builtin_fma(a, b, c);
    else return __builtin_fmaf(a, b, c);
}

template <typename T>
__device__ __forceinline__ void cmac(T &ar, T &ai, T hr, T hi, T gr, T gi)
{
    ar = fmadd<T>(hr, gr, ar);
    ar = fmadd<T>(-hi, gi, ar);
    ai = fmadd<T>(hr, gi, ai);
    ai = fmadd<T>(hi, gr, ai);
}

// Block row r of a row-major block as a byte offset from the lane's column
// base: one 32x32->64-bit multiply-add per gather (row_bytes = ld * entry
// size, checked on the host to fit 32 bits).
template <typename T>
__device__ __forceinline__ const T *row_at(const char *ub, uint32_t r, uint32_t row_bytes)
{
    return reinterpret_cast<const T *>(ub + (uint64_t)r * row_bytes);
}

constexpr int LS = kStageLen;   // staged entries per row; longer rows read the stream directly

// Accumulates one row of the sparse product from the LDS stage.  The stage
// keeps the SELL order (entry j of block row q at j*RPP + q) and pads every
// row past its length up to LS entries with the row itself and value 0, so
// all GB column indices and values of a batch can be read unguarded; all
// gathers of the batch are issued before the first value is used.
template <typename T, int NB, int GB, int RPP>
__device__ __forceinline__ void row_product_staged(const char *ub, uint32_t row_bytes, int cnt,
                                                   int len, const int32_t *scol, const T *sval,
                                                   T (&ar)[NB], T (&ai)[NB])
{
    static_assert(LS % GB == 0, "batches tile the LDS line");
#pragma unroll
    for (int e = 0; e < NB; ++e) ar[e] = ai[e] = T(0);
    for (int j = 0; j < len; j += GB) {
        int ci[GB];
#pragma unroll
        for (int i = 0; i < GB; ++i) ci[i] = scol[(j + i) * RPP];
        // the length is uniform over the workgroup: the guards are scalar
        // branches, and padded entries (row itself, value 0) past len are
        // neither gathered nor used
        Pack<T, NB> g[GB];
#pragma unroll
        for (int i = 0; i < GB; ++i) {
            if (j + i < len) {
                g[i] = load_pack_n<T, NB>(row_at<T>(ub, ci[i], row_bytes), cnt);
            } else {
#pragma unroll
                for (int e = 0; e < NB; ++e) g[i].re[e] = g[i].im[e] = T(0);
            }
        }
        // keep the whole batch in flight before the first use
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < GB; ++i) {
            T hr, hi;
            load_value<T>(sval, (int64_t)(j + i) * RPP, hr, hi);
#pragma unroll
            for (int e = 0; e < NB; ++e) cmac<T>(ar[e], ai[e], hr, hi, g[i].re[e], g[i].im[e]);
        }
    }
}

// The same from the global index stream (rows longer than the LDS stage).
template <typename T, int NB, int GB>
__device__ __forceinline__ void row_product_stream(const char *ub, uint32_t row_bytes, int cnt,
                                                   int len, const int32_t *__restrict__ col,
                                                   const T *__restrict__ val, int64_t e0,
                                                   int C, T (&ar)[NB], T (&ai)[NB])
{
#pragma unroll
    for (int e = 0; e < NB; ++e) ar[e] = ai[e] = T(0);
    for (int j = 0; j < len; j += GB) {
        Pack<T, NB> g[GB];
        T hr[GB], hi[GB];
#pragma unroll
        for (int i = 0; i < GB; ++i) {
            if (j + i < len) {
                const int64_t e = e0 + (int64_t)(j + i) * C;
                load_value<T>(val, e, hr[i], hi[i]);
                g[i] = load_pack_n<T, NB>(row_at<T>(ub, (uint32_t)col[e], row_bytes), cnt);
            }
        }
#pragma unroll
        for (int i = 0; i < GB; ++i) {
            if (j + i < len) {
#pragma unroll
                for (int e = 0; e < NB; ++e)
                    cmac<T>(ar[e], ai[e], hr[i], hi[i], g[i].re[e], g[i].im[e]);
            }
        }
    }
}

// Workgroup barrier that orders LDS only: the wave's outstanding global
// loads and stores stay in flight across it (a plain __syncthreads would
// wait for them).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// A unit of work: RB <= C consecutive rows of one chunk (a row block) times
// one column slab.  32-bit indices (the host checks the counts).
struct BlockLoc {
    uint32_t slab, rb, chunk, r0, len;
    int64_t base;
};

// Logical work item l -> block, slab-major: all row blocks of slab 0, then
// slab 1, ...  The row blocks per chunk are a power of two (2^lg_bpc).
__device__ __forceinline__ BlockLoc locate(uint32_t l, uint32_t nrb, int lg_bpc, int RB,
                                          const int64_t *__restrict__ chunk_ptr,
                                          const int32_t *__restrict__ chunk_len)
{
    BlockLoc L;
    L.slab = l / nrb;
    L.rb = l - L.slab * nrb;
    L.chunk = L.rb >> lg_bpc;
    L.r0 = (L.rb & ((1u << lg_bpc) - 1)) * RB;
    L.len = chunk_len[L.chunk];
    L.base = chunk_ptr[L.chunk];
    return L;
}

// The block's index/value stream in LDS, in SELL order: lane t carries
// entry t = j*RPP + q, so both the global loads (consecutive rows of one
// SELL column) and the LDS stores are contiguous.  Entries past a row's
// length become (row itself, 0).
template <typename T, int RPP>
struct Stage {
    static constexpr int PER = (RPP * LS + 255) / 256;
    int32_t cc[PER];
    T vr[PER], vi[PER];
    int32_t prow;   // perm entry of block row tid % RPP (-1: no row)
};

template <typename T, int RPP>
__device__ __forceinline__ void stage_load(Stage<T, RPP> &st, const BlockLoc &L, int tid, int C,
                                           int RB, const int32_t *__restrict__ perm,
                                           const int32_t *__restrict__ col,
                                           const T *__restrict__ val)
{
    static_assert(256 % RPP == 0, "a lane stages one block row");
    const int qq = tid % RPP;
    st.prow = qq < RB ? perm[(int64_t)L.chunk * C + L.r0 + qq] : -1;
#pragma unroll
    for (int k = 0; k < Stage<T, RPP>::PER; ++k) {
        const int t = tid + 256 * k, jj = t / RPP;
        if (t < RPP * LS && qq < RB && jj < (int)L.len) {
            const int64_t e = L.base + (int64_t)jj * C + L.r0 + qq;
            st.cc[k] = col[e];
            load_value<T>(val, e, st.vr[k], st.vi[k]);
        }
    }
}

template <typename T, int RPP>
__device__ __forceinline__ void stage_store(const Stage<T, RPP> &st, const BlockLoc &L, int tid,
                                            int RB, int32_t *s_col, T *s_val, int32_t *s_row)
{
    const int qq = tid % RPP;
#pragma unroll
    for (int k = 0; k < Stage<T, RPP>::PER; ++k) {
        const int t = tid + 256 * k, jj = t / RPP;
        if (t < RPP * LS && qq < RB) {
            const bool in = jj < (int)L.len;
            s_col[t] = in ? st.cc[k] : st.prow;
            store_value<T>(s_val + 2 * t, in ? st.vr[k] : T(0), in ? st.vi[k] : T(0));
        }
    }
    if (tid < RPP) s_row[tid] = st.prow;
}

// The fused step of one row given its product (ar, ai) and its own
// operands; the moment sums of the row are added to m0..m2.
template <typename T, int NB, int MODE, bool MOM, bool NT>
__device__ __forceinline__ void finish_row(int64_t off, int cnt, const T (&ar)[NB],
                                           const T (&ai)[NB], const Pack<T, NB> &uo,
                                           const Pack<T, NB> &wo, Pack<T, NB> yv, T *wout, T *y,
                                           T s_h, T s_u, const T (&g0)[NB], const T (&g1)[NB],
                                           const T (&g2)[NB], double (&m0)[NB],
                                           double (&m1)[NB], double (&m2)[NB])
{
    // explicit fused multiply-adds throughout, so that every kernel that
    // ends in this epilogue rounds identically
    Pack<T, NB> w;
#pragma unroll
    for (int e = 0; e < NB; ++e) {
        w.re[e] = fmadd<T>(s_h, ar[e], s_u * uo.re[e]);
        w.im[e] = fmadd<T>(s_h, ai[e], s_u * uo.im[e]);
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
        return;
    }
    if (MODE == MODE_SECOND) {
        Pack<T, NB> xn;
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            w.re[e] -= wo.re[e];
            w.im[e] -= wo.im[e];
            xn.re[e] = fmadd<T>(g2[e], w.re[e], fmadd<T>(g1[e], uo.re[e], g0[e] * wo.re[e]));
            xn.im[e] = fmadd<T>(g2[e], w.im[e], fmadd<T>(g1[e], uo.im[e], g0[e] * wo.im[e]));
        }
        store_pack_n<T, NB, NT>(wout + off, w, cnt);
        store_pack_n<T, NB, NT>(y + off, xn, cnt);
    } else {
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            w.re[e] -= wo.re[e];
            w.im[e] -= wo.im[e];
            yv.re[e] = fmadd<T>(g0[e], w.re[e], yv.re[e]);
            yv.im[e] = fmadd<T>(g0[e], w.im[e], yv.im[e]);
        }
        store_pack_n<T, NB, NT>(wout + off, w, cnt);
        store_pack_n<T, NB, NT>(y + off, yv, cnt);
    }
    if (MOM) {
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            m1[e] += (double)uo.re[e] * w.re[e] + (double)uo.im[e] * w.im[e];
            m2[e] += (double)w.re[e] * w.re[e] + (double)w.im[e] * w.im[e];
        }
    }
}

// The fused step on one row and one pack of columns (modes as above), with
// the moment dot products accumulated in m0..m2.
template <typename T, int NB, int MODE, bool MOM, bool NT, bool STAGED, int GB, int RPP, bool PC>
__device__ __forceinline__ void step_row(int row, int64_t c0, int cnt, int len,
                                         const int32_t *scol, const T *sval,
                                         const int32_t *__restrict__ col,
                                         const T *__restrict__ val, int64_t e0, int C,
                                         const T *__restrict__ u, const T *wold, T *wout, T *y,
                                         int64_t ld, T s_h, T s_u, T g0, T g1, T g2,
                                         const double *gcol, int64_t ldg, double (&m0)[NB],
                                         double (&m1)[NB], double (&m2)[NB])
{
    const uint32_t row_bytes = (uint32_t)(ld * 2 * sizeof(T));
    const char *ub = reinterpret_cast<const char *>(u + 2 * c0);
    // the row's own operands first: they do not depend on the product
    const int64_t off = 2 * ((int64_t)row * ld + c0);
    const Pack<T, NB> uo = load_pack_n<T, NB>(u + off, cnt);
    Pack<T, NB> wo, yv;
    if (MODE == MODE_SECOND || MODE == MODE_STEP) wo = load_pack_n<T, NB, NT>(wold + off, cnt);
    if (MODE == MODE_STEP) yv = load_pack_n<T, NB, NT>(y + off, cnt);
    T ar[NB], ai[NB];
    if (STAGED)
        row_product_staged<T, NB, GB, RPP>(ub, row_bytes, cnt, len, scol, sval, ar, ai);
    else
        row_product_stream<T, NB, GB>(ub, row_bytes, cnt, len, col, val, e0, C, ar, ai);
    T k0[NB], k1[NB], k2[NB];
    lane_coeffs<T, NB, MODE == MODE_SECOND, PC>(gcol, ldg, c0, cnt, g0, g1, g2, k0, k1, k2);
    finish_row<T, NB, MODE, MOM, NT>(off, cnt, ar, ai, uo, wo, yv, wout, y, s_h, s_u, k0, k1, k2,
                                     m0, m1, m2);
}

// Per-column moment partials of one row block: reduce over the rows of the
// wave (lanes with the same column), then over the four waves through LDS,
// in a fixed order; row block rb writes its own partial row.
template <int LPR, int NB>
__device__ __forceinline__ void moment_partials(double (&m0)[NB], double (&m1)[NB],
                                                double (&m2)[NB], double (*red)[64][3 * NB],
                                                int wave, int lane, int64_t rb, int64_t c0,
                                                int cnt, int64_t n_s, double *partials)
{
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
    lds_barrier();
    if (wave == 0 && lane < LPR && c0 < n_s) {
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            if (e >= cnt) continue;
            double *p = partials + 3 * (rb * n_s + c0 + e);
#pragma unroll
            for (int q = 0; q < 3; ++q)
                p[q] = red[0][lane][3 * e + q] + red[1][lane][3 * e + q] +
                       red[2][lane][3 * e + q] + red[3][lane][3 * e + q];
        }
    }
    lds_barrier();   // red is reused by the next block
}

// One row block per workgroup; rows longer than the LDS stage read the
// index stream directly.
template <typename T, int LPR, int NB, int MODE, bool MOM, bool NT, bool STAGED, int GB, bool PC>
__global__ __launch_bounds__(256) void k_step_sell(
    const int64_t *__restrict__ chunk_ptr, const int32_t *__restrict__ chunk_len,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ col,
    const T *__restrict__ val, int C, int RB, int lg_bpc, uint32_t nrb,
    const T *__restrict__ u, const T *wold, T *wout, T *y, int64_t n_s, int64_t ld, T s_h,
    T s_u, T g0, T g1, T g2, const double *__restrict__ gcol, int64_t ldg,
    double *__restrict__ partials, int lg_xg, int spw, int nslab)
{
    constexpr int RPW = 64 / LPR;        // rows per wave
    constexpr int RPP = 4 * RPW;         // rows per workgroup
    constexpr int SW = LPR * NB;         // slab width in complex columns
    __shared__ __align__(16) int32_t s_col[STAGED ? RPP * LS : 4];
    __shared__ __align__(16) T s_val[STAGED ? 2 * RPP * LS : 2];
    __shared__ int32_t s_row[RPP];
    __shared__ double red[MOM ? 4 : 1][64][3 * NB];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int rsub = lane / LPR, cl = lane % LPR;
    const BlockLoc L = locate(xcd_remap(blockIdx.x, gridDim.x, lg_xg), nrb, lg_bpc, RB,
                              chunk_ptr, chunk_len);
    {
        Stage<T, RPP> st;
        if (STAGED) {
            stage_load<T, RPP>(st, L, tid, C, RB, perm, col, val);
            stage_store<T, RPP>(st, L, tid, RB, s_col, s_val, s_row);
        } else if (tid < RPP) {
            s_row[tid] = tid < RB ? perm[(int64_t)L.chunk * C + L.r0 + tid] : -1;
        }
        lds_barrier();
    }
    const int q = wave * RPW + rsub;     // block row of this lane
    const int row = s_row[q];
    // the workgroup's slabs (a group of spw consecutive slabs) reuse the stage
    for (int sl = 0; sl < spw; ++sl) {
        const int slab = (int)L.slab * spw + sl;
        if (slab >= nslab) break;
        const int64_t c0 = (int64_t)slab * SW + (int64_t)cl * NB;
        const int cnt = (int)((n_s - c0) < NB ? (n_s - c0) : NB);   // valid columns of the pack
        double m0[NB], m1[NB], m2[NB];
#pragma unroll
        for (int e = 0; e < NB; ++e) m0[e] = m1[e] = m2[e] = 0.0;
        if (c0 < n_s && row >= 0)
            step_row<T, NB, MODE, MOM, NT, STAGED, GB, RPP, PC>(
                row, c0, cnt, L.len, s_col + q, s_val + 2 * q, col, val, L.base + L.r0 + q, C,
                u, wold, wout, y, ld, s_h, s_u, g0, g1, g2, gcol, ldg, m0, m1, m2);
        if (MOM)
            moment_partials<LPR, NB>(m0, m1, m2, red, wave, lane, L.rb, c0, cnt, n_s, partials);
    }
}

// ---------------------------------------------------------------------------
// Row groups.  A lane owns the G rows of one slot group (G consecutive slots
// of a chunk, G = 2 or 4) and one pack of columns.  Each entry of the
// group's column union is gathered once and applied to every row of the
// group with that row's value (zero where the row has no entry), so every
// row still sums its own entries in column order, as in the one-row kernel.
// For the lattice Hamiltonian the four orbital rows of a site gather 28
// distinct rows of u: 7 gathers per row instead of 13.

// The group block's index stream and value streams in LDS, in SELL order
// (entry j of group q at j*QPW + q), padded to LS entries with (first row, 0).
template <typename T, int G, int QPW>
struct StageG {
    static constexpr int PER = (QPW * LS + 255) / 256;
    int32_t cc[PER];
    T v[PER][2 * G];
    int32_t prow[G];
};

template <typename T, int G>
__device__ __forceinline__ void load_values_g(const T *val, int64_t e, T (&v)[2 * G])
{
#pragma unroll
    for (int k = 0; k < G; ++k) {
        const typename CVal<T>::V a =
            *reinterpret_cast<const typename CVal<T>::V *>(val + 2 * (G * e + k));
        v[2 * k] = a.x;
        v[2 * k + 1] = a.y;
    }
}

template <typename T, int G, int QPW>
__device__ __forceinline__ void stageg_load(StageG<T, G, QPW> &st, const BlockLoc &L, int tid,
                                            int P, int RB, const int32_t *__restrict__ perm,
                                            const int32_t *__restrict__ col,
                                            const T *__restrict__ val)
{
    static_assert(256 % QPW == 0, "a lane stages one group");
    const int qq = tid % QPW;
    const int64_t slot = ((int64_t)L.chunk * P + L.r0 + qq) * G;
#pragma unroll
    for (int k = 0; k < G; ++k) st.prow[k] = qq < RB ? perm[slot + k] : -1;
#pragma unroll
    for (int k = 0; k < StageG<T, G, QPW>::PER; ++k) {
        const int t = tid + 256 * k, jj = t / QPW;
        if (t < QPW * LS && qq < RB && jj < (int)L.len) {
            const int64_t e = L.base + (int64_t)jj * P + L.r0 + qq;
            st.cc[k] = col[e];
            load_values_g<T, G>(val, e, st.v[k]);
        }
    }
}

template <typename T, int G, int QPW>
__device__ __forceinline__ void stageg_store(const StageG<T, G, QPW> &st, const BlockLoc &L,
                                             int tid, int RB, int32_t *s_col, T *s_val,
                                             int32_t *s_row)
{
    const int qq = tid % QPW;
    const int32_t self = st.prow[0] >= 0 ? st.prow[0] : 0;
#pragma unroll
    for (int k = 0; k < StageG<T, G, QPW>::PER; ++k) {
        const int t = tid + 256 * k, jj = t / QPW;
        if (t < QPW * LS && qq < RB) {
            const bool in = jj < (int)L.len;
            s_col[t] = in ? st.cc[k] : self;
#pragma unroll
            for (int r = 0; r < G; ++r)
                store_value<T>(s_val + 2 * (G * t + r), in ? st.v[k][2 * r] : T(0),
                               in ? st.v[k][2 * r + 1] : T(0));
        }
    }
    if (tid < QPW)
#pragma unroll
        for (int r = 0; r < G; ++r) s_row[G * tid + r] = st.prow[r];
}

// The group's products from the LDS stage: all GB gathers of a batch are
// issued before the first value is used.
template <typename T, int NB, int G, int GB, int QPW>
__device__ __forceinline__ void group_product_staged(const char *ub, uint32_t row_bytes,
                                                     int cnt, int len, const int32_t *scol,
                                                     const T *sval, T (&ar)[G][NB],
                                                     T (&ai)[G][NB])
{
    static_assert(LS % GB == 0, "batches tile the LDS line");
#pragma unroll
    for (int k = 0; k < G; ++k)
#pragma unroll
        for (int e = 0; e < NB; ++e) ar[k][e] = ai[k][e] = T(0);
    for (int j = 0; j < len; j += GB) {
        int ci[GB];
#pragma unroll
        for (int i = 0; i < GB; ++i) ci[i] = scol[(j + i) * QPW];
        Pack<T, NB> g[GB];
#pragma unroll
        for (int i = 0; i < GB; ++i) {
            if (j + i < len) {
                g[i] = load_pack_n<T, NB>(row_at<T>(ub, ci[i], row_bytes), cnt);
            } else {
#pragma unroll
                for (int e = 0; e < NB; ++e) g[i].re[e] = g[i].im[e] = T(0);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < GB; ++i) {
#pragma unroll
            for (int k = 0; k < G; ++k) {
                T hr, hi;
                load_value<T>(sval + 2 * G * (j + i) * QPW + 2 * k, 0, hr, hi);
#pragma unroll
                for (int e = 0; e < NB; ++e)
                    cmac<T>(ar[k][e], ai[k][e], hr, hi, g[i].re[e], g[i].im[e]);
            }
        }
    }
}

// One block of RB <= QPW groups per workgroup (QPW = 4 * 64 / LPR groups).
template <typename T, int LPR, int NB, int G, int MODE, bool MOM, bool NT, int GB, bool PC>
__global__ __launch_bounds__(256) void k_step_sellg(
    const int64_t *__restrict__ chunk_ptr, const int32_t *__restrict__ chunk_len,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ col,
    const T *__restrict__ val, int P, int RB, int lg_bpc, uint32_t nrb,
    const T *__restrict__ u, const T *wold, T *wout, T *y, int64_t n_s, int64_t ld, T s_h,
    T s_u, T g0, T g1, T g2, const double *__restrict__ gcol, int64_t ldg,
    double *__restrict__ partials, int lg_xg, int spw, int nslab)
{
    constexpr int QPV = 64 / LPR;        // groups per wave
    constexpr int QPW = 4 * QPV;         // groups per workgroup
    constexpr int SW = LPR * NB;
    __shared__ __align__(16) int32_t s_col[QPW * LS];
    __shared__ __align__(16) T s_val[2 * G * QPW * LS];
    __shared__ int32_t s_row[G * QPW];
    __shared__ double red[MOM ? 4 : 1][64][3 * NB];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int qsub = lane / LPR, cl = lane % LPR;
    const BlockLoc L = locate(xcd_remap(blockIdx.x, gridDim.x, lg_xg), nrb, lg_bpc, RB,
                              chunk_ptr, chunk_len);
    {
        StageG<T, G, QPW> st;
        stageg_load<T, G, QPW>(st, L, tid, P, RB, perm, col, val);
        stageg_store<T, G, QPW>(st, L, tid, RB, s_col, s_val, s_row);
        lds_barrier();
    }
    const int q = wave * QPV + qsub;     // group of this lane
    int row[G];
#pragma unroll
    for (int k = 0; k < G; ++k) row[k] = s_row[G * q + k];
    const uint32_t row_bytes = (uint32_t)(ld * 2 * sizeof(T));
    // the workgroup's slabs (a group of spw consecutive slabs) reuse the stage
    for (int sl = 0; sl < spw; ++sl) {
        const int slab = (int)L.slab * spw + sl;
        if (slab >= nslab) break;
        const int64_t c0 = (int64_t)slab * SW + (int64_t)cl * NB;
        const int cnt = (int)((n_s - c0) < NB ? (n_s - c0) : NB);
        double m0[NB], m1[NB], m2[NB];
#pragma unroll
        for (int e = 0; e < NB; ++e) m0[e] = m1[e] = m2[e] = 0.0;
        if (c0 < n_s && row[0] >= 0) {
            const char *ub = reinterpret_cast<const char *>(u + 2 * c0);
            // the rows' own operands first (a missing row reads the first one)
            int64_t off[G];
            Pack<T, NB> uo[G], wo[G], yv[G];
#pragma unroll
            for (int k = 0; k < G; ++k) {
                off[k] = 2 * ((int64_t)(row[k] >= 0 ? row[k] : row[0]) * ld + c0);
                uo[k] = load_pack_n<T, NB>(u + off[k], cnt);
                if (MODE == MODE_SECOND || MODE == MODE_STEP)
                    wo[k] = load_pack_n<T, NB, NT>(wold + off[k], cnt);
                if (MODE == MODE_STEP) yv[k] = load_pack_n<T, NB, NT>(y + off[k], cnt);
            }
            T ar[G][NB], ai[G][NB];
            group_product_staged<T, NB, G, GB, QPW>(ub, row_bytes, cnt, L.len, s_col + q,
                                                    s_val + 2 * G * q, ar, ai);
            T k0[NB], k1[NB], k2[NB];
            lane_coeffs<T, NB, MODE == MODE_SECOND, PC>(gcol, ldg, c0, cnt, g0, g1, g2, k0, k1, k2);
#pragma unroll
            for (int k = 0; k < G; ++k)
                if (row[k] >= 0)
                    finish_row<T, NB, MODE, MOM, NT>(off[k], cnt, ar[k], ai[k], uo[k], wo[k],
                                                     yv[k], wout, y, s_h, s_u, k0, k1, k2, m0,
                                                     m1, m2);
        }
        if (MOM)
            moment_partials<LPR, NB>(m0, m1, m2, red, wave, lane, L.rb, c0, cnt, n_s, partials);
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

template <int LPR>
constexpr int rows_per_block()
{
    return 4 * (64 / LPR);
}

// Row blocks of one launch: a workgroup covers min(C, 4*64/LPR) rows of one
// chunk, or as many row groups of a grouped chunk (C/G groups).
int64_t sell_row_blocks(const Sell &S, int lpr)
{
    const int rpp = 4 * (64 / lpr);
    const int units = S.C / S.group;
    const int rb = units < rpp ? units : rpp;
    return S.nchunks * (units / rb);
}

// Launch geometry of the SELL kernel.
struct SellGeom {
    int RB, lg_bpc, lg_xg, spw;
    uint32_t nrb, nslab, ngroups;   // row blocks, slabs, slab groups of spw
};

template <int LPR, int NB>
int sell_geom(const chebfd_ctx *ctx, const Sell &S, const StepArgs &a, SellGeom &g)
{
    constexpr int SW = LPR * NB;
    constexpr int RPP = rows_per_block<LPR>();
    const int64_t nslab = (a.n_s + SW - 1) / SW;
    const int64_t nrb = sell_row_blocks(S, LPR);
    // a dispatch holds fewer than 2^32 work-items: < 2^24 workgroups of 256
    if (nrb * nslab >= ((int64_t)1 << 24) || a.ld * 16 >= ((int64_t)1 << 32))
        return fail(CHEBFD_ERR_UNSUPPORTED,
                    "fused step: more than 2^24 workgroups or a row stride above 2^32 bytes");
    const int units = S.C / S.group;   // rows or row groups per chunk
    g.RB = units < RPP ? units : RPP;
    g.lg_bpc = ilog2(units / g.RB);
    // default placement: the row blocks of one chunk share an XCD, or, in a
    // tiled lattice order, the row blocks of one strip
    const int64_t grp = S.group_rows > 0 ? S.group_rows / (g.RB * S.group) : units / g.RB;
    g.lg_xg = ctx->tune_xcd_group ? ilog2(ctx->tune_xcd_group) : ilog2_64(grp);
    g.nrb = (uint32_t)nrb;
    g.nslab = (uint32_t)nslab;
    // slabs per workgroup: the stage of a row block (its index and value
    // stream) is read from memory once per slab group; by default once per
    // launch (all slabs)
    g.spw = (int)std::min<int64_t>(nslab, ctx->tune_slabs > 0 ? ctx->tune_slabs : nslab);
    g.ngroups = (uint32_t)((nslab + g.spw - 1) / g.spw);
    return CHEBFD_OK;
}

template <typename T, int LPR, int NB, int MODE, bool MOM, bool NT, bool STAGED, int GB, bool PC>
void launch_sell_k(chebfd_ctx *ctx, const Sell &S, const StepArgs &a, const SellGeom &g)
{
    const T *val = std::is_same<T, double>::value ? (const T *)S.val64 : (const T *)S.val32;
    hipLaunchKernelGGL((k_step_sell<T, LPR, NB, MODE, MOM, NT, STAGED, GB, PC>),
                       dim3(g.nrb * g.ngroups), dim3(256), 0, ctx->stream, S.chunk_ptr,
                       S.chunk_len, S.perm, S.col, val, S.C, g.RB, g.lg_bpc, g.nrb,
                       (const T *)a.u, (const T *)a.wold, (T *)a.wout, (T *)a.y, a.n_s, a.ld,
                       (T)a.s_h, (T)a.s_u, (T)a.g0, (T)a.g1, (T)a.g2, a.gcol, a.ldg, a.partials,
                       g.lg_xg, g.spw, (int)g.nslab);
}

template <typename T, int LPR, int NB, int MODE, bool MOM, bool NT, bool PC = false>
int launch_sell_t(chebfd_ctx *ctx, const Sell &S, const StepArgs &a)
{
    SellGeom g;
    if (int rc = sell_geom<LPR, NB>(ctx, S, a, g)) return rc;
    if (S.group > 1) {
        const T *val = std::is_same<T, double>::value ? (const T *)S.val64 : (const T *)S.val32;
        const auto kern = S.group == 4 ? k_step_sellg<T, LPR, NB, 4, MODE, MOM, NT, 16, PC>
                                       : k_step_sellg<T, LPR, NB, 2, MODE, MOM, NT, 16, PC>;
        hipLaunchKernelGGL(kern, dim3(g.nrb * g.ngroups), dim3(256), 0, ctx->stream,
                           S.chunk_ptr, S.chunk_len, S.perm, S.col, val, S.C / S.group, g.RB,
                           g.lg_bpc, g.nrb, (const T *)a.u, (const T *)a.wold, (T *)a.wout,
                           (T *)a.y, a.n_s, a.ld, (T)a.s_h, (T)a.s_u, (T)a.g0, (T)a.g1, (T)a.g2,
                           a.gcol, a.ldg, a.partials, g.lg_xg, g.spw, (int)g.nslab);
        CHEBFD_CHECK_LAUNCH();
        return CHEBFD_OK;
    }
    // rows that fit the LDS stage -> staged variant, else the index stream
    if (S.max_len <= LS)
        launch_sell_k<T, LPR, NB, MODE, MOM, NT, true, 16, PC>(ctx, S, a, g);
    else
        launch_sell_k<T, LPR, NB, MODE, MOM, NT, false, 8, PC>(ctx, S, a, g);
    CHEBFD_CHECK_LAUNCH();
    return CHEBFD_OK;
}

template <typename T, int LPR, int NB, bool NT>
int launch_sell_mode(chebfd_ctx *ctx, const Sell &S, const StepArgs &a)
{
    const bool mom = a.partials != nullptr;
    if (a.gcol && a.mode != MODE_APPLY) {
        // per-column coefficients (complex64, no moments)
        if constexpr (std::is_same<T, float>::value) {
            if (mom) return fail(CHEBFD_ERR_UNSUPPORTED, "per-column coefficients: no moments");
            return a.mode == MODE_SECOND
                       ? launch_sell_t<T, LPR, NB, MODE_SECOND, false, NT, true>(ctx, S, a)
                       : launch_sell_t<T, LPR, NB, MODE_STEP, false, NT, true>(ctx, S, a);
        } else {
            return fail(CHEBFD_ERR_UNSUPPORTED, "per-column coefficients: complex64 only");
        }
    }
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

// Lanes per row (or per lattice site): the narrowest slab that still covers
// the block (fewer idle lanes for thin blocks such as the KPM vectors), else
// the tuned width, else 32 lanes (512-byte row segments in c128), and for
// the matrix-free step in c64 with more than 32 packs a whole wave per site
// (1 KB row segments: 16.4 against 17.5 ms per step at 256x256x64 with
// 128 columns; in c128 32 lanes stay fastest).
int pick_lpr(const chebfd_ctx *ctx, int64_t n_s, int nb, bool stencil)
{
    const int64_t packs = (n_s + nb - 1) / nb;
    if (packs <= 16) return 16;
    if (ctx->tune_lpr == 16 || ctx->tune_lpr == 32 || ctx->tune_lpr == 64) return ctx->tune_lpr;
    if (stencil && nb == 2 && packs > 32) return 64;
    return 32;
}

int launch_step(chebfd_ctx *ctx, const chebfd_matrix *H, const StepArgs &a, int64_t *n_part)
{
    if (H->storage == CHEBFD_STORAGE_STENCIL) return launch_stencil_step(ctx, H, a, n_part);
    const Sell &S = H->sell;
    const int nb = a.precision == CHEBFD_PREC_C128 ? 1 : 2;
    const int lpr = pick_lpr(ctx, a.n_s, nb, false);
    if (n_part) *n_part = sell_row_blocks(S, lpr);
    if (a.precision == CHEBFD_PREC_C128) return launch_sell_lpr<double, 1>(ctx, S, a, lpr);
    return launch_sell_lpr<float, 2>(ctx, S, a, lpr);
}

int64_t step_partial_blocks(const chebfd_ctx *ctx, const chebfd_matrix *H, int precision,
                            int64_t n_s)
{
    const int nb = precision == CHEBFD_PREC_C128 ? 1 : 2;
    const int lpr = pick_lpr(ctx, n_s, nb, H->storage == CHEBFD_STORAGE_STENCIL);
    if (H->storage == CHEBFD_STORAGE_SELL) return sell_row_blocks(H->sell, lpr);
    // the matrix-free step writes one partial row per workgroup of a slab
    return ti_shape(ctx, H->st, n_s, precision == CHEBFD_PREC_C128 ? 8 : 4, nb, lpr).nblk;
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
