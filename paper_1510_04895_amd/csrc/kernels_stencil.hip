// Fused Chebyshev filter step for the topological-insulator Hamiltonian of
// Sec. 5.1, Eq. (Ham), generated inside the kernel (the matrix is never
// stored; only the per-site potential V_n is read).  Same three modes as the
// SELL kernel.  A lane owns one lattice site (its four orbital rows) and NB
// consecutive complex columns: it reads the four rows of the site and of its
// six neighbours (28 packs for 4 output rows instead of 13 per row with an
// index stream) and writes the four output rows.
//
// Hopping blocks, orbital o = 2 tau + s, G0 = tau_z s_0, Gj = tau_x s_j:
//   H[n, n + e_j] = -t/2 (G0 + i Gj),  H[n, n - e_j] = -t/2 (G0 - i Gj),
// so the contribution of neighbour n + d e_j (d = +-1) to row o is
//   -t/2 ( G0[o][o] u[o] + d i Gj[o][o'] u[o'] ),
// with o' the single orbital coupled by Gj: tau flipped, and s flipped for
// j = x, y (s_x = 1, s_y = -i/+i) or kept for j = z (s_z = +1/-1).
#include <algorithm>
#include <type_traits>

#include "dispatch.h"
#include "internal.h"
#include "pack.h"

namespace chebfd {
namespace {

template <typename T, int NB>
struct Site {
    Pack<T, NB> o[4];
};

template <typename T, int NB>
__device__ __forceinline__ Site<T, NB> load_site(const T *u, int64_t site, int64_t ld,
                                                 int64_t c0, int cnt)
{
    Site<T, NB> s;
#pragma unroll
    for (int o = 0; o < 4; ++o)
        s.o[o] = load_pack_n<T, NB>(u + 2 * ((4 * site + o) * ld + c0), cnt);
    return s;
}

// acc[o] += th * (g0(o) un[o] + d * i * Gj[o][o'] un[o'])   (th = -t/2)
template <typename T, int NB, int J>
__device__ __forceinline__ void add_hop(Pack<T, NB> (&acc)[4], const Site<T, NB> &un, T th,
                                        T d)
{
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        const T g0 = (o < 2) ? T(1) : T(-1);
        const int tau = o >> 1, s = o & 1;
        const int op = ((1 - tau) << 1) | (J == 2 ? s : 1 - s);
        // c = d * i * Gj[o][o'] as (cr, ci)
        T cr, ci;
        if (J == 0) {            // s_x entry 1
            cr = T(0);
            ci = d;
        } else if (J == 1) {     // s_y entry -i (s=0) or +i (s=1): d*i*(-+i) = +-d
            cr = (s == 0) ? d : -d;
            ci = T(0);
        } else {                 // s_z entry +1 (s=0) or -1 (s=1)
            cr = T(0);
            ci = (s == 0) ? d : -d;
        }
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            const T vr = g0 * un.o[o].re[e] + cr * un.o[op].re[e] - ci * un.o[op].im[e];
            const T vi = g0 * un.o[o].im[e] + cr * un.o[op].im[e] + ci * un.o[op].re[e];
            acc[o].re[e] += th * vr;
            acc[o].im[e] += th * vi;
        }
    }
}

template <typename T, int LPS, int NB, int MODE, bool MOM, bool NT, bool PC>
__global__ __launch_bounds__(256) void k_step_ti(int Lx, int Ly, int Lz, int pbc, T th, T mm,
                                                 const T *__restrict__ pot, int64_t nsites,
                                                 int64_t nblk, const T *__restrict__ u,
                                                 const T *wold, T *wout, T *y, int64_t n_s,
                                                 int64_t ld, T s_h, T s_u, T g0, T g1, T g2,
                                                 const double *__restrict__ gcol, int64_t ldg,
                                                 double *__restrict__ partials, int order,
                                                 int64_t nslab, int lg_xg, int tile)
{
    constexpr int SPW = 64 / LPS;   // sites per wave
    constexpr int SPB = 4 * SPW;    // sites per workgroup
    constexpr int SW = LPS * NB;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int ssub = lane / LPS, cl = lane % LPS;
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x, lg_xg);
    int64_t slab, sb, site;
    bool in_lattice;
    if (order == 1) {
        // tiled lattice order: inside a strip row (the `tile` x-columns of
        // one y), sites run z fastest, then x; a block is SPB consecutive
        // sites of a strip row (the last one ragged); then y, then strips,
        // then slabs (tile divides Lx), so every neighbour of a site is
        // gathered at most one strip row of work apart, on the XCD that runs
        // the strip
        const int64_t row_sites = (int64_t)tile * Lz;
        const int64_t bpr = (row_sites + SPB - 1) / SPB;   // blocks per strip row
        const int64_t per_strip = bpr * Ly;
        const int64_t nper = (Lx / tile) * per_strip;
        slab = b / nper;
        sb = b - slab * nper;
        const int64_t strip = sb / per_strip;
        const int64_t r = sb - strip * per_strip;
        const int64_t yy0 = r / bpr;
        const int64_t sr = (r - yy0 * bpr) * SPB + wave * SPW + ssub;   // site in strip row
        in_lattice = sr < row_sites;
        const int64_t xl = sr / Lz;
        const int z = (int)(sr - xl * Lz);
        site = (strip * tile + xl) + (int64_t)Lx * (yy0 + (int64_t)Ly * z);
    } else {
        // column-slab major, sites in lattice order
        slab = b / nblk;
        sb = b - slab * nblk;
        site = sb * SPB + wave * SPW + ssub;
        in_lattice = site < nsites;
    }
    const int64_t c0 = slab * SW + (int64_t)cl * NB;
    const int cnt = (int)((n_s - c0) < NB ? (n_s - c0) : NB);
    const bool active = c0 < n_s && in_lattice;

    double m0[NB], m1[NB], m2[NB];
#pragma unroll
    for (int e = 0; e < NB; ++e) m0[e] = m1[e] = m2[e] = 0.0;

    if (active) {
        const int64_t lxy = (int64_t)Lx * Ly;
        const int z = (int)(site / lxy);
        const int64_t rem = site - (int64_t)z * lxy;
        const int yy = (int)(rem / Lx);
        const int x = (int)(rem - (int64_t)yy * Lx);
        const Site<T, NB> uo = load_site<T, NB>(u, site, ld, c0, cnt);
        // streamed operands of the four output rows
        Site<T, NB> wo, yo;
        if (MODE == MODE_SECOND || MODE == MODE_STEP)
#pragma unroll
            for (int o = 0; o < 4; ++o)
                wo.o[o] = load_pack_n<T, NB, NT>(wold + 2 * ((4 * site + o) * ld + c0), cnt);
        if (MODE == MODE_STEP)
#pragma unroll
            for (int o = 0; o < 4; ++o)
                yo.o[o] = load_pack_n<T, NB, NT>(y + 2 * ((4 * site + o) * ld + c0), cnt);
        const T vn = pot[site];
        Pack<T, NB> acc[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const T d = ((o < 2) ? mm : -mm) + vn;
#pragma unroll
            for (int e = 0; e < NB; ++e) {
                acc[o].re[e] = d * uo.o[o].re[e];
                acc[o].im[e] = d * uo.o[o].im[e];
            }
        }
        // The six neighbours, branch-free: a missing neighbour (open
        // boundary) reads the site itself with hopping weight 0.  All their
        // rows are requested before the first one is used.
        int64_t nb[6];
        T tw[6];
        {
            const int64_t lxy_ = (int64_t)Lx * Ly;
            const int co[3] = {x, yy, z};
            const int Ld[3] = {Lx, Ly, Lz};
            const int64_t stride[3] = {1, Lx, lxy_};
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const bool per = (pbc >> j) & 1;
                int cp = co[j] + 1, cm = co[j] - 1;
                const bool okp = cp < Ld[j] || per, okm = cm >= 0 || per;
                if (cp >= Ld[j]) cp -= Ld[j];
                if (cm < 0) cm += Ld[j];
                nb[2 * j] = okp ? site + (int64_t)(cp - co[j]) * stride[j] : site;
                nb[2 * j + 1] = okm ? site + (int64_t)(cm - co[j]) * stride[j] : site;
                tw[2 * j] = okp ? th : T(0);
                tw[2 * j + 1] = okm ? th : T(0);
            }
        }
        {
            Site<T, NB> un[6];
#pragma unroll
            for (int j = 0; j < 6; ++j) un[j] = load_site<T, NB>(u, nb[j], ld, c0, cnt);
            __builtin_amdgcn_sched_barrier(0);
            add_hop<T, NB, 0>(acc, un[0], tw[0], T(1));
            add_hop<T, NB, 0>(acc, un[1], tw[1], T(-1));
            add_hop<T, NB, 1>(acc, un[2], tw[2], T(1));
            add_hop<T, NB, 1>(acc, un[3], tw[3], T(-1));
            add_hop<T, NB, 2>(acc, un[4], tw[4], T(1));
            add_hop<T, NB, 2>(acc, un[5], tw[5], T(-1));
        }
        T k0[NB], k1[NB], k2[NB];
        lane_coeffs<T, NB, MODE == MODE_SECOND, PC>(gcol, ldg, c0, cnt, g0, g1, g2, k0, k1, k2);
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int64_t off = 2 * ((4 * site + o) * ld + c0);
            Pack<T, NB> w;
#pragma unroll
            for (int e = 0; e < NB; ++e) {
                w.re[e] = s_h * acc[o].re[e] + s_u * uo.o[o].re[e];
                w.im[e] = s_h * acc[o].im[e] + s_u * uo.o[o].im[e];
            }
            if (MODE == MODE_APPLY) {
                store_pack_n<T, NB, NT>(wout + off, w, cnt);
                if (MOM) {
#pragma unroll
                    for (int e = 0; e < NB; ++e) {
                        const double xr = uo.o[o].re[e], xi = uo.o[o].im[e];
                        const double wr = w.re[e], wi = w.im[e];
                        m0[e] += xr * xr + xi * xi;
                        m1[e] += xr * wr + xi * wi;
                        m2[e] += wr * wr + wi * wi;
                    }
                }
            } else if (MODE == MODE_SECOND) {
                const Pack<T, NB> xo = wo.o[o];
                Pack<T, NB> xn;
#pragma unroll
                for (int e = 0; e < NB; ++e) {
                    w.re[e] -= xo.re[e];
                    w.im[e] -= xo.im[e];
                    xn.re[e] = k0[e] * xo.re[e] + k1[e] * uo.o[o].re[e] + k2[e] * w.re[e];
                    xn.im[e] = k0[e] * xo.im[e] + k1[e] * uo.o[o].im[e] + k2[e] * w.im[e];
                }
                store_pack_n<T, NB, NT>(wout + off, w, cnt);
                store_pack_n<T, NB, NT>(y + off, xn, cnt);
                if (MOM) {
#pragma unroll
                    for (int e = 0; e < NB; ++e) {
                        m1[e] += (double)uo.o[o].re[e] * w.re[e] + (double)uo.o[o].im[e] * w.im[e];
                        m2[e] += (double)w.re[e] * w.re[e] + (double)w.im[e] * w.im[e];
                    }
                }
            } else {
                Pack<T, NB> yv = yo.o[o];
#pragma unroll
                for (int e = 0; e < NB; ++e) {
                    w.re[e] -= wo.o[o].re[e];
                    w.im[e] -= wo.o[o].im[e];
                    yv.re[e] += k0[e] * w.re[e];
                    yv.im[e] += k0[e] * w.im[e];
                }
                store_pack_n<T, NB, NT>(wout + off, w, cnt);
                store_pack_n<T, NB, NT>(y + off, yv, cnt);
                if (MOM) {
#pragma unroll
                    for (int e = 0; e < NB; ++e) {
                        m1[e] += (double)uo.o[o].re[e] * w.re[e] + (double)uo.o[o].im[e] * w.im[e];
                        m2[e] += (double)w.re[e] * w.re[e] + (double)w.im[e] * w.im[e];
                    }
                }
            }
        }
    }

    if (MOM) {
        __shared__ double red[4][64][3 * NB];
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            for (int off = LPS; off < 64; off <<= 1) {
                m0[e] += __shfl_xor(m0[e], off);
                m1[e] += __shfl_xor(m1[e], off);
                m2[e] += __shfl_xor(m2[e], off);
            }
            red[wave][lane][3 * e + 0] = m0[e];
            red[wave][lane][3 * e + 1] = m1[e];
            red[wave][lane][3 * e + 2] = m2[e];
        }
        __syncthreads();
        if (wave == 0 && lane < LPS && c0 < n_s) {
#pragma unroll
            for (int e = 0; e < NB; ++e) {
                if (e >= cnt) continue;
                double s[3];
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    s[q] = red[0][lane][3 * e + q] + red[1][lane][3 * e + q] +
                           red[2][lane][3 * e + q] + red[3][lane][3 * e + q];
                double *p = partials + 3 * (sb * n_s + c0 + e);
                p[0] = s[0];
                p[1] = s[1];
                p[2] = s[2];
            }
        }
    }
}

template <typename T, int LPS, int NB, int MODE, bool MOM, bool NT, bool PC = false>
int launch_ti_t(chebfd_ctx *ctx, const Stencil &S, const StepArgs &a, int64_t *n_part)
{
    constexpr int SW = LPS * NB;
    const int64_t nsites = (int64_t)S.L[0] * S.L[1] * S.L[2];
    const TiShape g = ti_shape(ctx, S, a.n_s, (int)sizeof(T), NB, LPS);
    const int order = g.order, tile = g.tile;
    const int64_t bpr = g.bpr, nblk = g.nblk;
    const int64_t nslab = (a.n_s + SW - 1) / SW;
    // a dispatch holds fewer than 2^32 work-items: < 2^24 workgroups of 256
    if (nblk * nslab >= ((int64_t)1 << 24))
        return fail(CHEBFD_ERR_UNSUPPORTED, "fused step: more than 2^24 workgroups");
    if (n_part) *n_part = nblk;
    // default placement in the tiled order: one strip of blocks per XCD group
    int lg_xg = ilog2(ctx->tune_xcd_group);
    if (order == 1 && !ctx->tune_xcd_group) lg_xg = ilog2_64(bpr * S.L[1]);
    const T *pot = std::is_same<T, double>::value ? (const T *)S.pot64 : (const T *)S.pot32;
    hipLaunchKernelGGL((k_step_ti<T, LPS, NB, MODE, MOM, NT, PC>), dim3((unsigned)(nblk * nslab)),
                       dim3(256), 0, ctx->stream, S.L[0], S.L[1], S.L[2], S.pbc,
                       (T)(-0.5 * S.t), (T)S.m, pot, nsites, nblk, (const T *)a.u,
                       (const T *)a.wold, (T *)a.wout, (T *)a.y, a.n_s, a.ld, (T)a.s_h,
                       (T)a.s_u, (T)a.g0, (T)a.g1, (T)a.g2, a.gcol, a.ldg, a.partials, order,
                       nslab, lg_xg, tile);
    CHEBFD_CHECK_LAUNCH();
    return CHEBFD_OK;
}

template <typename T, int LPS, int NB, bool NT>
int launch_ti_mode(chebfd_ctx *ctx, const Stencil &S, const StepArgs &a, int64_t *n_part)
{
    const bool mom = a.partials != nullptr;
    if (a.gcol && a.mode != MODE_APPLY) {
        // per-column coefficients (complex64, no moments)
        if constexpr (std::is_same<T, float>::value) {
            if (mom) return fail(CHEBFD_ERR_UNSUPPORTED, "per-column coefficients: no moments");
            return a.mode == MODE_SECOND
                       ? launch_ti_t<T, LPS, NB, MODE_SECOND, false, NT, true>(ctx, S, a, n_part)
                       : launch_ti_t<T, LPS, NB, MODE_STEP, false, NT, true>(ctx, S, a, n_part);
        } else {
            return fail(CHEBFD_ERR_UNSUPPORTED, "per-column coefficients: complex64 only");
        }
    }
    switch (a.mode) {
    case MODE_APPLY:
        return mom ? launch_ti_t<T, LPS, NB, MODE_APPLY, true, NT>(ctx, S, a, n_part)
                   : launch_ti_t<T, LPS, NB, MODE_APPLY, false, NT>(ctx, S, a, n_part);
    case MODE_SECOND:
        return mom ? launch_ti_t<T, LPS, NB, MODE_SECOND, true, NT>(ctx, S, a, n_part)
                   : launch_ti_t<T, LPS, NB, MODE_SECOND, false, NT>(ctx, S, a, n_part);
    default:
        return mom ? launch_ti_t<T, LPS, NB, MODE_STEP, true, NT>(ctx, S, a, n_part)
                   : launch_ti_t<T, LPS, NB, MODE_STEP, false, NT>(ctx, S, a, n_part);
    }
}

template <typename T, int NB>
int launch_ti_lps(chebfd_ctx *ctx, const Stencil &S, const StepArgs &a, int64_t *n_part, int lps)
{
    const bool nt = ctx->tune_nt != 0;
    switch (lps) {
    case 16:
        return nt ? launch_ti_mode<T, 16, NB, true>(ctx, S, a, n_part)
                  : launch_ti_mode<T, 16, NB, false>(ctx, S, a, n_part);
    case 64:
        return nt ? launch_ti_mode<T, 64, NB, true>(ctx, S, a, n_part)
                  : launch_ti_mode<T, 64, NB, false>(ctx, S, a, n_part);
    default:
        return nt ? launch_ti_mode<T, 32, NB, true>(ctx, S, a, n_part)
                  : launch_ti_mode<T, 32, NB, false>(ctx, S, a, n_part);
    }
}

}  // namespace

// Launch shape of the matrix-free step for a block of n_s columns with
// LPS lanes per site (NB columns of elem bytes per lane).
//
// Default block order.  Column-slab major, a site is gathered as the
// z-neighbour of the plane above and, two planes of work later, of the plane
// below; in between the step moves two planes of its five block streams over
// one slab.  Once that exceeds the memory-side cache (256 MB on MI355X) the
// second gather goes back to HBM, and the tiled order (strips of x-columns,
// z fastest: every neighbour at most one strip-row of work away, one strip
// per XCD) wins: 256x256x64 with 128 columns in complex128, 38.0 ms
// slab-major against 29.3 ms tiled.
TiShape ti_shape(const chebfd_ctx *ctx, const Stencil &S, int64_t n_s, int elem, int nb, int lps)
{
    TiShape g;
    const int spb = 4 * (64 / lps), sw = lps * nb;
    const int64_t row_bytes = (n_s < sw ? n_s : sw) * 2 * (int64_t)elem;
    g.order = ctx->tune_order >= 0 ? ctx->tune_order : (tiled_order_pays(S.L, row_bytes) ? 1 : 0);
    // tiled order: the largest strip width up to the default that divides Lx
    g.tile = std::min(default_tile(ctx, false), S.L[0]);
    while (g.tile > 1 && S.L[0] % g.tile) --g.tile;
    if (g.order == 1 && g.tile < 1) g.order = 0;
    // tiled blocks: spb consecutive sites of a strip row (the last ragged)
    g.bpr = ((int64_t)g.tile * S.L[2] + spb - 1) / spb;
    const int64_t nsites = (int64_t)S.L[0] * S.L[1] * S.L[2];
    g.nblk = g.order == 1 ? (int64_t)(S.L[0] / g.tile) * S.L[1] * g.bpr
                          : (nsites + spb - 1) / spb;
    return g;
}

int launch_stencil_step(chebfd_ctx *ctx, const chebfd_matrix *H, const StepArgs &a,
                        int64_t *n_part)
{
    const Stencil &S = H->st;
    if (a.precision == CHEBFD_PREC_C128)
        return launch_ti_lps<double, 1>(ctx, S, a, n_part, pick_lpr(ctx, a.n_s, 1, true));
    return launch_ti_lps<float, 2>(ctx, S, a, n_part, pick_lpr(ctx, a.n_s, 2, true));
}

}  // namespace chebfd
