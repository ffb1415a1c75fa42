// Sparse matrix handles: the topological-insulator Hamiltonian of Sec. 5.1
// (Eq. (Ham)), CSR -> SELL-C-sigma conversion (Sec. 4.2), Gershgorin bounds
// (Sec. 3.1 step 1) and upload to the device.
#include <algorithm>
#include <climits>
#include <iterator>
#include <cmath>
#include <complex>
#include <numeric>
#include <vector>

#include "internal.h"

namespace chebfd {

using cd = std::complex<double>;

namespace {

struct Entry {
    int64_t c;
    cd v;
};

// 4x4 blocks of Eq. (Ham) in the orbital basis o = 2 tau + s:
// onsite G0 = diag(1, 1, -1, -1); hop[j][0] = -t/2 (G0 + i Gj) couples n to
// n + e_j, hop[j][1] = -t/2 (G0 - i Gj) couples n to n - e_j.
struct TiBlocks {
    cd hop[3][2][4][4];
    double g0[4];
    TiBlocks(double t)
    {
        const cd I(0.0, 1.0);
        const cd sig[3][2][2] = {{{0.0, 1.0}, {1.0, 0.0}},
                                 {{0.0, -I}, {I, 0.0}},
                                 {{1.0, 0.0}, {0.0, -1.0}}};
        for (int o = 0; o < 4; ++o) g0[o] = (o < 2) ? 1.0 : -1.0;
        for (int j = 0; j < 3; ++j)
            for (int o = 0; o < 4; ++o)
                for (int p = 0; p < 4; ++p) {
                    const int to = o >> 1, so = o & 1, tp = p >> 1, sp = p & 1;
                    const cd gj = (to != tp) ? sig[j][so][sp] : cd(0.0);
                    const cd G0 = (o == p) ? cd(g0[o]) : cd(0.0);
                    hop[j][0][o][p] = -0.5 * t * (G0 + I * gj);
                    hop[j][1][o][p] = -0.5 * t * (G0 - I * gj);
                }
    }
};

// Merged, column-sorted entries of row (site, o) of the TI Hamiltonian.
void ti_row(const TiBlocks &B, const int L[3], int pbc, double m, double vn, int64_t site,
            int o, std::vector<Entry> &out)
{
    out.clear();
    const int64_t lxy = (int64_t)L[0] * L[1];
    const int r[3] = {(int)(site % L[0]), (int)((site / L[0]) % L[1]), (int)(site / lxy)};
    out.push_back({4 * site + o, cd(m * B.g0[o] + vn)});
    const int64_t stride[3] = {1, L[0], lxy};
    for (int j = 0; j < 3; ++j)
        for (int s = 0; s < 2; ++s) {
            const int d = s == 0 ? 1 : -1;
            int q = r[j] + d;
            if (q < 0 || q >= L[j]) {
                if (!((pbc >> j) & 1)) continue;
                q = (q + L[j]) % L[j];
            }
            const int64_t nb = site + (int64_t)(q - r[j]) * stride[j];
            for (int p = 0; p < 4; ++p) {
                const cd v = B.hop[j][s][o][p];
                if (v != cd(0.0)) out.push_back({4 * nb + p, v});
            }
        }
    std::sort(out.begin(), out.end(), [](const Entry &a, const Entry &b) { return a.c < b.c; });
    size_t w = 0;
    for (size_t i = 0; i < out.size(); ++i) {
        if (w > 0 && out[w - 1].c == out[i].c) out[w - 1].v += out[i].v;
        else out[w++] = out[i];
    }
    out.resize(w);
    out.erase(std::remove_if(out.begin(), out.end(), [](const Entry &e) { return e.v == cd(0.0); }),
              out.end());
}

template <typename T>
int upload(T **dst, const std::vector<T> &src)
{
    *dst = nullptr;
    if (src.empty()) return CHEBFD_OK;
    CHEBFD_HIP(hipMalloc((void **)dst, src.size() * sizeof(T)));
    CHEBFD_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return CHEBFD_OK;
}

void free_matrix(chebfd_matrix *H)
{
    Sell &S = H->sell;
    for (void *p : {(void *)S.chunk_ptr, (void *)S.chunk_len, (void *)S.perm, (void *)S.col,
                    (void *)S.val64, (void *)S.val32, (void *)H->st.pot64,
                    (void *)H->st.pot32})
        if (p) (void)hipFree(p);
}

// Builds SELL-C-sigma from a row generator.  rowfn(i, entries) fills row i.
// `order` (optional) is the sequence in which rows are cut into sigma windows
// and chunks (the traversal order of the fused step); nullptr = 0, 1, ...
// `grouped` asks for the row-group layout (see Sell): -1 where it pays (4,
// then 2 rows per group), 2 or 4 that group size whenever every union fits
// the LDS stage, 0 or 1 never; groups are consecutive slots (after the
// `pair_rows` placement, which puts rows with equal columns side by side).
template <typename RowFn>
int build_sell(chebfd_matrix *H, int64_t n, int C, int sigma, RowFn rowfn, bool pair_rows,
               const std::vector<int32_t> *order = nullptr, int grouped = 0)
{
    Sell &S = H->sell;
    S.n = n;
    S.C = C;
    S.sigma = sigma;
    S.nchunks = (n + C - 1) / C;
    const int64_t nslots = S.nchunks * C;
    // row lengths and the Gershgorin interval
    std::vector<int32_t> len(n);
    std::vector<Entry> row;
    double lo = INFINITY, hi = -INFINITY;
    int64_t nnz = 0;
    for (int64_t i = 0; i < n; ++i) {
        rowfn(i, row);
        len[i] = (int32_t)row.size();
        nnz += (int64_t)row.size();
        double d = 0.0, rad = 0.0;
        for (const Entry &e : row) {
            if (e.c == i) d += e.v.real();
            else rad += std::abs(e.v);
        }
        lo = std::min(lo, d - rad);
        hi = std::max(hi, d + rad);
    }
    H->g_lo = lo;
    H->g_hi = hi;
    S.nnz = nnz;
    // sort rows by descending length inside each sigma window (stable)
    std::vector<int32_t> perm(nslots, -1);
    for (int64_t w0 = 0; w0 < n; w0 += sigma) {
        const int64_t w1 = std::min(n, w0 + sigma);
        std::vector<int32_t> ids(w1 - w0);
        if (order) std::copy(order->begin() + w0, order->begin() + w1, ids.begin());
        else std::iota(ids.begin(), ids.end(), (int32_t)w0);
        std::stable_sort(ids.begin(), ids.end(), [&](int32_t a, int32_t b) { return len[a] > len[b]; });
        std::copy(ids.begin(), ids.end(), perm.begin() + w0);
    }
    // inside each chunk, place rows that gather the same columns at the same
    // entry positions next to each other: slots 2k and 2k+1 share one wave
    // instruction at 32 lanes per row, and equal addresses in one
    // instruction are one cache access (greedy pairing by the number of
    // positions with equal column index)
    if (pair_rows) {
        std::vector<std::vector<int64_t>> cols(C);
        std::vector<Entry> er;
        std::vector<int32_t> order;
        std::vector<char> used;
        for (int64_t c = 0; c < S.nchunks; ++c) {
            int nv = 0;
            for (int r = 0; r < C; ++r) {
                const int32_t i = perm[c * C + r];
                cols[r].clear();
                if (i < 0) continue;
                ++nv;
                rowfn(i, er);
                for (const Entry &e : er) cols[r].push_back(e.c);
            }
            if (nv < 3) continue;
            order.clear();
            used.assign(C, 0);
            for (int r = 0; r < nv; ++r) {
                if (used[r]) continue;
                used[r] = 1;
                order.push_back(perm[c * C + r]);
                int best = -1, bo = -1;
                for (int r2 = r + 1; r2 < nv; ++r2) {
                    if (used[r2]) continue;
                    const size_t m = std::min(cols[r].size(), cols[r2].size());
                    int ov = 0;
                    for (size_t j = 0; j < m; ++j) ov += cols[r][j] == cols[r2][j];
                    if (ov > bo) {
                        bo = ov;
                        best = r2;
                    }
                }
                if (best >= 0) {
                    used[best] = 1;
                    order.push_back(perm[c * C + best]);
                }
            }
            std::copy(order.begin(), order.end(), perm.begin() + c * C);
        }
    }
    if (grouped != 0 && grouped != 1) {
        // union columns of groups of G consecutive slots (each row's entries
        // are sorted by column); a group size is taken when every union fits
        // the kernel's LDS stage and (automatic choice) the unions save at
        // least a quarter of the gathers; the automatic choice tries 4, then 2
        std::vector<Entry> er;
        std::vector<int64_t> cur, nxt, rc;
        auto unions = [&](int G, std::vector<int32_t> &ulen, int64_t &sum_u, int64_t &sum_r,
                          int &max_u) {
            const int P = C / G;
            ulen.assign((size_t)S.nchunks * P, 0);
            sum_u = sum_r = 0;
            max_u = 0;
            for (int64_t c = 0; c < S.nchunks; ++c)
                for (int q = 0; q < P; ++q) {
                    cur.clear();
                    for (int k = 0; k < G; ++k) {
                        const int32_t i = perm[c * C + G * q + k];
                        if (i < 0) continue;
                        rowfn(i, er);
                        sum_r += (int64_t)er.size();
                        rc.clear();
                        for (const Entry &e : er) rc.push_back(e.c);
                        nxt.clear();
                        std::set_union(cur.begin(), cur.end(), rc.begin(), rc.end(),
                                       std::back_inserter(nxt));
                        cur.swap(nxt);
                    }
                    ulen[c * P + q] = (int32_t)cur.size();
                    sum_u += (int64_t)cur.size();
                    max_u = std::max(max_u, (int)cur.size());
                }
        };
        std::vector<int32_t> ulen;
        int64_t sum_u = 0, sum_r = 0;
        int max_u = 0, G = 0;
        for (int g : {4, 2}) {
            if (grouped > 0 && g != grouped) continue;
            if (C % g) continue;
            unions(g, ulen, sum_u, sum_r, max_u);
            if (max_u <= kStageLen && (grouped > 0 || 4 * sum_u <= 3 * sum_r)) {
                G = g;
                break;
            }
        }
        if (G > 0) {
            S.group = G;
            const int P = C / G;
            std::vector<int64_t> cptr(S.nchunks + 1, 0);
            std::vector<int32_t> clen(S.nchunks, 0);
            for (int64_t c = 0; c < S.nchunks; ++c) {
                int w = 0;
                for (int q = 0; q < P; ++q) w = std::max(w, ulen[c * P + q]);
                clen[c] = w;
                cptr[c + 1] = cptr[c] + (int64_t)w * P;
            }
            S.max_len = max_u;
            S.stored = cptr[S.nchunks];
            std::vector<int32_t> col(S.stored);
            std::vector<double> v64(2 * G * S.stored, 0.0);
            std::vector<float> v32(2 * G * S.stored, 0.0f);
            std::vector<std::vector<Entry>> rows(G);
            std::vector<size_t> at(G);
            for (int64_t c = 0; c < S.nchunks; ++c)
                for (int q = 0; q < P; ++q) {
                    int32_t self = -1;
                    for (int k = 0; k < G; ++k) {
                        const int32_t i = perm[c * C + G * q + k];
                        if (i >= 0) rowfn(i, rows[k]);
                        else rows[k].clear();
                        if (self < 0 && i >= 0) self = i;
                        at[k] = 0;
                    }
                    // padding: the group's first row (or row 0) with zero values
                    if (self < 0) self = 0;
                    for (int j = 0; j < clen[c]; ++j) {
                        const int64_t e = cptr[c] + (int64_t)j * P + q;
                        // next union column: the smallest pending one
                        int64_t cc = INT64_MAX;
                        for (int k = 0; k < G; ++k)
                            if (at[k] < rows[k].size()) cc = std::min(cc, rows[k][at[k]].c);
                        if (cc == INT64_MAX) {
                            col[e] = self;
                            continue;
                        }
                        col[e] = (int32_t)cc;
                        for (int k = 0; k < G; ++k)
                            if (at[k] < rows[k].size() && rows[k][at[k]].c == cc) {
                                const cd v = rows[k][at[k]++].v;
                                v64[2 * (G * e + k)] = v.real();
                                v64[2 * (G * e + k) + 1] = v.imag();
                                v32[2 * (G * e + k)] = (float)v.real();
                                v32[2 * (G * e + k) + 1] = (float)v.imag();
                            }
                    }
                }
            int rc2;
            if ((rc2 = upload(&S.chunk_ptr, cptr)) || (rc2 = upload(&S.chunk_len, clen)) ||
                (rc2 = upload(&S.perm, perm)) || (rc2 = upload(&S.col, col)) ||
                (rc2 = upload(&S.val64, v64)) || (rc2 = upload(&S.val32, v32)))
                return rc2;
            return CHEBFD_OK;
        }
    }
    std::vector<int64_t> cptr(S.nchunks + 1, 0);
    std::vector<int32_t> clen(S.nchunks, 0);
    int max_len = 0;
    for (int64_t c = 0; c < S.nchunks; ++c) {
        int w = 0;
        for (int r = 0; r < C; ++r) {
            const int32_t i = perm[c * C + r];
            if (i >= 0) w = std::max(w, len[i]);
        }
        clen[c] = w;
        max_len = std::max(max_len, w);
        cptr[c + 1] = cptr[c] + (int64_t)w * C;
    }
    S.max_len = max_len;
    S.stored = cptr[S.nchunks];
    std::vector<int32_t> col(S.stored);
    std::vector<double> v64(2 * S.stored, 0.0);
    std::vector<float> v32(2 * S.stored, 0.0f);
    for (int64_t c = 0; c < S.nchunks; ++c)
        for (int r = 0; r < C; ++r) {
            const int32_t i = perm[c * C + r];
            // padding entries point at the row itself (an access the row
            // makes anyway) with value zero; empty slots point at row 0
            const int32_t self = i >= 0 ? i : 0;
            if (i >= 0) rowfn(i, row);
            else row.clear();
            for (int j = 0; j < clen[c]; ++j) {
                const int64_t e = cptr[c] + (int64_t)j * C + r;
                if (j < (int)row.size()) {
                    col[e] = (int32_t)row[j].c;
                    v64[2 * e] = row[j].v.real();
                    v64[2 * e + 1] = row[j].v.imag();
                    v32[2 * e] = (float)row[j].v.real();
                    v32[2 * e + 1] = (float)row[j].v.imag();
                } else {
                    col[e] = self;
                }
            }
        }
    int rc;
    if ((rc = upload(&S.chunk_ptr, cptr)) || (rc = upload(&S.chunk_len, clen)) ||
        (rc = upload(&S.perm, perm)) || (rc = upload(&S.col, col)) ||
        (rc = upload(&S.val64, v64)) || (rc = upload(&S.val32, v32)))
        return rc;
    return CHEBFD_OK;
}

// Tiled lattice order of the rows: the lattice is cut into strips of `w`
// x-columns; strips run one after the other, inside a strip y-rows, inside a
// y-row the x-columns, and along each column z fastest, the four orbital rows
// of a site together.  Consecutive chunks are then z-runs of one column, and
// every neighbour of a site is at most one strip-row of work away.
std::vector<int32_t> ti_tiled_rows(const int L[3], int w)
{
    std::vector<int32_t> r;
    r.reserve((size_t)4 * L[0] * L[1] * L[2]);
    for (int x0 = 0; x0 < L[0]; x0 += w)
        for (int y = 0; y < L[1]; ++y)
            for (int x = x0; x < std::min(L[0], x0 + w); ++x)
                for (int z = 0; z < L[2]; ++z) {
                    const int64_t site = x + (int64_t)L[0] * (y + (int64_t)L[1] * z);
                    for (int o = 0; o < 4; ++o) r.push_back((int32_t)(4 * site + o));
                }
    return r;
}

}  // namespace

// Default strip width of the tiled lattice order (sites along x): 2 for the
// SELL row order, 4 for the matrix-free step (measured at 256x256x64).
int default_tile(const chebfd_ctx *ctx, bool sell)
{
    return ctx->tune_tile >= 0 ? ctx->tune_tile : (sell ? 2 : 4);
}

// Whether the tiled lattice order pays: in column-slab-major order a site's
// u row is gathered again two lattice planes of work later, during which the
// step moves two planes of its five block streams (slab_row bytes per row);
// beyond the 256 MB memory-side cache that second gather returns to HBM.
bool tiled_order_pays(const int L[3], int64_t slab_row)
{
    constexpr double kMallBytes = 256.0 * (1 << 20);
    return 2.0 * L[0] * L[1] * 4 * 5 * (double)slab_row > kMallBytes;
}

}  // namespace chebfd

using namespace chebfd;

extern "C" int chebfd_matrix_from_csr(chebfd_ctx *ctx, int64_t n, const int64_t *rowptr,
                                      const int32_t *col, const double *val, int sell_C,
                                      int sell_sigma, chebfd_matrix **out)
{
    if (!ctx || !out || !rowptr || (!col && n > 0) || (!val && n > 0))
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_matrix_from_csr: NULL argument");
    *out = nullptr;
    if (n < 1 || n >= (int64_t)INT32_MAX)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_matrix_from_csr: need 1 <= n < 2^31");
    if (sell_C < 1 || sell_C > 64 || (sell_C & (sell_C - 1)) || sell_sigma < 1 ||
        sell_sigma % sell_C)
        return fail(CHEBFD_ERR_INVALID_ARG,
                    "chebfd_matrix_from_csr: sell_C must be a power of two <= 64 and sell_sigma a multiple of it");
    if (rowptr[0] != 0)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_matrix_from_csr: rowptr[0] != 0");
    for (int64_t i = 0; i < n; ++i)
        if (rowptr[i + 1] < rowptr[i])
            return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_matrix_from_csr: decreasing rowptr");
    for (int64_t p = 0; p < rowptr[n]; ++p)
        if (col[p] < 0 || col[p] >= n)
            return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_matrix_from_csr: column index out of range");
    CHEBFD_HIP(hipSetDevice(ctx->device));
    auto *H = new chebfd_matrix();
    H->storage = CHEBFD_STORAGE_SELL;
    H->n = n;
    H->device = ctx->device;
    auto rowfn = [&](int64_t i, std::vector<Entry> &r) {
        r.clear();
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
            r.push_back({(int64_t)col[p], cd(val[2 * p], val[2 * p + 1])});
    };
    int rc = build_sell(H, n, sell_C, sell_sigma, rowfn, ctx->tune_pair_rows != 0, nullptr,
                        ctx->tune_row_group);
    if (rc) {
        free_matrix(H);
        delete H;
        return rc;
    }
    *out = H;
    return CHEBFD_OK;
}

extern "C" int chebfd_matrix_ti(chebfd_ctx *ctx, int Lx, int Ly, int Lz, int pbc_mask, double t,
                                double m, double V, uint64_t seed, int storage, int sell_C,
                                int sell_sigma, chebfd_matrix **out)
{
    if (!ctx || !out) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_matrix_ti: NULL argument");
    *out = nullptr;
    if (Lx < 1 || Ly < 1 || Lz < 1)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_matrix_ti: lattice extents must be >= 1");
    const int64_t nsites = (int64_t)Lx * Ly * Lz, n = 4 * nsites;
    if (n >= (int64_t)INT32_MAX)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_matrix_ti: N must be < 2^31");
    if (storage != CHEBFD_STORAGE_SELL && storage != CHEBFD_STORAGE_STENCIL)
        return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_matrix_ti: unknown storage");
    if (storage == CHEBFD_STORAGE_SELL &&
        (sell_C < 1 || sell_C > 64 || (sell_C & (sell_C - 1)) || sell_sigma < 1 ||
         sell_sigma % sell_C))
        return fail(CHEBFD_ERR_INVALID_ARG,
                    "chebfd_matrix_ti: sell_C must be a power of two <= 64 and sell_sigma a multiple of it");
    CHEBFD_HIP(hipSetDevice(ctx->device));
    const TiBlocks B(t);
    const int L[3] = {Lx, Ly, Lz};
    std::vector<double> pot(nsites);
    for (int64_t s = 0; s < nsites; ++s) pot[s] = V * (u01(seed, 0, (uint64_t)s) - 0.5);
    auto *H = new chebfd_matrix();
    H->storage = storage;
    H->n = n;
    H->device = ctx->device;
    auto rowfn = [&](int64_t i, std::vector<Entry> &r) {
        ti_row(B, L, pbc_mask, m, pot[i / 4], i / 4, (int)(i % 4), r);
    };
    int rc = CHEBFD_OK;
    if (storage == CHEBFD_STORAGE_SELL) {
        // the fused step's slab row: 32 lanes of 16 bytes
        const int w = ctx->tune_tile >= 0 || tiled_order_pays(L, 512)
                          ? std::min(default_tile(ctx, true), Lx) : 0;
        if (w > 0) {
            const std::vector<int32_t> order = ti_tiled_rows(L, w);
            rc = build_sell(H, n, sell_C, sell_sigma, rowfn, ctx->tune_pair_rows != 0, &order,
                            ctx->tune_row_group);
            H->sell.group_rows = (int64_t)4 * w * Ly * Lz;
        } else {
            rc = build_sell(H, n, sell_C, sell_sigma, rowfn, ctx->tune_pair_rows != 0, nullptr,
                            ctx->tune_row_group);
        }
    } else {
        Stencil &S = H->st;
        S.L[0] = Lx;
        S.L[1] = Ly;
        S.L[2] = Lz;
        S.pbc = pbc_mask;
        S.t = t;
        S.m = m;
        // Gershgorin interval from the merged rows
        std::vector<Entry> row;
        double lo = INFINITY, hi = -INFINITY;
        for (int64_t i = 0; i < n; ++i) {
            rowfn(i, row);
            double d = 0.0, rad = 0.0;
            for (const Entry &e : row) {
                if (e.c == i) d += e.v.real();
                else rad += std::abs(e.v);
            }
            lo = std::min(lo, d - rad);
            hi = std::max(hi, d + rad);
        }
        H->g_lo = lo;
        H->g_hi = hi;
        std::vector<float> pot32(nsites);
        for (int64_t s = 0; s < nsites; ++s) pot32[s] = (float)pot[s];
        if (!(rc = upload(&S.pot64, pot))) rc = upload(&S.pot32, pot32);
    }
    if (rc) {
        free_matrix(H);
        delete H;
        return rc;
    }
    *out = H;
    return CHEBFD_OK;
}

extern "C" int chebfd_matrix_info(const chebfd_matrix *H, int64_t *n, int64_t *nnz,
                                  int64_t *padded, double *g_lo, double *g_hi,
                                  int64_t *matrix_bytes_c128, int64_t *matrix_bytes_c64)
{
    if (!H) return fail(CHEBFD_ERR_INVALID_ARG, "chebfd_matrix_info: NULL matrix");
    const bool sell = H->storage == CHEBFD_STORAGE_SELL;
    int64_t nz = sell ? H->sell.nnz : 0;
    if (!sell) {
        // 13 entries per row minus the missing neighbours of open boundaries
        const int *L = H->st.L;
        int64_t per = 0;
        const int64_t ns = (int64_t)L[0] * L[1] * L[2];
        for (int j = 0; j < 3; ++j) {
            const int64_t links = ((H->st.pbc >> j) & 1) ? (int64_t)L[j] : (int64_t)L[j] - 1;
            per += 2 * links * (ns / L[j]);   // directed links along j
        }
        nz = 4 * ns + 8 * per;   // on-site + 2 entries per orbital row per directed link
    }
    if (n) *n = H->n;
    if (nnz) *nnz = nz;
    if (padded) *padded = sell ? H->sell.stored : 0;
    if (g_lo) *g_lo = H->g_lo;
    if (g_hi) *g_hi = H->g_hi;
    // one step reads every stored entry once: value + column index, plus the
    // chunk pointers/lengths and the slot permutation
    // (a row-group layout stores one index and G values per entry)
    const int64_t nv = sell && H->sell.group > 1 ? H->sell.group : 1;
    if (matrix_bytes_c128)
        *matrix_bytes_c128 = sell ? H->sell.stored * (nv * 16 + 4) : (H->n / 4) * 8;
    if (matrix_bytes_c64) *matrix_bytes_c64 = sell ? H->sell.stored * (nv * 8 + 4) : (H->n / 4) * 4;
    return CHEBFD_OK;
}

extern "C" int chebfd_matrix_destroy(chebfd_matrix *H)
{
    if (!H) return CHEBFD_OK;
    (void)hipSetDevice(H->device);
    free_matrix(H);
    delete H;
    return CHEBFD_OK;
}
