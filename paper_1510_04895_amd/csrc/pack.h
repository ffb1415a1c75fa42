// 16-byte packs of complex numbers for row-major block vectors: a lane moves
// NB consecutive complex columns with one global_load/store_dwordx4.  The NT
// variants carry the non-temporal hint, used for the streamed blocks (w and
// x of the filter step) so that they do not displace the gathered block u in
// the caches.
#pragma once
#include <hip/hip_runtime.h>

namespace chebfd {

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T, int NB>
struct Pack {
    T re[NB], im[NB];
};

template <typename T, int NB, bool NT>
struct PackIO;

template <bool NT>
struct PackIO<double, 1, NT> {
    static __device__ __forceinline__ Pack<double, 1> load(const double *p)
    {
        d2v d = NT ? __builtin_nontemporal_load(reinterpret_cast<const d2v *>(p))
                   : *reinterpret_cast<const d2v *>(p);
        Pack<double, 1> r;
        r.re[0] = d.x;
        r.im[0] = d.y;
        return r;
    }
    static __device__ __forceinline__ void store(double *p, const Pack<double, 1> &v)
    {
        d2v d = {v.re[0], v.im[0]};
        if (NT) __builtin_nontemporal_store(d, reinterpret_cast<d2v *>(p));
        else *reinterpret_cast<d2v *>(p) = d;
    }
};

template <bool NT>
struct PackIO<float, 2, NT> {
    static __device__ __forceinline__ Pack<float, 2> load(const float *p)
    {
        f4v d = NT ? __builtin_nontemporal_load(reinterpret_cast<const f4v *>(p))
                   : *reinterpret_cast<const f4v *>(p);
        Pack<float, 2> r;
        r.re[0] = d.x;
        r.im[0] = d.y;
        r.re[1] = d.z;
        r.im[1] = d.w;
        return r;
    }
    static __device__ __forceinline__ void store(float *p, const Pack<float, 2> &v)
    {
        f4v d = {v.re[0], v.im[0], v.re[1], v.im[1]};
        if (NT) __builtin_nontemporal_store(d, reinterpret_cast<f4v *>(p));
        else *reinterpret_cast<f4v *>(p) = d;
    }
};

// loads/stores of a possibly ragged last pack (only NB > 1 can be ragged)
template <typename T, int NB, bool NT = false>
__device__ __forceinline__ Pack<T, NB> load_pack_n(const T *p, int cnt)
{
    if (cnt >= NB) return PackIO<T, NB, NT>::load(p);
    Pack<T, NB> r;
#pragma unroll
    for (int e = 0; e < NB; ++e) {
        r.re[e] = e < cnt ? p[2 * e] : T(0);
        r.im[e] = e < cnt ? p[2 * e + 1] : T(0);
    }
    return r;
}

template <typename T, int NB, bool NT = false>
__device__ __forceinline__ void store_pack_n(T *p, const Pack<T, NB> &v, int cnt)
{
    if (cnt >= NB) {
        PackIO<T, NB, NT>::store(p, v);
        return;
    }
#pragma unroll
    for (int e = 0; e < NB; ++e)
        if (e < cnt) {
            p[2 * e] = v.re[e];
            p[2 * e + 1] = v.im[e];
        }
}

// The filter coefficients of a lane's columns c0 .. c0 + cnt - 1: the
// launch's scalars, or (PC) each column's own from the table gcol (row r at
// gcol + r * ldg; rows 0..2 in the second step, row 0 in later ones).  PC
// is a separate instantiation so that the plain step keeps its registers.
template <typename T, int NB, bool SECOND, bool PC>
__device__ __forceinline__ void lane_coeffs(const double *gcol, int64_t ldg, int64_t c0, int cnt,
                                            T g0, T g1, T g2, T (&k0)[NB], T (&k1)[NB],
                                            T (&k2)[NB])
{
#pragma unroll
    for (int e = 0; e < NB; ++e) {
        k0[e] = g0;
        k1[e] = g1;
        k2[e] = g2;
    }
    if (PC) {
#pragma unroll
        for (int e = 0; e < NB; ++e)
            if (e < cnt) {
                k0[e] = (T)gcol[c0 + e];
                if (SECOND) {
                    k1[e] = (T)gcol[ldg + c0 + e];
                    k2[e] = (T)gcol[2 * ldg + c0 + e];
                }
            }
    }
}

}  // namespace chebfd
