// Workgroup placement on the XCDs of gfx950.
//
// The dispatcher hands workgroup b of a launch to XCD b % 8, and each XCD
// has its own L2.  xcd_remap turns the hardware index into a logical one
// such that 2^lg consecutive logical workgroups run on the same XCD, so that
// neighbouring rows (which gather the same block rows) share one L2.  It is
// a bijection on [0, total); lg = 0 is the identity.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace chebfd {

constexpr int NUM_XCD = 8;
constexpr int LG_XCD = 3;

__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t total, int lg)
{
    if (lg <= 0) return b;
    const int span_lg = lg + LG_XCD;
    const uint32_t full = (total >> span_lg) << span_lg;
    if (b >= full) return b;   // the ragged tail keeps the hardware order
    const uint32_t xcd = b & (NUM_XCD - 1), k = b >> LG_XCD;
    return ((((k >> lg) << LG_XCD) + xcd) << lg) + (k & ((1u << lg) - 1));
}

// log2 of a power of two (0 for 0 and 1).
inline int ilog2(int g)
{
    int l = 0;
    while ((1 << (l + 1)) <= g) ++l;
    return l;
}

// the same for 64-bit counts
inline int ilog2_64(int64_t g)
{
    int l = 0;
    while (((int64_t)1 << (l + 1)) <= g) ++l;
    return l;
}

}  // namespace chebfd
