// Device helpers shared by the HIP kernels of libmh.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "mh_internal.h"

namespace mh {

// Calls f(std::integral_constant<int, 0>{}) ... f(<N-1>): a loop whose index
// is a compile-time constant in the body, independent of the unroller.
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// x mod p for any 64-bit x, by Barrett reduction (Barrett, CRYPTO 1986)
// with mu = floor((2^64 - 1) / p): the estimated quotient is at most two
// below the true one, so at most two corrections follow.
__device__ __forceinline__ uint32_t mod_u64(uint64_t x, uint32_t p, uint64_t mu)
{
    uint64_t q = __umul64hi(x, mu);
    uint64_t r = x - q * p;
    if (r >= p) r -= p;
    if (r >= p) r -= p;
    return uint32_t(r);
}

// x mod (2^31 - 1) for any 64-bit x: since 2^31 = 1 mod p, x = hi 2^31 + lo
// folds to hi + lo.  Two folds leave a value below 2^31 + 2^4, one
// conditional subtraction finishes.
__device__ __forceinline__ uint32_t mod_m31(uint64_t x)
{
    constexpr uint64_t M = 0x7FFFFFFFull;
    x = (x & M) + (x >> 31);
    x = (x & M) + (x >> 31);
    return uint32_t(x >= M ? x - M : x);
}

// Largest i in [lo, n) with prefix[i] <= t, given prefix[lo] <= t < prefix[n]
// (prefix non-decreasing).  A workgroup's popped work indices only grow, so
// it searches forward from its previous answer: a galloping search costs
// O(log distance) dependent loads instead of O(log n).
__device__ __forceinline__ int64_t find_from(const int64_t *prefix, int64_t n, int64_t lo,
                                             int64_t t)
{
    int64_t step = 1, hi = lo + 1;
    while (hi < n && prefix[hi] <= t) {
        lo = hi;
        step <<= 1;
        hi = lo + step;
    }
    if (hi > n) hi = n;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// Workgroup id -> output tile (gm, gn).  Workgroups are dispatched to the
// 8 XCDs round-robin; the first step gives each XCD a contiguous range of
// logical tile ids so that the workgroups sharing one XCD's L2 also share
// operand panels.  The second walks the tiles in groups of `group_m` tile
// rows, column by column, so concurrently running tiles reuse A slabs.
__device__ __forceinline__ void tile_of(int64_t bid, int64_t grid_m, int64_t grid_n, int group_m,
                                        int64_t &gm, int64_t &gn)
{
    const int64_t G = grid_m * grid_n;
    const int64_t per = G / 8, rem = G % 8;
    const int64_t x = bid % 8, idx = bid / 8;
    int64_t lid = (x < rem) ? x * (per + 1) + idx : rem * (per + 1) + (x - rem) * per + idx;
    const int64_t width = int64_t(group_m) * grid_n;
    const int64_t g = lid / width;
    const int64_t first = g * group_m;
    const int64_t gsz = (grid_m - first) < group_m ? (grid_m - first) : group_m;
    const int64_t in = lid - g * width;
    gm = first + in % gsz;
    gn = in / gsz;
}

}  // namespace mh
