// The plain kernel's 96-bit multiply-accumulate, shared with the probe that
// measures its issue rate.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mh {

// Four independent 96-bit multiply-accumulates: lo[q] += a * b[q] with the
// carry into hi[q] (v_mad_u64_u32 writes the carry to a lane mask, which
// v_addc_co_u32 adds to the 32-bit high word).  The four multiplies come
// first so that each carry mask is read three instructions after it is
// written.
__device__ __forceinline__ void mac4(uint64_t (&lo)[4], uint32_t (&hi)[4], uint32_t a,
                                     const uint32_t (&b)[4])
{
    uint64_t c0, c1, c2, c3;
    asm("v_mad_u64_u32 %0, %8, %12, %13, %0\n\t"
        "v_mad_u64_u32 %1, %9, %12, %14, %1\n\t"
        "v_mad_u64_u32 %2, %10, %12, %15, %2\n\t"
        "v_mad_u64_u32 %3, %11, %12, %16, %3\n\t"
        "v_addc_co_u32_e64 %4, %8, 0, %4, %8\n\t"
        "v_addc_co_u32_e64 %5, %9, 0, %5, %9\n\t"
        "v_addc_co_u32_e64 %6, %10, 0, %6, %10\n\t"
        "v_addc_co_u32_e64 %7, %11, 0, %7, %11"
        : "+v"(lo[0]), "+v"(lo[1]), "+v"(lo[2]), "+v"(lo[3]), "+v"(hi[0]), "+v"(hi[1]),
          "+v"(hi[2]), "+v"(hi[3]), "=&s"(c0), "=&s"(c1), "=&s"(c2), "=&s"(c3)
        : "v"(a), "v"(b[0]), "v"(b[1]), "v"(b[2]), "v"(b[3]));
}

}  // namespace mh
