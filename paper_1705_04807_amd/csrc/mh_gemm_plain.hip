// Plain uint32 modular GEMM: C := (C + A.B) mod p on the VALU.
//
// Each output keeps a 96-bit accumulator: a 64-bit low word updated with
// v_mad_u64_u32 (32x32 -> 64-bit multiply-add, carry out to a lane mask)
// and a 32-bit carry count updated with v_addc.  Products are below 2^62,
// so no reduction mod p is needed inside the k-loop; the accumulator is
// reduced once per output (Barrett) and added to C.
//
// A workgroup computes a 64 x 64 output block aligned to C's tile grid, so
// its writes stay inside whole C tiles (contained pieces, section 2.1).
// Operands are read either in place from the Morton-hybrid parents (when
// their tiles line up with the output tiles) or from tile-major panels
// written by the packing kernel.  32-deep slices of A and B are staged in
// LDS; each thread owns a 4 x 4 block of outputs.
#include "mh_device.h"

namespace mh {

namespace {

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int kAStride = 68;  // LDS words per depth row of A (transposed)

// Four independent 96-bit multiply-accumulates: lo[q] += a * b[q] with the
// carry into hi[q].  The four multiplies come first so that each carry
// mask is read three instructions after it is written.
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

// Address of view element (r, c): in-place Morton-hybrid parent whose view
// starts at tile (tr0, tc0), or a tile-major panel with ntc tile columns.
__device__ __forceinline__ uint64_t view_addr(int mhview, int64_t tr0, int64_t tc0, int64_t ntc,
                                              int64_t r, int64_t c, int logT)
{
    const uint64_t m = (1u << logT) - 1;
    const uint64_t inner = (uint64_t(r) & m) << logT | (uint64_t(c) & m);
    uint64_t tile;
    if (mhview)
        tile = tile_z(uint64_t(tr0 + (r >> logT)), uint64_t(tc0 + (c >> logT)));
    else
        tile = uint64_t(r >> logT) * uint64_t(ntc) + uint64_t(c >> logT);
    return (tile << (2 * logT)) | inner;
}

__global__ __launch_bounds__(256) void k_gemm_plain(PlainArgs a)
{
    __shared__ uint32_t As[BK * kAStride];  // As[kk][row]
    __shared__ uint32_t Bs[BK * BN];        // Bs[kk][col]
    const int t = threadIdx.x;
    const int tx = t & 15, ty = t >> 4;
    int64_t gm, gn;
    tile_of(blockIdx.x, a.grid_m, a.grid_n, 8, gm, gn);
    const int64_t rho0 = gm * BM, gam0 = gn * BN;

    uint64_t lo[4][4];
    uint32_t hi[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) lo[i][j] = 0, hi[i][j] = 0;

    const int64_t klo = a.sk, khi = a.sk + a.k;
    for (int64_t kap0 = (klo / BK) * BK; kap0 < khi; kap0 += BK) {
        // A slice: rows rho0.., depth kap0..; lanes along the depth
        {
            const int kk = t & 31;
            const int64_t kap = kap0 + kk;
            const bool kok = kap >= klo && kap < khi;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int rr = (t >> 5) + 8 * q;
                const int64_t rho = rho0 + rr;
                uint32_t v = 0;
                if (kok && rho >= a.sr && rho < a.sr + a.m)
                    v = a.A[view_addr(a.a_mh, a.a_tr0, a.a_tc0, a.a_ntc, rho, kap, a.logT)];
                As[kk * kAStride + rr] = v;
            }
        }
        // B slice: depth kap0.., columns gam0..; lanes along the columns
        {
            const int cc = t & 63;
            const int64_t gam = gam0 + cc;
            const bool cok = gam >= a.sc && gam < a.sc + a.n;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int kk = (t >> 6) + 4 * q;
                const int64_t kap = kap0 + kk;
                uint32_t v = 0;
                if (cok && kap >= klo && kap < khi)
                    v = a.B[view_addr(a.b_mh, a.b_tr0, a.b_tc0, a.b_ntc, kap, gam, a.logT)];
                Bs[kk * BN + cc] = v;
            }
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < BK; ++kk) {
            const uint4 av = *reinterpret_cast<const uint4 *>(&As[kk * kAStride + ty * 4]);
            const uint4 bv = *reinterpret_cast<const uint4 *>(&Bs[kk * BN + tx * 4]);
            const uint32_t b[4] = {bv.x, bv.y, bv.z, bv.w};
            mac4(lo[0], hi[0], av.x, b);
            mac4(lo[1], hi[1], av.y, b);
            mac4(lo[2], hi[2], av.z, b);
            mac4(lo[3], hi[3], av.w, b);
        }
        __syncthreads();
    }

    // 2^64 mod p, for folding the carry word
    uint32_t r64 = mod_u64(~uint64_t(0), a.p, a.mu) + 1;
    if (r64 == a.p) r64 = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t rho = rho0 + ty * 4 + i;
        if (rho < a.sr || rho >= a.sr + a.m) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t gam = gam0 + tx * 4 + j;
            if (gam < a.sc || gam >= a.sc + a.n) continue;
            const uint64_t hpart = uint64_t(mod_u64(hi[i][j], a.p, a.mu)) * r64;
            const uint32_t r = mod_u64(uint64_t(mod_u64(lo[i][j], a.p, a.mu)) + hpart, a.p, a.mu);
            const uint64_t off = mh_offset(uint64_t(a.row0C + rho), uint64_t(a.col0C + gam), a.logT);
            const uint32_t add = a.sub ? (r ? a.p - r : 0u) : r;  // C - r = C + (p - r)
            uint32_t c = a.C[off] + add;
            if (c >= a.p) c -= a.p;
            a.C[off] = c;
        }
    }
}

}  // namespace

hipError_t launch_gemm_plain(const PlainArgs &a, hipStream_t s)
{
    const int64_t groups = a.grid_m * a.grid_n;
    if (groups <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gemm_plain, dim3(unsigned(groups)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace mh
