// Plain uint32 modular GEMM: C := (C + A.B) mod p on the VALU.
//
// Each output keeps a 96-bit accumulator: a 64-bit low word updated with
// v_mad_u64_u32 (32x32 -> 64-bit multiply-add, carry out to a lane mask)
// and a 32-bit carry count updated with v_addc.  Products are below 2^62,
// so no reduction mod p is needed inside the k-loop; the accumulator is
// reduced once per output (Barrett, or shift-and-add folding for the
// Mersenne prime 2^31 - 1) and added to C.
//
// A workgroup computes a 64 x 64 output block aligned to C's tile grid, so
// its writes stay inside whole C tiles (contained pieces, section 2.1).
// Operands are read either in place from the Morton-hybrid parents (when
// their tiles line up with the output tiles) or from tile-major panels
// written by the packing kernel.  32-deep slices of A and B are staged in
// LDS; each thread owns a 4 x 4 block of outputs.
#include "mh_device.h"
#include "mh_mac.h"

namespace mh {

namespace {

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int kAStride = 68;  // LDS words per depth row of A (transposed)

// Operand views (one kernel instance each):
enum View {
    kPanel = 0,        // tile-major panel with ntc tile columns
    kInPlace = 1,      // Morton-hybrid parent, view starting at tile (tr0, tc0)
    kElementwise = 2,  // Morton-hybrid parent, view starting at element (tr0, tc0),
                       // every element addressed by its own encoding
};

// Address of view element (r, c).  Parents have at most 2^18 rows and
// T >= 16, so tile coordinates stay below 2^14 (32-bit dilation) and tile
// indices below 2^28.
template <int VIEW>
__device__ __forceinline__ uint64_t view_addr(int64_t tr0, int64_t tc0, int64_t ntc, int64_t r,
                                              int64_t c, int logT)
{
    if (VIEW == kElementwise) return mh_offset(uint64_t(tr0 + r), uint64_t(tc0 + c), logT);
    const uint32_t m = (1u << logT) - 1;
    const uint32_t inner = (uint32_t(r) & m) << logT | (uint32_t(c) & m);
    const uint32_t tr = uint32_t(r) >> logT, tc = uint32_t(c) >> logT;
    const uint32_t tile = VIEW == kInPlace
                              ? (spread16(uint32_t(tr0) + tr) << 1) | spread16(uint32_t(tc0) + tc)
                              : tr * uint32_t(ntc) + tc;
    return (uint64_t(tile) << (2 * logT)) | inner;
}

// kElementwise is the comparator for the locality argument of section 2.1
// (problems P1 and P2): the same arithmetic with the planner taken out.  The
// output blocks follow the product's own coordinates instead of C's tile
// grid, and A, B and C are read and written where they lie, each element
// through a full Morton-hybrid encoding, so a block that straddles tiles is
// traversed across them.
template <int VIEW>
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
                    v = a.A[view_addr<VIEW>(a.a_tr0, a.a_tc0, a.a_ntc, rho, kap, a.logT)];
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
                    v = a.B[view_addr<VIEW>(a.b_tr0, a.b_tc0, a.b_ntc, kap, gam, a.logT)];
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
    // p = 2^31 - 1 (the prime of the large-prime workloads): 2^64 = 4 mod p
    // and shifts and adds replace the Barrett products.
    const bool mersenne = a.p == 0x7FFFFFFFu;
    // Per output row, the C loads of its four words first, then the stores:
    // in the other order each load would wait for the store before it (the
    // compiler cannot tell the words apart).
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t rho = rho0 + ty * 4 + i;
        if (rho < a.sr || rho >= a.sr + a.m) continue;
        auto inside = [&](int j) {
            const int64_t gam = gam0 + tx * 4 + j;
            return gam >= a.sc && gam < a.sc + a.n;
        };
        auto offset = [&](int j) {
            return mh_offset(uint64_t(a.row0C + rho), uint64_t(a.col0C + gam0 + tx * 4 + j),
                             a.logT);
        };
        uint32_t cv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) cv[j] = inside(j) ? a.C[offset(j)] : 0u;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!inside(j)) continue;
            uint32_t r;
            if (mersenne) {
                r = mod_m31(uint64_t(mod_m31(lo[i][j])) + (uint64_t(hi[i][j]) << 2));
            } else {
                const uint64_t hpart = uint64_t(mod_u64(hi[i][j], a.p, a.mu)) * r64;
                r = mod_u64(uint64_t(mod_u64(lo[i][j], a.p, a.mu)) + hpart, a.p, a.mu);
            }
            const uint32_t add = a.sub ? (r ? a.p - r : 0u) : r;  // C - r = C + (p - r)
            uint32_t c = cv[j] + add;
            if (c >= a.p) c -= a.p;
            a.C[offset(j)] = c;
        }
    }
}

}  // namespace

hipError_t launch_gemm_plain(const PlainArgs &a, hipStream_t s)
{
    const int64_t groups = a.grid_m * a.grid_n;
    if (groups <= 0) return hipSuccess;
    // A and B are both panels, both in place, or both elementwise.
    if (a.a_mh != a.b_mh) return hipErrorInvalidValue;
    switch (a.a_mh) {
    case kPanel:
        hipLaunchKernelGGL(k_gemm_plain<kPanel>, dim3(unsigned(groups)), dim3(256), 0, s, a);
        break;
    case kInPlace:
        hipLaunchKernelGGL(k_gemm_plain<kInPlace>, dim3(unsigned(groups)), dim3(256), 0, s, a);
        break;
    default:
        hipLaunchKernelGGL(k_gemm_plain<kElementwise>, dim3(unsigned(groups)), dim3(256), 0, s,
                           a);
    }
    return hipGetLastError();
}

}  // namespace mh
