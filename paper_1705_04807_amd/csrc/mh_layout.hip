// Layout conversion kernels: Cartesian row-major <-> Morton-hybrid.
//
// One workgroup converts whole tiles.  The Morton-hybrid side of a tile is
// T*T contiguous words (section 1; Prop. 2.5 row-major tiles), so it is read
// or written as one contiguous run; the Cartesian side is T row segments of
// T words.  The tile coordinates come from de-interleaving each tile's Z
// index once, into a table in LDS, never per element.  HBM-bound: 4 bytes read and
// 4 bytes written per word.
#include "mh_internal.h"

namespace mh {

namespace {

constexpr int kThreads = 256;

// Tiles handled by one workgroup: at least 4096 words per group.
__host__ __device__ constexpr int tiles_per_group(int logT)
{
    return (2 * logT >= 12) ? 1 : (1 << (12 - 2 * logT));
}
constexpr int kMaxTilesPerGroup = tiles_per_group(4);  // T = 16, the smallest edge

// Cartesian side: rows x cols words (row length ld); the Morton-hybrid
// parent is padded beyond them: TO_MH writes zeros there, the other way
// leaves the Cartesian words outside rows x cols untouched.  VEC moves four
// words at once and requires cols to be a multiple of four.
template <bool TO_MH, bool VEC>
__global__ __launch_bounds__(kThreads) void k_layout(uint32_t *__restrict__ dst,
                                                     const uint32_t *__restrict__ src,
                                                     int64_t ld, int64_t rows, int64_t cols,
                                                     int logT, uint64_t ntiles)
{
    const int T = 1 << logT;
    const int tpg = tiles_per_group(logT);
    const uint64_t tile0 = uint64_t(blockIdx.x) * tpg;
    const int words = T << logT;                 // per tile
    const int per_group = tpg * words;
    constexpr int W = VEC ? 4 : 1;
    // The group's tiles, de-interleaved once each: tile coordinates are
    // below 2^14 (N <= 2^18, T >= 16), so Z indices fit 32 bits.
    __shared__ uint32_t tileI[kMaxTilesPerGroup], tileJ[kMaxTilesPerGroup];
    if (int(threadIdx.x) < tpg) {
        const uint32_t tz = uint32_t(tile0 + threadIdx.x);
        tileI[threadIdx.x] = compact16(tz >> 1);
        tileJ[threadIdx.x] = compact16(tz);
    }
    __syncthreads();
    for (int e = threadIdx.x * W; e < per_group; e += kThreads * W) {
        const int tl = e >> (2 * logT);
        const uint64_t tz = tile0 + tl;
        if (tz >= ntiles) break;
        const int r = (e >> logT) & (T - 1);
        const int c = e & (T - 1);
        const int64_t gi = (int64_t(tileI[tl]) << logT) + r, gj = (int64_t(tileJ[tl]) << logT) + c;
        const bool inside = gi < rows && gj < cols;  // whole group when VEC
        const uint64_t cart = uint64_t(gi) * uint64_t(ld) + uint64_t(gj);
        const uint64_t mh = (tz << (2 * logT)) + (uint64_t(r) << logT) + c;
        if (VEC) {
            if (TO_MH) {
                uint4 v = make_uint4(0, 0, 0, 0);
                if (inside) v = *reinterpret_cast<const uint4 *>(src + cart);
                *reinterpret_cast<uint4 *>(dst + mh) = v;
            } else if (inside) {
                uint4 v = *reinterpret_cast<const uint4 *>(src + mh);
                *reinterpret_cast<uint4 *>(dst + cart) = v;
            }
        } else {
            if (TO_MH)
                dst[mh] = inside ? src[cart] : 0u;
            else if (inside)
                dst[cart] = src[mh];
        }
    }
}

template <bool TO_MH>
hipError_t launch(uint32_t *dst, const uint32_t *src, int64_t ld, int64_t rows, int64_t cols,
                  int64_t N, int logT, hipStream_t s)
{
    const uint64_t q = uint64_t(N) >> logT;
    const uint64_t ntiles = q * q;
    const int tpg = tiles_per_group(logT);
    const uint64_t groups = (ntiles + tpg - 1) / tpg;
    const bool vec = (ld % 4 == 0) && (cols % 4 == 0) && ((uintptr_t)src % 16 == 0) &&
                     ((uintptr_t)dst % 16 == 0);
    if (vec)
        hipLaunchKernelGGL((k_layout<TO_MH, true>), dim3(unsigned(groups)), dim3(kThreads), 0, s,
                           dst, src, ld, rows, cols, logT, ntiles);
    else
        hipLaunchKernelGGL((k_layout<TO_MH, false>), dim3(unsigned(groups)), dim3(kThreads), 0, s,
                           dst, src, ld, rows, cols, logT, ntiles);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_layout_from(uint32_t *dst, const uint32_t *src, int64_t ld, int64_t rows,
                              int64_t cols, int64_t N, int logT, hipStream_t s)
{
    return launch<true>(dst, src, ld, rows, cols, N, logT, s);
}

hipError_t launch_layout_to(uint32_t *dst, int64_t ld, int64_t rows, int64_t cols,
                            const uint32_t *src, int64_t N, int logT, hipStream_t s)
{
    return launch<false>(dst, src, ld, rows, cols, N, logT, s);
}

}  // namespace mh
