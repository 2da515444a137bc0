// Operand packing kernels.
//
// A non-aligned operand block is copied once into a panel whose tiles line
// up with the output's tile grid, so that the GEMM kernels afterwards only
// read contiguous, aligned data (the section 2.1 locality argument: base
// cases should read row-major pieces, never per-element Morton-hybrid
// encodes).  Within the source, every row segment of a tile is contiguous;
// the Morton-hybrid address of an element is split into a row part and a
// column part, so one encode is shared by a whole row or column of the
// workgroup's chunk.
//
// pack_u32:  tile-major uint32 panel for the plain kernel.
// pack_limb: signed 8-bit limb planes in MFMA operand order for the int8
//            MFMA kernel (balanced base-256 digits of the centred residue).
#include "mh_device.h"

namespace mh {

namespace {

__device__ __forceinline__ uint64_t row_part(uint64_t r, int logT)
{
    return (uint64_t(spread16(uint32_t(r >> logT))) << (2 * logT + 1)) |
           ((r & ((1u << logT) - 1)) << logT);
}

__device__ __forceinline__ uint64_t col_part(uint64_t c, int logT)
{
    return (uint64_t(spread16(uint32_t(c >> logT))) << (2 * logT)) | (c & ((1u << logT) - 1));
}

// ------------------------------------------------------------ u32 panel

// Panel of prow x pcol words in T x T tiles, tile-major: tile (tr, tc) at
// dst + (tr * pcol/T + tc) * T^2.  Panel entry (r, c) holds source entry
// (srow0 + r, scol0 + c) when r in [vr0, vr1) and c in [vc0, vc1), else 0.
// One workgroup per tile.
__global__ __launch_bounds__(256) void k_pack_u32(uint32_t *__restrict__ dst, int64_t ntc,
                                                  const uint32_t *__restrict__ src, int64_t srow0,
                                                  int64_t scol0, int64_t vr0, int64_t vr1,
                                                  int64_t vc0, int64_t vc1, int logT)
{
    const int T = 1 << logT;
    const int64_t tr = blockIdx.y, tc = blockIdx.x;
    uint32_t *out = dst + (tr * ntc + tc) * (int64_t(T) << logT);
    for (int e = threadIdx.x; e < (T << logT); e += 256) {
        const int64_t r = (tr << logT) + (e >> logT);
        const int64_t c = (tc << logT) + (e & (T - 1));
        uint32_t v = 0;
        if (r >= vr0 && r < vr1 && c >= vc0 && c < vc1)
            v = src[row_part(uint64_t(srow0 + r), logT) | col_part(uint64_t(scol0 + c), logT)];
        out[e] = v;
    }
}

// ------------------------------------------------------------ limb panel

constexpr int kChunk = 64;         // panel rows x depth per workgroup
constexpr int kLdsStride = 68;     // words per LDS row (padding against bank conflicts)

template <int L>
__device__ __forceinline__ void digits16(const uint32_t *x, uint32_t p, int32_t H, uint4 *out)
{
    // out[t] holds digit t of the 16 residues, one byte each (element e in
    // byte e%4 of word e/4).
    uint32_t w[L][4];
#pragma unroll
    for (int t = 0; t < L; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) w[t][q] = 0;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        int32_t v = int32_t(x[e]);
        v = v > H ? v - int32_t(p) : v;  // centred residue
#pragma unroll
        for (int t = 0; t < L; ++t) {
            const int32_t d = int32_t(int8_t(v & 0xFF));  // balanced digit in [-128, 127]
            w[t][e >> 2] |= (uint32_t(d) & 0xFFu) << (8 * (e & 3));
            v = (v - d) >> 8;
        }
    }
#pragma unroll
    for (int t = 0; t < L; ++t) out[t] = make_uint4(w[t][0], w[t][1], w[t][2], w[t][3]);
}

// Limb panel layout: 32-row slabs x 32-deep k-blocks x L limbs, 1 KiB per
// (slab, kb, limb); lane q of a block holds row (q & 31), depth
// (q >> 5) * 16 .. +15.  One workgroup packs 64 panel rows x 64 depth
// (2 slabs x 2 k-blocks).  trans = 0: panel (rho, kap) <- src(r0 + rho -
// shift, c0 + kap); trans = 1: src(r0 + kap - kshift, c0 + rho - shift).
// Entries with rho outside [shift, shift + R) or kap outside [kshift,
// kshift + K) are zero (kshift = 0 when trans = 0).
template <int L, bool TRANS>
__device__ __forceinline__ void pack_chunk(int8_t *__restrict__ dst, int64_t nkb,
                                           const uint32_t *__restrict__ src, int64_t r0,
                                           int64_t c0, int64_t shift, int64_t R, int64_t K,
                                           int logT, uint32_t p, int32_t H, int64_t rho0,
                                           int64_t kap0, uint32_t *tile, int neg, int64_t kshift)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;

    // The chunk's source rectangle is read as aligned 16-byte groups: a
    // window of 17 groups (68 words) along the contiguous source direction
    // covers the 64 needed words whatever their alignment (16 groups when
    // the window starts on a group boundary).  An aligned group
    // never crosses a tile row (T is a multiple of 4), so each group is one
    // contained piece; groups wholly outside the block are not read (they may
    // lie beyond the parent), and words outside it are stored as zero.
    //   !TRANS: contiguous direction = depth kap (source column c0 + kap),
    //           other direction = panel row rho (source row r0 + rho - shift).
    //   TRANS:  contiguous direction = panel row rho (source column
    //           c0 + rho - shift), other = depth kap (source row r0 + kap).
    {
        const int64_t cfirst = TRANS ? c0 + rho0 - shift : c0 + kap0;  // source col of slot 0
        const int64_t clo = c0;                                         // block's columns:
        const int64_t chi = TRANS ? c0 + R : c0 + K;                    //   [clo, chi)
        const int64_t gbase = cfirst & ~int64_t(3);
        const int mis = int(cfirst - gbase);
        constexpr int G = 17;
#pragma unroll
        for (int q = 0; q < (kChunk * G + 255) / 256; ++q) {
            const int gi = int(threadIdx.x) + 256 * q;
            if (gi >= kChunk * G) break;
            const int other = gi / G, g = gi - other * G;
            const int64_t gcol = gbase + 4 * g;
            int64_t srow;
            bool ok;
            if (!TRANS) {
                const int64_t rho = rho0 + other;
                ok = rho >= shift && rho < shift + R;
                srow = r0 + rho - shift;
            } else {
                const int64_t kap = kap0 + other;
                ok = kap >= kshift && kap < kshift + K;
                srow = r0 + kap - kshift;
            }
            // the 17th group is needed only when the window starts inside a group
            ok = ok && gcol + 4 > clo && gcol < chi && (mis != 0 || g < G - 1);
            uint4 v = make_uint4(0, 0, 0, 0);
            if (ok)
                v = *reinterpret_cast<const uint4 *>(
                    src + (row_part(uint64_t(srow), logT) | col_part(uint64_t(gcol), logT)));
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int slot = 4 * g + e - mis;  // position along the contiguous direction
                const int64_t col = gcol + e;
                if (slot < 0 || slot >= kChunk) continue;
                const uint32_t x = (col >= clo && col < chi) ? w[e] : 0u;
                if (!TRANS)
                    tile[other * kLdsStride + slot] = ok ? x : 0u;
                else
                    tile[slot * kLdsStride + other] = ok ? x : 0u;
            }
        }
    }
    __syncthreads();

    const int sl = wave >> 1, kbl = wave & 1;
    const int64_t kb = kap0 / 32 + kbl;
    if (kb >= nkb) return;
    const int rr = sl * 32 + (lane & 31);
    const int kk = kbl * 32 + (lane >> 5) * 16;
    uint32_t x[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint4 v = *reinterpret_cast<const uint4 *>(&tile[rr * kLdsStride + kk + 4 * q]);
        x[4 * q] = v.x;
        x[4 * q + 1] = v.y;
        x[4 * q + 2] = v.z;
        x[4 * q + 3] = v.w;
    }
    if (neg) {
#pragma unroll
        for (int e = 0; e < 16; ++e) x[e] = x[e] ? p - x[e] : 0u;  // (p - x) mod p
    }
    uint4 d[L];
    digits16<L>(x, p, H, d);
    const int64_t slab = rho0 / 32 + sl;
    uint4 *o = reinterpret_cast<uint4 *>(dst + ((slab * nkb + kb) * L) * 1024) + lane;
#pragma unroll
    for (int t = 0; t < L; ++t) o[t * 64] = d[t];
}

template <int L, bool TRANS>
__global__ __launch_bounds__(256) void k_pack_limb(int8_t *__restrict__ dst, int64_t nkb,
                                                   const uint32_t *__restrict__ src, int64_t r0,
                                                   int64_t c0, int64_t shift, int64_t R, int64_t K,
                                                   int logT, uint32_t p, int32_t H, int neg)
{
    __shared__ uint32_t tile[kChunk * kLdsStride];
    pack_chunk<L, TRANS>(dst, nkb, src, r0, c0, shift, R, K, logT, p, H,
                         int64_t(blockIdx.y) * kChunk, int64_t(blockIdx.x) * kChunk, tile, neg, 0);
}

// Persistent form for a batch: workgroups pop runs of 64 x 64 chunks of all
// the A panels (TRANS = false: tasks [0, ncalls)) or the B panels (TRANS =
// true: tasks [ncalls, 2 ncalls)) of the batch through an atomic counter; a
// forward search over the per-operand prefix sums finds the operand of a
// run's first chunk, and the following chunks step forward from it.
// Barriers between chunks (and after reading the popped index) order the
// reuse of the LDS tile.  One instance per direction, the popped index read
// as a scalar, and the queue arrays as separate read-only parameters (so
// that a task's fields load into scalar registers) keep the register count,
// and so the number of resident workgroups, of the single-operand kernel.
template <int L, bool TRANS>
__global__ __launch_bounds__(256) void k_pack_limb_batched(const BatchHeader *__restrict__ hdr,
                                                           const PackTask *__restrict__ packs,
                                                           const int64_t *__restrict__ pack_prefix,
                                                           uint64_t *counter)
{
    constexpr int64_t kGrab = 8;  // chunks per pop: one atomic and one search per 8 chunks
    __shared__ uint32_t tile[kChunk * kLdsStride];
    __shared__ uint32_t chunk_s;
    const int64_t ncalls = hdr->ncalls;
    const int64_t first = TRANS ? ncalls : 0, last = TRANS ? 2 * ncalls : ncalls;  // tasks
    const int64_t base = pack_prefix[first], total = pack_prefix[last];            // chunks
    const uint32_t p = hdr->p;
    const int32_t H = int32_t(limb_threshold(L));
    int64_t lo = first;
    for (;;) {
        // (chunk counts stay below 2^31: a batch has fewer chunks)
        if (threadIdx.x == 0)
            chunk_s = uint32_t(atomicAdd((unsigned long long *)counter,
                                         (unsigned long long)kGrab));
        __syncthreads();
        const int64_t c0 = base + int64_t(__builtin_amdgcn_readfirstlane(chunk_s));
        __syncthreads();
        if (c0 >= total) break;
        lo = find_from(pack_prefix, last, lo, c0);
        const int64_t c1 = c0 + kGrab < total ? c0 + kGrab : total;
        for (int64_t c = c0; c < c1; ++c) {
            while (pack_prefix[lo + 1] <= c) ++lo;  // the next chunks may start the next operand
            const PackTask t = packs[lo];
            const int64_t local = c - pack_prefix[lo];
            const int64_t kchunks = (t.nkb + 1) / 2;
            const int64_t rho0 = (local / kchunks) * kChunk, kap0 = (local % kchunks) * kChunk;
            if (c > c0) __syncthreads();  // the previous chunk's LDS reads are done
            pack_chunk<L, TRANS>(t.dst, t.nkb, t.src, t.r0, t.c0, t.shift, t.R, t.K, t.logT, p, H,
                                 rho0, kap0, tile, t.neg, TRANS ? int64_t(t.kshift) : 0);
        }
    }
}

template <int L>
hipError_t launch_limb_L(int8_t *dst, int64_t prow, int64_t nkb, const uint32_t *src, int64_t r0,
                         int64_t c0, int64_t shift, int64_t R, int64_t K, int trans, int neg,
                         int logT, uint32_t p, hipStream_t s)
{
    const int32_t H = int32_t(limb_threshold(L));
    dim3 grid(unsigned((nkb + 1) / 2), unsigned(prow / kChunk));
    if (trans)
        hipLaunchKernelGGL((k_pack_limb<L, true>), grid, dim3(256), 0, s, dst, nkb, src, r0, c0,
                           shift, R, K, logT, p, H, neg);
    else
        hipLaunchKernelGGL((k_pack_limb<L, false>), grid, dim3(256), 0, s, dst, nkb, src, r0, c0,
                           shift, R, K, logT, p, H, neg);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pack_u32(uint32_t *dst, int64_t prow, int64_t pcol, const uint32_t *src,
                           int64_t srow0, int64_t scol0, int64_t vr0, int64_t vr1, int64_t vc0,
                           int64_t vc1, int logT, hipStream_t s)
{
    const int64_t ntr = prow >> logT, ntc = pcol >> logT;
    if (ntr <= 0 || ntc <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_u32, dim3(unsigned(ntc), unsigned(ntr)), dim3(256), 0, s, dst, ntc,
                       src, srow0, scol0, vr0, vr1, vc0, vc1, logT);
    return hipGetLastError();
}

hipError_t launch_pack_limb_batched(int L, const QueueView &q, uint64_t *counters, int num_cu,
                                    hipStream_t s)
{
    // A panels with counters[0], then B panels with counters[1].
    auto go = [&](auto kern_a, auto kern_b) {
        hipError_t e = hipSuccess;
        int i = 0;
        for (auto kern : {kern_a, kern_b}) {
            int per_cu = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0) !=
                    hipSuccess ||
                per_cu < 1)
                per_cu = 1;
            hipLaunchKernelGGL(kern, dim3(unsigned(num_cu * per_cu)), dim3(256), 0, s, q.hdr,
                               q.packs, q.pack_prefix, counters + i++);
            if ((e = hipGetLastError()) != hipSuccess) break;
        }
        return e;
    };
    switch (L) {
    case 1: return go(k_pack_limb_batched<1, false>, k_pack_limb_batched<1, true>);
    case 2: return go(k_pack_limb_batched<2, false>, k_pack_limb_batched<2, true>);
    case 3: return go(k_pack_limb_batched<3, false>, k_pack_limb_batched<3, true>);
    default: return go(k_pack_limb_batched<4, false>, k_pack_limb_batched<4, true>);
    }
}

hipError_t launch_pack_limb(int8_t *dst, int64_t prow, int64_t nkb, const uint32_t *src,
                            int64_t r0, int64_t c0, int64_t shift, int64_t R, int64_t K, int trans,
                            int neg, int logT, uint32_t p, int L, hipStream_t s)
{
    if (prow <= 0 || nkb <= 0) return hipSuccess;
    switch (L) {
    case 1: return launch_limb_L<1>(dst, prow, nkb, src, r0, c0, shift, R, K, trans, neg, logT, p, s);
    case 2: return launch_limb_L<2>(dst, prow, nkb, src, r0, c0, shift, R, K, trans, neg, logT, p, s);
    case 3: return launch_limb_L<3>(dst, prow, nkb, src, r0, c0, shift, R, K, trans, neg, logT, p, s);
    default: return launch_limb_L<4>(dst, prow, nkb, src, r0, c0, shift, R, K, trans, neg, logT, p, s);
    }
}

}  // namespace mh
