// int8-limb MFMA GEMM with fused mod-p epilogue: C := (C + A.B) mod p.
//
// Every residue has been split by the packing kernel into L balanced
// base-256 digits in [-128, 127] (A = sum_t A_t 256^t, B = sum_u B_u 256^u
// with the centred residues), so
//     A.B = sum_s 256^s T_s,   T_s = sum_{t+u=s} A_t . B_u,  s = 0 .. 2L-2.
// Each T_s is an int8 x int8 -> int32 product, run on the gfx950 MFMA
// v_mfma_i32_32x32x32_i8.  A k-block is short enough (kblock_for) that no
// T_s can leave int32; after each k-block the shifts are combined by Horner
// (r <- 256 r + T_s mod p, highest s first) into a residue, and at the end
// the residue is added to C mod p.  Exact: the error against the definition
// is zero.
//
// Operand panels are in MFMA operand order (1 KiB per 32x32 block and limb,
// lane q holding 16 consecutive depths of row q mod 32), so every fragment
// is one coalesced 16-byte load per lane straight from global memory / L2;
// the L digit planes of a block are adjacent, and consecutive k-blocks
// follow each other.  A wave computes WM x WN blocks of 32 x 32 outputs and
// keeps (2L-1) int32 accumulator tiles per block.  The epilogue writes
// whole C tile pieces (the workgroup's output block is aligned to C's tile
// grid) with masked read-modify-write.
#include "mh_device.h"

namespace mh {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

template <int L, int WM, int WN, int WAVES_M, int WAVES_N>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N) void k_gemm_limb(LimbArgs a)
{
    constexpr int S = 2 * L - 1;
    constexpr int BM = 32 * WM * WAVES_M, BN = 32 * WN * WAVES_N;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wmi = wave / WAVES_N, wni = wave % WAVES_N;
    int64_t gm, gn;
    tile_of(blockIdx.x, a.grid_m, a.grid_n, 8, gm, gn);

    const int64_t slabA = gm * (WM * WAVES_M) + wmi * WM;
    const int64_t slabB = gn * (WN * WAVES_N) + wni * WN;
    const int64_t nkb = a.nkb;
    // v4i units: block (slab, kb, limb) starts at ((slab * nkb + kb) * L + limb) * 64
    const v4i *pa = reinterpret_cast<const v4i *>(a.Ap) + slabA * nkb * L * 64 + lane;
    const v4i *pb = reinterpret_cast<const v4i *>(a.Bp) + slabB * nkb * L * 64 + lane;
    const int64_t slab_stride = nkb * L * 64;

    v16i acc[S][WM][WN];
    static_for<S>([&](auto s) {
        static_for<WM>([&](auto i) { static_for<WN>([&](auto j) { acc[s][i][j] = v16i{0}; }); });
    });

    // Combine the shift accumulators of one k-block by Horner into residues
    // (highest shift first: r <- 256 r + T_s mod p, so each shift's registers
    // are free once consumed), then add them to C with a masked
    // read-modify-write inside C's tiles, and clear the accumulators.
    // Output (row, col) of a 32x32 block sits in lane col + 32 * ((row / 4) & 1),
    // register 4 * (row / 8) + row % 4.
    auto flush = [&]() {
        uint32_t r[WM][WN][16];
        static_for<WM>([&](auto i) {
            static_for<WN>([&](auto j) { static_for<16>([&](auto v) { r[i][j][v] = 0; }); });
        });
        static_for<S>([&](auto q) {
            constexpr int s = S - 1 - q;
            static_for<WM>([&](auto i) {
                static_for<WN>([&](auto j) {
                    static_for<16>([&](auto v) {
                        const uint64_t x =
                            (uint64_t(r[i][j][v]) << 8) + a.bias + int64_t(acc[s][i][j][int(v)]);
                        r[i][j][v] = mod_u64(x, a.p, a.mu);
                    });
                    acc[s][i][j] = v16i{0};
                });
            });
        });
        static_for<WM>([&](auto i) {
            static_for<WN>([&](auto j) {
                const int64_t gam = gn * BN + (wni * WN + j) * 32 + (lane & 31);
                if (gam < a.sc || gam >= a.sc + a.n) return;
                const uint64_t ccol = uint64_t(a.col0C + gam);
                static_for<16>([&](auto v) {
                    const int row = (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
                    const int64_t rho = gm * BM + (wmi * WM + i) * 32 + row;
                    if (rho < a.sr || rho >= a.sr + a.m) return;
                    const uint64_t off = mh_offset(uint64_t(a.row0C + rho), ccol, a.logT);
                    uint32_t c = a.C[off] + r[i][j][v];
                    if (c >= a.p) c -= a.p;
                    a.C[off] = c;
                });
            });
        });
    };

    for (int64_t kb0 = 0; kb0 < nkb; kb0 += a.kb_per_red) {
        const int64_t kb1 = (kb0 + a.kb_per_red < nkb) ? kb0 + a.kb_per_red : nkb;
        for (int64_t kb = kb0; kb < kb1; ++kb) {
            v4i fa[WM][L], fb[WN][L];
            static_for<WM>([&](auto i) {
                static_for<L>([&](auto t) { fa[i][t] = pa[i * slab_stride + (kb * L + t) * 64]; });
            });
            static_for<WN>([&](auto j) {
                static_for<L>([&](auto u) { fb[j][u] = pb[j * slab_stride + (kb * L + u) * 64]; });
            });
            static_for<L>([&](auto t) {
                static_for<L>([&](auto u) {
                    static_for<WM>([&](auto i) {
                        static_for<WN>([&](auto j) {
                            acc[t + u][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                fa[i][t], fb[j][u], acc[t + u][i][j], 0, 0, 0);
                        });
                    });
                });
            });
        }
        flush();
    }
}

template <int L, int WM, int WN, int WAVES_M, int WAVES_N>
hipError_t launch_one(const LimbArgs &a, hipStream_t s)
{
    const int64_t groups = a.grid_m * a.grid_n;
    if (groups <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_gemm_limb<L, WM, WN, WAVES_M, WAVES_N>), dim3(unsigned(groups)),
                       dim3(64 * WAVES_M * WAVES_N), 0, s, a);
    return hipGetLastError();
}

// Configuration table.  (2L-1) * WM * WN accumulator tiles of 16 registers
// must fit beside the fragments: at most 14 tiles.
const LimbKernelCfg kCfgs[] = {
    {0, 1, 2, 2, 2},  // 64 x 128
    {1, 1, 1, 2, 2},  // 64 x 64
    {2, 2, 1, 2, 2},  // 128 x 64
    {3, 2, 2, 2, 2},  // 128 x 128 (L <= 2)
};

bool cfg_fits(int L, const LimbKernelCfg &c) { return (2 * L - 1) * c.wm * c.wn <= 14; }

template <int L>
hipError_t dispatch_L(int cfg, const LimbArgs &a, hipStream_t s)
{
    switch (cfg) {
    case 0: return launch_one<L, 1, 2, 2, 2>(a, s);
    case 1: return launch_one<L, 1, 1, 2, 2>(a, s);
    case 2: return launch_one<L, 2, 1, 2, 2>(a, s);
    case 3:
        if constexpr (L <= 2) return launch_one<L, 2, 2, 2, 2>(a, s);
        return hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

}  // namespace

int limb_cfg_count() { return int(sizeof(kCfgs) / sizeof(kCfgs[0])); }
const LimbKernelCfg &limb_cfg(int idx) { return kCfgs[idx]; }

int limb_cfg_default(int L, int64_t m, int64_t n, int64_t k)
{
    (void)k;
    if (m * n <= int64_t(512) * 512) return 1;
    if (L <= 2) return 3;
    return 0;
}

hipError_t launch_gemm_limb(int cfg, int L, const LimbArgs &a, hipStream_t s)
{
    if (cfg < 0 || cfg >= limb_cfg_count() || !cfg_fits(L, kCfgs[cfg])) return hipErrorInvalidValue;
    switch (L) {
    case 1: return dispatch_L<1>(cfg, a, s);
    case 2: return dispatch_L<2>(cfg, a, s);
    case 3: return dispatch_L<3>(cfg, a, s);
    case 4: return dispatch_L<4>(cfg, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace mh
