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

// C through a global-address-space pointer: its loads and stores are then
// global (vector memory counter only) rather than flat, which the compiler
// also counts as LDS accesses, so that every wait for a fragment read from
// LDS would wait for the C traffic as well.
typedef __attribute__((address_space(1))) uint32_t gu32;

// Stages between the early C loads and the epilogue (persistent kernel, one
// 32 x 32 block per wave, L <= 2).
constexpr int kCLead = 2;

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// One workgroup's output block (gm, gn) of the product described by `a`.
// PIPE (LDS path): fragment reads one k-block ahead of the MFMAs, with a
// second fragment set.
template <int L, int WM, int WN, int WAVES_M, int WAVES_N, int KS, bool LDS, int NBUF, bool PIPE,
          bool EARLYC = false, bool APAR = false>
__device__ __forceinline__ void gemm_tile(const LimbArgs &a, int64_t gm, int64_t gn)
{
    constexpr int S = 2 * L - 1;
    constexpr int BM = 32 * WM * WAVES_M, BN = 32 * WN * WAVES_N;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wmi = wave / WAVES_N, wni = wave % WAVES_N;
    gu32 *const Cg = (gu32 *)a.C;

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

    // C words of the wave's outputs loaded kCLead stages ahead of the
    // epilogue (one 32 x 32 block per wave, at L <= 2 in the persistent
    // kernel: a block there is a short pipeline, and its C round trip would
    // otherwise stall the waves between two blocks).  The launch selects
    // this form for T >= 32 and C parents of at most 2^30 words, so 32
    // consecutive rows (columns) lie in at most two tile rows (columns), and
    // every word has a 32-bit byte offset from the parent's base: per lane,
    // the offsets of its column in the two tile rows, and per output a
    // select, keep the 16 loads within a few registers.  Rows and columns
    // are clamped into the output block (a wave wholly outside it takes the
    // block's first rows and columns), so every wave issues all 16 loads,
    // to valid words, without branches, and the stage waits can count them;
    // out-of-block outputs discard theirs.
    constexpr bool kEarlyC = EARLYC && LDS && !PIPE && WM * WN == 1;
    uint32_t cpre[16];
    auto c_tile = [&](auto &&f) {
        // f(v, inside, base, byte offset) for the lane's 16 outputs
        const int lt = a.logT;
        const uint32_t tmask = (1u << lt) - 1;
        const int wu = __builtin_amdgcn_readfirstlane(wave);  // (wave-uniform: scalar)
        const int64_t rho0 = gm * BM + (wu / WAVES_N) * 32, gam0 = gn * BN + (wu % WAVES_N) * 32;
        const bool any = rho0 < a.sr + a.m && rho0 + 32 > a.sr && gam0 < a.sc + a.n &&
                         gam0 + 32 > a.sc;
        const uint32_t rlo = uint32_t(a.row0C + a.sr), rhi = rlo + uint32_t(a.m) - 1;
        const uint32_t clo = uint32_t(a.col0C + a.sc), chi = clo + uint32_t(a.n) - 1;
        const uint32_t R0 = any ? uint32_t(a.row0C + rho0) : rlo;
        const uint32_t C0 = any ? uint32_t(a.col0C + gam0) : clo;
        const uint32_t tr0 = R0 >> lt, tc0 = C0 >> lt;
        const uint32_t bR = (tr0 + 1) << lt, bC = (tc0 + 1) << lt;  // next tile row / column
        uint32_t col = C0 + uint32_t(lane & 31);
        const bool col_in = any && col >= clo && col <= chi;
        col = col < clo ? clo : (col > chi ? chi : col);
        const uint32_t tcl = col >= bC ? tc0 + 1 : tc0;
        // word offsets of the lane's column in tile rows tr0 and tr0 + 1 (the
        // second is used only by rows that lie there, so its tile exists)
        uint32_t baseU = ((((spread16(tr0) << 1) | spread16(tcl)) << (2 * lt)) | (col & tmask));
        uint32_t baseL = ((((spread16(tr0 + 1) << 1) | spread16(tcl)) << (2 * lt)) | (col & tmask));
        // (computed where used: hoisted out of the k loop, the addresses
        // would hold registers through it)
        asm volatile("" : "+v"(baseU), "+v"(baseL));
        const uint32_t rl = R0 + uint32_t((lane >> 5) * 4);
        static_for<16>([&](auto v) {
            constexpr int drow = (int(v) >> 2) * 8 + (int(v) & 3);
            uint32_t row = rl + uint32_t(drow);
            const bool in = col_in && row >= rlo && row <= rhi;
            row = row < rlo ? rlo : (row > rhi ? rhi : row);
            f(v, in, Cg, ((row >= bR ? baseL : baseU) + ((row & tmask) << lt)) << 2);
        });
    };
    auto word = [](gu32 *base, uint32_t byte_off) -> gu32 & {
        return *(gu32 *)((__attribute__((address_space(1))) char *)base + byte_off);
    };
    auto fetch_c = [&]() {
        if constexpr (kEarlyC) {
                c_tile([&](auto v, bool, gu32 *base, uint32_t off) { cpre[int(v)] = word(base, off); });
        }
    };

    // Combine the shift accumulators of one k-block by Horner into residues
    // (highest shift first: r <- 256 r + T_s mod p, so each shift's registers
    // are free once consumed), then add them to C with a masked
    // read-modify-write inside C's tiles, and clear the accumulators.
    // Output (row, col) of a 32x32 block sits in lane col + 32 * ((row / 4) & 1),
    // register 4 * (row / 8) + row % 4.
    auto flush = [&]() {
        // Horner in fp64, two shifts per reduction: with r < p < 2^31 and
        // |T_s| < 2^31, x = 65536 r + 256 T_s + T_{s-1} has |x| < 2^48, so x and
        // x - q p are exact doubles; q = floor(x / p) from the rounded
        // reciprocal is off by at most one (|x / p| error < 2^-4), which the two
        // corrections absorb.  Result: r = sum_s 256^s T_s mod p in [0, p).
        const double pd = double(a.p), pinv = a.pinv;
        auto red = [&](double x) {
            const double q = floor(x * pinv);
            double r = fma(-q, pd, x);
            r = r < 0.0 ? r + pd : r;
            r = r >= pd ? r - pd : r;
            return r;
        };
        // Three shifts (L = 2) need one reduction: 65536 T_2 + 256 T_1 + T_0
        // is below 2^48 in magnitude as well.
        constexpr int S0 = S == 3 ? 3 : 1;  // shifts taken by the first reduction
        if constexpr (kEarlyC) {
            // One output at a time, from its accumulators to its early C word.
            c_tile([&](auto v, bool in, gu32 *base, uint32_t off) {
                double x = double(acc[S - 1][0][0][int(v)]);
                if constexpr (S0 == 3)
                    x = fma(x, 65536.0, fma(double(acc[1][0][0][int(v)]), 256.0,
                                            double(acc[0][0][0][int(v)])));
                double rv = red(x);
                static_for<(S - S0) / 2>([&](auto q) {
                    constexpr int hi = S - 2 - 2 * q, lo = hi - 1;
                    rv = red(fma(rv, 65536.0, fma(double(acc[hi][0][0][int(v)]), 256.0,
                                                  double(acc[lo][0][0][int(v)]))));
                });
                if (in) {
                    uint32_t c = cpre[int(v)] + uint32_t(rv);
                    if (c >= a.p) c -= a.p;
                    word(base, off) = c;
                }
            });
            static_for<S>([&](auto t) { acc[t][0][0] = v16i{0}; });
            return;
        }
        double r[WM][WN][16];
        static_for<WM>([&](auto i) {
            static_for<WN>([&](auto j) {
                static_for<16>([&](auto v) {
                    double x = double(acc[S - 1][i][j][int(v)]);
                    if constexpr (S0 == 3)
                        x = fma(x, 65536.0, fma(double(acc[1][i][j][int(v)]), 256.0,
                                                double(acc[0][i][j][int(v)])));
                    r[i][j][v] = red(x);
                });
                static_for<S0>([&](auto t) { acc[S - 1 - t][i][j] = v16i{0}; });
            });
        });
        static_for<(S - S0) / 2>([&](auto q) {
            constexpr int hi = S - 2 - 2 * q, lo = hi - 1;
            static_for<WM>([&](auto i) {
                static_for<WN>([&](auto j) {
                    static_for<16>([&](auto v) {
                        const double x = fma(r[i][j][v], 65536.0,
                                             fma(double(acc[hi][i][j][int(v)]), 256.0,
                                                 double(acc[lo][i][j][int(v)])));
                        r[i][j][v] = red(x);
                    });
                    acc[hi][i][j] = v16i{0};
                    acc[lo][i][j] = v16i{0};
                });
            });
        });
        // Word offsets in C with 32-bit dilation (parents have at most 2^18
        // rows and T >= 16, so tile coordinates stay below 2^14).  The column
        // part is the lane's.  A 32-row block starts on a multiple of
        // min(T, 32) in C (the panel shift), so its rows 0-15 and 16-31 each
        // lie in one tile row: two dilations per block serve its 16 outputs.
        const uint32_t tmask = (1u << a.logT) - 1;
        static_for<WM>([&](auto i) {
            const int64_t rho0 = gm * BM + (wmi * WM + i) * 32;  // first panel row of the block
            const uint32_t rowC0 = uint32_t(a.row0C + rho0);
            const uint32_t rowbits[2] = {spread16(rowC0 >> a.logT) << 1,
                                         spread16((rowC0 + 16) >> a.logT) << 1};
            static_for<WN>([&](auto j) {
                const int64_t gam = gn * BN + (wni * WN + j) * 32 + (lane & 31);
                if (gam < a.sc || gam >= a.sc + a.n) return;
                const uint32_t colC = uint32_t(a.col0C + gam);
                const uint32_t colbits = spread16(colC >> a.logT), colin = colC & tmask;
                auto row_of = [&](int v) { return (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3); };
                auto inside = [&](int v) {
                    const int64_t rho = rho0 + row_of(v);
                    return rho >= a.sr && rho < a.sr + a.m;
                };
                auto offset = [&](int v) {
                    const uint32_t rowC = rowC0 + uint32_t(row_of(v));
                    const uint32_t tile = rowbits[v >= 8 ? 1 : 0] | colbits;
                    return (uint64_t(tile) << (2 * a.logT)) | ((rowC & tmask) << a.logT) | colin;
                };
                if constexpr (WM * WN == 1) {
                    // The C loads of eight outputs first, then their
                    // stores: in the other order each load would wait for
                    // the store before it (the compiler cannot tell the
                    // words apart), one memory round trip per output.
                    static_for<2>([&](auto h) {
                        uint32_t cv[8];
                        static_for<8>([&](auto u) {
                            constexpr int v = int(h) * 8 + int(u);
                            cv[u] = inside(v) ? Cg[offset(v)] : 0u;
                        });
                        static_for<8>([&](auto u) {
                            constexpr int v = int(h) * 8 + int(u);
                            if (!inside(v)) return;
                            uint32_t c = cv[u] + uint32_t(r[i][j][v]);
                            if (c >= a.p) c -= a.p;
                            Cg[offset(v)] = c;
                        });
                    });
                } else {
                    // (larger wave tiles have no registers to spare for that)
                    static_for<16>([&](auto v) {
                        const int row = (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
                        const int64_t rho = rho0 + row;
                        if (rho < a.sr || rho >= a.sr + a.m) return;
                        const uint32_t rowC = rowC0 + uint32_t(row);
                        const uint32_t tile = rowbits[v >= 8 ? 1 : 0] | colbits;
                        const uint64_t off = (uint64_t(tile) << (2 * a.logT)) |
                                             ((rowC & tmask) << a.logT) | colin;
                        uint32_t c = Cg[off] + uint32_t(r[i][j][v]);
                        if (c >= a.p) c -= a.p;
                        Cg[off] = c;
                    });
                }
            });
        });
    };

    // Fragments of k-blocks kb .. kb+KS-1: WM A slabs and WN B slabs, L digit
    // planes each.
    using FragA = v4i[KS][WM][L];
    using FragB = v4i[KS][WN][L];
    auto load = [&](FragA &fa, FragB &fb, int64_t kb) {
        static_for<KS>([&](auto q) {
            static_for<WM>([&](auto i) {
                static_for<L>([&](auto t) {
                    fa[q][i][t] = pa[i * slab_stride + ((kb + q) * L + t) * 64];
                });
            });
            static_for<WN>([&](auto j) {
                static_for<L>([&](auto u) {
                    fb[q][j][u] = pb[j * slab_stride + ((kb + q) * L + u) * 64];
                });
            });
        });
    };
    auto mma = [&](const FragA &fa, const FragB &fb) {
        static_for<KS>([&](auto q) {
            static_for<L>([&](auto t) {
                static_for<L>([&](auto u) {
                    static_for<WM>([&](auto i) {
                        static_for<WN>([&](auto j) {
                            acc[t + u][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                fa[q][i][t], fb[q][j][u], acc[t + u][i][j], 0, 0, 0);
                        });
                    });
                });
            });
        });
    };

    if constexpr (!LDS) {
        // Two register sets: the loads of the next stage (KS k-blocks) are in
        // flight while the MFMAs of the current one run.  nkb and kb_per_red
        // are multiples of KS.
        FragA fa0, fa1;
        FragB fb0, fb1;
        for (int64_t kb0 = 0; kb0 < nkb; kb0 += a.kb_per_red) {
            const int64_t kb1 = (kb0 + a.kb_per_red < nkb) ? kb0 + a.kb_per_red : nkb;
            load(fa0, fb0, kb0);
            int64_t kb = kb0;
            for (; kb + 2 * KS <= kb1; kb += 2 * KS) {
                load(fa1, fb1, kb + KS);
                mma(fa0, fb0);
                if (kb + 2 * KS < kb1) load(fa0, fb0, kb + 2 * KS);
                mma(fa1, fb1);
            }
            if (kb < kb1) mma(fa0, fb0);
            flush();
        }
    } else {
        // The workgroup's blocks of one stage (all A slabs, then all B slabs,
        // KS k-blocks x L limbs each) go global -> LDS with one 16-byte
        // buffer_load ... lds per lane and block, spread over the waves; LDS
        // holds NBUF stages.  Blocks land in lane order, so each wave reads
        // its fragments back with conflict-free 16-byte LDS reads, and every
        // A or B block crosses the L2 once per workgroup instead of once per
        // wave that uses it.  The buffer form (descriptor: the block's slab,
        // so the hardware bounds every access) rather than global_load_lds:
        // the compiler counts a global load into LDS as a FLAT access of
        // either counter and then waits for all loads and LDS reads to drain
        // at every wait, where the buffer form keeps its counts exact (with
        // the bare barrier below, about 6 % faster at L = 2).
        extern __shared__ v4i lds_buf[];  // [NBUF][NBLK][64]
        constexpr int NW = WAVES_M * WAVES_N;
        // A from a whole-parent panel (APAR): the launch starts the panel
        // rows on a parent slab, so the A blocks of a stage are the parent's.
        constexpr bool kApar = APAR;
        constexpr int NA = WM * WAVES_M * KS * L;
        constexpr int NBLK = (WM * WAVES_M + WN * WAVES_N) * KS * L;
        constexpr int R = (NBLK + NW - 1) / NW;  // 16-byte loads per wave and stage (at most)
        // With more than two buffers, the wait below lets this wave's loads of
        // the later stages stay outstanding; waves issue R or R - 1 loads per
        // stage, so it counts the smaller number (waiting a little longer
        // where a wave issued more is still correct).
        constexpr int RMIN = NBLK / NW;
        static_assert((NBUF - 2) * RMIN < 64, "vmcnt count");
        const int wv = __builtin_amdgcn_readfirstlane(wave);
        const int64_t slabA0 = gm * (WM * WAVES_M), slabB0 = gn * (WN * WAVES_N);
        // Block addresses are wave-uniform (scalar registers); only the lane's
        // 16-byte offset is per lane.
        const char *ga = reinterpret_cast<const char *>(a.Ap);
        const char *gb = reinterpret_cast<const char *>(a.Bp);
        const uint32_t lane_off = uint32_t(lane) * 16u;
        const int slab_bytes = int(nkb * L) << 10;  // < 2^31 (nkb <= 2^13)
        auto issue = [&](int64_t st, int buf) {
            const int64_t kb = st * KS;
            static_for<R>([&](auto r) {
                const int b = wv + NW * r;
                if (NBLK % NW == 0 || b < NBLK) {
                    const bool isb = b >= NA;
                    const int bb = isb ? b - NA : b;
                    const int sl = bb / (KS * L), q = (bb / L) % KS, t = bb % L;
                    const int64_t slab = (isb ? slabB0 : slabA0) + sl;
                    __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                        (void *)((isb ? gb : ga) + ((slab * nkb * L) << 10)), 0, slab_bytes,
                        0x00020000);
                    int off = int(((kb + q) * L + t) << 10);
                    if constexpr (kApar) {
                        if (!isb) {
                            // the parent's slab (the panel has guard slabs after
                            // the parent's rows: rows past the parent only feed
                            // discarded outputs, and depths past the product, read
                            // from the next slab, meet zero rows of B)
                            const int64_t ps = a.a_slab0 + gm * WAVES_M + sl;
                            rs = __builtin_amdgcn_make_buffer_rsrc(
                                (void *)(ga + ps * ((a.a_nkbp * L) << 10)), 0, 0x7FFFFFFF,
                                0x00020000);
                            off = int(((a.a_kb0 + kb + q) * L + t) << 10);
                        }
                    }
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(
                        rs,
                        (__attribute__((address_space(3))) void *)(lds_buf +
                                                                    (buf * NBLK + b) * 64),
                        16, int(lane_off), off, 0, 0);
                }
            });
        };
        // s_waitcnt vmcnt(n) lgkmcnt(0), expcnt left free
        constexpr int kWaitInFlight = ((NBUF - 2) * RMIN & 15) | (7 << 4) |
                                      (((NBUF - 2) * RMIN >> 4) << 14);
        constexpr int kWaitAll = 7 << 4;  // vmcnt(0) lgkmcnt(0)
        constexpr int kWaitC = (1 << 14) | (7 << 4);  // vmcnt(16) lgkmcnt(0): the early C loads
        static_assert(KS % 2 == 0, "fragment sets alternate within and across stages");
        const int64_t nst = nkb / KS, st_red = a.kb_per_red / KS;

        // Make stage s readable: this wave's blocks of s have landed (loads
        // complete in order, so it suffices that at most the NBUF - 2 later
        // stages are outstanding; the last stages, and the first stage after
        // an epilogue, whose C accesses were issued after the prefetches,
        // wait for everything), and its own LDS reads of the previous stage
        // are done; then every wave has done the same, so buffer (s - 1) mod
        // NBUF is free again and stage s + NBUF - 1 goes into it.  A bare
        // barrier: the fence of __syncthreads() would make the compiler wait
        // for the later stages' loads as well.  The empty asm statements keep
        // memory accesses on their side.
        auto enter_stage = [&](int64_t s, bool after_epilogue, bool c_pending = false) {
            if (NBUF > 2 && s + NBUF - 2 < nst && !after_epilogue)
                __builtin_amdgcn_s_waitcnt(kWaitInFlight);
            else if (c_pending)
                __builtin_amdgcn_s_waitcnt(kWaitC);
            else
                __builtin_amdgcn_s_waitcnt(kWaitAll);
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            if (s + NBUF - 1 < nst) issue(s + NBUF - 1, int((s + NBUF - 1) % NBUF));
        };
        // Fragments of k-block q of stage s, from LDS.
        using FragA1 = v4i[WM][L];
        using FragB1 = v4i[WN][L];
        auto read = [&](FragA1 &fa, FragB1 &fb, int64_t s, int q) {
            const v4i *sb = lds_buf + (s % NBUF) * (NBLK * 64) + lane;
            static_for<WM>([&](auto i) {
                static_for<L>([&](auto t) {
                    fa[i][t] = sb[(((wmi * WM + i) * KS + q) * L + t) * 64];
                });
            });
            static_for<WN>([&](auto j) {
                static_for<L>([&](auto u) {
                    fb[j][u] = sb[(NA + ((wni * WN + j) * KS + q) * L + u) * 64];
                });
            });
        };
        auto mma1 = [&](const FragA1 &fa, const FragB1 &fb) {
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
        };

        // NBUF - 1 stages in flight ahead of the one being multiplied
        static_for<NBUF - 1>([&](auto s0) {
            if (int64_t(s0) < nst) issue(int64_t(s0), int(s0));
        });
        if constexpr (PIPE) {
            // Two fragment sets: the LDS reads of the next k-block (of this
            // stage, or the first of the next one) are in flight while the
            // current one's MFMAs run; the next stage is entered before the
            // last k-block of the current one is multiplied.
            FragA1 fa[2];
            FragB1 fb[2];
            for (int64_t st0 = 0; st0 < nst; st0 += st_red) {
                const int64_t st1 = (st0 + st_red < nst) ? st0 + st_red : nst;
                enter_stage(st0, st0 > 0);
                read(fa[0], fb[0], st0, 0);
                for (int64_t st = st0; st < st1; ++st) {
                    static_for<KS>([&](auto q) {
                        constexpr int cur = int(q) & 1, nxt = cur ^ 1;
                        if constexpr (int(q) + 1 < KS) {
                            read(fa[nxt], fb[nxt], st, int(q) + 1);
                        } else {
                            if (st + 1 < st1) {
                                enter_stage(st + 1, false);
                                read(fa[nxt], fb[nxt], st + 1, 0);
                            }
                        }
                        mma1(fa[cur], fb[cur]);
                    });
                }
                flush();
            }
        } else {
            // One fragment set, read right before its MFMAs.
            for (int64_t st0 = 0; st0 < nst; st0 += st_red) {
                const int64_t st1 = (st0 + st_red < nst) ? st0 + st_red : nst;
                // The early C loads go out with the first k-block of stage
                // st_c, after the loads of stage st_c + 1: entering that
                // stage waits for all but those 16 loads (loads complete in
                // order), so their latency hides behind whole stages.
                // (Stage st_c comes after the loop: inside it, the loads'
                // registers would look busy on the loop's back edge, and the
                // compiler would wait for all loads before reusing them.)
                const int64_t st_c = st1 - kCLead > st0 ? st1 - kCLead : st0;
                auto body = [&](int64_t st, bool fetch) {
                    static_for<KS>([&](auto q) {
                        FragA1 fa;
                        FragB1 fb;
                        read(fa, fb, st, int(q));
                        if (int(q) == 0 && fetch) fetch_c();
                        mma1(fa, fb);
                    });
                };
                for (int64_t st = st0; st < (kEarlyC ? st_c : st1); ++st) {
                    enter_stage(st, st == st0 && st0 > 0);
                    body(st, false);
                }
                if constexpr (kEarlyC) {
                    enter_stage(st_c, st_c == st0 && st0 > 0);
                    body(st_c, true);
                    for (int64_t st = st_c + 1; st < st1; ++st) {
                        enter_stage(st, false, st == st_c + 1);
                        body(st, false);
                    }
                }
                flush();
            }
        }
    }
}

// At L >= 3 the four-wave 32 x 32 LDS configuration asks for two waves per
// SIMD (it then fits 217 registers without spilling), so that two of its
// workgroups, each with its own stage barrier, share a compute unit.
template <int L, int WM, int WN, int WAVES_M, int WAVES_N, int KS, bool LDS, int NBUF>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N,
                             (LDS && WAVES_M * WAVES_N == 4 && WM * WN == 1 && L >= 3) ? 2 : 1) void
k_gemm_limb(LimbArgs a)
{
    int64_t gm, gn;
    tile_of(blockIdx.x, a.grid_m, a.grid_n, 8, gm, gn);
    gemm_tile<L, WM, WN, WAVES_M, WAVES_N, KS, LDS, NBUF, true>(a, gm, gn);
}

// Persistent form for a batch of products.  The output blocks come in
// kXcdGroups groups of whole products (numbered call by call in the queue's
// order, largest k first within a group).  Workgroups are dispatched to the
// XCDs round-robin, so workgroup b runs on XCD b mod 8: it pops blocks of
// group b mod 8 through that group's atomic counter until the group is
// done, then helps the other groups in turn, and exits when all are done
// (the exit test is the same for all waves of the group).  A group's
// operand panels are thus read by one XCD and stay in its L2.  The pop of
// the next block is issued when a block starts and read when it ends, so
// its latency hides behind the block.  A forward search over the per-call
// prefix sums finds the call of a block.
template <int L, int WM, int WN, int WAVES_M, int WAVES_N, int KS, bool LDS, int NBUF, bool EARLYC,
          bool APAR>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N,
                             (WAVES_M * WAVES_N == 8 && WM * WN == 1 && L <= 2) ? 4 : 1) void
k_gemm_limb_batched(
    const BatchHeader *__restrict__ hdr, const LimbArgs *__restrict__ calls,
    const int64_t *__restrict__ tile_prefix, uint64_t *counters)
{
    // (The queue arrays are separate read-only parameters, so that loads
    // from them at uniform addresses can be scalar.)
    __shared__ uint32_t task_s;
    const int64_t ncalls = hdr->ncalls;
    const int g0 = int(blockIdx.x % kXcdGroups);
    // Block indices and counter values stay below 2^31 (a batch has fewer
    // output blocks, and each counter passes its group's size at most once
    // per workgroup).
    auto pop = [&](int g) {
        return uint32_t(atomicAdd((unsigned long long *)(counters + g), 1ull));
    };
    // The block index is the same for all lanes: read it as a scalar, so
    // that the product's arguments load into scalar registers.
    auto publish = [&](uint32_t v) {
        if (threadIdx.x == 0) task_s = v;
        __syncthreads();
        const uint32_t r = __builtin_amdgcn_readfirstlane(task_s);
        __syncthreads();
        return r;
    };
    for (int gi = 0; gi < kXcdGroups; ++gi) {
        const int g = (g0 + gi) % kXcdGroups;
        const int64_t first = hdr->group_tile[g], size = hdr->group_tile[g + 1] - first;
        int64_t lo = hdr->group_call[g];
        uint32_t cur = publish(threadIdx.x == 0 ? pop(g) : 0u);
        while (int64_t(cur) < size) {
            uint32_t next = 0;
            if (threadIdx.x == 0) next = pop(g);  // read after the block
            const int64_t t = first + cur;
            lo = find_from(tile_prefix, ncalls, lo, t);
            const LimbArgs a = calls[lo];
            const int64_t local = t - tile_prefix[lo];
            // The queue state takes registers: only the eight-wave 32 x 32
            // configurations have room for the second fragment set here, and
            // at L <= 2 they rather keep to 128 registers (launch bounds), so
            // that two workgroups share a compute unit and one's epilogue
            // and first loads overlap the other's MFMAs.
            constexpr bool kPipe = WAVES_M * WAVES_N <= 8 && WM * WN == 1 && L > 2;
            gemm_tile<L, WM, WN, WAVES_M, WAVES_N, KS, LDS, NBUF, kPipe, EARLYC, APAR>(
                a, local / a.grid_n, local % a.grid_n);
            cur = publish(next);
        }
    }
}

template <int L, int WM, int WN, int WAVES_M, int WAVES_N, int KS, bool LDS, int NBUF>
constexpr size_t lds_bytes()
{
    return LDS ? size_t(NBUF) * (WM * WAVES_M + WN * WAVES_N) * KS * L * 1024 : 0;
}

template <int L, int WM, int WN, int WAVES_M, int WAVES_N, int KS, bool LDS, int NBUF = 2>
hipError_t launch_one(const LimbArgs &a, hipStream_t s)
{
    const int64_t groups = a.grid_m * a.grid_n;
    if (groups <= 0) return hipSuccess;
    if (a.nkb % KS || a.kb_per_red % KS) return hipErrorInvalidValue;
    auto kern = k_gemm_limb<L, WM, WN, WAVES_M, WAVES_N, KS, LDS, NBUF>;
    const size_t shm = lds_bytes<L, WM, WN, WAVES_M, WAVES_N, KS, LDS, NBUF>();
    if (shm > 65536) {
        static bool set = false;
        if (!set && hipFuncSetAttribute((const void *)kern,
                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                        int(shm)) != hipSuccess)
            return hipErrorInvalidValue;
        set = true;
    }
    hipLaunchKernelGGL(kern, dim3(unsigned(groups)), dim3(64 * WAVES_M * WAVES_N), shm, s, a);
    return hipGetLastError();
}

// Configuration table: {id, WM, WN, waves_m, waves_n, KS, LDS, NBUF, LMAX}.
// (2L-1) * WM * WN accumulator tiles of 16 registers must fit beside the
// fragments: at most 14 tiles.  NBUF: LDS stage buffers (NBUF - 1 stages in
// flight while one is multiplied).  LMAX: largest limb count the
// configuration is built for (LDS capacity).
const LimbKernelCfg kCfgs[] = {
    {0, 1, 2, 2, 2, 1, 0},  // 64 x 128
    {1, 1, 1, 2, 2, 1, 0},  // 64 x 64
    {2, 2, 1, 2, 2, 1, 0},  // 128 x 64
    {3, 2, 2, 2, 2, 1, 0},  // 128 x 128 (L <= 2)
    {4, 1, 2, 2, 2, 2, 0},  // 64 x 128, 64-deep stages
    {5, 2, 2, 2, 2, 2, 0},  // 128 x 128, 64-deep stages (L <= 2)
    {6, 1, 1, 2, 2, 2, 0},  // 64 x 64, 64-deep stages
    {7, 1, 2, 2, 2, 2, 1},   // 64 x 128, LDS-shared stages
    {8, 2, 2, 2, 2, 2, 1},   // 128 x 128, LDS-shared stages (L <= 2)
    {9, 1, 1, 2, 2, 2, 1},   // 64 x 64, LDS-shared stages
    {10, 2, 1, 2, 2, 2, 1},  // 128 x 64, LDS-shared stages
    {11, 1, 1, 2, 4, 2, 1},        // 64 x 128, 8 waves of 32 x 32, LDS-shared stages
    {12, 1, 1, 4, 2, 2, 1},        // 128 x 64, 8 waves of 32 x 32, LDS-shared stages
    {13, 1, 1, 4, 4, 2, 1, 2, 2},  // 128 x 128, 16 waves of 32 x 32, LDS-shared stages (L <= 2)
    {14, 1, 1, 4, 4, 2, 1, 3, 2},  // the same, two stages in flight (L <= 2)
    {15, 1, 2, 4, 2, 2, 1, 2, 2},  // 128 x 128, 8 waves of 32 x 64, LDS-shared stages (L <= 2)
};

bool cfg_fits(int L, const LimbKernelCfg &c)
{
    return (2 * L - 1) * c.wm * c.wn <= 14 && L <= c.lmax;
}

template <int L, int WM, int WN, int WAVES_M, int WAVES_N, int KS, bool LDS, int NBUF = 2,
          bool CAN_APAR = false>
hipError_t launch_batched_one(bool early_c, bool a_parent, const QueueView &q, uint64_t *counters,
                              int num_cu, hipStream_t s)
{
    // The early-C form exists where the kernel multiplies without a second
    // fragment set, one 32 x 32 block per wave; the A-parent form for the
    // configurations that name it.
    constexpr bool kCan = LDS && WM * WN == 1 && L <= 2;
    constexpr bool kCanA = kCan && CAN_APAR;
    using Kern = void (*)(const BatchHeader *, const LimbArgs *, const int64_t *, uint64_t *);
    Kern kern = k_gemm_limb_batched<L, WM, WN, WAVES_M, WAVES_N, KS, LDS, NBUF, false, false>;
    const size_t shm = lds_bytes<L, WM, WN, WAVES_M, WAVES_N, KS, LDS, NBUF>();
    if constexpr (kCan) {
        if (early_c) kern = k_gemm_limb_batched<L, WM, WN, WAVES_M, WAVES_N, KS, LDS, NBUF, true, false>;
    }
    if constexpr (kCanA) {
        if (a_parent) {
            kern = early_c
                       ? k_gemm_limb_batched<L, WM, WN, WAVES_M, WAVES_N, KS, LDS, NBUF, true, true>
                       : k_gemm_limb_batched<L, WM, WN, WAVES_M, WAVES_N, KS, LDS, NBUF, false, true>;
        }
    }
    // (the host drops the panel shifts for the early-C form: a kernel without
    // it would misplace the outputs)
    if ((early_c && !kCan) || (a_parent && !kCanA)) return hipErrorInvalidValue;
    // (called while a graph is captured, once per graph)
    if (shm > 65536 && hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           int(shm)) != hipSuccess)
        return hipErrorInvalidValue;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * WAVES_M * WAVES_N, shm) !=
            hipSuccess || per_cu < 1)
        per_cu = 1;
    hipLaunchKernelGGL(kern, dim3(unsigned(num_cu * per_cu)), dim3(64 * WAVES_M * WAVES_N), shm,
                       s, q.hdr, q.calls, q.tile_prefix, counters);
    return hipGetLastError();
}

template <int L>
hipError_t dispatch_batched_L(int cfg, bool early_c, bool a_parent, const QueueView &q,
                              uint64_t *counters, int num_cu, hipStream_t s)
{
    switch (cfg) {
    case 0: return launch_batched_one<L, 1, 2, 2, 2, 1, false>(early_c, a_parent, q, counters, num_cu, s);
    case 1: return launch_batched_one<L, 1, 1, 2, 2, 1, false>(early_c, a_parent, q, counters, num_cu, s);
    case 2: return launch_batched_one<L, 2, 1, 2, 2, 1, false>(early_c, a_parent, q, counters, num_cu, s);
    case 3:
        if constexpr (L <= 2) return launch_batched_one<L, 2, 2, 2, 2, 1, false>(early_c, a_parent, q, counters, num_cu, s);
        return hipErrorInvalidValue;
    case 4: return launch_batched_one<L, 1, 2, 2, 2, 2, false>(early_c, a_parent, q, counters, num_cu, s);
    case 5:
        if constexpr (L <= 2) return launch_batched_one<L, 2, 2, 2, 2, 2, false>(early_c, a_parent, q, counters, num_cu, s);
        return hipErrorInvalidValue;
    case 6: return launch_batched_one<L, 1, 1, 2, 2, 2, false>(early_c, a_parent, q, counters, num_cu, s);
    case 7: return launch_batched_one<L, 1, 2, 2, 2, 2, true>(early_c, a_parent, q, counters, num_cu, s);
    case 8:
        if constexpr (L <= 2) return launch_batched_one<L, 2, 2, 2, 2, 2, true>(early_c, a_parent, q, counters, num_cu, s);
        return hipErrorInvalidValue;
    case 9: return launch_batched_one<L, 1, 1, 2, 2, 2, true>(early_c, a_parent, q, counters, num_cu, s);
    case 10: return launch_batched_one<L, 2, 1, 2, 2, 2, true>(early_c, a_parent, q, counters, num_cu, s);
    case 11:
        return launch_batched_one<L, 1, 1, 2, 4, 2, true, 2, true>(early_c, a_parent, q, counters,
                                                                  num_cu, s);
    case 12:
        return launch_batched_one<L, 1, 1, 4, 2, 2, true, 2, true>(early_c, a_parent, q, counters,
                                                                  num_cu, s);
    case 13:
        if constexpr (L <= 2)
            return launch_batched_one<L, 1, 1, 4, 4, 2, true, 2, true>(early_c, a_parent, q,
                                                                      counters, num_cu, s);
        return hipErrorInvalidValue;
    case 14:
        if constexpr (L <= 2)
            return launch_batched_one<L, 1, 1, 4, 4, 2, true, 3>(early_c, a_parent, q, counters, num_cu, s);
        return hipErrorInvalidValue;
    case 15:
        if constexpr (L <= 2) return launch_batched_one<L, 1, 2, 4, 2, 2, true>(early_c, a_parent, q, counters, num_cu, s);
        return hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

template <int L>
hipError_t dispatch_L(int cfg, const LimbArgs &a, hipStream_t s)
{
    switch (cfg) {
    case 0: return launch_one<L, 1, 2, 2, 2, 1, false>(a, s);
    case 1: return launch_one<L, 1, 1, 2, 2, 1, false>(a, s);
    case 2: return launch_one<L, 2, 1, 2, 2, 1, false>(a, s);
    case 3:
        if constexpr (L <= 2) return launch_one<L, 2, 2, 2, 2, 1, false>(a, s);
        return hipErrorInvalidValue;
    case 4: return launch_one<L, 1, 2, 2, 2, 2, false>(a, s);
    case 5:
        if constexpr (L <= 2) return launch_one<L, 2, 2, 2, 2, 2, false>(a, s);
        return hipErrorInvalidValue;
    case 6: return launch_one<L, 1, 1, 2, 2, 2, false>(a, s);
    case 7: return launch_one<L, 1, 2, 2, 2, 2, true>(a, s);
    case 8:
        if constexpr (L <= 2) return launch_one<L, 2, 2, 2, 2, 2, true>(a, s);
        return hipErrorInvalidValue;
    case 9: return launch_one<L, 1, 1, 2, 2, 2, true>(a, s);
    case 10: return launch_one<L, 2, 1, 2, 2, 2, true>(a, s);
    case 11: return launch_one<L, 1, 1, 2, 4, 2, true>(a, s);
    case 12: return launch_one<L, 1, 1, 4, 2, 2, true>(a, s);
    case 13:
        if constexpr (L <= 2) return launch_one<L, 1, 1, 4, 4, 2, true>(a, s);
        return hipErrorInvalidValue;
    case 14:
        if constexpr (L <= 2) return launch_one<L, 1, 1, 4, 4, 2, true, 3>(a, s);
        return hipErrorInvalidValue;
    case 15:
        if constexpr (L <= 2) return launch_one<L, 1, 2, 4, 2, 2, true>(a, s);
        return hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

}  // namespace

int limb_cfg_count() { return int(sizeof(kCfgs) / sizeof(kCfgs[0])); }
const LimbKernelCfg &limb_cfg(int idx) { return kCfgs[idx]; }
bool limb_cfg_fits(int L, int idx)
{
    return idx >= 0 && idx < limb_cfg_count() && cfg_fits(L, kCfgs[idx]);
}

int limb_cfg_default(int L, int64_t m, int64_t n, int64_t k)
{
    (void)k;
    if (m * n <= int64_t(512) * 512) return 6;  // 64 x 64 output blocks
    // 64 x 128, 8 waves sharing LDS stages; at L >= 3, 64 x 64 blocks of 4
    // waves held to two waves per SIMD, so that two workgroups (each with
    // its own barrier) share a compute unit
    return L <= 2 ? 11 : 9;
}

bool limb_batched_early_c(int logT, int64_t max_nc)
{
    return logT >= 5 && max_nc <= (int64_t(1) << 15);
}
bool limb_batched_a_parent(int cfg, int L) { return L <= 2 && cfg >= 11 && cfg <= 13; }

hipError_t launch_gemm_limb_batched(int cfg, int L, bool early_c, bool a_parent,
                                    const QueueView &q, uint64_t *counters, int num_cu,
                                    hipStream_t s)
{
    if (cfg < 0 || cfg >= limb_cfg_count() || !cfg_fits(L, kCfgs[cfg])) return hipErrorInvalidValue;
    if (a_parent && !limb_batched_a_parent(cfg, L)) return hipErrorInvalidValue;
    switch (L) {
    case 1: return dispatch_batched_L<1>(cfg, early_c, a_parent, q, counters, num_cu, s);
    case 2: return dispatch_batched_L<2>(cfg, early_c, a_parent, q, counters, num_cu, s);
    case 3: return dispatch_batched_L<3>(cfg, false, false, q, counters, num_cu, s);
    case 4: return dispatch_batched_L<4>(cfg, false, false, q, counters, num_cu, s);
    }
    return hipErrorInvalidValue;
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
