// FP64-MFMA modular GEMM for primes below 2^26: C := (C +/- A.B) mod p.
//
// Residues are centred, x' = x or x - p in [-(p-1)/2, (p-1)/2], and
// multiplied as doubles with v_mfma_f64_16x16x4f64.  Every product and
// every partial sum is an integer; a double holds integers of magnitude up
// to 2^53 exactly, so the MFMA's sums are exact as long as the accumulator
// (at most p - 1 after a reduction) plus the products added since stays
// within 2^53.  With H = max |x'|, that allows red_steps = (2^53 - p) /
// (4 H^2) MFMA steps of depth 4 between reductions mod p: at least 2 for
// p < 2^26, about 2^21 (no reduction in practice) for p = 65521.  The
// reduction is r = x - floor(x / p) p in double arithmetic (the quotient
// estimate is off by at most one, corrected after an exact fused
// multiply-add).
//
// Operand access is the plain kernel's: A and B are read in place from the
// Morton-hybrid parents when their tiles line up with the output tiles, or
// from tile-major u32 panels written by the packing kernel.  A workgroup
// computes a 128 x 128 output block aligned to C's tile grid (so its writes
// stay inside whole C tiles); four waves each own 64 x 64 (4 x 4 MFMA
// tiles).  32-deep slices of A and B are staged in LDS as centred int32,
// double-buffered, with one barrier per slice.
#include "mh_device.h"

namespace mh {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 32;
constexpr int kStride = BK + 4;  // LDS words per row (BK depths + 4 padding)

__device__ __forceinline__ int32_t centre(uint32_t v, uint32_t p, uint32_t H)
{
    return v > H ? int32_t(v) - int32_t(p) : int32_t(v);
}

// x mod p in [0, p) for an integer-valued double |x| <= 2^53.
__device__ __forceinline__ double reduce_f64(double x, double p, double pinv)
{
    const double q = floor(x * pinv);
    double r = fma(-q, p, x);
    r = r < 0.0 ? r + p : r;
    r = r >= p ? r - p : r;
    return r;
}

constexpr int NQ = BK / 8;  // 16-byte groups per thread per operand per slice

// Per-thread parts of the operand addresses that do not change along k.
// A: thread t reads rows rho0 + (t >> 3) + 32 q, depth group 4 (t & 7) of
// every slice.  B: depth rows (t >> 5) + 8 q of every slice, columns
// gam0 + 4 (t & 31) .. +3.
struct Lanes {
    uint32_t a_row[NQ];    // MH: spread tile row << 1; panel: tile row * ntc
    uint32_t a_inner[NQ];  // (row mod T) << logT
    uint32_t a_ok;         // bit q: row q lies in the product
    uint32_t b_col;        // MH: spread tile column; panel: tile column
    uint32_t b_inner;      // column mod T
    uint32_t b_cmask;      // bit e: column gam + e lies in the product
};

// Word offset of (tile bits, inner) in a Morton-hybrid parent or panel.
__device__ __forceinline__ uint64_t word(uint32_t tile, uint32_t inner, int logT)
{
    return (uint64_t(tile) << (2 * logT)) | inner;
}

__device__ __forceinline__ uint32_t row_bits(int mh, uint32_t tr, uint32_t ntc)
{
    return mh ? spread16(tr) << 1 : tr * ntc;
}

__device__ __forceinline__ uint32_t col_bits(int mh, uint32_t tc)
{
    return mh ? spread16(tc) : tc;
}

// Panel coordinates of one workgroup fit in 32 bits (below 2^18 + 2^8).
struct Geo {
    int32_t sr, er, sc, ec, klo, khi;  // valid rows [sr, er), columns [sc, ec), depths [klo, khi)
    uint32_t a_tr0, a_tc0, a_ntc, b_tr0, b_tc0, b_ntc;
    int a_mh, b_mh, logT;
};

__device__ __forceinline__ void lanes_init(const Geo &g, int32_t rho0, int32_t gam0, int t,
                                           Lanes &ln)
{
    const uint32_t m = (1u << g.logT) - 1;
    ln.a_ok = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int32_t rho = rho0 + (t >> 3) + 32 * q;
        ln.a_row[q] = row_bits(g.a_mh, g.a_tr0 + (uint32_t(rho) >> g.logT), g.a_ntc);
        ln.a_inner[q] = (uint32_t(rho) & m) << g.logT;
        ln.a_ok |= (rho >= g.sr && rho < g.er) ? 1u << q : 0u;
    }
    const int32_t gam = gam0 + 4 * (t & 31);
    ln.b_col = col_bits(g.b_mh, g.b_tc0 + (uint32_t(gam) >> g.logT));
    ln.b_inner = uint32_t(gam) & m;
    ln.b_cmask = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) ln.b_cmask |= (gam + e >= g.sc && gam + e < g.ec) ? 1u << e : 0u;
}

struct Slice {
    uint4 a[NQ], b[NQ];
    uint32_t am, bm;  // bit 4q + e: element e of group q lies in the product
};

// Global loads of one BK-deep slice, four consecutive depths (A) or columns
// (B) per 16-byte load.  A group is read from its own address only when its
// first entry lies in the product's rows (A) or depths (B) and not past the
// end of its depths (A) or columns (B): the group of four then lies in one
// tile that exists.  Other groups read the operand's first 16 bytes
// instead, so every load is unconditional and no wait follows it; the
// per-element masks are applied when the slice is stored to LDS.
__device__ __forceinline__ void load_slice(const PlainArgs &a, const Geo &g, const Lanes &ln,
                                           int32_t kap0, int t, Slice &s)
{
    const uint32_t m = (1u << g.logT) - 1;
    // A: one depth group per thread, the same for its NQ rows
    const int32_t kap = kap0 + 4 * (t & 7);
    uint32_t km = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) km |= (kap + e >= g.klo && kap + e < g.khi) ? 1u << e : 0u;
    const uint32_t acol = col_bits(g.a_mh, g.a_tc0 + (uint32_t(kap) >> g.logT));
    s.am = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const bool ok = ((ln.a_ok >> q) & 1u) && kap < g.khi;
        const uint64_t off =
            ok ? word(ln.a_row[q] + acol, ln.a_inner[q] | (uint32_t(kap) & m), g.logT) : 0;
        s.a[q] = *reinterpret_cast<const uint4 *>(a.A + off);
        s.am |= ok ? km << (4 * q) : 0u;
    }
    // B: NQ depth rows per thread, the same four columns
    s.bm = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int32_t kb = kap0 + (t >> 5) + 8 * q;
        const bool ok = kb >= g.klo && kb < g.khi && ln.b_cmask != 0;
        const uint32_t brow = row_bits(g.b_mh, g.b_tr0 + (uint32_t(kb) >> g.logT), g.b_ntc);
        const uint64_t off =
            ok ? word(brow + ln.b_col, ((uint32_t(kb) & m) << g.logT) | ln.b_inner, g.logT) : 0;
        s.b[q] = *reinterpret_cast<const uint4 *>(a.B + off);
        s.bm |= ok ? ln.b_cmask << (4 * q) : 0u;
    }
}

__device__ __forceinline__ int32_t masked(uint32_t v, uint32_t mk, int bit, uint32_t p,
                                          uint32_t H)
{
    return (mk >> bit) & 1u ? centre(v, p, H) : 0;
}

// Centred int32 into LDS: As[row][depth], Bs[col][depth] (depth contiguous).
__device__ __forceinline__ void store_slice(const Slice &s, int t, int32_t *As, int32_t *Bs,
                                            uint32_t p, uint32_t H)
{
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int row = (t >> 3) + 32 * q, grp = t & 7;
        const uint4 v = s.a[q];
        const int4 w = make_int4(masked(v.x, s.am, 4 * q + 0, p, H),
                                 masked(v.y, s.am, 4 * q + 1, p, H),
                                 masked(v.z, s.am, 4 * q + 2, p, H),
                                 masked(v.w, s.am, 4 * q + 3, p, H));
        *reinterpret_cast<int4 *>(&As[row * kStride + 4 * grp]) = w;
    }
    const int c = 4 * (t & 31);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int kk = (t >> 5) + 8 * q;
        const uint4 v = s.b[q];
        Bs[(c + 0) * kStride + kk] = masked(v.x, s.bm, 4 * q + 0, p, H);
        Bs[(c + 1) * kStride + kk] = masked(v.y, s.bm, 4 * q + 1, p, H);
        Bs[(c + 2) * kStride + kk] = masked(v.z, s.bm, 4 * q + 2, p, H);
        Bs[(c + 3) * kStride + kk] = masked(v.w, s.bm, 4 * q + 3, p, H);
    }
}

constexpr size_t kLdsBytes = size_t(2) * (BM + BN) * kStride * sizeof(int32_t);

// RED2: primes whose reduction interval is below one slice (red_steps <
// BK / 4, p above about 2^25) reduce after every second MFMA step; the
// others reduce every red_steps / (BK / 4) slices, outside the slice loop,
// so that the accumulators stay in the accumulation registers in between.
template <bool RED2>
__global__ __launch_bounds__(256) void k_gemm_f64(PlainArgs a)
{
    extern __shared__ int32_t lds[];  // A buffers [2][BM][kStride], then B [2][BN][kStride]
    auto As = [&](int b) { return lds + b * BM * kStride; };
    auto Bs = [&](int b) { return lds + 2 * BM * kStride + b * BN * kStride; };
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int lr = lane & 15, lg = lane >> 4;
    int64_t gm, gn;
    tile_of(blockIdx.x, a.grid_m, a.grid_n, 8, gm, gn);
    const int32_t rho0 = int32_t(gm * BM), gam0 = int32_t(gn * BN);
    Geo g;
    g.sr = int32_t(a.sr);
    g.er = int32_t(a.sr + a.m);
    g.sc = int32_t(a.sc);
    g.ec = int32_t(a.sc + a.n);
    g.klo = int32_t(a.sk);
    g.khi = int32_t(a.sk + a.k);
    g.a_tr0 = uint32_t(a.a_tr0);
    g.a_tc0 = uint32_t(a.a_tc0);
    g.a_ntc = uint32_t(a.a_ntc);
    g.b_tr0 = uint32_t(a.b_tr0);
    g.b_tc0 = uint32_t(a.b_tc0);
    g.b_ntc = uint32_t(a.b_ntc);
    g.a_mh = a.a_mh;
    g.b_mh = a.b_mh;
    g.logT = a.logT;
    const uint32_t H = (a.p - 1) / 2;
    const double pd = double(a.p);
    Lanes ln;
    lanes_init(g, rho0, gam0, t, ln);

    v4d acc[4][4];
    static_for<4>([&](auto i) {
        static_for<4>([&](auto j) { acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0}; });
    });
    auto reduce_all = [&]() {
        static_for<4>([&](auto i) {
            static_for<4>([&](auto j) {
                static_for<4>([&](auto v) {
                    acc[i][j][int(v)] = reduce_f64(acc[i][j][int(v)], pd, a.pinv);
                });
            });
        });
    };

    int32_t kap0 = (g.klo / BK) * BK;
    Slice s;
    load_slice(a, g, ln, kap0, t, s);
    store_slice(s, t, As(0), Bs(0), a.p, H);
    __syncthreads();
    int buf = 0;
    const int per_red = RED2 ? 0x7FFFFFFF : a.red_steps / (BK / 4);  // slices between reductions
    bool more = true;
    while (more) {
        for (int left = per_red; left > 0; --left) {
            const int32_t next = kap0 + BK;
            more = next < g.khi;
            // Lane (lr, lg) feeds MFMA step e of half h with depth
            // 16 h + 4 lg + e of the slice, for A row lr and B column lr of
            // each 16 x 16 tile.
            static_for<BK / 16>([&](auto h) {
                int4 af[4], bf[4];
                static_for<4>([&](auto i) {
                    af[i] = *reinterpret_cast<const int4 *>(
                        &As(buf)[(wr * 64 + 16 * i + lr) * kStride + 16 * h + 4 * lg]);
                    bf[i] = *reinterpret_cast<const int4 *>(
                        &Bs(buf)[(wc * 64 + 16 * i + lr) * kStride + 16 * h + 4 * lg]);
                });
                static_for<4>([&](auto e) {
                    // the next slice's loads go out after the first step's MFMAs
                    if (h == 0 && e == 1 && more) load_slice(a, g, ln, next, t, s);
                    double ad[4], bd[4];
                    static_for<4>([&](auto i) {
                        const int4 x = af[i], y = bf[i];
                        ad[i] = double(e == 0 ? x.x : e == 1 ? x.y : e == 2 ? x.z : x.w);
                        bd[i] = double(e == 0 ? y.x : e == 1 ? y.y : e == 2 ? y.z : y.w);
                    });
                    static_for<4>([&](auto i) {
                        static_for<4>([&](auto j) {
                            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ad[i], bd[j],
                                                                             acc[i][j], 0, 0, 0);
                        });
                    });
                    if (RED2 && (e == 1 || e == 3)) reduce_all();
                });
            });
            if (!more) break;
            store_slice(s, t, As(buf ^ 1), Bs(buf ^ 1), a.p, H);
            __syncthreads();
            buf ^= 1;
            kap0 = next;
        }
        if (more) reduce_all();
    }

    // Tile (i, j), lane (lr, lg), element v: row 16 i + lg + 4 v, column 16 j + lr
    // (the result layout of v_mfma_f64_16x16x4f64).
    // Per row group i, the C loads of its 16 outputs first, then the
    // stores: in the other order each load would wait for the store before
    // it (the compiler cannot tell the words apart).
    static_for<4>([&](auto i) {
        auto rho_of = [&](int v) { return rho0 + wr * 64 + 16 * int(i) + lg + 4 * v; };
        auto gam_of = [&](int j) { return gam0 + wc * 64 + 16 * j + lr; };
        auto inside = [&](int v, int j) {
            const int64_t rho = rho_of(v), gam = gam_of(j);
            return rho >= a.sr && rho < a.sr + a.m && gam >= a.sc && gam < a.sc + a.n;
        };
        auto offset = [&](int v, int j) {
            return mh_offset(uint64_t(a.row0C + rho_of(v)), uint64_t(a.col0C + gam_of(j)), a.logT);
        };
        uint32_t cv[4][4];
        static_for<4>([&](auto v) {
            static_for<4>([&](auto j) { cv[v][j] = inside(v, j) ? a.C[offset(v, j)] : 0u; });
        });
        static_for<4>([&](auto v) {
            static_for<4>([&](auto j) {
                if (!inside(v, j)) return;
                const uint32_t r = uint32_t(reduce_f64(acc[i][j][int(v)], pd, a.pinv));
                const uint32_t add = a.sub ? (r ? a.p - r : 0u) : r;
                uint32_t c = cv[v][j] + add;
                if (c >= a.p) c -= a.p;
                a.C[offset(v, j)] = c;
            });
        });
    });
}

template <bool RED2>
hipError_t launch_f64(const PlainArgs &a, int64_t groups, hipStream_t s)
{
    static bool set = false;
    if (!set && hipFuncSetAttribute((const void *)k_gemm_f64<RED2>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    int(kLdsBytes)) != hipSuccess)
        return hipErrorInvalidValue;
    set = true;
    hipLaunchKernelGGL(k_gemm_f64<RED2>, dim3(unsigned(groups)), dim3(256), kLdsBytes, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_f64(const PlainArgs &a, hipStream_t s)
{
    const int64_t groups = a.grid_m * a.grid_n;
    if (groups <= 0) return hipSuccess;
    return a.red_steps < BK / 4 ? launch_f64<true>(a, groups, s) : launch_f64<false>(a, groups, s);
}

}  // namespace mh
