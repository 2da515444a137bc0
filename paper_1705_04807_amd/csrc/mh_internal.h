// Internal declarations shared by the host runtime and the HIP kernels of
// libmh.  Not part of the public interface (include/mh.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <string>
#include <vector>

#include "mh.h"

namespace mh {

// ------------------------------------------------------------- index math
//
// Morton-hybrid index (section 1; section 2.2 Step 1 quadrant order NW, NE,
// SW, SE; Prop. 2.5 row-major tiles):
//   z(i,j) = Z(i>>logT, j>>logT) << 2logT | (i & (T-1)) << logT | (j & (T-1))
// where Z interleaves the tile coordinates, row bit above column bit.  The
// interleave uses dilated integers (bit spreading by masks), so an index
// costs a constant number of word operations (Prop. 2.6 on work).

__host__ __device__ __forceinline__ uint64_t spread32(uint64_t x)
{
    x &= 0xFFFFFFFFull;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

__host__ __device__ __forceinline__ uint64_t compact32(uint64_t x)
{
    x &= 0x5555555555555555ull;
    x = (x | (x >> 1)) & 0x3333333333333333ull;
    x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
    x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
    x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
    return x;
}

// 32-bit spread for tile coordinates below 2^16 (device hot paths).
__host__ __device__ __forceinline__ uint32_t spread16(uint32_t x)
{
    x &= 0xFFFFu;
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

__host__ __device__ __forceinline__ uint32_t compact16(uint32_t x)
{
    x &= 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0F0F0F0Fu;
    x = (x | (x >> 4)) & 0x00FF00FFu;
    x = (x | (x >> 8)) & 0x0000FFFFu;
    return x;
}

// Z index of tile (I, J): row bit more significant.
__host__ __device__ __forceinline__ uint64_t tile_z(uint64_t I, uint64_t J)
{
    return (spread32(I) << 1) | spread32(J);
}

__host__ __device__ __forceinline__ uint64_t mh_offset(uint64_t i, uint64_t j, int logT)
{
    const uint64_t m = (1ull << logT) - 1;
    return (tile_z(i >> logT, j >> logT) << (2 * logT)) | ((i & m) << logT) | (j & m);
}

constexpr int64_t kMaxN = int64_t(1) << 18;  // largest parent edge accepted

// ------------------------------------------------------- limb arithmetic
//
// A residue x in [0,p) is centred, x' = x if x <= H_L else x - p with
// H_L = 127 (256^L - 1) / 255, and written as x' = sum_t d_t 256^t with
// every d_t in [-128, 127] (balanced base-256 digits).  L digits cover the
// window [-128 (256^L-1)/255, H_L] of 256^L integers, which holds every
// centred residue exactly when p <= 256^L.
inline int limbs_for(uint32_t p)
{
    if (p <= 256u) return 1;
    if (p <= 65536u) return 2;
    if (p <= (1u << 24)) return 3;
    return 4;
}

__host__ __device__ inline int64_t limb_threshold(int L)
{
    int64_t h = 0, w = 1;
    for (int t = 0; t < L; ++t) { h += 127 * w; w *= 256; }
    return h;
}

// Longest k-block (multiple of 64, two MFMA depths) whose shift accumulators
// T_s = sum_{t+u=s} A_t B_u cannot leave int32: |d_t d_u| <= 2^14 and at most
// L digit pairs meet in one shift, so |T_s| <= kappa * L * 2^14 < 2^31.
inline int kblock_for(int L)
{
    int64_t kap = ((int64_t(1) << 31) - 1) / (int64_t(L) << 14);
    return int(kap / 64 * 64);
}

// ------------------------------------------------------------- geometry
//
// Product coordinates: i in [0,m) (rows of C and A), l in [0,k) (inner),
// j in [0,n) (columns of C and B).  The GEMM kernels work on "panel"
// coordinates shifted so that panel row 0 and panel column 0 fall on a C
// tile boundary: panel row rho = i + sr with sr = rc mod T, panel column
// gamma = j + sc with sc = cc mod T.  Then every workgroup's output block
// (tile_m x tile_n, aligned in panel coordinates) covers whole C tiles or
// lies inside one, and its writes stay inside C tiles (contained).

struct Product {
    uint32_t *C;
    const uint32_t *A, *B;
    int64_t NC, rc, cc, NA, ra, ca, NB, rb, cb, m, k, n;
    uint32_t p;
    int32_t T, logT;
};

// Launch parameters of the limb GEMM family (one template instance each).
struct LimbKernelCfg {
    int id;
    int wm, wn;          // 32x32 MFMA tiles per wave (rows, cols)
    int waves_m, waves_n;
    int ks;              // 32-deep k-blocks per pipeline stage
    int lds;             // 1: stages shared through LDS by the workgroup's waves
    int nbuf = 2;        // stage buffers (LDS, or register sets)
    int lmax = 4;        // largest limb count built for this configuration
    int tile_m() const { return 32 * wm * waves_m; }
    int tile_n() const { return 32 * wn * waves_n; }
};

// Device-side description of one packed operand panel.
//   Limb panel: 32-row slabs x 32-deep k-blocks x L limbs, 1 KiB each, in the
//   lane order of the MFMA operand: lane q holds row (q mod 32), depth
//   (q div 32)*16 .. +15 of the block.  Address of (slab, kb, limb):
//   base + ((slab * nkb + kb) * L + limb) * 1024.
struct PanelDesc {
    int8_t *base;
    int64_t rows;  // padded panel rows (multiple of the workgroup tile)
    int64_t nkb;   // k-blocks of 32
};

struct Plan {
    Product pr;
    int mode;
    int L;
    int kblock;
    int64_t sr, sc;          // panel shifts (see above)
    int64_t row0C, col0C;    // C coordinates of panel (0,0)
    int64_t prow, pcol;      // padded panel extent (multiple of tile_m / tile_n)
    int64_t kpad;            // padded k
    int tile_m, tile_n;
    int64_t grid_m, grid_n;  // workgroup tiles
    bool in_place;           // plain mode reads A and B tiles in the parents
    int64_t sk;              // plain in-place: k shift (ca mod T)
    int limb_cfg;            // index into the limb kernel table
    bool sub;                // C := C - A.B (B is negated while packing)
};

// ------------------------------------------------------ host prototypes

bool valid_T(int32_t T);
int log2i(int64_t x);
mh_status check_parent(int64_t N, int32_t T);
mh_status validate_product(const Product &p, bool need_ptrs);
void plan_product(const Product &p, int mode, Plan &out, int forced_cfg = -1);

// mode argument of the ABI: arithmetic form in the low byte, MH_SUBTRACT flag.
inline bool parse_mode(int32_t mode, int &form, bool &sub)
{
    form = mode & 0xFF;
    sub = (mode & MH_SUBTRACT) != 0;
    return (mode & ~(0xFF | MH_SUBTRACT)) == 0 && form >= MH_MODE_AUTO && form <= MH_MODE_PLAIN_ELEMENTWISE;
}
void segments(int64_t len, int64_t offA, int64_t offB, int32_t T, std::vector<int64_t> &cuts);

// limb kernel table
int limb_cfg_count();
const LimbKernelCfg &limb_cfg(int idx);
bool limb_cfg_fits(int L, int idx);  // accumulators fit and the instance is built for L
int limb_cfg_default(int L, int64_t m, int64_t n, int64_t k);

// ------------------------------------------------------ kernel launchers
// All return hipSuccess or the launch error; they do not synchronise.

// rows x cols Cartesian words <-> N x N Morton-hybrid parent (zero padded).
hipError_t launch_layout_from(uint32_t *dst, const uint32_t *src, int64_t ld, int64_t rows,
                              int64_t cols, int64_t N, int logT, hipStream_t s);
hipError_t launch_layout_to(uint32_t *dst, int64_t ld, int64_t rows, int64_t cols,
                            const uint32_t *src, int64_t N, int logT, hipStream_t s);

// u32 tile panel for the plain kernel: view rows x cols of T x T tiles,
// tile-major.  Source element of panel (r, c): trans ? (o0 + c, i0 + r)
// : (o0 + r, i0 + c) ... see mh_pack.hip.
hipError_t launch_pack_u32(uint32_t *dst, int64_t prow, int64_t pcol, const uint32_t *src,
                           int64_t srow0, int64_t scol0, int64_t vr0, int64_t vr1,
                           int64_t vc0, int64_t vc1, int logT, hipStream_t s);

// Limb panel (see PanelDesc).  For operand A (trans = 0) panel row rho and
// depth kap read source (r0 + rho - shift, c0 + kap); for B (trans = 1)
// source (r0 + kap, c0 + rho - shift).  Entries outside rows [shift,
// shift+R) or depths [0,K) are zero.
hipError_t launch_pack_limb(int8_t *dst, int64_t prow, int64_t nkb, const uint32_t *src,
                            int64_t r0, int64_t c0, int64_t shift, int64_t R, int64_t K,
                            int trans, int neg, int logT, uint32_t p, int L, hipStream_t s);

struct PlainArgs {
    const uint32_t *A;   // MH parent (in place) or tile-major panel
    const uint32_t *B;
    uint32_t *C;
    int a_mh, b_mh;      // 1: MH parent; 0: panel; 2: MH parent, view at any element
    int64_t a_tr0, a_tc0, a_ntc;  // A view origin in tiles (MH) / tile columns (panel)
    int64_t b_tr0, b_tc0, b_ntc;
    int64_t sr, sc, sk;  // valid panel rows [sr, sr+m), cols [sc, sc+n), depth [sk, sk+k)
    int64_t m, n, k, kpad;
    int64_t row0C, col0C;
    int64_t grid_m, grid_n;
    uint32_t p;
    uint64_t mu;         // floor((2^64 - 1) / p)
    int logT;
    int sub;             // C := C - A.B
    int red_steps;       // FP64 form: MFMA steps (depth 4) between reductions mod p
    double pinv;         // FP64 form: 1.0 / p rounded to nearest
};
hipError_t launch_gemm_plain(const PlainArgs &a, hipStream_t s);
hipError_t launch_gemm_f64(const PlainArgs &a, hipStream_t s);

// FP64 form: largest p accepted, and the MFMA steps of depth 4 between
// reductions so that |partial sum| <= (p - 1) + 4 steps H^2 <= 2^53 with
// H = max |centred residue|.
constexpr uint32_t kF64MaxP = (1u << 26) - 1;
inline int f64_red_steps(uint32_t p)
{
    const double H = p == 2u ? 1.0 : double((p - 1) / 2);
    const double steps = std::floor((9007199254740992.0 - double(p)) / (4.0 * H * H));
    return steps > double(1 << 30) ? (1 << 30) : int(steps);
}
inline mh_status check_form_modulus(int form, uint32_t p)
{
    return (form == MH_MODE_FP64 && p > kF64MaxP) ? MH_E_MODULUS : MH_OK;
}

struct LimbArgs {
    const int8_t *Ap, *Bp;
    int64_t nkb;         // k-blocks of 32 in the panels
    int kb_per_red;      // k-blocks between reductions mod p
    uint32_t *C;
    int64_t row0C, col0C, sr, sc, m, n;
    int64_t grid_m, grid_n;
    uint32_t p;
    uint64_t mu;         // floor((2^64 - 1) / p)
    uint64_t bias;       // multiple of p, >= 2^31
    double pinv;         // 1.0 / p rounded to nearest
    int logT;
    // Batched form with A read from a whole-parent limb panel (Ap: its slab
    // 0, with kAParentGuard slabs after the parent's): panel row 0 of the
    // product is the parent's row 32 a_slab0, its k-block 0 the parent's
    // k-block a_kb0; a slab holds a_nkbp k-blocks.
    int64_t a_slab0, a_kb0, a_nkbp;
};
hipError_t launch_gemm_limb(int cfg, int L, const LimbArgs &a, hipStream_t s);
// Guard slabs after a whole-parent A panel: a product's panel rows end at
// most 128 rows after the parent's, and its last k-block reaches at most one
// k-block into the following slab.
constexpr int64_t kAParentGuard = 6;

// ------------------------------------------------------------ batch queue
//
// Device-resident description of a batch of products, laid out in one
// buffer with room for `cap` products: a header, one PackTask per operand
// panel (A then B of each product), their chunk prefix sums, one LimbArgs
// per product (in launch order: largest k first) and their output-block
// prefix sums.

struct PackTask {
    const uint32_t *src;
    int8_t *dst;
    int64_t r0, c0, shift, R, K, prow, nkb;
    int32_t trans, logT;
    int32_t neg;        // pack (p - x) mod p
    int32_t kshift;     // (trans only) depth kap holds source row r0 + kap - kshift
};

// Output blocks of a batch are split into kXcdGroups groups of whole
// products, one per XCD of the device (a persistent workgroup pops its
// XCD's group first, so the group's operand panels stay in that XCD's L2).
constexpr int kXcdGroups = 8;

struct BatchHeader {
    int64_t npack, ncalls, pack_chunks, gemm_tiles;
    uint32_t p;
    int32_t L;
    int64_t group_tile[kXcdGroups + 1];  // group g: output blocks [group_tile[g], group_tile[g+1])
    int64_t group_call[kXcdGroups];      // first product of group g (queue order)
    int64_t pad[1];
};

struct QueueView {
    BatchHeader *hdr;
    PackTask *packs;        // [2 cap]
    int64_t *pack_prefix;   // [2 cap + 1]
    LimbArgs *calls;        // [cap]
    int64_t *tile_prefix;   // [cap + 1]
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline size_t queue_bytes(int64_t cap)
{
    return align256(sizeof(BatchHeader)) + align256(sizeof(PackTask) * 2 * cap) +
           align256(sizeof(int64_t) * (2 * cap + 1)) + align256(sizeof(LimbArgs) * cap) +
           align256(sizeof(int64_t) * (cap + 1));
}

inline QueueView queue_view(void *base, int64_t cap)
{
    char *b = (char *)base;
    QueueView q;
    q.hdr = (BatchHeader *)b;
    b += align256(sizeof(BatchHeader));
    q.packs = (PackTask *)b;
    b += align256(sizeof(PackTask) * 2 * cap);
    q.pack_prefix = (int64_t *)b;
    b += align256(sizeof(int64_t) * (2 * cap + 1));
    q.calls = (LimbArgs *)b;
    b += align256(sizeof(LimbArgs) * cap);
    q.tile_prefix = (int64_t *)b;
    return q;
}

// Work counters of one batched graph: A packing, B packing, then one GEMM
// counter per XCD group.
constexpr int kBatchCounters = 2 + kXcdGroups;
hipError_t launch_pack_limb_batched(int L, const QueueView &q, uint64_t *counters, int num_cu,
                                    hipStream_t s);
// early_c: the form that loads C ahead of the epilogue (valid when
// limb_batched_early_c(logT, largest C parent) holds); a_parent: the form
// that reads A from whole-parent panels (configurations for which
// limb_batched_a_parent(cfg, L) holds, with early_c, and panel rows that
// start on a 32-row slab of the A parent).
bool limb_batched_early_c(int logT, int64_t max_nc);
bool limb_batched_a_parent(int cfg, int L);
hipError_t launch_gemm_limb_batched(int cfg, int L, bool early_c, bool a_parent,
                                    const QueueView &q, uint64_t *counters, int num_cu,
                                    hipStream_t s);
hipError_t launch_reset_counters(uint64_t *counters, hipStream_t s);

}  // namespace mh
