/*
 * mh.h -- Morton-hybrid modular matrix multiplication on AMD MI355X (gfx950).
 *
 * The operation (Abu Salem and Al Arab, "Cache-oblivious Matrix
 * Multiplication for Exact Factorisation", section 2): a product of
 * rectangular sub-matrices of Morton-hybrid parents over the prime field
 * F_p, in accumulating form (section 2.2):
 *
 *     C[rc+i][cc+j] := (C[rc+i][cc+j] + sum_{l<k} A[ra+i][ca+l] * B[rb+l][cb+j]) mod p
 *
 * for 0 <= i < m, 0 <= j < n.  The paper names the output A and the factors
 * B, C; this library names the output C and the factors A (m x k) and
 * B (k x n).
 *
 * Morton-hybrid layout (section 1; section 2.2 Step 1; Prop. 2.5).  An
 * N x N parent, N = T * 2^q, is cut into T x T tiles.  Tiles are stored in
 * Z (Morton) order, quadrants NW, NE, SW, SE (row bit more significant);
 * each tile is T*T contiguous words in row-major order.  Entry (i,j) sits at
 *     z(i,j) = Z(i/T, j/T) * T^2 + (i mod T) * T + (j mod T),
 *     Z(I,J) = sum_b (2*I_b + J_b) * 4^b.
 * The index does not depend on N.  Supported T: 16, 32, 64, 128.
 *
 * Conventions for every call below.
 *  - Matrix pointers are device pointers to uint32 words owned by the
 *    caller.  Entries must be residues in [0,p); this is not checked.  The
 *    A and B parents of a product must be 16-byte aligned (hipMalloc gives
 *    256), C 4-byte aligned (else MH_E_INVALID).
 *  - Arguments are validated synchronously before anything is enqueued; a
 *    call that returns an error has no effect.
 *  - Device calls are asynchronous on the caller's `stream` (0 = the null
 *    stream) and return without synchronising.  Faults detected later are
 *    reported by mh_ctx_last_device_error.
 *  - A context is used by one host thread at a time.  It owns all device
 *    workspace (limb panels, task queues, captured graphs); nothing the
 *    library allocates is visible to the caller.
 *  - The products of one context are ordered among themselves even when
 *    they are issued on different streams: a product on another stream than
 *    the context's previous one first makes its stream wait (on the device,
 *    not the host) for that previous product, since both use the context's
 *    workspace.  Products on different contexts are independent.  When the
 *    workspace grows, the host waits for the context's own earlier work
 *    only, never for the whole device.
 *  - Workspace limit: a product whose operand panels would exceed the
 *    context's limit (mh_ctx_set_workspace_limit; by default 1/8 of the
 *    device memory) is run as consecutive sub-products over chunks of its
 *    depth, then of its output rows and columns, accumulated into C in
 *    turn; the result is the same.
 *  - No C++ exception crosses this interface.
 *  - Two environment variables override the limb form's choices, for
 *    tuning and testing: MH_LIMB_CFG=<index> forces a kernel configuration
 *    (ignored if it does not fit the limb count) and MH_LIMB_KBLOCK=<depth>
 *    (a multiple of 64) shortens the k-blocks between reductions below the
 *    int32 bound.  Both keep results exact.
 */
#ifndef MH_H
#define MH_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mh_ctx mh_ctx;

typedef enum {
    MH_OK = 0,
    MH_E_INVALID = 1,      /* null pointer, negative size, bad flag */
    MH_E_SHAPE = 2,        /* parent size N is not T * 2^q */
    MH_E_BOUNDS = 3,       /* a block reaches outside its parent */
    MH_E_MODULUS = 4,      /* p outside [2, 2^31 - 1] */
    MH_E_ALIAS = 5,        /* an output region overlaps an input region or another output */
    MH_E_UNSUPPORTED = 6,  /* T not in {16,32,64,128}, or a mode/size the build lacks */
    MH_E_NOMEM = 7,        /* device or pinned allocation failed */
    MH_E_DEVICE = 8        /* a HIP call failed */
} mh_status;

/* Flags of mh_classify_submatrix.  Scattered == !MH_CONTAINED. */
enum {
    MH_ALIGNED = 1u,   /* Def. "aligned" (section 2): starts at the first entry of a
                          T x T tile and is 2^a T x 2^b T (a, b >= 0) */
    MH_CONTAINED = 2u, /* Def. "contained" (section 2.1): lies inside one T x T tile */
    MH_QUADRANT = 4u   /* one of the blocks of the quadrant recursion of section 2.2
                          Step 1 (the parent or a quadrant of one): rows = cols = 2^a T
                          and row, col multiples of rows; its entries are the index
                          range [alpha, alpha + lambda) */
};

/* Arithmetic forms of the product (the low byte of `mode`).  All are exact;
 * they differ in speed and in the moduli they accept. */
enum {
    MH_MODE_AUTO = 0,      /* pick by shape */
    MH_MODE_PLAIN_U32 = 1, /* VALU kernel, 64-bit multiply-accumulate with carry word */
    MH_MODE_LIMB_I8 = 2,   /* residues split into signed 8-bit limbs; int8 MFMA with
                              int32 accumulators; mod-p reduction once per k-block */
    MH_MODE_FP64 = 3,      /* p < 2^26 only (else MH_E_MODULUS): centred residues as
                              doubles, FP64 MFMA, mod-p reduction deferred while every
                              partial sum stays an integer below 2^53 in magnitude */
    MH_MODE_PLAIN_ELEMENTWISE = 4 /* comparator, not a production form: the plain kernel
                              without the planner, every element of A, B and C addressed
                              by its own Morton-hybrid encoding where it lies (the
                              default algorithm of section 2.2 on scattered blocks,
                              problems P1 and P2 of section 2.1) */
};

/* Or-ed into `mode`: subtractive update C := (C - A.B) mod p, the Schur
 * complement step of an LU / TU elimination (the caller side of section 1's
 * TU recursion). */
#define MH_SUBTRACT 0x100

/* Kernel classes reported by mh_ctx_kernel_time. */
enum {
    MH_K_LAYOUT_FROM = 0,
    MH_K_LAYOUT_TO = 1,
    MH_K_PACK = 2,         /* operand packing of one product, A and B together
                              (limb split or u32 panel copy) */
    MH_K_GEMM_PLAIN = 3,
    MH_K_GEMM_LIMB = 4,
    MH_K_BATCHED = 5,      /* one batched graph: persistent pack + persistent GEMM */
    MH_K_GEMM_F64 = 6,     /* FP64-MFMA form (plain and elementwise forms: MH_K_GEMM_PLAIN) */
    MH_K_COUNT = 7
};

/* ---------------------------------------------------------------- context */

/* Create a context bound to HIP device `hip_device`.  *out is set on success.
 * Errors: MH_E_INVALID (out null), MH_E_DEVICE (no such device). */
mh_status mh_ctx_create(mh_ctx **out, int hip_device);

/* Synchronise the context's pending work, free its workspace and graphs. */
mh_status mh_ctx_destroy(mh_ctx *ctx);

/* Static text for a status code (never null). */
const char *mh_status_string(mh_status s);

/* First asynchronous HIP error seen by the context since the last call
 * (sticky until read, then cleared).  Queries the device without blocking. */
mh_status mh_ctx_last_device_error(mh_ctx *ctx);

/* Largest device workspace (bytes) one call of the context may hold for its
 * operand panels: products (and batches) that would need more are split into
 * sub-products that fit, as described above.  0 = no limit; otherwise at
 * least 1 MiB (else MH_E_INVALID).  A held workspace above a new limit is
 * released after the context's pending work (host wait on that work only). */
mh_status mh_ctx_set_workspace_limit(mh_ctx *ctx, uint64_t bytes);

/* The context's workspace limit (0 = none) and the bytes it holds now; either
 * pointer may be null. */
mh_status mh_ctx_workspace_info(mh_ctx *ctx, uint64_t *limit, uint64_t *held);

/* Enable (1) or disable (0) timing: when on, every library kernel launch is
 * bracketed by HIP events recorded on the stream it is launched on. */
mh_status mh_ctx_set_timing(mh_ctx *ctx, int enable);

/* Sum of the recorded durations (ms) and the number of launches of kernel
 * class `kernel` (MH_K_*) since the last reset.  Blocks until the recorded
 * events have completed.  reset != 0 clears the record afterwards. */
mh_status mh_ctx_kernel_time(mh_ctx *ctx, int kernel, double *total_ms, int64_t *launches,
                             int reset);

/* The individual durations (ms, in launch order) of kernel class `kernel`
 * since the last reset: at most `cap` are written to ms_out (host array),
 * *launches is set to the number recorded.  Blocks like mh_ctx_kernel_time;
 * does not reset. */
mh_status mh_ctx_kernel_times(mh_ctx *ctx, int kernel, double *ms_out, int64_t cap,
                              int64_t *launches);

/* ------------------------------------------------------------ diagnostics */

/* Sustained int8 MFMA rate of the context's device, the ceiling a dense
 * int8 kernel can approach there: one workgroup of four waves per compute
 * unit keeps eight independent 32x32 accumulators busy with
 * v_mfma_i32_32x32x32_i8 on random register operands, rotated from one
 * MFMA to the next, with no memory traffic in the loop; each wave issues
 * 8 * iters MFMAs.  One untimed launch of the same size runs first (the
 * clock settles under the load), then the timed one, bracketed by HIP
 * events on `stream`.  *pops receives int8 operations per second
 * (2 x 32^3 per MFMA).  The published peak assumes the full engine clock;
 * under this load the device may lower its clock to stay within its power
 * limit, which this figure includes.  Synchronises `stream`; allocates and
 * frees a small device buffer.
 * Errors: MH_E_INVALID (ctx or pops null; iters odd, below 2 or above
 * 2^24), MH_E_NOMEM, MH_E_DEVICE. */
mh_status mh_probe_mfma_i8(mh_ctx *ctx, int32_t iters, double *pops, hipStream_t stream);

/* Sustained issue rate of the plain form's 96-bit multiply-accumulate (the
 * v_mad_u64_u32 + v_addc_co_u32 pair of the plain kernel, one shared
 * helper): eight workgroups of 256 threads per compute unit, sixteen
 * independent accumulators per lane, `iters` rounds each, no memory traffic
 * in the loop; one untimed launch, then the timed one (HIP events on
 * `stream`).  *macs receives multiply-accumulates per second: the ceiling
 * the plain kernel's VALU-bound loop can approach.  Synchronises `stream`;
 * allocates and frees a small device buffer.
 * Errors: MH_E_INVALID (ctx or macs null; iters below 1 or above 2^24),
 * MH_E_NOMEM, MH_E_DEVICE. */
mh_status mh_probe_valu_mac(mh_ctx *ctx, int32_t iters, double *macs, hipStream_t stream);

/* Autotuning of the limb kernels' configuration (workgroup and wave tile,
 * pipeline depth, LDS sharing) per shape bucket: single products by limbs,
 * T and ceil(log2) of m, k, n; batches by limbs, T and ceil(log2) of their
 * mean output area and mean k.  mode 0: built-in defaults; 1: use choices
 * already in the context's cache; 2: as 1, and time every configuration on
 * the first call of an uncached bucket (on the caller's operands, writing a
 * scratch output, so C is unaffected; that call synchronises `stream`).
 * Tuning runs the product once per configuration, so it should be enabled
 * for representative calls, not for one-off products. */
mh_status mh_ctx_set_autotune(mh_ctx *ctx, int mode);

/* Configuration (MH_* kernel table index) cached for the single-product
 * bucket of (p, T, m, k, n), or -1 in *cfg if none. */
mh_status mh_ctx_tune_lookup(mh_ctx *ctx, uint32_t p, int32_t T, int64_t m, int64_t k,
                             int64_t n, int32_t *cfg);

/* Write the context's cache to a JSON file (tagged with the device name,
 * CU count and HIP runtime version); replace it atomically. */
mh_status mh_ctx_tune_cache_save(mh_ctx *ctx, const char *path);

/* Merge the entries of a file written by mh_ctx_tune_cache_save for the same
 * device tag into the context's cache; *loaded (may be null) is set to the
 * number of entries taken.  MH_E_INVALID if the file cannot be read. */
mh_status mh_ctx_tune_cache_load(mh_ctx *ctx, const char *path, int32_t *loaded);

/* ------------------------------------------------------ host index math */

/* Morton-hybrid index of Cartesian (i,j) for tile edge T (a power of two);
 * i, j < 2^31.  The paper's encode (section 2.2 Step 2). */
uint64_t mh_encode(uint64_t i, uint64_t j, uint32_t T);

/* Inverse of mh_encode: the paper's extract_i and extract_j. */
void mh_extract(uint64_t z, uint32_t T, uint64_t *i, uint64_t *j);

/* Flags (MH_ALIGNED | MH_CONTAINED | MH_QUADRANT) of the rows x cols block
 * whose first entry is (row, col) in an N x N parent with tile edge T.
 * O(1), host only.  Errors: MH_E_UNSUPPORTED (T), MH_E_SHAPE (N),
 * MH_E_INVALID (rows or cols < 1, flags_out null), MH_E_BOUNDS. */
mh_status mh_classify_submatrix(int64_t N, int32_t T, int64_t row, int64_t col, int64_t rows,
                                int64_t cols, uint32_t *flags_out);

/* ---------------------------------------------------------------- layout */

/* dst_mh (N*N words, Morton-hybrid) <- src (Cartesian row-major, row length
 * ld_src >= N).  Both device pointers; they must not overlap. */
mh_status mh_layout_from_cartesian(mh_ctx *ctx, uint32_t *dst_mh, const uint32_t *src,
                                   int64_t ld_src, int64_t N, int32_t T, hipStream_t stream);

/* dst (Cartesian row-major, row length ld_dst >= N) <- src_mh (N*N words). */
mh_status mh_layout_to_cartesian(mh_ctx *ctx, uint32_t *dst, int64_t ld_dst,
                                 const uint32_t *src_mh, int64_t N, int32_t T,
                                 hipStream_t stream);

/* Rectangular or non-power-of-two matrices (the caller side of the TU
 * recursion, section 1, whose matrices have any shape): they are embedded in
 * the top-left corner of the smallest Morton-hybrid parent, zero padded.
 * mh_parent_size: *N = the smallest T * 2^q >= max(rows, cols), host only;
 * MH_E_INVALID (rows or cols < 1, N null), MH_E_UNSUPPORTED (T, or N above
 * 2^18). */
mh_status mh_parent_size(int64_t rows, int64_t cols, int32_t T, int64_t *N);

/* dst_mh (N*N words) <- the rows x cols Cartesian matrix src (row length
 * ld_src >= cols) in its top-left corner, zeros elsewhere.  rows, cols <= N.
 * Device pointers that must not overlap.  Errors as mh_layout_from_cartesian,
 * MH_E_INVALID for rows or cols outside [1, N]. */
mh_status mh_layout_from_cartesian_padded(mh_ctx *ctx, uint32_t *dst_mh, int64_t N,
                                          const uint32_t *src, int64_t ld_src, int64_t rows,
                                          int64_t cols, int32_t T, hipStream_t stream);

/* The rows x cols top-left corner of src_mh (N*N words) -> dst (row length
 * ld_dst >= cols); words of dst outside rows x cols are not written. */
mh_status mh_layout_to_cartesian_padded(mh_ctx *ctx, uint32_t *dst, int64_t ld_dst,
                                        int64_t rows, int64_t cols, const uint32_t *src_mh,
                                        int64_t N, int32_t T, hipStream_t stream);

/* --------------------------------------------------------------- product */

/*
 * C[rc:rc+m, cc:cc+n] := (C + A[ra:ra+m, ca:ca+k] . B[rb:rb+k, cb:cb+n]) mod p
 * on Morton-hybrid parents C (NC x NC), A (NA x NA), B (NB x NB), all with
 * tile edge T.  Blocks may be aligned, contained or scattered.  k = 0 leaves
 * C unchanged; m = 0 or n = 0 is a no-op.  A, B and C may be the same
 * buffer provided the C block overlaps neither the A nor the B block (the
 * Schur update of a TU step writes one block of a matrix from two others).
 * The result is canonical (in [0,p)) and identical for every mode.
 * Errors: MH_E_INVALID, MH_E_SHAPE, MH_E_BOUNDS, MH_E_MODULUS (p outside
 * [2, 2^31-1], or p >= 2^26 with MH_MODE_FP64), MH_E_ALIAS, MH_E_UNSUPPORTED
 * (bits of mode other than a form and MH_SUBTRACT), MH_E_NOMEM.
 */
mh_status mh_matmul_modp(mh_ctx *ctx, uint32_t *C, int64_t NC, int64_t rc, int64_t cc,
                         const uint32_t *A, int64_t NA, int64_t ra, int64_t ca,
                         const uint32_t *B, int64_t NB, int64_t rb, int64_t cb, int64_t m,
                         int64_t k, int64_t n, uint32_t p, int32_t T, int32_t mode,
                         hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product, arguments, result and errors as mh_matmul_modp, but the operand
 * panels live in a fixed 128 MiB device array of the library (one per GPU,
 * held until the process ends) instead of the context's workspace, and the
 * call makes no device allocation of any kind (no hipMalloc or hipFree, no
 * autotuning runs -- configurations already in the context's tuning cache
 * are used -- and no timing events even with timing on).  A product whose
 * panels exceed 128 MiB runs as consecutive sub-products over chunks of its
 * depth, then of its output rows and columns, each within the array; should
 * even the smallest chunk not fit, the call returns MH_E_NOMEM before
 * anything is enqueued for it.  The array's contents are left from the last
 * call and never relied on (packing writes every panel byte it reads).
 * Calls through one context are ordered as the context's other calls are;
 * calls through different contexts (or host threads) on the same GPU share
 * the one array and race if they may overlap on the device: the caller
 * must order them (one stream, or events).  MH_E_DEVICE if the array's
 * device address could not be obtained when the context was created.
 */
mh_status mh_matmul_modp_noalloc(mh_ctx *ctx, uint32_t *C, int64_t NC, int64_t rc, int64_t cc,
                                 const uint32_t *A, int64_t NA, int64_t ra, int64_t ca,
                                 const uint32_t *B, int64_t NB, int64_t rb, int64_t cb,
                                 int64_t m, int64_t k, int64_t n, uint32_t p, int32_t T,
                                 int32_t mode, hipStream_t stream);

/* One independent product of a batch (same meaning as mh_matmul_modp). */
typedef struct {
    uint32_t *C;
    const uint32_t *A, *B;
    int64_t NC, NA, NB;
    int64_t rc, cc, ra, ca, rb, cb;
    int64_t m, k, n;
} mh_mm_desc;

/*
 * `count` independent products sharing p and T, run as one persistent
 * launch over a device task queue (section 2.2, Prop. 2.6: the calls of one
 * recursion level are independent).  descs is a host array.  No C block may
 * overlap another C block or any A or B block of the batch (MH_E_ALIAS); A
 * and B blocks may be shared.  The launch sequence (counter reset,
 * persistent packing kernels for the A and the B blocks, persistent GEMM
 * kernel, whose workgroups serve the products of their own XCD's group
 * first) is captured once into a HIP graph per context and replayed; only
 * the queue contents change between calls, through one host-to-device copy
 * on `stream`; a graph is kept per kernel configuration and limb count, so
 * batches of different shapes or moduli do not re-capture each other's.  Like
 * every product of the context, a batch is ordered after the context's
 * previous call, also across streams.  Products whose panels together exceed
 * the workspace limit go out as several consecutive graphs.  mode:
 * MH_MODE_AUTO and MH_MODE_LIMB_I8 run the limb form; the other forms run the
 * products one after another with their own kernels.
 */
mh_status mh_matmul_modp_batched(mh_ctx *ctx, const mh_mm_desc *descs, int32_t count,
                                 uint32_t p, int32_t T, int32_t mode, hipStream_t stream);

/* The checks of mh_matmul_modp_batched without the product, host only: each
 * product's sizes, bounds, modulus and form as for mh_matmul_modp (pointers
 * must be non-null and aligned but are never dereferenced), and no output
 * block sharing a word with another output block or any input block of the
 * batch (section 2.2, Prop. 2.6: the independent calls of one recursion
 * level write disjoint blocks).  Returns what mh_matmul_modp_batched would
 * return before any device work: MH_OK, MH_E_INVALID, MH_E_SHAPE,
 * MH_E_BOUNDS, MH_E_MODULUS, MH_E_ALIAS or MH_E_UNSUPPORTED.  The aliasing
 * check sorts the blocks of each parent by first row and sweeps them, so a
 * batch of n products costs O(n log n) plus the pairs whose rows overlap. */
mh_status mh_validate_batch(const mh_mm_desc *descs, int32_t count, uint32_t p, int32_t T,
                            int32_t mode);

/* Kernel configuration (index into the limb kernel table, as reported by
 * mh_plan_info.kernel_cfg), limb count and GEMM forms of the last batched
 * graph the context launched for a caller (tuning runs excluded); -1, 0 and
 * 0 if none.  forms: MH_BATCH_FORM_EARLY_C if the GEMM loaded C ahead of its
 * epilogue, MH_BATCH_FORM_A_PARENT if it read A from panels of whole
 * parents (each A parent packed once for the batch).  Any pointer may be
 * null. */
#define MH_BATCH_FORM_EARLY_C 1
#define MH_BATCH_FORM_A_PARENT 2
mh_status mh_ctx_last_batch_config(mh_ctx *ctx, int32_t *cfg, int32_t *limbs, int32_t *forms);

/* ------------------------------------------------------ planner, host only */

/* What the planner makes of one product (no device work, no validation of
 * pointers; sizes and bounds are validated as for mh_matmul_modp). */
typedef struct {
    int64_t row_segments;   /* segments of [0,m) cut by C's and A's tile rows */
    int64_t inner_segments; /* segments of [0,k) cut by A's tile columns and B's tile rows */
    int64_t col_segments;   /* segments of [0,n) cut by C's and B's tile columns */
    int64_t leaves;         /* base cases of the section 2.2 recursion: the product of the three */
    int64_t c_tiles;        /* C tiles the output block touches (each written by one task) */
    int64_t gemm_tasks;     /* output blocks handed to workgroups */
    int64_t pack_chunks;    /* operand chunks handed to the packing kernel (0 if none) */
    int32_t mode;           /* mode the call would run in */
    int32_t in_place;       /* 1 if the plain kernel reads A and B tiles in place */
    int32_t tile_m, tile_n; /* output block of one workgroup */
    int32_t limbs;          /* limbs per residue (limb mode) */
    int32_t kblock;         /* depth between reductions mod p (limb and FP64 forms) */
    int32_t kernel_cfg;     /* limb GEMM configuration the call would launch (-1: none) */
} mh_plan_info;

mh_status mh_plan_describe(int64_t NC, int64_t rc, int64_t cc, int64_t NA, int64_t ra,
                           int64_t ca, int64_t NB, int64_t rb, int64_t cb, int64_t m,
                           int64_t k, int64_t n, uint32_t p, int32_t T, int32_t mode,
                           mh_plan_info *out);

/*
 * The leaves themselves: box q is out[6q..6q+5] = (i0, ni, l0, nl, j0, nj)
 * in product coordinates; C piece rows [i0,i0+ni) x cols [j0,j0+nj), A piece
 * [i0..) x [l0..), B piece [l0..) x [j0..).  Every piece lies in one tile.
 * Writes at most `cap` boxes and sets *count to the total.
 */
mh_status mh_plan_leaves(int64_t NC, int64_t rc, int64_t cc, int64_t NA, int64_t ra,
                         int64_t ca, int64_t NB, int64_t rb, int64_t cb, int64_t m, int64_t k,
                         int64_t n, int32_t T, int64_t *out, int64_t cap, int64_t *count);

/*
 * The output blocks of the workgroups: task q is out[4q..4q+3] =
 * (i0, ni, j0, nj) in product coordinates.  They partition [0,m) x [0,n)
 * and each lies inside C tiles it writes whole (clipped to the block).
 */
mh_status mh_plan_gemm_tasks(int64_t NC, int64_t rc, int64_t cc, int64_t NA, int64_t ra,
                             int64_t ca, int64_t NB, int64_t rb, int64_t cb, int64_t m,
                             int64_t k, int64_t n, uint32_t p, int32_t T, int32_t mode,
                             int64_t *out, int64_t cap, int64_t *count);

#ifdef __cplusplus
}
#endif

#endif /* MH_H */
