// Host runtime of libmh: context, validation, index math, classification,
// planner and dispatch of the single-product path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "mh_ctx.h"
#include "mh_internal.h"

using namespace mh;

// ================================================================ statuses

extern "C" const char *mh_status_string(mh_status s)
{
    // A C caller may pass any int: read the argument's bits as one, since
    // loading an enum value outside the enumerators' range is undefined in C++.
    int v;
    std::memcpy(&v, &s, sizeof v);
    switch (v) {
    case MH_OK: return "ok";
    case MH_E_INVALID: return "invalid argument";
    case MH_E_SHAPE: return "parent size is not T * 2^q";
    case MH_E_BOUNDS: return "block outside its parent";
    case MH_E_MODULUS: return "modulus outside [2, 2^31-1]";
    case MH_E_ALIAS: return "output region overlaps an input or another output";
    case MH_E_UNSUPPORTED: return "unsupported tile edge, mode or size";
    case MH_E_NOMEM: return "out of device or pinned memory";
    case MH_E_DEVICE: return "HIP call failed";
    }
    return "unknown status";
}

// ================================================================ context

namespace mh {

DeviceGuard::DeviceGuard(int dev)
{
    prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
}
DeviceGuard::~DeviceGuard()
{
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
}

mh_status note_error(mh_ctx *ctx, hipError_t e)
{
    if (e == hipSuccess) return MH_OK;
    if (e == hipErrorOutOfMemory) return MH_E_NOMEM;
    if (ctx && ctx->sticky == MH_OK) ctx->sticky = MH_E_DEVICE;
    return MH_E_DEVICE;
}

hipEvent_t take_event(mh_ctx *ctx)
{
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void record_start(mh_ctx *ctx, int kernel, hipStream_t s, TimedLaunch &t)
{
    t.kernel = kernel;
    t.a = t.b = nullptr;
    if (!ctx->timing || ctx->no_timing) return;
    t.a = take_event(ctx);
    t.b = take_event(ctx);
    if (t.a) (void)hipEventRecord(t.a, s);
}

void record_end(mh_ctx *ctx, hipStream_t s, TimedLaunch &t)
{
    if (!ctx->timing || ctx->no_timing || !t.a || !t.b) return;
    (void)hipEventRecord(t.b, s);
    ctx->records.push_back(t);
}

void use_begin(mh_ctx *ctx, hipStream_t s)
{
    if (ctx->used && ctx->last_use && ctx->last_stream != s)
        (void)hipStreamWaitEvent(s, ctx->last_use, 0);
    ctx->in_call = true;
    ctx->cur_stream = s;
}

void use_end(mh_ctx *ctx, hipStream_t s)
{
    ctx->in_call = false;
    if (ctx->last_use && hipEventRecord(ctx->last_use, s) == hipSuccess) {
        ctx->last_stream = s;
        ctx->used = true;
    }
}

// Inside a call, the work this call has already enqueued counts too: the
// event is recorded on the call's stream first (which waited for the
// previous call in use_begin), so the wait covers both.
mh_status drain(mh_ctx *ctx)
{
    if (!ctx->last_use) return MH_OK;
    if (ctx->in_call && hipEventRecord(ctx->last_use, ctx->cur_stream) == hipSuccess) {
        ctx->last_stream = ctx->cur_stream;
        ctx->used = true;
    }
    if (!ctx->used) return MH_OK;
    return note_error(ctx, hipEventSynchronize(ctx->last_use));
}

// Device workspace owned by the context, grown on demand.  Growing waits
// for the context's earlier work (the old block may still be in use by it);
// the caller's current call has enqueued nothing into the old block yet.
void *workspace(mh_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->ws_size) return ctx->ws;
    if (ctx->ws) {
        (void)drain(ctx);
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_size = 0;
    }
    size_t want = bytes + bytes / 8 + (size_t(1) << 20);
    want = (want + 0xFFFFF) & ~size_t(0xFFFFF);
    if (ctx->ws_limit && want > ctx->ws_limit) want = std::max(bytes, ctx->ws_limit);
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    ctx->ws = p;
    ctx->ws_size = want;
    return p;
}

char *ws_get(mh_ctx *ctx, const WsSource &src, size_t bytes)
{
    if (src.fixed) return bytes <= src.cap ? src.fixed : nullptr;
    return (char *)workspace(ctx, bytes);
}

}  // namespace mh

extern "C" mh_status mh_ctx_create(mh_ctx **out, int hip_device)
{
    if (!out) return MH_E_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) {
        (void)hipGetLastError();
        return MH_E_DEVICE;
    }
    mh_ctx *c = new (std::nothrow) mh_ctx();
    if (!c) return MH_E_NOMEM;
    c->device = hip_device;
    DeviceGuard g(hip_device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess) {
        c->num_cu = prop.multiProcessorCount;
        c->ws_limit = prop.totalGlobalMem / 8;  // default workspace limit
    }
    if (hipEventCreateWithFlags(&c->last_use, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return MH_E_DEVICE;
    }
    // the no-allocation entry point's panel scratch on this device
    c->noalloc_ws = noalloc_scratch_init(hip_device);
    *out = c;
    return MH_OK;
}

extern "C" mh_status mh_ctx_destroy(mh_ctx *ctx)
{
    if (!ctx) return MH_E_INVALID;
    {
        DeviceGuard g(ctx->device);
        (void)drain(ctx);
        for (auto &r : ctx->records) {
            if (r.b) (void)hipEventSynchronize(r.b);
            if (r.a) (void)hipEventDestroy(r.a);
            if (r.b) (void)hipEventDestroy(r.b);
        }
        for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
        batched_release(ctx);
        if (ctx->ws) (void)hipFree(ctx->ws);
        if (ctx->tune_scratch) (void)hipFree(ctx->tune_scratch);
        if (ctx->last_use) (void)hipEventDestroy(ctx->last_use);
    }
    delete ctx;
    return MH_OK;
}

extern "C" mh_status mh_ctx_last_device_error(mh_ctx *ctx)
{
    if (!ctx) return MH_E_INVALID;
    DeviceGuard g(ctx->device);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess && ctx->sticky == MH_OK) ctx->sticky = MH_E_DEVICE;
    mh_status s = ctx->sticky;
    ctx->sticky = MH_OK;
    return s;
}

extern "C" mh_status mh_ctx_set_workspace_limit(mh_ctx *ctx, uint64_t bytes)
{
    if (!ctx) return MH_E_INVALID;
    if (bytes != 0 && bytes < (uint64_t(1) << 20)) return MH_E_INVALID;
    ctx->ws_limit = size_t(bytes);
    if (ctx->ws && ctx->ws_limit && ctx->ws_size > ctx->ws_limit) {
        // a held block above the new limit is released once the context's work is done
        DeviceGuard g(ctx->device);
        mh_status st = drain(ctx);
        if (st != MH_OK) return st;
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_size = 0;
    }
    return MH_OK;
}

extern "C" mh_status mh_ctx_workspace_info(mh_ctx *ctx, uint64_t *limit, uint64_t *held)
{
    if (!ctx) return MH_E_INVALID;
    if (limit) *limit = ctx->ws_limit;
    if (held) *held = ctx->ws_size;
    return MH_OK;
}

extern "C" mh_status mh_ctx_set_timing(mh_ctx *ctx, int enable)
{
    if (!ctx) return MH_E_INVALID;
    ctx->timing = enable != 0;
    return MH_OK;
}

extern "C" mh_status mh_ctx_kernel_time(mh_ctx *ctx, int kernel, double *total_ms,
                                        int64_t *launches, int reset)
{
    if (!ctx || kernel < 0 || kernel >= MH_K_COUNT) return MH_E_INVALID;
    DeviceGuard g(ctx->device);
    double tot = 0.0;
    int64_t cnt = 0;
    for (auto &r : ctx->records) {
        if (r.kernel != kernel) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) return note_error(ctx, hipErrorUnknown);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            tot += ms;
            ++cnt;
        }
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = cnt;
    if (reset) {
        std::vector<TimedLaunch> keep;
        for (auto &r : ctx->records) {
            if (r.kernel == kernel) {
                ctx->event_pool.push_back(r.a);
                ctx->event_pool.push_back(r.b);
            } else {
                keep.push_back(r);
            }
        }
        ctx->records.swap(keep);
    }
    return MH_OK;
}

extern "C" mh_status mh_ctx_kernel_times(mh_ctx *ctx, int kernel, double *ms_out, int64_t cap,
                                         int64_t *launches)
{
    if (!ctx || kernel < 0 || kernel >= MH_K_COUNT || cap < 0 || (cap > 0 && !ms_out))
        return MH_E_INVALID;
    DeviceGuard g(ctx->device);
    int64_t cnt = 0;
    for (auto &r : ctx->records) {
        if (r.kernel != kernel) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) return note_error(ctx, hipErrorUnknown);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
        if (cnt < cap) ms_out[cnt] = ms;
        ++cnt;
    }
    if (launches) *launches = cnt;
    return MH_OK;
}

// ================================================================ index math

namespace mh {

bool valid_T(int32_t T) { return T == 16 || T == 32 || T == 64 || T == 128; }

int log2i(int64_t x)
{
    int l = 0;
    while ((int64_t(1) << l) < x) ++l;
    return l;
}

mh_status check_parent(int64_t N, int32_t T)
{
    if (!valid_T(T)) return MH_E_UNSUPPORTED;
    if (N < T || N % T) return MH_E_SHAPE;
    int64_t q = N / T;
    if (q & (q - 1)) return MH_E_SHAPE;
    if (N > kMaxN) return MH_E_UNSUPPORTED;
    return MH_OK;
}

}  // namespace mh

extern "C" uint64_t mh_encode(uint64_t i, uint64_t j, uint32_t T)
{
    int logT = log2i(T);
    return mh_offset(i, j, logT);
}

extern "C" void mh_extract(uint64_t z, uint32_t T, uint64_t *i, uint64_t *j)
{
    int logT = log2i(T);
    uint64_t t = z >> (2 * logT), r = z & ((uint64_t(1) << (2 * logT)) - 1);
    uint64_t I = compact32(t >> 1), J = compact32(t);
    if (i) *i = (I << logT) | (r >> logT);
    if (j) *j = (J << logT) | (r & (T - 1));
}

static bool pow2_multiple(int64_t x, int64_t T)
{
    if (x <= 0 || x % T) return false;
    int64_t q = x / T;
    return (q & (q - 1)) == 0;
}

extern "C" mh_status mh_classify_submatrix(int64_t N, int32_t T, int64_t row, int64_t col,
                                           int64_t rows, int64_t cols, uint32_t *flags_out)
{
    if (!flags_out) return MH_E_INVALID;
    mh_status s = check_parent(N, T);
    if (s != MH_OK) return s;
    if (rows < 1 || cols < 1 || row < 0 || col < 0) return MH_E_INVALID;
    if (row + rows > N || col + cols > N) return MH_E_BOUNDS;
    uint32_t f = 0;
    // Def. "aligned" (section 2) with Cor. 2.1: first entry (k1 T, k2 T), size 2^a T x 2^b T.
    if (row % T == 0 && col % T == 0 && pow2_multiple(rows, T) && pow2_multiple(cols, T))
        f |= MH_ALIGNED;
    // Def. "contained" (section 2.1): first and last rows in one tile row, same for columns.
    if (row / T == (row + rows - 1) / T && col / T == (col + cols - 1) / T) f |= MH_CONTAINED;
    // A block of the quadrant recursion (section 2.2 Step 1).
    if (rows == cols && pow2_multiple(rows, T) && row % rows == 0 && col % cols == 0)
        f |= MH_QUADRANT;
    *flags_out = f;
    return MH_OK;
}

// ================================================================ validation

namespace mh {

static bool ranges_overlap(int64_t a0, int64_t an, int64_t b0, int64_t bn)
{
    return an > 0 && bn > 0 && a0 < b0 + bn && b0 < a0 + an;
}

// Does the output block of one product share memory with an input block?
static bool output_aliases(const uint32_t *C, int64_t NC, int64_t rc, int64_t cc, int64_t m,
                           int64_t n, const uint32_t *X, int64_t NX, int64_t rx, int64_t cx,
                           int64_t xr, int64_t xc)
{
    if (m <= 0 || n <= 0 || xr <= 0 || xc <= 0) return false;
    uintptr_t c0 = (uintptr_t)C, c1 = c0 + 4 * (uintptr_t)(NC * NC);
    uintptr_t x0 = (uintptr_t)X, x1 = x0 + 4 * (uintptr_t)(NX * NX);
    if (c1 <= x0 || x1 <= c0) return false;  // different allocations
    if (C != X || NC != NX) return true;    // overlapping storage of another shape
    return ranges_overlap(rc, m, rx, xr) && ranges_overlap(cc, n, cx, xc);
}

mh_status validate_product(const Product &p, bool need_ptrs)
{
    if (!valid_T(p.T)) return MH_E_UNSUPPORTED;
    mh_status s;
    if ((s = check_parent(p.NC, p.T)) != MH_OK) return s;
    if ((s = check_parent(p.NA, p.T)) != MH_OK) return s;
    if ((s = check_parent(p.NB, p.T)) != MH_OK) return s;
    if (p.m < 0 || p.k < 0 || p.n < 0) return MH_E_INVALID;
    if (p.rc < 0 || p.cc < 0 || p.ra < 0 || p.ca < 0 || p.rb < 0 || p.cb < 0)
        return MH_E_BOUNDS;
    if (p.rc + p.m > p.NC || p.cc + p.n > p.NC) return MH_E_BOUNDS;
    if (p.ra + p.m > p.NA || p.ca + p.k > p.NA) return MH_E_BOUNDS;
    if (p.rb + p.k > p.NB || p.cb + p.n > p.NB) return MH_E_BOUNDS;
    if (p.p < 2u || p.p > 0x7FFFFFFFu) return MH_E_MODULUS;
    if (need_ptrs && (!p.C || !p.A || !p.B)) return MH_E_INVALID;
    // A and B are read with 16-byte loads, C with 4-byte ones.
    if (need_ptrs && (((uintptr_t)p.A & 15) || ((uintptr_t)p.B & 15) || ((uintptr_t)p.C & 3)))
        return MH_E_INVALID;
    if (need_ptrs) {
        if (output_aliases(p.C, p.NC, p.rc, p.cc, p.m, p.n, p.A, p.NA, p.ra, p.ca, p.m, p.k))
            return MH_E_ALIAS;
        if (output_aliases(p.C, p.NC, p.rc, p.cc, p.m, p.n, p.B, p.NB, p.rb, p.cb, p.k, p.n))
            return MH_E_ALIAS;
    }
    return MH_OK;
}

bool outputs_alias(const Product &x, const Product &y)
{
    return output_aliases(x.C, x.NC, x.rc, x.cc, x.m, x.n, y.C, y.NC, y.rc, y.cc, y.m, y.n);
}

// ================================================================ planner
//
// The section 2.2 recursion divides the aligned parents A, B, C into
// quadrants down to T x T tiles and keeps, for each of the up-to-64
// quadrant combinations, the compatible parts of the three sub-matrices.
// Reading Step 4 as interval intersection in product coordinates, the base
// cases it reaches are exactly the boxes of the grid obtained by cutting
//   rows  [0,m) where C or A starts a tile row,
//   inner [0,k) where A starts a tile column or B a tile row,
//   cols  [0,n) where C or B starts a tile column,
// and every piece of such a box lies in one tile (Cor. 2.4).  The planner
// computes that grid in closed form instead of recursing.

void segments(int64_t len, int64_t offA, int64_t offB, int32_t T, std::vector<int64_t> &cuts)
{
    cuts.clear();
    cuts.push_back(0);
    if (len <= 0) return;
    int64_t a = (T - offA % T) % T, b = (T - offB % T) % T;
    if (a == 0) a = T;
    if (b == 0) b = T;
    while (a < len || b < len) {
        int64_t x = std::min(a, b);
        if (x >= len) break;
        cuts.push_back(x);
        if (a == x) a += T;
        if (b == x) b += T;
    }
    cuts.push_back(len);
}

void plan_product(const Product &p, int mode, Plan &pl, int forced_cfg)
{
    pl.pr = p;
    pl.sub = false;
    const int64_t T = p.T;
    if (mode == MH_MODE_AUTO) {
        double work = double(p.m) * double(p.n) * double(p.k);
        mode = work < double(1 << 21) ? MH_MODE_PLAIN_U32 : MH_MODE_LIMB_I8;
    }
    pl.mode = mode;
    pl.L = limbs_for(p.p);
    pl.kblock = kblock_for(pl.L);
    if (const char *e = std::getenv("MH_LIMB_KBLOCK")) {
        // shorter k-blocks than the bound allows (always exact; used by tests
        // to run the epilogue between k-blocks at small sizes)
        const int v = std::atoi(e);
        if (v >= 64 && v % 64 == 0 && v < pl.kblock) pl.kblock = v;
    }
    if (mode == MH_MODE_LIMB_I8) {
        pl.limb_cfg = limb_cfg_default(pl.L, p.m, p.n, p.k);
        if (const char *e = std::getenv("MH_LIMB_CFG")) {  // explicit override (tuning runs)
            int c = std::atoi(e);
            if (limb_cfg_fits(pl.L, c))
                pl.limb_cfg = c;
        }
        // a forced configuration (tuner, tune cache) that does not fit L is ignored
        if (limb_cfg_fits(pl.L, forced_cfg)) pl.limb_cfg = forced_cfg;
        const LimbKernelCfg &c = limb_cfg(pl.limb_cfg);
        pl.tile_m = c.tile_m();
        pl.tile_n = c.tile_n();
    } else {
        pl.limb_cfg = -1;
        pl.tile_m = mode == MH_MODE_FP64 ? 128 : 64;
        pl.tile_n = pl.tile_m;
    }
    // The elementwise comparator works in the product's own coordinates.
    const bool ew = mode == MH_MODE_PLAIN_ELEMENTWISE;
    pl.sr = ew ? 0 : p.rc % std::min<int64_t>(T, pl.tile_m);
    pl.sc = ew ? 0 : p.cc % std::min<int64_t>(T, pl.tile_n);
    pl.row0C = p.rc - pl.sr;
    pl.col0C = p.cc - pl.sc;
    pl.prow = (pl.sr + p.m + pl.tile_m - 1) / pl.tile_m * pl.tile_m;
    pl.pcol = (pl.sc + p.n + pl.tile_n - 1) / pl.tile_n * pl.tile_n;
    pl.grid_m = pl.prow / pl.tile_m;
    pl.grid_n = pl.pcol / pl.tile_n;
    if (mode == MH_MODE_LIMB_I8) {
        pl.sk = 0;
        pl.kpad = (p.k + 63) / 64 * 64;  // an even number of 32-deep k-blocks
        pl.in_place = false;
    } else if (ew) {
        pl.sk = 0;
        pl.kpad = p.k;
        pl.in_place = true;
    } else {
        // In place when A's tile rows line up with the panel rows, B's tile
        // columns with the panel columns, and A's tile columns with B's tile rows.
        pl.sk = p.ca % T;
        pl.in_place = ((p.ra - pl.sr) % T == 0) && (p.ra >= pl.sr) && ((p.cb - pl.sc) % T == 0) &&
                      (p.cb >= pl.sc) && ((p.rb - pl.sk) % T == 0) && (p.rb >= pl.sk) &&
                      p.C != p.A && p.C != p.B;
        if (!pl.in_place) pl.sk = 0;
        int64_t kq = std::max<int64_t>(T, 64);
        pl.kpad = (pl.sk + p.k + kq - 1) / kq * kq;
    }
}

}  // namespace mh

// ------------------------------------------------------- planner queries

Product mh::make_product(uint32_t *C, int64_t NC, int64_t rc, int64_t cc, const uint32_t *A,
                        int64_t NA, int64_t ra, int64_t ca, const uint32_t *B, int64_t NB,
                        int64_t rb, int64_t cb, int64_t m, int64_t k, int64_t n, uint32_t p,
                        int32_t T)
{
    Product pr;
    pr.C = C;
    pr.A = A;
    pr.B = B;
    pr.NC = NC;
    pr.rc = rc;
    pr.cc = cc;
    pr.NA = NA;
    pr.ra = ra;
    pr.ca = ca;
    pr.NB = NB;
    pr.rb = rb;
    pr.cb = cb;
    pr.m = m;
    pr.k = k;
    pr.n = n;
    pr.p = p;
    pr.T = T;
    pr.logT = valid_T(T) ? log2i(T) : 0;
    return pr;
}

extern "C" mh_status mh_plan_describe(int64_t NC, int64_t rc, int64_t cc, int64_t NA, int64_t ra,
                                      int64_t ca, int64_t NB, int64_t rb, int64_t cb, int64_t m,
                                      int64_t k, int64_t n, uint32_t p, int32_t T, int32_t mode,
                                      mh_plan_info *out)
{
    if (!out) return MH_E_INVALID;
    int form;
    bool sub;
    if (!parse_mode(mode, form, sub)) return MH_E_UNSUPPORTED;
    mode = form;
    Product pr = make_product(nullptr, NC, rc, cc, nullptr, NA, ra, ca, nullptr, NB, rb, cb, m,
                              k, n, p, T);
    mh_status s = validate_product(pr, false);
    if (s == MH_OK) s = check_form_modulus(form, p);
    if (s != MH_OK) return s;
    std::vector<int64_t> rcut, kcut, ccut;
    segments(m, rc, ra, T, rcut);
    segments(k, ca, rb, T, kcut);
    segments(n, cc, cb, T, ccut);
    std::memset(out, 0, sizeof(*out));
    out->row_segments = m > 0 ? int64_t(rcut.size()) - 1 : 0;
    out->inner_segments = k > 0 ? int64_t(kcut.size()) - 1 : 0;
    out->col_segments = n > 0 ? int64_t(ccut.size()) - 1 : 0;
    out->leaves = out->row_segments * out->inner_segments * out->col_segments;
    if (m > 0 && n > 0)
        out->c_tiles = ((rc + m - 1) / T - rc / T + 1) * ((cc + n - 1) / T - cc / T + 1);
    Plan pl;
    plan_product(pr, mode, pl);
    out->mode = pl.mode;
    out->in_place = pl.in_place ? 1 : 0;
    out->tile_m = pl.tile_m;
    out->tile_n = pl.tile_n;
    out->limbs = pl.mode == MH_MODE_LIMB_I8 ? pl.L : 0;
    out->kblock = pl.mode == MH_MODE_LIMB_I8 ? pl.kblock
                : pl.mode == MH_MODE_FP64     ? int32_t(std::min<int64_t>(
                                                    int64_t(4) * f64_red_steps(p), INT32_MAX / 4 * 4))
                                              : 0;
    out->kernel_cfg = pl.mode == MH_MODE_LIMB_I8 ? pl.limb_cfg : -1;
    out->gemm_tasks = (m > 0 && n > 0) ? pl.grid_m * pl.grid_n : 0;
    if (pl.mode == MH_MODE_LIMB_I8 && m > 0 && n > 0 && k > 0) {
        int64_t nkb = pl.kpad / 32;
        out->pack_chunks = (pl.prow / 64) * ((nkb + 1) / 2) + (pl.pcol / 64) * ((nkb + 1) / 2);
    } else if (!pl.in_place && m > 0 && n > 0 && k > 0) {
        out->pack_chunks = 2;
    }
    return MH_OK;
}

extern "C" mh_status mh_plan_leaves(int64_t NC, int64_t rc, int64_t cc, int64_t NA, int64_t ra,
                                    int64_t ca, int64_t NB, int64_t rb, int64_t cb, int64_t m,
                                    int64_t k, int64_t n, int32_t T, int64_t *out, int64_t cap,
                                    int64_t *count)
{
    if (!count || (cap > 0 && !out)) return MH_E_INVALID;
    Product pr = make_product(nullptr, NC, rc, cc, nullptr, NA, ra, ca, nullptr, NB, rb, cb, m,
                              k, n, 2, T);
    mh_status s = validate_product(pr, false);
    if (s != MH_OK) return s;
    *count = 0;
    if (m == 0 || n == 0 || k == 0) return MH_OK;
    std::vector<int64_t> rcut, kcut, ccut;
    segments(m, rc, ra, T, rcut);
    segments(k, ca, rb, T, kcut);
    segments(n, cc, cb, T, ccut);
    int64_t q = 0;
    for (size_t a = 0; a + 1 < rcut.size(); ++a)
        for (size_t b = 0; b + 1 < kcut.size(); ++b)
            for (size_t c = 0; c + 1 < ccut.size(); ++c, ++q) {
                if (q >= cap) continue;
                int64_t *o = out + 6 * q;
                o[0] = rcut[a];
                o[1] = rcut[a + 1] - rcut[a];
                o[2] = kcut[b];
                o[3] = kcut[b + 1] - kcut[b];
                o[4] = ccut[c];
                o[5] = ccut[c + 1] - ccut[c];
            }
    *count = q;
    return MH_OK;
}

extern "C" mh_status mh_plan_gemm_tasks(int64_t NC, int64_t rc, int64_t cc, int64_t NA,
                                        int64_t ra, int64_t ca, int64_t NB, int64_t rb,
                                        int64_t cb, int64_t m, int64_t k, int64_t n, uint32_t p,
                                        int32_t T, int32_t mode, int64_t *out, int64_t cap,
                                        int64_t *count)
{
    if (!count || (cap > 0 && !out)) return MH_E_INVALID;
    int form;
    bool sub;
    if (!parse_mode(mode, form, sub)) return MH_E_UNSUPPORTED;
    mode = form;
    Product pr = make_product(nullptr, NC, rc, cc, nullptr, NA, ra, ca, nullptr, NB, rb, cb, m,
                              k, n, p, T);
    mh_status s = validate_product(pr, false);
    if (s == MH_OK) s = check_form_modulus(form, p);
    if (s != MH_OK) return s;
    *count = 0;
    if (m == 0 || n == 0) return MH_OK;
    Plan pl;
    plan_product(pr, mode, pl);
    int64_t q = 0;
    for (int64_t gm = 0; gm < pl.grid_m; ++gm)
        for (int64_t gn = 0; gn < pl.grid_n; ++gn) {
            int64_t i0 = std::max<int64_t>(0, gm * pl.tile_m - pl.sr);
            int64_t i1 = std::min<int64_t>(m, (gm + 1) * pl.tile_m - pl.sr);
            int64_t j0 = std::max<int64_t>(0, gn * pl.tile_n - pl.sc);
            int64_t j1 = std::min<int64_t>(n, (gn + 1) * pl.tile_n - pl.sc);
            if (i1 <= i0 || j1 <= j0) continue;
            if (q < cap) {
                int64_t *o = out + 4 * q;
                o[0] = i0;
                o[1] = i1 - i0;
                o[2] = j0;
                o[3] = j1 - j0;
            }
            ++q;
        }
    *count = q;
    return MH_OK;
}

// ================================================================ layout

// Shared by the square and the padded conversions: dst/src are checked for
// overlap over the bytes each side really touches.
static mh_status layout_common(mh_ctx *ctx, bool to_mh, uint32_t *mhbuf, uint32_t *cart,
                               int64_t ld, int64_t rows, int64_t cols, int64_t N, int32_t T,
                               hipStream_t stream)
{
    if (!ctx || !mhbuf || !cart) return MH_E_INVALID;
    mh_status s = check_parent(N, T);
    if (s != MH_OK) return s;
    if (rows < 1 || cols < 1 || rows > N || cols > N || ld < cols) return MH_E_INVALID;
    uintptr_t m0 = (uintptr_t)mhbuf, m1 = m0 + 4 * (uintptr_t)(N * N);
    uintptr_t c0 = (uintptr_t)cart, c1 = c0 + 4 * (uintptr_t)((rows - 1) * ld + cols);
    if (m0 < c1 && c0 < m1) return MH_E_ALIAS;
    DeviceGuard g(ctx->device);
    TimedLaunch t;
    record_start(ctx, to_mh ? MH_K_LAYOUT_FROM : MH_K_LAYOUT_TO, stream, t);
    hipError_t e = to_mh ? launch_layout_from(mhbuf, cart, ld, rows, cols, N, log2i(T), stream)
                         : launch_layout_to(cart, ld, rows, cols, mhbuf, N, log2i(T), stream);
    record_end(ctx, stream, t);
    return note_error(ctx, e);
}

extern "C" mh_status mh_layout_from_cartesian(mh_ctx *ctx, uint32_t *dst_mh, const uint32_t *src,
                                              int64_t ld_src, int64_t N, int32_t T,
                                              hipStream_t stream)
{
    if (ld_src < N) return MH_E_INVALID;
    return layout_common(ctx, true, dst_mh, const_cast<uint32_t *>(src), ld_src, N, N, N, T,
                         stream);
}

extern "C" mh_status mh_layout_to_cartesian(mh_ctx *ctx, uint32_t *dst, int64_t ld_dst,
                                            const uint32_t *src_mh, int64_t N, int32_t T,
                                            hipStream_t stream)
{
    if (ld_dst < N) return MH_E_INVALID;
    return layout_common(ctx, false, const_cast<uint32_t *>(src_mh), dst, ld_dst, N, N, N, T,
                         stream);
}

extern "C" mh_status mh_parent_size(int64_t rows, int64_t cols, int32_t T, int64_t *N)
{
    if (!N || rows < 1 || cols < 1) return MH_E_INVALID;
    if (!valid_T(T)) return MH_E_UNSUPPORTED;
    int64_t n = T;
    while (n < rows || n < cols) {
        if (n >= kMaxN) return MH_E_UNSUPPORTED;
        n *= 2;
    }
    *N = n;
    return MH_OK;
}

extern "C" mh_status mh_layout_from_cartesian_padded(mh_ctx *ctx, uint32_t *dst_mh, int64_t N,
                                                     const uint32_t *src, int64_t ld_src,
                                                     int64_t rows, int64_t cols, int32_t T,
                                                     hipStream_t stream)
{
    return layout_common(ctx, true, dst_mh, const_cast<uint32_t *>(src), ld_src, rows, cols, N,
                         T, stream);
}

extern "C" mh_status mh_layout_to_cartesian_padded(mh_ctx *ctx, uint32_t *dst, int64_t ld_dst,
                                                   int64_t rows, int64_t cols,
                                                   const uint32_t *src_mh, int64_t N, int32_t T,
                                                   hipStream_t stream)
{
    return layout_common(ctx, false, const_cast<uint32_t *>(src_mh), dst, ld_dst, rows, cols, N,
                         T, stream);
}

// ================================================================ product

namespace mh {

uint64_t barrett_mu(uint32_t p) { return ~uint64_t(0) / p; }

static uint64_t horner_bias(uint32_t p)
{
    uint64_t b = ((uint64_t(1) << 31) + p - 1) / p * p;
    return b;
}

// Device bytes of a plan's operand panels (0 when it reads A and B in place).
size_t plan_ws_bytes(const Plan &pl)
{
    const Product &p = pl.pr;
    if (p.m <= 0 || p.n <= 0 || p.k <= 0) return 0;
    if (pl.mode == MH_MODE_LIMB_I8) {
        const size_t per_row = size_t(pl.kpad) * size_t(pl.L);  // nkb * 32 * L
        return align256(size_t(pl.prow) * per_row) + align256(size_t(pl.pcol) * per_row) + 256;
    }
    if (pl.mode == MH_MODE_PLAIN_ELEMENTWISE || pl.in_place) return 0;
    const int64_t T = p.T;
    const int64_t prow = (pl.prow + T - 1) / T * T, pcol = (pl.pcol + T - 1) / T * T;
    return align256(size_t(prow) * size_t(pl.kpad) * 4) +
           align256(size_t(pl.kpad) * size_t(pcol) * 4) + 256;
}

mh_status run_plain(mh_ctx *ctx, const Plan &pl, char *ws, hipStream_t s)
{
    const Product &p = pl.pr;
    const int64_t T = p.T;
    PlainArgs a;
    std::memset(&a, 0, sizeof(a));
    a.C = p.C;
    a.sr = pl.sr;
    a.sc = pl.sc;
    a.sk = pl.sk;
    a.m = p.m;
    a.n = p.n;
    a.k = p.k;
    a.kpad = pl.kpad;
    a.row0C = pl.row0C;
    a.col0C = pl.col0C;
    a.grid_m = pl.grid_m;
    a.grid_n = pl.grid_n;
    a.p = p.p;
    a.mu = barrett_mu(p.p);
    a.logT = p.logT;
    a.sub = pl.sub ? 1 : 0;
    a.red_steps = f64_red_steps(p.p);
    a.pinv = 1.0 / double(p.p);
    if (pl.mode == MH_MODE_PLAIN_ELEMENTWISE) {
        a.A = p.A;
        a.B = p.B;
        a.a_mh = a.b_mh = 2;
        a.a_tr0 = p.ra;  // element origins
        a.a_tc0 = p.ca;
        a.b_tr0 = p.rb;
        a.b_tc0 = p.cb;
    } else if (pl.in_place) {
        a.A = p.A;
        a.B = p.B;
        a.a_mh = a.b_mh = 1;
        a.a_tr0 = (p.ra - pl.sr) / T;
        a.a_tc0 = (p.ca - pl.sk) / T;
        a.b_tr0 = (p.rb - pl.sk) / T;
        a.b_tc0 = (p.cb - pl.sc) / T;
    } else {
        // u32 panels, tile-major, of prow x kpad (A) and kpad x pcol (B).
        int64_t prow = (pl.prow + T - 1) / T * T, pcol = (pl.pcol + T - 1) / T * T;
        size_t abytes = size_t(prow) * size_t(pl.kpad) * 4;
        if (!ws) return MH_E_NOMEM;
        uint32_t *Ap = (uint32_t *)ws;
        uint32_t *Bp = (uint32_t *)(ws + align256(abytes));
        TimedLaunch t;
        record_start(ctx, MH_K_PACK, s, t);
        // A panel (rho, kap) <- A(ra - sr + rho, ca + kap) for rho in [sr, sr+m), kap < k
        hipError_t e = launch_pack_u32(Ap, prow, pl.kpad, p.A, p.ra - pl.sr, p.ca, pl.sr,
                                       pl.sr + p.m, 0, p.k, p.logT, s);
        // B panel (kap, gam) <- B(rb + kap, cb - sc + gam) for kap < k, gam in [sc, sc+n)
        if (e == hipSuccess)
            e = launch_pack_u32(Bp, pl.kpad, pcol, p.B, p.rb, p.cb - pl.sc, 0, p.k, pl.sc,
                                pl.sc + p.n, p.logT, s);
        record_end(ctx, s, t);
        if (e != hipSuccess) return note_error(ctx, e);
        a.A = Ap;
        a.B = Bp;
        a.a_mh = a.b_mh = 0;
        a.a_ntc = pl.kpad / T;
        a.b_ntc = pcol / T;
    }
    const bool f64 = pl.mode == MH_MODE_FP64;
    TimedLaunch t;
    record_start(ctx, f64 ? MH_K_GEMM_F64 : MH_K_GEMM_PLAIN, s, t);
    hipError_t e = f64 ? launch_gemm_f64(a, s) : launch_gemm_plain(a, s);
    record_end(ctx, s, t);
    return note_error(ctx, e);
}

mh_status run_limb(mh_ctx *ctx, const Plan &pl, char *ws, hipStream_t s)
{
    const Product &p = pl.pr;
    const int L = pl.L;
    const int64_t nkb = pl.kpad / 32;
    size_t abytes = size_t(pl.prow) * size_t(nkb) * 32 * L;
    if (!ws) return MH_E_NOMEM;
    int8_t *Ap = (int8_t *)ws;
    int8_t *Bp = (int8_t *)(ws + align256(abytes));
    TimedLaunch t;
    record_start(ctx, MH_K_PACK, s, t);
    hipError_t e = launch_pack_limb(Ap, pl.prow, nkb, p.A, p.ra, p.ca, pl.sr, p.m, p.k, 0, 0,
                                    p.logT, p.p, L, s);
    // C - A.B = C + A.(-B): the subtractive update negates B while packing it.
    if (e == hipSuccess)
        e = launch_pack_limb(Bp, pl.pcol, nkb, p.B, p.rb, p.cb, pl.sc, p.n, p.k, 1,
                             pl.sub ? 1 : 0, p.logT, p.p, L, s);
    record_end(ctx, s, t);
    if (e != hipSuccess) return note_error(ctx, e);
    LimbArgs a;
    std::memset(&a, 0, sizeof(a));
    a.Ap = Ap;
    a.Bp = Bp;
    a.nkb = nkb;
    a.kb_per_red = pl.kblock / 32;
    a.C = p.C;
    a.row0C = pl.row0C;
    a.col0C = pl.col0C;
    a.sr = pl.sr;
    a.sc = pl.sc;
    a.m = p.m;
    a.n = p.n;
    a.grid_m = pl.grid_m;
    a.grid_n = pl.grid_n;
    a.p = p.p;
    a.mu = barrett_mu(p.p);
    a.bias = horner_bias(p.p);
    a.pinv = 1.0 / double(p.p);
    a.logT = p.logT;
    record_start(ctx, MH_K_GEMM_LIMB, s, t);
    e = launch_gemm_limb(pl.limb_cfg, L, a, s);
    record_end(ctx, s, t);
    return note_error(ctx, e);
}

// Plan of one product, with the tuner's configuration where it has one.
// Timing runs of the tuner (mode 2) only when the caller lets the library
// allocate (they write a scratch output parent).
static void plan_tuned(mh_ctx *ctx, const Product &pr, int form, bool sub, bool may_tune,
                       hipStream_t s, Plan &pl)
{
    plan_product(pr, form, pl);
    if (pl.mode == MH_MODE_LIMB_I8 && ctx->autotune) {
        int cfg = tune_get(ctx, tune_key_single(pl.L, pr));
        if (cfg < 0 && ctx->autotune == 2 && may_tune) cfg = tune_single(ctx, pr, s);
        if (cfg >= 0) plan_product(pr, MH_MODE_LIMB_I8, pl, cfg);
    }
    pl.sub = sub;
}

static mh_status run_plan(mh_ctx *ctx, const Plan &pl, const WsSource &src, hipStream_t s)
{
    const size_t need = plan_ws_bytes(pl);
    char *ws = need ? ws_get(ctx, src, need) : nullptr;
    if (need && !ws) return MH_E_NOMEM;
    return pl.mode == MH_MODE_LIMB_I8 ? run_limb(ctx, pl, ws, s) : run_plain(ctx, pl, ws, s);
}

// Sub-product of pr: rows [i0, i0+mi), inner [l0, l0+kl), columns [j0, j0+nj)
// in product coordinates.
static Product sub_product(const Product &pr, int64_t i0, int64_t mi, int64_t l0, int64_t kl,
                           int64_t j0, int64_t nj)
{
    Product q = pr;
    q.rc = pr.rc + i0;
    q.ra = pr.ra + i0;
    q.cc = pr.cc + j0;
    q.cb = pr.cb + j0;
    q.ca = pr.ca + l0;
    q.rb = pr.rb + l0;
    q.m = mi;
    q.k = kl;
    q.n = nj;
    return q;
}

// Chunk edges (mb, kc, nb) whose panels fit `cap` bytes.  Every chunk
// boundary falls on a multiple of T in rows and columns and of max(64, T)
// in depth, so each chunk has the panel shifts of the whole product and no
// chunk needs more than the first.  Depth is split first (down to 1024),
// then the longer of the two output edges (down to 1024), then depth to
// its granule, then the output edges to T.  false if even that does not fit.
static bool choose_chunks(const Product &pr, int form, size_t cap, int64_t &mb, int64_t &kc,
                          int64_t &nb)
{
    const int64_t T = pr.T, kq = std::max<int64_t>(64, T);
    auto up = [](int64_t x, int64_t q) { return (x + q - 1) / q * q; };
    auto bytes = [&]() {
        Plan pl;
        plan_product(sub_product(pr, 0, std::min(mb, pr.m), 0, std::min(kc, pr.k), 0,
                                 std::min(nb, pr.n)),
                     form, pl);
        return plan_ws_bytes(pl);
    };
    auto half_k = [&]() { kc = std::max(kq, up((kc + 1) / 2, kq)); };
    auto half_mn = [&]() {
        int64_t &x = mb >= nb ? mb : nb;
        x = std::max(T, up((x + 1) / 2, T));
    };
    mb = pr.m;
    kc = pr.k;
    nb = pr.n;
    while (bytes() > cap && kc > 1024) half_k();
    while (bytes() > cap && std::max(mb, nb) > 1024) half_mn();
    while (bytes() > cap && kc > kq) half_k();
    while (bytes() > cap && std::max(mb, nb) > T) half_mn();
    return bytes() <= cap;
}

mh_status run_product(mh_ctx *ctx, const Product &pr, int form, bool sub, const WsSource &src,
                      hipStream_t s)
{
    if (pr.m == 0 || pr.n == 0 || pr.k == 0) return MH_OK;
    Plan pl;
    plan_tuned(ctx, pr, form, sub, !src.fixed, s, pl);
    const size_t cap = src.fixed ? src.cap : (ctx->ws_limit ? ctx->ws_limit : SIZE_MAX);
    if (plan_ws_bytes(pl) <= cap) return run_plan(ctx, pl, src, s);
    // Too large for the workspace allowed: sub-products over chunks of the
    // rows, the depth and the columns, each accumulated into C in turn
    // (addition mod p is associative, so the result is the same; for the
    // subtractive update every chunk subtracts its part).
    form = pl.mode;  // the whole product's form, also for small trailing chunks
    int64_t mb, kc, nb;
    if (!choose_chunks(pr, form, cap, mb, kc, nb)) return MH_E_NOMEM;
    for (int64_t i0 = 0; i0 < pr.m; i0 += mb)
        for (int64_t j0 = 0; j0 < pr.n; j0 += nb)
            for (int64_t l0 = 0; l0 < pr.k; l0 += kc) {
                const Product q = sub_product(pr, i0, std::min(mb, pr.m - i0), l0,
                                              std::min(kc, pr.k - l0), j0, std::min(nb, pr.n - j0));
                Plan ql;
                plan_tuned(ctx, q, form, sub, !src.fixed, s, ql);
                if (plan_ws_bytes(ql) > cap) plan_product(q, form, ql);  // built-in tile
                ql.sub = sub;
                if (plan_ws_bytes(ql) > cap) return MH_E_NOMEM;
                mh_status st = run_plan(ctx, ql, src, s);
                if (st != MH_OK) return st;
            }
    return MH_OK;
}

}  // namespace mh

extern "C" mh_status mh_matmul_modp(mh_ctx *ctx, uint32_t *C, int64_t NC, int64_t rc, int64_t cc,
                                    const uint32_t *A, int64_t NA, int64_t ra, int64_t ca,
                                    const uint32_t *B, int64_t NB, int64_t rb, int64_t cb,
                                    int64_t m, int64_t k, int64_t n, uint32_t p, int32_t T,
                                    int32_t mode, hipStream_t stream)
{
    if (!ctx) return MH_E_INVALID;
    int form;
    bool sub;
    if (!parse_mode(mode, form, sub)) return MH_E_UNSUPPORTED;
    Product pr = make_product(C, NC, rc, cc, A, NA, ra, ca, B, NB, rb, cb, m, k, n, p, T);
    mh_status s = validate_product(pr, true);
    if (s == MH_OK) s = check_form_modulus(form, p);
    if (s != MH_OK) return s;
    if (m == 0 || n == 0 || k == 0) return MH_OK;
    DeviceGuard g(ctx->device);
    CtxUse use(ctx, stream);
    return run_product(ctx, pr, form, sub, WsSource{}, stream);
}
