// Batched products: one persistent launch over a device task queue,
// captured once into a HIP graph and replayed.
//
// The calls of one recursion level of a TU factorisation are independent
// (section 2.2, Prop. 2.6: the recursive calls can be cast in parallel), so
// a whole batch runs as
//   reset counters -> persistent pack kernels (A, then B panels) ->
//   persistent GEMM kernel
// on one stream.  Each persistent kernel has a fixed grid (CUs x occupancy)
// and pops work items through atomic counters until the queue is empty,
// so the graph's topology never changes: a new batch only rewrites the
// queue (one host-to-device copy from pinned staging memory) before the
// graph is launched again.  The products are split into one group per XCD,
// balanced by work, so that each group's operand panels are read through
// one L2; within a group they are queued largest k first, so the longest
// output blocks start first (longest-processing-time order).
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>

#include "mh_ctx.h"
#include "mh_device.h"

namespace mh {

namespace {

__global__ void k_reset_counters(uint64_t *c)
{
    if (threadIdx.x < kBatchCounters) c[threadIdx.x] = 0;
}

void release_graphs(BatchedState &b)
{
    for (auto &g : b.graphs) {
        if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
        if (g.second.graph) (void)hipGraphDestroy(g.second.graph);
    }
    b.graphs.clear();
}

int batch_cfg(int L, const std::vector<Plan> &plans)
{
    double area = 0.0;
    for (const Plan &p : plans) area += double(p.pr.m) * double(p.pr.n);
    area /= std::max<size_t>(plans.size(), 1);
    // 64 x 128 blocks of 8 waves sharing LDS stages when the products are
    // large enough (at L <= 2 two such workgroups share a compute unit, and
    // one's epilogue overlaps the other's MFMAs); else small per-product
    // blocks keep padding and tails low.
    int cfg = area <= 512.0 * 512.0 ? 6 : (L <= 2 ? 11 : 4);
    if (const char *e = std::getenv("MH_LIMB_CFG")) {  // explicit override (tuning runs)
        int c = std::atoi(e);
        if (limb_cfg_fits(L, c))
            cfg = c;
    }
    return cfg;
}

// Capacity (products) of the queue buffers, reallocating them if needed.
mh_status ensure_queue(mh_ctx *ctx, int64_t ncalls)
{
    BatchedState &b = ctx->batched;
    if (b.queue_dev && ncalls <= b.queue_cap) return MH_OK;
    int64_t cap = 64;
    while (cap < ncalls) cap *= 2;
    // The captured graphs read the old queue: wait for the context's
    // launches to finish before destroying them and freeing it.
    mh_status st = drain(ctx);
    if (st != MH_OK) return st;
    release_graphs(b);
    if (b.queue_dev) (void)hipFree(b.queue_dev);
    if (b.queue_host) (void)hipHostFree(b.queue_host);
    b.queue_dev = b.queue_host = nullptr;
    b.queue_cap = 0;
    const size_t bytes = queue_bytes(cap);
    if (hipMalloc(&b.queue_dev, bytes) != hipSuccess) {
        b.queue_dev = nullptr;
        (void)hipGetLastError();
        return MH_E_NOMEM;
    }
    if (hipHostMalloc(&b.queue_host, bytes, hipHostMallocDefault) != hipSuccess) {
        b.queue_host = nullptr;
        (void)hipGetLastError();
        return MH_E_NOMEM;
    }
    if (!b.counters &&
        hipMalloc((void **)&b.counters, kBatchCounters * sizeof(uint64_t)) != hipSuccess) {
        b.counters = nullptr;
        (void)hipGetLastError();
        return MH_E_NOMEM;
    }
    if (!b.staging_free && hipEventCreateWithFlags(&b.staging_free, hipEventDisableTiming) !=
                               hipSuccess) {
        b.staging_free = nullptr;
        return MH_E_DEVICE;
    }
    if (!b.capture_stream &&
        hipStreamCreateWithFlags(&b.capture_stream, hipStreamNonBlocking) != hipSuccess) {
        b.capture_stream = nullptr;
        return MH_E_DEVICE;
    }
    b.queue_cap = cap;
    return MH_OK;
}

// Capture reset -> pack -> GEMM for kernel configuration cfg, L limbs and
// the GEMM's forms (C loaded early, A from whole-parent panels), once per
// context, queue buffer and key; returns the executable graph.
hipGraphExec_t ensure_graph(mh_ctx *ctx, int cfg, int L, bool early_c, bool a_parent)
{
    BatchedState &b = ctx->batched;
    const int key = ((cfg * 8 + L) * 2 + (early_c ? 1 : 0)) * 2 + (a_parent ? 1 : 0);
    auto it = b.graphs.find(key);
    if (it != b.graphs.end()) return it->second.exec;
    const QueueView q = queue_view(b.queue_dev, b.queue_cap);
    hipStream_t cs = b.capture_stream;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return nullptr;
    hipError_t e1 = launch_reset_counters(b.counters, cs);
    hipError_t e2 = launch_pack_limb_batched(L, q, b.counters, ctx->num_cu, cs);
    hipError_t e3 =
        launch_gemm_limb_batched(cfg, L, early_c, a_parent, q, b.counters + 2, ctx->num_cu, cs);
    hipGraph_t g = nullptr;
    hipError_t e4 = hipStreamEndCapture(cs, &g);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return nullptr;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return nullptr;
    }
    b.graphs[key] = BatchedState::Captured{g, ex};
    return ex;
}

// One rectangle of a batch in the storage of a parent: an output block
// (is_c) or an input block.
struct Rect {
    int64_t r0, r1, c0, c1;  // rows [r0, r1), columns [c0, c1)
    bool is_c;
};

// MH_E_ALIAS if an output block of the batch shares a word with another
// output block or with any input block, else MH_OK; the rule of
// output_aliases applied to every pair, in O(n log n + overlaps) instead of
// O(n^2) (a TU level has hundreds of products).  Blocks of different parent
// allocations never share words; if two different parents' storage
// overlaps (another base or edge), any block of one against an output block
// of the other counts as overlapping, as it does for a single product.
mh_status check_batch_aliasing(const std::vector<Product> &prods)
{
    struct Parent {
        const uint32_t *base;
        int64_t N;
        std::vector<Rect> rects;
        bool has_c = false;
    };
    std::vector<Parent> parents;
    auto parent_of = [&](const uint32_t *base, int64_t N) -> Parent & {
        for (Parent &q : parents)
            if (q.base == base && q.N == N) return q;
        parents.push_back(Parent{base, N, {}, false});
        return parents.back();
    };
    auto add = [&](const uint32_t *base, int64_t N, int64_t r, int64_t c, int64_t rows,
                   int64_t cols, bool is_c) {
        if (rows <= 0 || cols <= 0) return;
        Parent &q = parent_of(base, N);
        q.rects.push_back(Rect{r, r + rows, c, c + cols, is_c});
        q.has_c = q.has_c || is_c;
    };
    for (const Product &x : prods) {
        if (x.m > 0 && x.n > 0) add(x.C, x.NC, x.rc, x.cc, x.m, x.n, true);
        add(x.A, x.NA, x.ra, x.ca, x.m, x.k, false);
        add(x.B, x.NB, x.rb, x.cb, x.k, x.n, false);
    }
    // Distinct parents whose storage overlaps: sweep over start addresses.
    std::vector<size_t> by_addr(parents.size());
    std::iota(by_addr.begin(), by_addr.end(), 0);
    auto lo = [&](size_t q) { return (uintptr_t)parents[q].base; };
    auto hi = [&](size_t q) { return lo(q) + 4 * (uintptr_t)(parents[q].N * parents[q].N); };
    std::sort(by_addr.begin(), by_addr.end(), [&](size_t a, size_t b) { return lo(a) < lo(b); });
    for (size_t u = 0; u < by_addr.size(); ++u)
        for (size_t v = u + 1; v < by_addr.size() && lo(by_addr[v]) < hi(by_addr[u]); ++v)
            if (parents[by_addr[u]].has_c || parents[by_addr[v]].has_c) return MH_E_ALIAS;
    // Within one parent: sweep the rectangles by first row, keeping those
    // whose rows are still open; a pair counts when one is an output block.
    for (Parent &q : parents) {
        if (!q.has_c) continue;
        std::vector<Rect> &rs = q.rects;
        std::sort(rs.begin(), rs.end(), [](const Rect &a, const Rect &b) { return a.r0 < b.r0; });
        std::vector<const Rect *> open;
        for (const Rect &x : rs) {
            size_t keep = 0;
            for (const Rect *y : open)
                if (y->r1 > x.r0) open[keep++] = y;
            open.resize(keep);
            for (const Rect *y : open)
                if ((x.is_c || y->is_c) && x.c0 < y->c1 && y->c0 < x.c1) return MH_E_ALIAS;
            open.push_back(&x);
        }
    }
    return MH_OK;
}

}  // namespace

hipError_t launch_reset_counters(uint64_t *counters, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, counters);
    return hipGetLastError();
}

void batched_release(mh_ctx *ctx)
{
    BatchedState &b = ctx->batched;
    release_graphs(b);
    if (b.capture_stream) (void)hipStreamDestroy(b.capture_stream);
    if (b.queue_dev) (void)hipFree(b.queue_dev);
    if (b.queue_host) (void)hipHostFree(b.queue_host);
    if (b.counters) (void)hipFree(b.counters);
    if (b.staging_free) (void)hipEventDestroy(b.staging_free);
    b = BatchedState();
}

}  // namespace mh

namespace mh {

// Runs products already planned with kernel configuration cfg as one
// batched graph on `stream`.  With c_override set, every output goes to that
// buffer instead (tuning runs).
mh_status launch_batch(mh_ctx *ctx, const std::vector<Plan> &plans0, int cfg, int L, uint32_t p,
                       hipStream_t stream, uint32_t *c_override)
{
    if (plans0.empty()) return MH_OK;
    // C loaded ahead of the epilogue: where the configuration has that form
    // (one 32 x 32 block per wave, LDS stages, L <= 2), tile size and C
    // parents permitting.
    int64_t max_nc = 0;
    for (const Plan &pl : plans0) max_nc = std::max<int64_t>(max_nc, pl.pr.NC);
    const LimbKernelCfg &kc = limb_cfg(cfg);
    const bool early_c = kc.lds && kc.wm * kc.wn == 1 && L <= 2 &&
                         limb_batched_early_c(plans0[0].pr.logT, max_nc);

    // A operands from whole-parent panels: each distinct A parent is packed
    // once, and the GEMM reads every product's A block out of its parent's
    // panel (a TU level's products are blocks of a few shared parents, each
    // word of which lies in many products' A blocks).  Chosen when the A
    // blocks hold at least as many words as their parents (MH_BATCH_APARENT
    // = 0 never, 1 whenever the configuration has that form), with the
    // early-C form, and every parent panel below 2 GiB.  Each product's panel
    // rows then start on a 32-row slab of its A parent (row shift ra mod 32
    // instead of C's tile phase: the early-C epilogue addresses C rows of
    // any phase), and B's panels start their depth at the phase ca mod 32 of
    // A's columns in the parent's k-blocks.
    struct AParent {
        const uint32_t *A;
        int64_t N, nslab, nkbp;
        size_t off;
    };
    std::vector<AParent> apars;
    std::vector<int> apar_of(plans0.size(), -1);
    bool a_parent = early_c && limb_batched_a_parent(cfg, L);
    if (a_parent) {
        const char *env = std::getenv("MH_BATCH_APARENT");
        const int want = env ? std::atoi(env) : -1;
        double words = 0.0, pwords = 0.0;
        for (size_t q = 0; q < plans0.size() && a_parent; ++q) {
            const Product &pr = plans0[q].pr;
            words += double(pr.m) * double(pr.k);
            int idx = -1;
            for (size_t u = 0; u < apars.size(); ++u)
                if (apars[u].A == pr.A && apars[u].N == pr.NA) idx = int(u);
            if (idx < 0) {
                AParent ap;
                ap.A = pr.A;
                ap.N = pr.NA;
                ap.nslab = (pr.NA + 63) / 64 * 2;  // rows in whole 64-row pack chunks
                ap.nkbp = (pr.NA + 63) / 64 * 2;   // an even number of k-blocks
                ap.off = 0;
                if ((ap.nslab + kAParentGuard) * ap.nkbp * L * 1024 >= (int64_t(1) << 31))
                    a_parent = false;
                pwords += double(pr.NA) * double(pr.NA);
                apars.push_back(ap);
                idx = int(apars.size()) - 1;
            }
            apar_of[q] = idx;
        }
        a_parent = a_parent && want != 0 && (want == 1 || words >= pwords);
        // within the context's workspace limit: the parents' panels and the
        // products' B panels (whose depth grows by at most one k-block)
        if (a_parent && ctx->ws_limit) {
            size_t need = 0;
            for (const AParent &ap : apars)
                need += align256(size_t(ap.nslab + kAParentGuard) * size_t(ap.nkbp) * size_t(L) *
                                 1024);
            for (const Plan &pl : plans0)
                need += align256(size_t(pl.pcol) * size_t(pl.kpad + 64) * size_t(L));
            if (need + 256 > ctx->ws_limit) a_parent = false;
        }
    }
    // The early-C epilogue addresses C rows at any phase, so the row shift
    // need not align the output blocks with C's tile rows: none (fewer
    // padded rows), or A's slab phase.  The column shift stays: with C's
    // columns on its tile grid, each row of a wave's 32 outputs is one
    // 128-byte line.
    std::vector<Plan> shifted;
    if (early_c) {
        shifted = plans0;
        for (Plan &pl : shifted) {
            pl.sr = a_parent ? pl.pr.ra % 32 : 0;
            pl.row0C = pl.pr.rc - pl.sr;
            pl.prow = (pl.sr + pl.pr.m + pl.tile_m - 1) / pl.tile_m * pl.tile_m;
            pl.grid_m = pl.prow / pl.tile_m;
        }
    }
    const std::vector<Plan> &plans = early_c ? shifted : plans0;

    // Longest-processing-time order: every output block of a product costs
    // its k, so products with the longest k go first.  In that order each
    // product joins the XCD group with the least work so far (blocks x k);
    // the queue then holds the groups one after another, each in LPT order.
    std::vector<size_t> order(plans.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return plans[a].kpad > plans[b].kpad; });
    std::vector<int> grp(plans.size());
    double work[kXcdGroups] = {};
    int64_t group_tiles[kXcdGroups] = {}, group_calls[kXcdGroups] = {};
    for (size_t i : order) {
        int g = 0;
        for (int h = 1; h < kXcdGroups; ++h)
            if (work[h] < work[g]) g = h;
        const int64_t tiles = plans[i].grid_m * plans[i].grid_n;
        grp[i] = g;
        work[g] += double(tiles) * double(plans[i].kpad);
        group_tiles[g] += tiles;
        group_calls[g] += 1;
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return grp[a] < grp[b]; });

    // GEMM k-blocks of each product (A-parent form: from the phase of ca)
    std::vector<int64_t> nkbs(plans.size());
    for (size_t q = 0; q < plans.size(); ++q) {
        const Product &pr = plans[q].pr;
        nkbs[q] = a_parent ? (pr.ca % 32 + pr.k + 63) / 64 * 2 : plans[q].kpad / 32;
    }

    // Panels in the context workspace: the parents' (A-parent form), then
    // every product's own.
    std::vector<size_t> aoff(plans.size()), boff(plans.size());
    size_t total = 0;
    if (a_parent)
        for (AParent &ap : apars) {
            const size_t slab = size_t(ap.nkbp) * size_t(L) * 1024;
            ap.off = total;
            total += align256((size_t(ap.nslab) + size_t(kAParentGuard)) * slab);
        }
    for (size_t q = 0; q < plans.size(); ++q) {
        const Plan &pl = plans[q];
        const size_t nkb = size_t(nkbs[q]);
        aoff[q] = a_parent ? apars[apar_of[q]].off : total;
        if (!a_parent) total += align256(size_t(pl.prow) * nkb * 32 * L);
        boff[q] = total;
        total += align256(size_t(pl.pcol) * nkb * 32 * L);
    }
    const int64_t ncalls = int64_t(plans.size());
    mh_status s = ensure_queue(ctx, ncalls);
    if (s != MH_OK) return s;
    char *ws = (char *)workspace(ctx, total + 256);
    if (!ws) return MH_E_NOMEM;
    BatchedState &b = ctx->batched;

    // The staging buffer may still be read by the previous batch's copy.
    if (hipEventSynchronize(b.staging_free) != hipSuccess) return note_error(ctx, hipErrorUnknown);
    const QueueView hq = queue_view(b.queue_host, b.queue_cap);
    int64_t pack_total = 0, tile_total = 0;
    for (int64_t q = 0; q < ncalls; ++q) {
        const Plan &pl = plans[order[q]];
        const Product &pr = pl.pr;
        const int64_t nkb = nkbs[order[q]];
        int8_t *Ap = (int8_t *)(ws + aoff[order[q]]);
        int8_t *Bp = (int8_t *)(ws + boff[order[q]]);
        const int32_t kshift = a_parent ? int32_t(pr.ca % 32) : 0;
        // A panels are tasks [0, ncalls), B panels [ncalls, 2 ncalls); in the
        // A-parent form the first A tasks pack the parents and the rest are empty
        if (!a_parent)
            hq.packs[q] =
                PackTask{pr.A, Ap, pr.ra, pr.ca, pl.sr, pr.m, pr.k, pl.prow, nkb, 0, pr.logT, 0, 0};
        else if (q < int64_t(apars.size()))
            hq.packs[q] = PackTask{apars[q].A, (int8_t *)(ws + apars[q].off), 0, 0, 0,
                                   apars[q].N, apars[q].N, apars[q].nslab * 32, apars[q].nkbp,
                                   0, pr.logT, 0, 0};
        else
            hq.packs[q] = PackTask{nullptr, nullptr, 0, 0, 0, 0, 0, 0, 0, 0, pr.logT, 0, 0};
        hq.packs[ncalls + q] = PackTask{pr.B, Bp, pr.rb, pr.cb, pl.sc, pr.n, pr.k, pl.pcol, nkb,
                                        1, pr.logT, pl.sub ? 1 : 0, kshift};
        LimbArgs &a = hq.calls[q];
        std::memset(&a, 0, sizeof(a));
        a.Ap = Ap;
        a.Bp = Bp;
        a.nkb = nkb;
        a.kb_per_red = pl.kblock / 32;
        a.C = c_override ? c_override : pr.C;
        a.row0C = pl.row0C;
        a.col0C = pl.col0C;
        a.sr = pl.sr;
        a.sc = pl.sc;
        a.m = pr.m;
        a.n = pr.n;
        a.grid_m = pl.grid_m;
        a.grid_n = pl.grid_n;
        a.p = p;
        a.mu = ~uint64_t(0) / p;
        a.bias = ((uint64_t(1) << 31) + p - 1) / p * p;
        a.pinv = 1.0 / double(p);
        a.logT = pr.logT;
        if (a_parent) {
            const AParent &ap = apars[apar_of[order[q]]];
            a.a_slab0 = (pr.ra - pl.sr) / 32;  // (ra - sr is a multiple of 32)
            a.a_kb0 = pr.ca / 32;
            a.a_nkbp = ap.nkbp;
        }
        hq.tile_prefix[q] = tile_total;
        tile_total += pl.grid_m * pl.grid_n;
    }
    for (int64_t t = 0; t < 2 * ncalls; ++t) {
        const PackTask &pt = hq.packs[t];
        hq.pack_prefix[t] = pack_total;
        pack_total += (pt.prow / 64) * ((pt.nkb + 1) / 2);
    }
    hq.pack_prefix[2 * ncalls] = pack_total;
    hq.tile_prefix[ncalls] = tile_total;
    BatchHeader &h = *hq.hdr;
    std::memset(&h, 0, sizeof(h));
    h.npack = 2 * ncalls;
    h.ncalls = ncalls;
    h.pack_chunks = pack_total;
    h.gemm_tiles = tile_total;
    h.p = p;
    h.L = L;
    int64_t first_call = 0;
    for (int g = 0; g < kXcdGroups; ++g) {
        h.group_tile[g + 1] = h.group_tile[g] + group_tiles[g];
        h.group_call[g] = std::min<int64_t>(first_call, ncalls - 1);  // unused if empty
        first_call += group_calls[g];
    }

    hipGraphExec_t exec = ensure_graph(ctx, cfg, L, early_c, a_parent);
    if (!exec) return MH_E_DEVICE;
    hipError_t e = hipMemcpyAsync(b.queue_dev, b.queue_host, queue_bytes(b.queue_cap),
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(b.staging_free, stream);
    if (e != hipSuccess) return note_error(ctx, e);
    TimedLaunch t;
    record_start(ctx, MH_K_BATCHED, stream, t);
    e = hipGraphLaunch(exec, stream);
    record_end(ctx, stream, t);
    if (e == hipSuccess && !c_override) {
        b.last_cfg = cfg;
        b.last_L = L;
        b.last_forms = (early_c ? MH_BATCH_FORM_EARLY_C : 0) |
                       (a_parent ? MH_BATCH_FORM_A_PARENT : 0);
    }
    return note_error(ctx, e);
}

}  // namespace mh

using namespace mh;

extern "C" mh_status mh_ctx_last_batch_config(mh_ctx *ctx, int32_t *cfg, int32_t *limbs,
                                               int32_t *forms)
{
    if (!ctx) return MH_E_INVALID;
    if (cfg) *cfg = ctx->batched.last_cfg;
    if (limbs) *limbs = ctx->batched.last_L;
    if (forms) *forms = ctx->batched.last_forms;
    return MH_OK;
}

// Validation of a batched call, host only: every product as for a single
// call, then the aliasing rule over the whole batch.
static mh_status validate_batch(const mh_mm_desc *d, int32_t count, uint32_t p, int32_t T,
                                int32_t mode, std::vector<Product> &prods, int &form, bool &sub)
{
    if (count < 0 || (count > 0 && !d)) return MH_E_INVALID;
    if (!parse_mode(mode, form, sub)) return MH_E_UNSUPPORTED;
    if (!valid_T(T)) return MH_E_UNSUPPORTED;
    if (p < 2u || p > 0x7FFFFFFFu) return MH_E_MODULUS;
    if (check_form_modulus(form, p) != MH_OK) return MH_E_MODULUS;
    // Validate every product first: a failing call has no effect.
    prods.assign(size_t(count), Product{});
    for (int32_t i = 0; i < count; ++i) {
        Product &pr = prods[i];
        pr.C = d[i].C;
        pr.A = d[i].A;
        pr.B = d[i].B;
        pr.NC = d[i].NC;
        pr.NA = d[i].NA;
        pr.NB = d[i].NB;
        pr.rc = d[i].rc;
        pr.cc = d[i].cc;
        pr.ra = d[i].ra;
        pr.ca = d[i].ca;
        pr.rb = d[i].rb;
        pr.cb = d[i].cb;
        pr.m = d[i].m;
        pr.k = d[i].k;
        pr.n = d[i].n;
        pr.p = p;
        pr.T = T;
        pr.logT = log2i(T);
        mh_status s = validate_product(pr, true);
        if (s != MH_OK) return s;
    }
    // No output block may overlap another output block or any input block.
    return check_batch_aliasing(prods);
}

extern "C" mh_status mh_validate_batch(const mh_mm_desc *d, int32_t count, uint32_t p, int32_t T,
                                       int32_t mode)
{
    std::vector<Product> prods;
    int form;
    bool sub;
    return validate_batch(d, count, p, T, mode, prods, form, sub);
}

extern "C" mh_status mh_matmul_modp_batched(mh_ctx *ctx, const mh_mm_desc *d, int32_t count,
                                            uint32_t p, int32_t T, int32_t mode,
                                            hipStream_t stream)
{
    if (!ctx) return MH_E_INVALID;
    std::vector<Product> prods;
    int form;
    bool sub;
    if (mh_status st = validate_batch(d, count, p, T, mode, prods, form, sub); st != MH_OK)
        return st;
    mode = form;
    DeviceGuard g(ctx->device);
    std::vector<int32_t> live;
    for (int32_t i = 0; i < count; ++i)
        if (prods[i].m > 0 && prods[i].n > 0 && prods[i].k > 0) live.push_back(i);
    if (live.empty()) return MH_OK;
    CtxUse use(ctx, stream);

    if (mode != MH_MODE_AUTO && mode != MH_MODE_LIMB_I8) {
        // The plain, FP64 and elementwise forms have no batched kernel:
        // products run one after another.
        for (int32_t i : live) {
            mh_status s = run_product(ctx, prods[i], mode, sub, WsSource{}, stream);
            if (s != MH_OK) return s;
        }
        return MH_OK;
    }

    const int L = limbs_for(p);
    std::vector<Plan> plans(live.size());
    for (size_t q = 0; q < live.size(); ++q) plan_product(prods[live[q]], MH_MODE_LIMB_I8, plans[q]);
    const size_t cap = ctx->ws_limit ? ctx->ws_limit : SIZE_MAX;
    size_t total = 0;
    for (const Plan &pl : plans) total += plan_ws_bytes(pl);
    int cfg = -1;
    if (ctx->autotune) {
        cfg = tune_get(ctx, tune_key_batch(L, T, plans));
        if (cfg < 0 && ctx->autotune == 2 && total <= cap) cfg = tune_batch(ctx, plans, L, p, stream);
    }
    if (!limb_cfg_fits(L, cfg)) cfg = batch_cfg(L, plans);  // none cached, or unusable for L
    for (size_t q = 0; q < live.size(); ++q) {
        plan_product(prods[live[q]], MH_MODE_LIMB_I8, plans[q], cfg);
        plans[q].sub = sub;
    }
    // Within the workspace limit: consecutive runs of products whose panels
    // fit together go out as one batched graph each; a product whose own
    // panels exceed the limit runs alone in chunks (run_product).
    std::vector<Plan> part;
    size_t part_bytes = 0;
    auto flush_part = [&]() -> mh_status {
        if (part.empty()) return MH_OK;
        mh_status s = launch_batch(ctx, part, cfg, L, p, stream, nullptr);
        part.clear();
        part_bytes = 0;
        return s;
    };
    for (size_t q = 0; q < plans.size(); ++q) {
        const size_t need = plan_ws_bytes(plans[q]);
        if (need > cap) {
            mh_status s = run_product(ctx, prods[live[q]], MH_MODE_LIMB_I8, sub, WsSource{}, stream);
            if (s != MH_OK) return s;
            continue;
        }
        if (part_bytes + need > cap) {
            mh_status s = flush_part();
            if (s != MH_OK) return s;
        }
        part.push_back(plans[q]);
        part_bytes += need;
    }
    return flush_part();
}
