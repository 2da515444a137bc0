// Autotuner: per shape bucket, the limb GEMM configuration (workgroup
// tile, wave tile, pipeline depth, LDS sharing) that ran fastest on this
// device, measured with HIP events on the caller's data, kept in the
// context and persisted as a small JSON file.
//
// Buckets: a single product by (limbs, T, ceil(log2) of m, k, n); a batch by
// (limbs, T, ceil(log2) of its mean output area and of its mean k).  The
// paper fixes its truncation size by citation (T' = 32, section 2.2
// performance analysis); here T is the caller's, and the tuner chooses the
// GPU-side blocking around it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mh_ctx.h"
#include "mh_internal.h"

namespace mh {

namespace {

int clog2(double x)
{
    int l = 0;
    while (double(int64_t(1) << l) < x && l < 62) ++l;
    return l;
}

std::string device_tag(mh_ctx *ctx)
{
    hipDeviceProp_t prop;
    char buf[160];
    if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess) return "unknown";
    int rt = 0;
    (void)hipRuntimeGetVersion(&rt);
    std::snprintf(buf, sizeof(buf), "%s cu=%d hip=%d", prop.gcnArchName, prop.multiProcessorCount,
                  rt);
    for (char *c = buf; *c; ++c)
        if (*c == '"' || *c == '\\') *c = '_';
    return buf;
}


// Scratch output parent for tuning runs (the caller's C is never written).
uint32_t *tune_scratch(mh_ctx *ctx, int64_t N)
{
    const size_t bytes = size_t(N) * size_t(N) * 4;
    if (bytes > ctx->tune_scratch_size) {
        (void)drain(ctx);
        if (ctx->tune_scratch) (void)hipFree(ctx->tune_scratch);
        ctx->tune_scratch = nullptr;
        ctx->tune_scratch_size = 0;
        if (hipMalloc(&ctx->tune_scratch, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        ctx->tune_scratch_size = bytes;
    }
    return (uint32_t *)ctx->tune_scratch;
}

// Average time (ms) of `reps` runs of f on stream s, after one warm-up run.
template <class F>
double time_ms(hipStream_t s, F &&f, int reps)
{
    if (f() != MH_OK) return -1.0;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.0;
    (void)hipEventRecord(a, s);
    bool ok = true;
    for (int r = 0; r < reps && ok; ++r) ok = f() == MH_OK;
    (void)hipEventRecord(b, s);
    float ms = -1.f;
    if (ok && hipEventSynchronize(b) == hipSuccess) (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ok ? double(ms) / reps : -1.0;
}

}  // namespace

std::string tune_key_single(int L, const Product &p)
{
    char buf[128];
    std::snprintf(buf, sizeof(buf), "single L=%d T=%d m=%d k=%d n=%d", L, p.T, clog2(double(p.m)),
                  clog2(double(p.k)), clog2(double(p.n)));
    return buf;
}

std::string tune_key_batch(int L, int T, const std::vector<Plan> &plans)
{
    double area = 0.0, k = 0.0;
    for (const Plan &q : plans) {
        area += double(q.pr.m) * double(q.pr.n);
        k += double(q.pr.k);
    }
    const double n = double(std::max<size_t>(plans.size(), 1));
    char buf[128];
    std::snprintf(buf, sizeof(buf), "batch L=%d T=%d area=%d k=%d", L, T, clog2(area / n),
                  clog2(k / n));
    return buf;
}

int tune_get(mh_ctx *ctx, const std::string &key)
{
    auto it = ctx->tune.find(key);
    return it == ctx->tune.end() ? -1 : it->second.cfg;
}

void tune_put(mh_ctx *ctx, const std::string &key, int cfg, double ms)
{
    ctx->tune[key] = TuneEntry{cfg, ms};
}

// Time every configuration that fits L on product p (output redirected to a
// scratch parent); returns the fastest.  Synchronises the stream.
int tune_single(mh_ctx *ctx, const Product &p, hipStream_t s)
{
    const int L = limbs_for(p.p);
    Product q = p;
    q.C = tune_scratch(ctx, p.NC);
    if (!q.C) return -1;
    const bool timing = ctx->timing;
    ctx->timing = false;
    int best = -1;
    double best_ms = 0.0;
    for (int cfg = 0; cfg < limb_cfg_count(); ++cfg) {
        if (!limb_cfg_fits(L, cfg)) continue;
        Plan pl;
        plan_product(q, MH_MODE_LIMB_I8, pl, cfg);
        const size_t need = plan_ws_bytes(pl);
        if (ctx->ws_limit && need > ctx->ws_limit) continue;  // would not run unchunked
        char *ws = (char *)workspace(ctx, need);
        if (!ws) continue;
        const double ms = time_ms(s, [&] { return run_limb(ctx, pl, ws, s); }, 2);
        if (ms > 0.0 && (best < 0 || ms < best_ms)) {
            best = cfg;
            best_ms = ms;
        }
    }
    ctx->timing = timing;
    if (best >= 0) tune_put(ctx, tune_key_single(L, p), best, best_ms);
    return best;
}

// Same for a batch: each configuration runs the whole batched graph with
// every output redirected to one scratch parent.
int tune_batch(mh_ctx *ctx, std::vector<Plan> &plans, int L, uint32_t p, hipStream_t s)
{
    int64_t nmax = 0;
    for (const Plan &q : plans) nmax = std::max(nmax, q.pr.NC);
    uint32_t *scratch = tune_scratch(ctx, nmax);
    if (!scratch) return -1;
    const bool timing = ctx->timing;
    ctx->timing = false;
    int best = -1;
    double best_ms = 0.0;
    for (int cfg = 0; cfg < limb_cfg_count(); ++cfg) {
        if (!limb_cfg_fits(L, cfg)) continue;
        for (Plan &q : plans) {
            const bool sub = q.sub;
            plan_product(q.pr, MH_MODE_LIMB_I8, q, cfg);
            q.sub = sub;
        }
        const double ms =
            time_ms(s, [&] { return launch_batch(ctx, plans, cfg, L, p, s, scratch); }, 2);
        if (ms > 0.0 && (best < 0 || ms < best_ms)) {
            best = cfg;
            best_ms = ms;
        }
    }
    ctx->timing = timing;
    if (best >= 0) tune_put(ctx, tune_key_batch(L, plans.empty() ? 64 : plans[0].pr.T, plans),
                            best, best_ms);
    return best;
}

}  // namespace mh

using namespace mh;

extern "C" mh_status mh_ctx_set_autotune(mh_ctx *ctx, int mode)
{
    if (!ctx || mode < 0 || mode > 2) return MH_E_INVALID;
    ctx->autotune = mode;
    return MH_OK;
}

extern "C" mh_status mh_ctx_tune_lookup(mh_ctx *ctx, uint32_t p, int32_t T, int64_t m, int64_t k,
                                        int64_t n, int32_t *cfg)
{
    if (!ctx || !cfg) return MH_E_INVALID;
    Product pr{};
    pr.p = p;
    pr.T = T;
    pr.m = m;
    pr.k = k;
    pr.n = n;
    *cfg = tune_get(ctx, tune_key_single(limbs_for(p), pr));
    return MH_OK;
}

extern "C" mh_status mh_ctx_tune_cache_save(mh_ctx *ctx, const char *path)
{
    if (!ctx || !path) return MH_E_INVALID;
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return MH_E_INVALID;
    std::fprintf(f, "{\"format\": \"mh-tune-1\", \"device\": \"%s\",\n \"entries\": [\n",
                 device_tag(ctx).c_str());
    size_t i = 0;
    for (auto &e : ctx->tune)
        std::fprintf(f, "  {\"key\": \"%s\", \"cfg\": %d, \"ms\": %.6f}%s\n", e.first.c_str(),
                     e.second.cfg, e.second.ms, ++i < ctx->tune.size() ? "," : "");
    std::fprintf(f, " ]}\n");
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path) != 0) return MH_E_INVALID;
    return MH_OK;
}

extern "C" mh_status mh_ctx_tune_cache_load(mh_ctx *ctx, const char *path, int32_t *loaded)
{
    if (!ctx || !path) return MH_E_INVALID;
    if (loaded) *loaded = 0;
    FILE *f = std::fopen(path, "r");
    if (!f) return MH_E_INVALID;
    const std::string want = "\"device\": \"" + device_tag(ctx) + "\"";
    char line[512];
    bool device_ok = false;
    int32_t n = 0;
    while (std::fgets(line, sizeof(line), f)) {
        if (std::strstr(line, "\"device\"")) device_ok = std::strstr(line, want.c_str()) != nullptr;
        const char *k = std::strstr(line, "{\"key\": \"");
        if (!k || !device_ok) continue;
        k += 9;
        const char *e = std::strchr(k, '"');
        if (!e) continue;
        std::string key(k, e - k);
        int cfg = -1;
        double ms = 0.0;
        if (std::sscanf(e, "\", \"cfg\": %d, \"ms\": %lf", &cfg, &ms) == 2 && cfg >= 0 &&
            cfg < limb_cfg_count()) {
            ctx->tune[key] = TuneEntry{cfg, ms};
            ++n;
        }
    }
    std::fclose(f);
    if (loaded) *loaded = n;
    return MH_OK;
}
