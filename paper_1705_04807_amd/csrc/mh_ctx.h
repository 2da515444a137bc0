// The context object behind the opaque mh_ctx handle, and host helpers
// shared by the host runtime files.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "mh_internal.h"

namespace mh {

struct TimedLaunch {
    hipEvent_t a, b;
    int kernel;
};

// State of the batched path (persistent kernels, queue, graph).
struct BatchedState {
    void *queue_dev = nullptr;          // device copy of the task queue
    void *queue_host = nullptr;         // pinned staging buffer of the same layout
    int64_t queue_cap = 0;              // products the queue buffers hold
    hipEvent_t staging_free = nullptr;  // recorded after the last host-to-device queue copy
    uint64_t *counters = nullptr;       // device work counters (pack, GEMM)
    hipStream_t capture_stream = nullptr;
    // One captured graph per (kernel configuration, limbs, C-load form of
    // the GEMM): a batch whose key differs from the previous one's replays
    // its own graph, so
    // no graph is destroyed while a launch of it may still run.  All of them
    // embed the queue's address and are destroyed together when the queue
    // is reallocated (after the context's work has drained).
    struct Captured {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::map<int, Captured> graphs;
    int last_cfg = -1;                  // configuration, limbs and GEMM forms of the
    int last_L = 0;                     //   last batched graph
    int last_forms = 0;
};

struct DeviceGuard {
    int prev;
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
};

mh_status note_error(mh_ctx *ctx, hipError_t e);

// Ordering of the calls of one context.  Every call that uses memory the
// context owns (workspace panels, the batch queue, tuning scratch) runs
// between use_begin and use_end on its stream: use_begin makes the stream
// wait for the previous such call when that one ran on another stream, and
// use_end records the context's last-use event there.  So the calls of a
// context are ordered even across streams, and drain (a host wait on that
// one event) covers all of the context's work without synchronising the
// whole device.
void use_begin(mh_ctx *ctx, hipStream_t s);
void use_end(mh_ctx *ctx, hipStream_t s);
mh_status drain(mh_ctx *ctx);
struct CtxUse {
    mh_ctx *ctx;
    hipStream_t s;
    CtxUse(mh_ctx *c, hipStream_t st) : ctx(c), s(st) { use_begin(ctx, s); }
    ~CtxUse() { use_end(ctx, s); }
};
// Inside a call that must not allocate, timing is off (it would create HIP
// events).
struct NoTiming {
    mh_ctx *ctx;
    explicit NoTiming(mh_ctx *c);
    ~NoTiming();
};
void record_start(mh_ctx *ctx, int kernel, hipStream_t s, TimedLaunch &t);
void record_end(mh_ctx *ctx, hipStream_t s, TimedLaunch &t);
void *workspace(mh_ctx *ctx, size_t bytes);
// Device memory for a product's panels: the context's growing workspace
// (fixed == nullptr), or a fixed buffer of `cap` bytes that is never grown.
struct WsSource {
    char *fixed = nullptr;
    size_t cap = 0;  // bytes usable; for the context's workspace, its limit (0: none)
};
size_t plan_ws_bytes(const Plan &pl);
char *ws_get(mh_ctx *ctx, const WsSource &src, size_t bytes);
mh_status run_product(mh_ctx *ctx, const Product &pr, int form, bool sub, const WsSource &src,
                      hipStream_t s);
bool outputs_alias(const Product &x, const Product &y);
Product make_product(uint32_t *C, int64_t NC, int64_t rc, int64_t cc, const uint32_t *A,
                     int64_t NA, int64_t ra, int64_t ca, const uint32_t *B, int64_t NB,
                     int64_t rb, int64_t cb, int64_t m, int64_t k, int64_t n, uint32_t p,
                     int32_t T);
// Panel scratch of the no-allocation entry point (mh_noalloc.hip): its size,
// and its device address on `device` (looked up once per device with that
// device current; nullptr if unavailable).
size_t noalloc_scratch_bytes();
void *noalloc_scratch_init(int device);
void batched_release(mh_ctx *ctx);
mh_status run_plain(mh_ctx *ctx, const Plan &pl, char *ws, hipStream_t s);
mh_status run_limb(mh_ctx *ctx, const Plan &pl, char *ws, hipStream_t s);
mh_status launch_batch(mh_ctx *ctx, const std::vector<Plan> &plans, int cfg, int L, uint32_t p,
                       hipStream_t stream, uint32_t *c_override);

// Autotuner (mh_tune.cpp).
struct TuneEntry {
    int cfg;
    double ms;
};
std::string tune_key_single(int L, const Product &p);
std::string tune_key_batch(int L, int T, const std::vector<Plan> &plans);
int tune_get(mh_ctx *ctx, const std::string &key);
int tune_single(mh_ctx *ctx, const Product &p, hipStream_t s);
int tune_batch(mh_ctx *ctx, std::vector<Plan> &plans, int L, uint32_t p, hipStream_t s);

}  // namespace mh

struct mh_ctx {
    int device = 0;
    int num_cu = 256;
    void *ws = nullptr;
    size_t ws_size = 0;
    bool timing = false;
    std::vector<mh::TimedLaunch> records;
    std::vector<hipEvent_t> event_pool;
    mh_status sticky = MH_OK;
    mh::BatchedState batched;
    int autotune = 0;                          // 0 off, 1 cached choices, 2 tune on first use
    std::map<std::string, mh::TuneEntry> tune; // shape bucket -> configuration
    void *tune_scratch = nullptr;              // output parent for tuning runs
    size_t tune_scratch_size = 0;
    size_t ws_limit = 0;                       // largest workspace (bytes) a call may hold; 0: none
    hipEvent_t last_use = nullptr;             // see use_begin / use_end
    hipStream_t last_stream = nullptr;
    bool used = false;
    bool in_call = false;                      // between use_begin and use_end
    hipStream_t cur_stream = nullptr;          // the current call's stream
    void *noalloc_ws = nullptr;                // device address of the no-allocation scratch
    bool no_timing = false;                    // inside mh_matmul_modp_noalloc
};

inline mh::NoTiming::NoTiming(mh_ctx *c) : ctx(c) { ctx->no_timing = true; }
inline mh::NoTiming::~NoTiming() { ctx->no_timing = false; }
