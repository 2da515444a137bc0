// mh_matmul_modp_noalloc: the single product of mh_matmul_modp with its
// operand panels in a fixed device array of this file instead of the
// context's growing workspace, for callers that cannot allocate device
// memory.  The kernels are the ones mh_matmul_modp launches; they receive
// the array's device address as their panel pointer.
#include "mh_ctx.h"

#include <mutex>

namespace mh {

namespace {

constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kMaxDevices = 64;

// Panel scratch: one copy per GPU the library runs on, held until the
// process ends.  In host code its name is only a stand-in for the symbol;
// kernels get the device address obtained below.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_lock;
void *g_addr[kMaxDevices];
bool g_done[kMaxDevices];

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

// Device address of `scratch` on `device` (nullptr if it cannot be had).
// Looked up once per device, with that device current; the caller (context
// creation) has made it current.
void *noalloc_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_lock);
    if (!g_done[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            ptr = nullptr;
        }
        g_addr[device] = ptr;
        g_done[device] = true;
    }
    return g_addr[device];
}

}  // namespace mh

extern "C" mh_status mh_matmul_modp_noalloc(mh_ctx *ctx, uint32_t *C, int64_t NC, int64_t rc,
                                            int64_t cc, const uint32_t *A, int64_t NA,
                                            int64_t ra, int64_t ca, const uint32_t *B,
                                            int64_t NB, int64_t rb, int64_t cb, int64_t m,
                                            int64_t k, int64_t n, uint32_t p, int32_t T,
                                            int32_t mode, hipStream_t stream)
{
    using namespace mh;
    if (!ctx) return MH_E_INVALID;
    int form;
    bool sub;
    if (!parse_mode(mode, form, sub)) return MH_E_UNSUPPORTED;
    Product pr = make_product(C, NC, rc, cc, A, NA, ra, ca, B, NB, rb, cb, m, k, n, p, T);
    mh_status s = validate_product(pr, true);
    if (s == MH_OK) s = check_form_modulus(form, p);
    if (s != MH_OK) return s;
    if (m == 0 || n == 0 || k == 0) return MH_OK;
    if (!ctx->noalloc_ws) return MH_E_DEVICE;
    DeviceGuard g(ctx->device);
    NoTiming quiet(ctx);  // timing would create HIP events
    CtxUse use(ctx, stream);
    return run_product(ctx, pr, form, sub,
                       WsSource{static_cast<char *>(ctx->noalloc_ws), kScratchBytes}, stream);
}
