// Diagnostics: the rates this device sustains for the two arithmetic
// paths, int8 MFMA and the plain kernel's 96-bit VALU multiply-accumulate.
//
// The published int8 peak assumes the full engine clock.  Under a dense
// int8 MFMA load on random operands the device lowers its clock to stay
// within its power limit, so the rate a GEMM can approach is lower.  The
// MFMA probe measures that ceiling: every wave keeps eight independent
// 32x32 accumulators busy with v_mfma_i32_32x32x32_i8 on random operands
// held in registers and rotated from one MFMA to the next (so the
// multipliers see new random bytes each time, as in a GEMM), with no memory
// traffic inside the loop.  The sums are written out so that nothing is
// optimised away.
#include "mh_ctx.h"
#include "mh_device.h"
#include "mh_mac.h"

namespace mh {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint32_t hash32(uint32_t x)
{
    // 32-bit integer hash (lowbias32 constants)
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

constexpr int kProbeThreads = 256;  // four waves: one per SIMD of a compute unit

__global__ __launch_bounds__(kProbeThreads) void k_probe_mfma_i8(int32_t pairs, uint32_t seed,
                                                                 int32_t *out)
{
    v4i a[8], b[8];
    uint32_t h = hash32(seed * 7919u + blockIdx.x * kProbeThreads + threadIdx.x);
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 4; ++j) {
            h = hash32(h + 0x9e3779b9u);
            a[i][j] = int32_t(h);
            h = hash32(h + 0x9e3779b9u);
            b[i][j] = int32_t(h);
        }
    v16i acc[8];
    for (int i = 0; i < 8; ++i) acc[i] = v16i{0};
    for (int32_t it = 0; it < pairs; ++it) {
        static_for<8>([&](auto i) {
            acc[i] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[(i + 1) & 7], acc[i], 0, 0, 0);
        });
        static_for<8>([&](auto i) {
            acc[i] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[(i + 3) & 7], b[(i + 6) & 7], acc[i],
                                                           0, 0, 0);
        });
    }
    int32_t s = 0;
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 16; ++j) s += acc[i][j];
    out[blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

// The plain kernel's multiply-accumulate pair (mac4: v_mad_u64_u32 +
// v_addc_co_u32), sixteen independent 96-bit accumulators per lane, no
// memory traffic in the loop.
constexpr int kValuThreads = 256;
constexpr int kValuGroupsPerCu = 8;  // eight waves per SIMD

__global__ __launch_bounds__(kValuThreads) void k_probe_valu_mac(int32_t iters, uint32_t seed,
                                                                 uint64_t *out)
{
    uint64_t lo[4][4] = {};
    uint32_t hi[4][4] = {};
    uint32_t h = hash32(seed * 7919u + blockIdx.x * kValuThreads + threadIdx.x);
    uint32_t a[4], b[4];
    for (int i = 0; i < 4; ++i) {
        h = hash32(h + 0x9e3779b9u);
        a[i] = h;
        h = hash32(h + 0x9e3779b9u);
        b[i] = h;
    }
    for (int32_t it = 0; it < iters; ++it) {
        static_for<4>([&](auto i) { mac4(lo[i], hi[i], a[i], b); });
    }
    uint64_t s = 0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) s += lo[i][j] + hi[i][j];
    out[blockIdx.x * kValuThreads + threadIdx.x] = s;
}

}  // namespace

// Runs launch(1) untimed (the clock settles under the load), then launch(2)
// bracketed by HIP events on `stream`; ms receives the timed duration.
template <typename F>
hipError_t time_twice(hipStream_t stream, F launch, float &ms)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch(1u);
    if (e == hipSuccess) e = hipEventRecord(e0, stream);
    if (e == hipSuccess) e = launch(2u);
    if (e == hipSuccess) e = hipEventRecord(e1, stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return e;
}

}  // namespace mh

using namespace mh;

extern "C" mh_status mh_probe_mfma_i8(mh_ctx *ctx, int32_t iters, double *pops,
                                      hipStream_t stream)
{
    if (!ctx || !pops || iters < 2 || (iters & 1) || iters > (1 << 24)) return MH_E_INVALID;
    DeviceGuard g(ctx->device);
    const int grid = ctx->num_cu;
    int32_t *out = nullptr;
    if (hipMalloc((void **)&out, size_t(grid) * kProbeThreads * sizeof(int32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return MH_E_NOMEM;
    }
    float ms = 0.0f;
    const hipError_t e = time_twice(
        stream,
        [&](uint32_t seed) {
            hipLaunchKernelGGL(k_probe_mfma_i8, dim3(grid), dim3(kProbeThreads), 0, stream,
                               iters / 2, seed, out);
            return hipGetLastError();
        },
        ms);
    (void)hipFree(out);
    if (e != hipSuccess) return note_error(ctx, e);
    if (!(ms > 0.0f)) return MH_E_DEVICE;
    // 16 MFMAs per pair and wave, 2 x 32^3 int8 operations each
    const double waves = double(grid) * (kProbeThreads / 64);
    *pops = 2.0 * 32 * 32 * 32 * 8.0 * double(iters) * waves / (double(ms) * 1e-3);
    return MH_OK;
}

extern "C" mh_status mh_probe_valu_mac(mh_ctx *ctx, int32_t iters, double *macs,
                                       hipStream_t stream)
{
    if (!ctx || !macs || iters < 1 || iters > (1 << 24)) return MH_E_INVALID;
    DeviceGuard g(ctx->device);
    const int grid = ctx->num_cu * kValuGroupsPerCu;
    uint64_t *out = nullptr;
    if (hipMalloc((void **)&out, size_t(grid) * kValuThreads * sizeof(uint64_t)) != hipSuccess) {
        (void)hipGetLastError();
        return MH_E_NOMEM;
    }
    float ms = 0.0f;
    const hipError_t e = time_twice(
        stream,
        [&](uint32_t seed) {
            hipLaunchKernelGGL(k_probe_valu_mac, dim3(grid), dim3(kValuThreads), 0, stream,
                               iters, seed, out);
            return hipGetLastError();
        },
        ms);
    (void)hipFree(out);
    if (e != hipSuccess) return note_error(ctx, e);
    if (!(ms > 0.0f)) return MH_E_DEVICE;
    // 16 multiply-accumulates per iteration and lane
    *macs = 16.0 * double(iters) * double(grid) * kValuThreads / (double(ms) * 1e-3);
    return MH_OK;
}
