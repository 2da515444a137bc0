// Diagnostics: the int8 MFMA rate this device sustains.
//
// The published int8 peak assumes the full engine clock.  Under a dense
// int8 MFMA load on random operands the device lowers its clock to stay
// within its power limit, so the rate a GEMM can approach is lower.  This
// kernel measures that ceiling: every wave keeps eight independent
// 32x32 accumulators busy with v_mfma_i32_32x32x32_i8 on random operands
// held in registers and rotated from one MFMA to the next (so the
// multipliers see new random bytes each time, as in a GEMM), with no memory
// traffic inside the loop.  The sums are written out so that nothing is
// optimised away.
#include "mh_ctx.h"
#include "mh_device.h"

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

}  // namespace

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
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float ms = 0.0f;
    if (e == hipSuccess) {
        // untimed launch of the same size: clocks settle under the load
        hipLaunchKernelGGL(k_probe_mfma_i8, dim3(grid), dim3(kProbeThreads), 0, stream,
                           iters / 2, 1u, out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e0, stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_probe_mfma_i8, dim3(grid), dim3(kProbeThreads), 0, stream,
                           iters / 2, 2u, out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (e != hipSuccess) return note_error(ctx, e);
    if (!(ms > 0.0f)) return MH_E_DEVICE;
    // 16 MFMAs per pair and wave, 2 x 32^3 int8 operations each
    const double waves = double(grid) * (kProbeThreads / 64);
    *pops = 2.0 * 32 * 32 * 32 * 8.0 * double(iters) * waves / (double(ms) * 1e-3);
    return MH_OK;
}
