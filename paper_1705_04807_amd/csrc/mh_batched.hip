// Batched products (placeholder: one product after another).
#include "mh_ctx.h"
#include "mh_device.h"

namespace mh {

void batched_release(mh_ctx *ctx) { (void)ctx; }

}  // namespace mh

using namespace mh;

extern "C" mh_status mh_matmul_modp_batched(mh_ctx *ctx, const mh_mm_desc *d, int32_t count,
                                            uint32_t p, int32_t T, int32_t mode,
                                            hipStream_t stream)
{
    if (!ctx || (count > 0 && !d) || count < 0) return MH_E_INVALID;
    for (int32_t i = 0; i < count; ++i) {
        mh_status s = mh_matmul_modp(ctx, d[i].C, d[i].NC, d[i].rc, d[i].cc, d[i].A, d[i].NA,
                                     d[i].ra, d[i].ca, d[i].B, d[i].NB, d[i].rb, d[i].cb, d[i].m,
                                     d[i].k, d[i].n, p, T, mode, stream);
        if (s != MH_OK) return s;
    }
    return MH_OK;
}
