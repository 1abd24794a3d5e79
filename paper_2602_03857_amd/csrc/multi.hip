// Multi-model forward (placeholder until the MFMA path lands).
#include "api_internal.h"

namespace grav {
uint64_t multi_workspace_need(const Mesh &g, int64_t n, grav_prec prec, int K) {
    (void)g; (void)n; (void)prec; (void)K;
    return 0;
}
}  // namespace grav

extern "C" int grav_forward_multi(grav_ctx *ctx, const grav_mesh *mesh, const grav_obs *obs,
                                  const float *models, int32_t K, float *D, grav_prec prec,
                                  grav_stream stream) {
    (void)mesh; (void)obs; (void)models; (void)K; (void)D; (void)prec; (void)stream;
    if (!ctx) return GRAV_EINVAL;
    return grav::fail(ctx, GRAV_EINVAL, "multi-model forward not available");
}
