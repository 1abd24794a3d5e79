// Diagnostic: sustained issue rate of the instruction classes the edge-segment
// sweeps are made of (FP32 FMA, the v_log / v_rcp / v_sqrt transcendentals,
// FP64 FMA).  Each lane runs eight independent
// dependency chains of one instruction class, so the rate measured is the
// issue limit, not the latency; the grid holds 8 waves on every SIMD.  The
// ratios between classes are the weights of the sweeps' issue-slot roofline.
#include <hip/hip_runtime.h>

#include "api_internal.h"

namespace grav {

namespace {

constexpr int kProbeIters = 2048;
constexpr int kProbeChains = 8;

enum ProbeOp {
    kOpFma32 = 0, kOpLog = 1, kOpRcp = 2, kOpSqrt = 3, kOpFma64 = 4, kOpAdd32 = 5, kNumProbeOps = 6
};

// Every chain step is one short (4-byte) instruction: the FMA chains add k*b
// with k in a scalar register (v_fmac), the transcendental chains add an
// inline constant; the step loop is unrolled so scalar loop control is rare.
template <int OP>
__global__ __launch_bounds__(256) void k_issue_rate(float *__restrict__ out, int iters, float k,
                                                    double k64) {
    const float s = 1.1f + threadIdx.x * 1e-3f;
    if constexpr (OP == kOpFma64) {
        double a[kProbeChains];
        const double b = 1e-9 * s;
#pragma unroll
        for (int c = 0; c < kProbeChains; ++c) a[c] = s + 0.1 * c;
#pragma unroll 4
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int c = 0; c < kProbeChains; ++c) a[c] = fma(k64, b, a[c]);
        }
        double r = 0.0;
#pragma unroll
        for (int c = 0; c < kProbeChains; ++c) r += a[c];
        out[blockIdx.x * blockDim.x + threadIdx.x] = static_cast<float>(r);
    } else {
        float a[kProbeChains];
        const float b = 1e-7f * s;
#pragma unroll
        for (int c = 0; c < kProbeChains; ++c) a[c] = s + 0.1f * c;
#pragma unroll 4
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int c = 0; c < kProbeChains; ++c) {
                if constexpr (OP == kOpFma32) a[c] = fmaf(k, b, a[c]);
                if constexpr (OP == kOpLog) a[c] = __builtin_amdgcn_logf(a[c]) + 2.0f;
                if constexpr (OP == kOpRcp) a[c] = __builtin_amdgcn_rcpf(a[c]) + 2.0f;
                if constexpr (OP == kOpSqrt) a[c] = __builtin_amdgcn_sqrtf(a[c]) + 1.0f;
                if constexpr (OP == kOpAdd32) a[c] = a[c] + k;
            }
        }
        float r = 0.0f;
#pragma unroll
        for (int c = 0; c < kProbeChains; ++c) r += a[c];
        out[blockIdx.x * blockDim.x + threadIdx.x] = r;
    }
}

template <int OP>
hipError_t launch_probe(float *out, int blocks, hipStream_t st) {
    k_issue_rate<OP><<<blocks, 256, 0, st>>>(out, kProbeIters, 0.999f, 0.999);
    return hipGetLastError();
}

}  // namespace

// Rates in chain steps per lane per second, summed over lanes.  An FMA or add
// step is one instruction; a transcendental step is the transcendental plus
// the FP32 add that keeps its chain going, so its issue cost in FMA slots is
// rate(FMA32) / rate(step) - rate(FMA32) / rate(add).
int op_issue_rates(grav_ctx *ctx, double *rates, hipStream_t st) {
    int cus = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "device attribute");
    const int blocks = cus * 8;            // 8 waves on each of the 4 SIMDs of every CU
    Arena ar = ctx_arena(ctx);
    float *out = ar.take<float>((size_t)blocks * 256);
    if (ar.failed) return fail(ctx, GRAV_ENOMEM, "workspace too small for the probe");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(ctx, e, "event create");
    }
    hipError_t (*launchers[kNumProbeOps])(float *, int, hipStream_t) = {
        launch_probe<kOpFma32>, launch_probe<kOpLog>, launch_probe<kOpRcp>,
        launch_probe<kOpSqrt>, launch_probe<kOpFma64>, launch_probe<kOpAdd32>};
    const double lane_ops = (double)blocks * 256 * kProbeIters * kProbeChains;
    int rc = GRAV_OK;
    for (int op = 0; op < kNumProbeOps && rc == GRAV_OK; ++op) {
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && rc == GRAV_OK; ++rep) {   // the first run warms up
            if ((e = hipEventRecord(e0, st)) != hipSuccess || (e = launchers[op](out, blocks, st)) != hipSuccess ||
                (e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
                (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
                rc = hip_fail(ctx, e, "probe");
        }
        if (rc == GRAV_OK) rates[op] = lane_ops / (ms * 1e-3);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

}  // namespace grav
