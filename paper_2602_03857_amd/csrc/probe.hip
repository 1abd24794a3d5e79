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

// Pairs of classes: FP32 FMA chains with transcendental (v_log_f32 + add)
// chains, and FP32 FMA chains with compare-and-select (v_cmp + v_cndmask +
// add) chains, either on alternating waves (odd waves one class, even waves
// the other) or interleaved in every wave (four chains of each).  Against the
// rate of the two halves run one after the other, the excess is the work the
// SIMD issues together from different waves or from one wave.
enum PairOp { kPairTrans = 0, kPairSelect = 1 };

template <int B>
__device__ __forceinline__ void pair_step(float (&a)[4], float k, float b) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if constexpr (B == kPairTrans) a[c] = __builtin_amdgcn_logf(a[c]) + 2.0f;
        if constexpr (B == kPairSelect) a[c] = a[c] + ((a[c] > b) ? -k : k);
    }
}

__device__ __forceinline__ void fma_step(float (&a)[4], float k, float b) {
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] = fmaf(k, b, a[c]);
}

// kAlone: every wave runs class B only (its single-class rate).
template <int B, bool kInterleaved, bool kAlone = false>
__global__ __launch_bounds__(256) void k_issue_pair(float *__restrict__ out, int iters, float k) {
    const float s = 1.1f + threadIdx.x * 1e-3f;
    float a0[4], a1[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        a0[c] = s + 0.1f * c;
        a1[c] = s + 0.2f * c;
    }
    const float b = 1e-7f * s;
    if (kInterleaved) {
#pragma unroll 4
        for (int i = 0; i < iters; ++i) {
            fma_step(a0, k, b);
            pair_step<B>(a1, k, b);
        }
    } else if (kAlone || ((threadIdx.x >> 6) & 1)) {
#pragma unroll 4
        for (int i = 0; i < iters; ++i) {
            pair_step<B>(a0, k, b);
            pair_step<B>(a1, k, b);
        }
    } else {
#pragma unroll 4
        for (int i = 0; i < iters; ++i) {
            fma_step(a0, k, b);
            fma_step(a1, k, b);
        }
    }
    float r = 0.0f;
#pragma unroll
    for (int c = 0; c < 4; ++c) r += a0[c] + a1[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

template <int B, bool kInterleaved, bool kAlone = false>
hipError_t launch_pair(float *out, int blocks, hipStream_t st) {
    k_issue_pair<B, kInterleaved, kAlone><<<blocks, 256, 0, st>>>(out, kProbeIters, 0.999f);
    return hipGetLastError();
}

// One timed launch (after a warm-up launch) of `launch`; lane_ops / seconds.
int time_probe(grav_ctx *ctx, hipError_t (*launch)(float *, int, hipStream_t), float *out,
               int blocks, double lane_ops, hipStream_t st, double *rate) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(ctx, e, "event create");
    }
    int rc = GRAV_OK;
    float ms = 0.0f;
    for (int rep = 0; rep < 2 && rc == GRAV_OK; ++rep) {
        if ((e = hipEventRecord(e0, st)) != hipSuccess || (e = launch(out, blocks, st)) != hipSuccess ||
            (e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
            (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
            rc = hip_fail(ctx, e, "probe");
    }
    if (rc == GRAV_OK) *rate = lane_ops / (ms * 1e-3);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

}  // namespace

// Rates in chain steps per second summed over lanes (each lane runs eight
// chains): [0] FMA + transcendental on alternating waves, [1] interleaved in
// every wave, [2] FMA + compare-and-select on alternating waves,
// [3] interleaved, [4] compare-and-select alone.
int op_issue_pair_rates(grav_ctx *ctx, double *rates, hipStream_t st) {
    int cus = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "device attribute");
    const int blocks = cus * 8;
    Arena ar = ctx_arena(ctx);
    float *out = ar.take<float>((size_t)blocks * 256);
    if (ar.failed) return fail(ctx, GRAV_ENOMEM, "workspace too small for the probe");
    hipError_t (*launchers[5])(float *, int, hipStream_t) = {
        launch_pair<kPairTrans, false>, launch_pair<kPairTrans, true>,
        launch_pair<kPairSelect, false>, launch_pair<kPairSelect, true>,
        launch_pair<kPairSelect, false, true>};
    const double lane_ops = (double)blocks * 256 * kProbeIters * kProbeChains;
    for (int i = 0; i < 5; ++i) {
        const int rc = time_probe(ctx, launchers[i], out, blocks, lane_ops, st, &rates[i]);
        if (rc) return rc;
    }
    return GRAV_OK;
}

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
    hipError_t (*launchers[kNumProbeOps])(float *, int, hipStream_t) = {
        launch_probe<kOpFma32>, launch_probe<kOpLog>, launch_probe<kOpRcp>,
        launch_probe<kOpSqrt>, launch_probe<kOpFma64>, launch_probe<kOpAdd32>};
    const double lane_ops = (double)blocks * 256 * kProbeIters * kProbeChains;
    for (int op = 0; op < kNumProbeOps; ++op) {
        const int rc = time_probe(ctx, launchers[op], out, blocks, lane_ops, st, &rates[op]);
        if (rc) return rc;
    }
    return GRAV_OK;
}

}  // namespace grav
