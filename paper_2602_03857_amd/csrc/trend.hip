// Regional-residual separation: least-squares polynomial trend surface of
// degree 1 or 2 in the horizontal station coordinates (the second-degree
// trend removal of the paper's field workflow, Section 2.2; the same fit over
// the whole domain joins independently inverted sections, Section 4.5).
//
// The fit is done in the centred, scaled frame u = (x - x0) / L,
// w = (y - y0) / L (bounding-box centre, half the larger side), where the
// normal matrix of the monomials (1, u, w, u^2, u w, w^2) is well conditioned.
// Every reduction uses a fixed tree over kDotBlocks block partials, so the
// result is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "api_internal.h"

namespace grav {

namespace {

constexpr int kMaxBasis = 6;
constexpr int kMaxSums = kMaxBasis * (kMaxBasis + 1) / 2 + kMaxBasis;   // Gram upper triangle + rhs

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_down(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    return v;
}

__device__ __forceinline__ void basis(double u, double w, double *phi) {
    phi[0] = 1.0;
    phi[1] = u;
    phi[2] = w;
    phi[3] = u * u;
    phi[4] = u * w;
    phi[5] = w * w;
}

// Per-block bounding box and a non-finite flag: part[blk*5 + {xmin, xmax, ymin, ymax, bad}].
__global__ __launch_bounds__(256) void k_trend_bbox(const double *__restrict__ x,
                                                    const double *__restrict__ y,
                                                    const double *__restrict__ v, int64_t n,
                                                    double *__restrict__ part) {
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY, bad = 0.0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kDotBlocks * 256) {
        const double xi = x[i], yi = y[i], vi = v[i];
        if (!isfinite(xi) || !isfinite(yi) || !isfinite(vi)) bad = 1.0;
        x0 = fmin(x0, xi);
        x1 = fmax(x1, xi);
        y0 = fmin(y0, yi);
        y1 = fmax(y1, yi);
    }
    __shared__ double s[4][5];
    const double r[5] = {wave_min(x0), wave_max(x1), wave_min(y0), wave_max(y1), wave_max(bad)};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int j = 0; j < 5; ++j) s[wave][j] = r[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        part[blockIdx.x * 5 + 0] = fmin(fmin(s[0][0], s[1][0]), fmin(s[2][0], s[3][0]));
        part[blockIdx.x * 5 + 1] = fmax(fmax(s[0][1], s[1][1]), fmax(s[2][1], s[3][1]));
        part[blockIdx.x * 5 + 2] = fmin(fmin(s[0][2], s[1][2]), fmin(s[2][2], s[3][2]));
        part[blockIdx.x * 5 + 3] = fmax(fmax(s[0][3], s[1][3]), fmax(s[2][3], s[3][3]));
        part[blockIdx.x * 5 + 4] = fmax(fmax(s[0][4], s[1][4]), fmax(s[2][4], s[3][4]));
    }
}

// One block: frame = {x0, y0, L}; flag = 1 for non-finite input.
__global__ __launch_bounds__(256) void k_trend_frame(const double *__restrict__ part,
                                                     double *__restrict__ frame,
                                                     int *__restrict__ flag) {
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY, bad = 0.0;
    for (int b = threadIdx.x; b < kDotBlocks; b += 256) {
        x0 = fmin(x0, part[b * 5 + 0]);
        x1 = fmax(x1, part[b * 5 + 1]);
        y0 = fmin(y0, part[b * 5 + 2]);
        y1 = fmax(y1, part[b * 5 + 3]);
        bad = fmax(bad, part[b * 5 + 4]);
    }
    __shared__ double s[4][5];
    const double r[5] = {wave_min(x0), wave_max(x1), wave_min(y0), wave_max(y1), wave_max(bad)};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int j = 0; j < 5; ++j) s[wave][j] = r[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        const double a = fmin(fmin(s[0][0], s[1][0]), fmin(s[2][0], s[3][0]));
        const double b = fmax(fmax(s[0][1], s[1][1]), fmax(s[2][1], s[3][1]));
        const double c = fmin(fmin(s[0][2], s[1][2]), fmin(s[2][2], s[3][2]));
        const double d = fmax(fmax(s[0][3], s[1][3]), fmax(s[2][3], s[3][3]));
        const double e = fmax(fmax(s[0][4], s[1][4]), fmax(s[2][4], s[3][4]));
        const double half = 0.5 * fmax(b - a, d - c);
        frame[0] = 0.5 * (a + b);
        frame[1] = 0.5 * (c + d);
        frame[2] = half > 0.0 ? half : 1.0;    // a single point: any scale
        *flag = e > 0.0 ? 1 : 0;
    }
}

// Per-block sums of phi_i phi_j (i <= j) and phi_i v:
// part[blk*kMaxSums + k], k over the upper triangle row by row, then the rhs.
template <int NB>
__global__ __launch_bounds__(256) void k_trend_gram(const double *__restrict__ x,
                                                    const double *__restrict__ y,
                                                    const double *__restrict__ v, int64_t n,
                                                    const double *__restrict__ frame,
                                                    double *__restrict__ part) {
    constexpr int NS = NB * (NB + 1) / 2 + NB;
    const double x0 = frame[0], y0 = frame[1], il = 1.0 / frame[2];
    double acc[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] = 0.0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kDotBlocks * 256) {
        double phi[kMaxBasis];
        basis((x[i] - x0) * il, (y[i] - y0) * il, phi);
        const double vi = v[i];
        int k = 0;
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = a; b < NB; ++b, ++k) acc[k] = fma(phi[a], phi[b], acc[k]);
#pragma unroll
        for (int a = 0; a < NB; ++a, ++k) acc[k] = fma(phi[a], vi, acc[k]);
    }
    __shared__ double s[4][NS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const double t = wave_sum(acc[k]);
        if (lane == 0) s[wave][k] = t;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < NS; k += 256)
        part[blockIdx.x * kMaxSums + k] = (s[0][k] + s[1][k]) + (s[2][k] + s[3][k]);
}

// One block: reduce the partials, solve the normal equations by Cholesky.
// coef (kMaxBasis doubles) receives the coefficients (zeros beyond NB);
// flag |= 2 when the normal matrix is numerically singular.
template <int NB>
__global__ __launch_bounds__(256) void k_trend_solve(const double *__restrict__ part,
                                                     double *__restrict__ coef,
                                                     int *__restrict__ flag) {
    constexpr int NS = NB * (NB + 1) / 2 + NB;
    __shared__ double tot[NS];
    // one wave per sum, lanes over blocks in a fixed order
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = wave; k < NS; k += 4) {
        double a = 0.0;
        for (int b = lane; b < kDotBlocks; b += 64) a += part[b * kMaxSums + k];
        a = wave_sum(a);
        if (lane == 0) tot[k] = a;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double A[NB][NB], rhs[NB];
    int k = 0;
    for (int a = 0; a < NB; ++a)
        for (int b = a; b < NB; ++b) {
            A[a][b] = tot[k];
            A[b][a] = tot[k];
            ++k;
        }
    for (int a = 0; a < NB; ++a) rhs[a] = tot[k++];
    double dmax = 0.0;
    for (int a = 0; a < NB; ++a) dmax = fmax(dmax, A[a][a]);
    // in-place Cholesky A = L L^T (lower triangle)
    bool ok = dmax > 0.0;
    for (int j = 0; j < NB && ok; ++j) {
        double d = A[j][j];
        for (int p = 0; p < j; ++p) d -= A[j][p] * A[j][p];
        if (!(d > 1e-12 * dmax)) { ok = false; break; }
        const double ljj = sqrt(d);
        A[j][j] = ljj;
        for (int i = j + 1; i < NB; ++i) {
            double t = A[i][j];
            for (int p = 0; p < j; ++p) t -= A[i][p] * A[j][p];
            A[i][j] = t / ljj;
        }
    }
    double c[NB];
    if (ok) {
        for (int i = 0; i < NB; ++i) {           // L z = rhs
            double t = rhs[i];
            for (int p = 0; p < i; ++p) t -= A[i][p] * c[p];
            c[i] = t / A[i][i];
        }
        for (int i = NB - 1; i >= 0; --i) {      // L^T c = z
            double t = c[i];
            for (int p = i + 1; p < NB; ++p) t -= A[p][i] * c[p];
            c[i] = t / A[i][i];
        }
    } else {
        for (int i = 0; i < NB; ++i) c[i] = 0.0;
        *flag |= 2;
    }
    for (int i = 0; i < kMaxBasis; ++i) coef[i] = i < NB ? c[i] : 0.0;
}

// trend[i] = T(x_i, y_i); resid[i] = v[i] - T (either may be null; resid may alias v).
__global__ __launch_bounds__(256) void k_trend_apply(const double *__restrict__ x,
                                                     const double *__restrict__ y, const double *v,
                                                     int64_t n, const double *__restrict__ frame,
                                                     const double *__restrict__ coef, double *resid,
                                                     double *__restrict__ trend) {
    const double x0 = frame[0], y0 = frame[1], il = 1.0 / frame[2];
    double c[kMaxBasis];
    for (int j = 0; j < kMaxBasis; ++j) c[j] = coef[j];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double phi[kMaxBasis];
        basis((x[i] - x0) * il, (y[i] - y0) * il, phi);
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < kMaxBasis; ++j) t = fma(c[j], phi[j], t);
        if (trend) trend[i] = t;
        if (resid) resid[i] = v[i] - t;
    }
}

}  // namespace

uint64_t trend_workspace_need() {
    Counter c;
    c.take<double>((size_t)kDotBlocks * kMaxSums);
    c.take<double>(16);
    return c.off;
}

int op_trend_surface(grav_ctx *ctx, const double *x, const double *y, const double *v, int64_t n,
                     int degree, double *coef, double *frame, double *resid, double *trend,
                     hipStream_t st) {
    Arena ar = ctx_arena(ctx);
    double *part = ar.take<double>((size_t)kDotBlocks * kMaxSums);
    double *dev = ar.take<double>(16);     // frame [0,3), coefficients [4,10)
    if (ar.failed) return fail(ctx, GRAV_ENOMEM, "workspace too small for the trend-surface sums");
    int *flag = reinterpret_cast<int *>(ctx->ws);
    hipError_t e = hipSuccess;
    k_trend_bbox<<<kDotBlocks, 256, 0, st>>>(x, y, v, n, part);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(ctx, e, "trend bbox");
    k_trend_frame<<<1, 256, 0, st>>>(part, dev, flag);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(ctx, e, "trend frame");
    if (degree == 2) {
        k_trend_gram<6><<<kDotBlocks, 256, 0, st>>>(x, y, v, n, dev, part);
        if ((e = hipGetLastError()) == hipSuccess) k_trend_solve<6><<<1, 256, 0, st>>>(part, dev + 4, flag);
    } else {
        k_trend_gram<3><<<kDotBlocks, 256, 0, st>>>(x, y, v, n, dev, part);
        if ((e = hipGetLastError()) == hipSuccess) k_trend_solve<3><<<1, 256, 0, st>>>(part, dev + 4, flag);
    }
    if (e != hipSuccess || (e = hipGetLastError()) != hipSuccess) return hip_fail(ctx, e, "trend fit");
    if (resid || trend) {
        unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
        k_trend_apply<<<grid, 256, 0, st>>>(x, y, v, n, dev, dev + 4, resid, trend);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(ctx, e, "trend apply");
    }
    double *h = ctx->h_scal;    // pinned staging: frame [0,3), coefficients [4,10)
    if ((e = hipMemcpyAsync(h, dev, 10 * sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hip_fail(ctx, e, "trend copy");
    if ((e = hipMemcpyAsync(ctx->h_flags, flag, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hip_fail(ctx, e, "trend copy");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(ctx, e, "trend sync");
    if (*ctx->h_flags & 1) return fail(ctx, GRAV_EINVAL, "x, y or v holds a non-finite value");
    if (*ctx->h_flags & 2)
        return fail(ctx, GRAV_EINVAL, "the points do not determine a trend surface of this degree");
    for (int i = 0; i < 3; ++i) frame[i] = h[i];
    for (int i = 0; i < kMaxBasis; ++i) coef[i] = h[4 + i];
    return GRAV_OK;
}

}  // namespace grav
