// FP64 vector kernels of the data-space conjugate-gradient solver
// (Eq. 11 solved iteratively): dot products with a fixed reduction tree
// (bitwise reproducible), and the CG updates reading their step lengths from
// device memory so that an iteration needs no host round trip.
#include "grav_internal.h"

namespace grav {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Block sum of `v` over 256 threads; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double part[4];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) part[wave] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (part[0] + part[1]) + (part[2] + part[3]);
    return r;
}

__global__ __launch_bounds__(256) void k_dot(const double *__restrict__ a,
                                             const double *__restrict__ b, int64_t n,
                                             double *__restrict__ partials) {
    double acc = 0.0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kDotBlocks * 256)
        acc = b ? fma(a[i], b[i], acc) : acc + a[i];
    const double s = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_dot_finish(const double *__restrict__ partials,
                                                    double *__restrict__ scal, int mode, int slot) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < kDotBlocks; i += 256) acc += partials[i];
    const double s = block_sum(acc);
    if (threadIdx.x == 0) {
        switch (mode) {
            case kFinishInit:          // r0 . r0 : ||delta_d||^2
                scal[kRR] = s;
                scal[kB2] = s;
                scal[kRRNew] = s;
                break;
            case kFinishPQ:            // alpha = (r.r) / (p.Ap); 0 once r = 0
                scal[kPQ] = s;
                scal[kAlpha] = s > 0.0 ? scal[kRR] / s : 0.0;
                break;
            case kFinishRRNew:         // beta = (r'.r') / (r.r), then r.r <- r'.r'
                scal[kRRNew] = s;
                scal[kBeta] = scal[kRR] > 0.0 ? s / scal[kRR] : 0.0;
                scal[kRR] = s;
                break;
            case kFinishPQPrecond:
                scal[kPQ] = s;
                scal[kAlpha] = s > 0.0 ? scal[kRZ] / s : 0.0;
                break;
            case kFinishRZNew:
                scal[kBeta] = scal[kRZ] > 0.0 ? s / scal[kRZ] : 0.0;
                scal[kRZ] = s;
                break;
            default:
                scal[slot] = s;
                break;
        }
    }
}

__global__ __launch_bounds__(256) void k_cg_update_yr(double *__restrict__ y, double *__restrict__ r,
                                                      const double *__restrict__ p,
                                                      const double *__restrict__ q, int64_t n,
                                                      const double *__restrict__ scal,
                                                      double *__restrict__ partials) {
    const double alpha = scal[kAlpha];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kDotBlocks * 256) {
        y[i] = fma(alpha, p[i], y[i]);
        const double ri = fma(-alpha, q[i], r[i]);
        r[i] = ri;
        acc = fma(ri, ri, acc);
    }
    const double s = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_pcg_setup(const double *__restrict__ diag, double lambda,
                                                   double *__restrict__ dinv,
                                                   const double *__restrict__ r,
                                                   double *__restrict__ z, double *__restrict__ p,
                                                   int64_t n, double *__restrict__ part_rr,
                                                   double *__restrict__ part_rz) {
    double arr = 0.0, arz = 0.0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kDotBlocks * 256) {
        const double di = 1.0 / (diag[i] + lambda);
        dinv[i] = di;
        const double ri = r[i], zi = di * ri;
        z[i] = zi;
        p[i] = zi;
        arr = fma(ri, ri, arr);
        arz = fma(ri, zi, arz);
    }
    const double s1 = block_sum(arr);
    __syncthreads();
    const double s2 = block_sum(arz);
    if (threadIdx.x == 0) {
        part_rr[blockIdx.x] = s1;
        part_rz[blockIdx.x] = s2;
    }
}

__global__ __launch_bounds__(256) void k_pcg_update_yrz(double *__restrict__ y, double *__restrict__ r,
                                                        double *__restrict__ z,
                                                        const double *__restrict__ p,
                                                        const double *__restrict__ q,
                                                        const double *__restrict__ dinv, int64_t n,
                                                        const double *__restrict__ scal,
                                                        double *__restrict__ part_rr,
                                                        double *__restrict__ part_rz) {
    const double alpha = scal[kAlpha];
    double arr = 0.0, arz = 0.0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kDotBlocks * 256) {
        y[i] = fma(alpha, p[i], y[i]);
        const double ri = fma(-alpha, q[i], r[i]);
        r[i] = ri;
        const double zi = dinv[i] * ri;
        z[i] = zi;
        arr = fma(ri, ri, arr);
        arz = fma(ri, zi, arz);
    }
    const double s1 = block_sum(arr);
    __syncthreads();
    const double s2 = block_sum(arz);
    if (threadIdx.x == 0) {
        part_rr[blockIdx.x] = s1;
        part_rz[blockIdx.x] = s2;
    }
}

__global__ __launch_bounds__(256) void k_cg_update_p(double *__restrict__ p,
                                                     const double *__restrict__ r, int64_t n,
                                                     const double *__restrict__ scal) {
    const double beta = scal[kBeta];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = fma(beta, p[i], r[i]);
}

__global__ void k_sub(const double *__restrict__ a, const double *__restrict__ b,
                      double *__restrict__ dst, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = b ? a[i] - b[i] : a[i];
}

// dst = ca a + cb b; dst may alias a or b (element-wise).
__global__ void k_lincomb(double *dst, double ca, const double *a, double cb, const double *b,
                          int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = fma(ca, a[i], cb * b[i]);
}

__global__ void k_fill(double *__restrict__ dst, double value, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = value;
}

inline unsigned grid_vec(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_dot(const double *a, const double *b, int64_t n, double *partials,
                      hipStream_t st) {
    k_dot<<<kDotBlocks, 256, 0, st>>>(a, b, n, partials);
    return hipGetLastError();
}

hipError_t launch_dot_finish(const double *partials, double *scal, int mode, int slot,
                             hipStream_t st) {
    k_dot_finish<<<1, 256, 0, st>>>(partials, scal, mode, slot);
    return hipGetLastError();
}

hipError_t launch_cg_update_yr(double *y, double *r, const double *p, const double *q, int64_t n,
                               const double *scal, double *partials, hipStream_t st) {
    k_cg_update_yr<<<kDotBlocks, 256, 0, st>>>(y, r, p, q, n, scal, partials);
    return hipGetLastError();
}

hipError_t launch_pcg_setup(const double *diag, double lambda, double *dinv, const double *r,
                            double *z, double *p, int64_t n, double *part_rr, double *part_rz,
                            hipStream_t st) {
    k_pcg_setup<<<kDotBlocks, 256, 0, st>>>(diag, lambda, dinv, r, z, p, n, part_rr, part_rz);
    return hipGetLastError();
}

hipError_t launch_pcg_update_yrz(double *y, double *r, double *z, const double *p, const double *q,
                                 const double *dinv, int64_t n, const double *scal,
                                 double *part_rr, double *part_rz, hipStream_t st) {
    k_pcg_update_yrz<<<kDotBlocks, 256, 0, st>>>(y, r, z, p, q, dinv, n, scal, part_rr, part_rz);
    return hipGetLastError();
}

hipError_t launch_cg_update_p(double *p, const double *r, int64_t n, const double *scal,
                              hipStream_t st) {
    k_cg_update_p<<<grid_vec(n), 256, 0, st>>>(p, r, n, scal);
    return hipGetLastError();
}

hipError_t launch_sub(const double *a, const double *b, double *dst, int64_t n, hipStream_t st) {
    k_sub<<<grid_vec(n), 256, 0, st>>>(a, b, dst, n);
    return hipGetLastError();
}

hipError_t launch_lincomb(double *dst, double ca, const double *a, double cb, const double *b,
                          int64_t n, hipStream_t st) {
    k_lincomb<<<grid_vec(n), 256, 0, st>>>(dst, ca, a, cb, b, n);
    return hipGetLastError();
}

hipError_t launch_fill(double *dst, double value, int64_t n, hipStream_t st) {
    k_fill<<<grid_vec(n), 256, 0, st>>>(dst, value, n);
    return hipGetLastError();
}

}  // namespace grav
