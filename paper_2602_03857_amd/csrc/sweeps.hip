// Sweep kernels of the matrix-free prism-gravity operators (paper Eq. 1-6):
// forward d = G m, adjoint G^T v, the weighted row sums that give
// trace(G C G^T), and the O(M) stencils around them.
//
// Layouts (all device memory, C order):
//   cell    (i, j, k)  -> (i*ny + j)*nz + k          M = nx*ny*nz
//   segment (a, b, k)  -> (a*(ny+1) + b)*nz + k      vertical edge of node column (a, b), layer k
//   node    (a, b, c)  -> (a*(ny+1) + b)*(nz+1) + c
//
// Mixed path.  Summing Eq. 1 over the two vertical corners of a prism gives
// the edge-segment term S = Psi(z_bottom) - Psi(z_top) for each of the four
// vertical edges, with parity (-1)^(p+q) in (x, y):
//   G_ok = gamma * sum_{p,q in {0,1}} (-1)^(p+q) S(o; column (i+p, j+q), layer k).
// Summing over cells (Eq. 5) therefore moves the (x, y) parity onto the
// density, W2(a,b,k) = sum_{p,q} (-1)^(p+q) m(a-p, b-q, k) (zero outside the
// mesh), and d_o = gamma * sum_segments S * W2 - one S per vertical edge
// segment, shared by the (up to) four prisms around it.  The adjoint runs
// the same sum the other way: U(segment) = sum_o v_o S, then
// (G^T v)_cell = gamma * sum_{p,q} (-1)^(p+q) U.
//
// FP64 path.  The same regrouping over all three axes: node weight
// W = B m (up to 8 cells per node, parity (-1)^(p+q+r) of Eq. 1) and
// d_o = gamma * sum_nodes Psi(node - o) * W.
#include <type_traits>

#include "grav_internal.h"
#include "edge_math.h"
#include "sweep_bodies.h"

namespace grav {

namespace {

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------------ O(M)

// Layer table (layout at layer_table_len): hk[k] = thickness of layer k,
// then (as an int) the first layer index from which every layer is "deep"
// (its top at least kDeepRatio thicknesses below the mesh top), then the
// node depths Z_{k+1} - Z_0.
__global__ void k_layer_thickness(const double *__restrict__ zn, int nz, float *__restrict__ hk) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nz) {
        hk[k] = static_cast<float>(zn[k + 1] - zn[k]);
        hk[nz + 1 + k] = static_cast<float>(zn[k + 1] - zn[0]);
    }
    if (k == 0) {
        int kdeep = nz;
        while (kdeep > 0 && (zn[kdeep - 1] - zn[0]) >= kDeepRatio * (zn[kdeep] - zn[kdeep - 1]) &&
               (zn[kdeep - 1] - zn[0]) >= kDeepMinDepth)
            --kdeep;
        reinterpret_cast<int *>(hk + nz)[0] = kdeep;
    }
}

// W2(a,b,k) = m(a,b) - m(a-1,b) - m(a,b-1) + m(a-1,b-1), zero-padded.
__global__ void k_edge_weights(const double *__restrict__ m, int nx, int ny, int nz,
                               double *__restrict__ w2) {
    const int64_t total = (int64_t)(nx + 1) * (ny + 1) * nz;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < total;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(s % nz);
        const int64_t col = s / nz;
        const int b = (int)(col % (ny + 1));
        const int a = (int)(col / (ny + 1));
        double acc = 0.0;
        const bool a0 = a < nx, a1 = a >= 1, b0 = b < ny, b1 = b >= 1;
        if (a0 && b0) acc += m[((int64_t)a * ny + b) * nz + k];
        if (a1 && b0) acc -= m[((int64_t)(a - 1) * ny + b) * nz + k];
        if (a0 && b1) acc -= m[((int64_t)a * ny + (b - 1)) * nz + k];
        if (a1 && b1) acc += m[((int64_t)(a - 1) * ny + (b - 1)) * nz + k];
        w2[s] = acc;
    }
}

// W(a,b,c) = sum over cells (a-p', b-q', c-r') with p',q',r' in {0,1} of
// -(-1)^(p'+q'+r') m  (the vertex parity of Eq. 1 with vertex index p = p'+1).
__global__ void k_node_weights(const double *__restrict__ m, int nx, int ny, int nz,
                               double *__restrict__ wn) {
    const int64_t total = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < total;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(s % (nz + 1));
        const int64_t col = s / (nz + 1);
        const int b = (int)(col % (ny + 1));
        const int a = (int)(col / (ny + 1));
        double acc = 0.0;
        for (int p = 0; p < 2; ++p) {
            const int i = a - p;
            if (i < 0 || i >= nx) continue;
            for (int q = 0; q < 2; ++q) {
                const int j = b - q;
                if (j < 0 || j >= ny) continue;
                for (int r = 0; r < 2; ++r) {
                    const int k = c - r;
                    if (k < 0 || k >= nz) continue;
                    const double v = m[((int64_t)i * ny + j) * nz + k];
                    acc += ((p + q + r) & 1) ? v : -v;
                }
            }
        }
        wn[s] = acc;
    }
}

__global__ void k_reduce_parts(const double *__restrict__ part, int nparts, int64_t len,
                               double scale, const double *__restrict__ add, double coef,
                               double *__restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int p = 0; p < nparts; ++p) acc += part[(int64_t)p * len + i];
        double r = scale * acc;
        if (add) r = fma(coef, add[i], r);
        out[i] = r;
    }
}

// out(i,j,k) = base + scale * C * [U(i,j) - U(i+1,j) - U(i,j+1) + U(i+1,j+1)](k)
__global__ void k_adjoint_finish_edges(const double *__restrict__ U, int nx, int ny, int nz,
                                       double scale, const double *__restrict__ wdepth,
                                       const double *__restrict__ base, double *__restrict__ out) {
    const int64_t total = (int64_t)nx * ny * nz;
    const int64_t ny1 = ny + 1;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < total;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(s % nz);
        const int64_t ij = s / nz;
        const int64_t j = ij % ny;
        const int64_t i = ij / ny;
        const int64_t c00 = (i * ny1 + j) * nz + k;
        const int64_t c10 = ((i + 1) * ny1 + j) * nz + k;
        const double g = (U[c00] - U[c10]) - (U[c00 + nz] - U[c10 + nz]);
        double f = scale * g;
        if (wdepth) {
            const double w = wdepth[s];
            f = f / (w * w);
        }
        if (base) f += base[s];
        out[s] = f;
    }
}

// out(i,j,k) = base + scale * C * sum_{p',q',r'} -(-1)^(p'+q'+r') P(i+p', j+q', k+r')
__global__ void k_adjoint_finish_nodes(const double *__restrict__ P, int nx, int ny, int nz,
                                       double scale, const double *__restrict__ wdepth,
                                       const double *__restrict__ base, double *__restrict__ out) {
    const int64_t total = (int64_t)nx * ny * nz;
    const int64_t ny1 = ny + 1, nz1 = nz + 1;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < total;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = s % nz;
        const int64_t ij = s / nz;
        const int64_t j = ij % ny;
        const int64_t i = ij / ny;
        double g = 0.0;
        for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) {
                const int64_t base_idx = ((i + p) * ny1 + (j + q)) * nz1 + k;
                const double lo = P[base_idx], hi = P[base_idx + 1];
                // r' = 0 (top): sign -(-1)^(p+q); r' = 1 (bottom): sign +(-1)^(p+q)
                const double e = hi - lo;
                g += ((p + q) & 1) ? -e : e;
            }
        double f = scale * g;
        if (wdepth) {
            const double w = wdepth[s];
            f = f / (w * w);
        }
        if (base) f += base[s];
        out[s] = f;
    }
}

// ------------------------------------------------------------------ sweeps

// Mixed forward sweep.  Lane = observation.  Block row = a contiguous chunk of
// node columns (block index modulo nchunk, so with nchunk a multiple of 8 each
// XCD only ever touches its own chunks' W2).  All mesh data is wave-uniform.
__global__ __launch_bounds__(kBlock) void k_forward_mixed(
    const double *__restrict__ xn, const double *__restrict__ yn, const double *__restrict__ zn,
    int ny1, int nz, const float *__restrict__ hk, const double *__restrict__ ox,
    const double *__restrict__ oy, const double *__restrict__ oz, int64_t n,
    const double *__restrict__ w2, int64_t ncols, int64_t cols_per_chunk, int nchunk,
    double *__restrict__ partial) {
    forward_mixed_block(xn, yn, zn, ny1, nz, hk, ox, oy, oz, n, w2, ncols, cols_per_chunk,
                        (int)(blockIdx.x % nchunk), (int64_t)(blockIdx.x / nchunk), partial,
                        (int)threadIdx.x);
}

// FP64 forward sweep over nodes: lane = observation, chunk of node columns.
__global__ __launch_bounds__(kBlock) void k_forward_f64(
    const double *__restrict__ xn, const double *__restrict__ yn, const double *__restrict__ zn,
    int ny1, int nz, const double *__restrict__ ox, const double *__restrict__ oy,
    const double *__restrict__ oz, int64_t n, const double *__restrict__ wn, int64_t ncols,
    int64_t cols_per_chunk, int nchunk, double *__restrict__ partial) {
    const int chunk = (int)(blockIdx.x % nchunk);
    const int64_t o = (int64_t)(blockIdx.x / nchunk) * kBlock + threadIdx.x;
    const int64_t oc = o < n ? o : n - 1;
    const double xo = ox[oc], yo = oy[oc], zo = oz[oc];
    const int64_t c0 = (int64_t)chunk * cols_per_chunk;
    const int64_t c1 = c0 + cols_per_chunk < ncols ? c0 + cols_per_chunk : ncols;
    const int nz1 = nz + 1;
    double acc = 0.0;
    int a = (int)(c0 / ny1), b = (int)(c0 - (int64_t)a * ny1);
    for (int64_t col = c0; col < c1; ++col) {
        const double x = xn[a] - xo, y = yn[b] - yo;
        const double *__restrict__ w = wn + col * nz1;
        for (int c = 0; c < nz1; ++c) acc = fma(psi_f64(x, y, zn[c] - zo), w[c], acc);
        if (++b == ny1) { b = 0; ++a; }
    }
    if (o < n) partial[(int64_t)chunk * n + o] = acc;
}

// Mixed adjoint sweep.  Lane = (node column, chunk of <= kAdjLayers layers).
// Bounded to 64 VGPRs so that 8 waves fit on a SIMD (the few values it spills
// are read once per observation, outside the layer steps).
#ifndef GRAV_ADJ_WAVES
#define GRAV_ADJ_WAVES 8
#endif
#if GRAV_ADJ_WAVES > 0
#define GRAV_ADJ_OCCUPANCY __attribute__((amdgpu_waves_per_eu(GRAV_ADJ_WAVES, GRAV_ADJ_WAVES)))
#else
#define GRAV_ADJ_OCCUPANCY
#endif
__global__ __launch_bounds__(kBlock) GRAV_ADJ_OCCUPANCY
void k_adjoint_mixed(
    const double *__restrict__ xn, const double *__restrict__ yn, const double *__restrict__ zn,
    int ny1, int nz, const float *__restrict__ hk, const double *__restrict__ ox,
    const double *__restrict__ oy, const double *__restrict__ oz, const double *__restrict__ v,
    int64_t n, int64_t obs_per_part, int nparts, int64_t ncols, int nkc,
    double *__restrict__ upart) {
    unsigned bid = blockIdx.x;
    const int part = (int)(bid % (unsigned)nparts);
    bid /= (unsigned)nparts;
    const int kc = (int)(bid % (unsigned)nkc);
    bid /= (unsigned)nkc;
    adjoint_mixed_block(xn, yn, zn, ny1, nz, hk, ox, oy, oz, v, n, obs_per_part, ncols, nkc, part,
                        kc, bid, upart, (int)threadIdx.x);
}

// FP64 adjoint sweep: lane = node, P(node) = sum_{o in part} v_o Psi(node - o).
__global__ __launch_bounds__(kBlock) void k_adjoint_f64(
    const double *__restrict__ xn, const double *__restrict__ yn, const double *__restrict__ zn,
    int ny1, int nz, const double *__restrict__ ox, const double *__restrict__ oy,
    const double *__restrict__ oz, const double *__restrict__ v, int64_t n, int64_t obs_per_part,
    int nparts, int64_t nnodes, double *__restrict__ ppart) {
    const int part = (int)(blockIdx.x % nparts);
    const int64_t node = (int64_t)(blockIdx.x / nparts) * kBlock + threadIdx.x;
    const int64_t nd = node < nnodes ? node : nnodes - 1;
    const int nz1 = nz + 1;
    const int c = (int)(nd % nz1);
    const int64_t col = nd / nz1;
    const int b = (int)(col % ny1);
    const int a = (int)(col / ny1);
    const double X = xn[a], Y = yn[b], Z = zn[c];
    const int64_t o0 = (int64_t)part * obs_per_part;
    const int64_t o1 = o0 + obs_per_part < n ? o0 + obs_per_part : n;
    double acc = 0.0;
    for (int64_t o = o0; o < o1; ++o) acc = fma(v[o], psi_f64(X - ox[o], Y - oy[o], Z - oz[o]), acc);
    if (node < nnodes) ppart[(int64_t)part * nnodes + node] = acc;
}

// Mixed weighted row sums: lane = observation; chunk = range of prism rows i.
// For each (i, k) the sweep walks j carrying the two edge terms of the
// previous column pair, so each prism costs two new edge segments.
// partial[chunk][o] = sum_{cells in chunk} C * (sum_pq (-1)^(p+q) S)^2  (no gamma^2)
__global__ __launch_bounds__(kBlock) void k_trace_mixed(
    const double *__restrict__ xn, const double *__restrict__ yn, const double *__restrict__ zn,
    int nx, int ny, int nz, const float *__restrict__ hk, const double *__restrict__ wdepth,
    const double *__restrict__ ox, const double *__restrict__ oy, const double *__restrict__ oz,
    int64_t n, int64_t rows_per_chunk, int nchunk, double *__restrict__ partial) {
    const int chunk = (int)(blockIdx.x % nchunk);
    const int64_t o = (int64_t)(blockIdx.x / nchunk) * kBlock + threadIdx.x;
    const int64_t oc = o < n ? o : n - 1;
    const double xo = ox[oc], yo = oy[oc], zo = oz[oc];
    const int i0 = (int)(chunk * rows_per_chunk);
    const int i1 = (int)(i0 + rows_per_chunk < nx ? i0 + rows_per_chunk : nx);
    const float ztop = static_cast<float>(zn[0] - zo);
    const float *__restrict__ zrel = hk + nz + 1;
    const int kdeep = reinterpret_cast<const int *>(hk + nz)[0];
    double acc = 0.0;
    for (int i = i0; i < i1; ++i) {
        const double Xa = xn[i], Xb = xn[i + 1];
        for (int k = 0; k < nz; ++k) {
            const float z1 = node_depth(zrel, k, ztop);
            const float z2 = node_depth(zrel, k + 1, ztop);
            const float h = hk[k];
            // one row of prisms (i, all j, k); deep layers take the shorter
            // edge formula (k is uniform, so the branch is too)
            auto row = [&](auto deep) {
                constexpr bool kDeep = decltype(deep)::value;
                Column ca = make_column(Xa, yn[0], xo, yo);
                Column cb = make_column(Xb, yn[0], xo, yo);
                float Sa = edge_segment<kDeep>(ca, make_node(ca, z1), make_node(ca, z2), h);
                float Sb = edge_segment<kDeep>(cb, make_node(cb, z1), make_node(cb, z2), h);
                for (int j = 0; j < ny; ++j) {
                    ca = make_column(Xa, yn[j + 1], xo, yo);
                    cb = make_column(Xb, yn[j + 1], xo, yo);
                    const float Sa1 = edge_segment<kDeep>(ca, make_node(ca, z1), make_node(ca, z2), h);
                    const float Sb1 = edge_segment<kDeep>(cb, make_node(cb, z1), make_node(cb, z2), h);
                    const double g = ((double)Sa - (double)Sb) - ((double)Sa1 - (double)Sb1);
                    const double w = wdepth[((int64_t)i * ny + j) * nz + k];
                    acc = fma(g * g, 1.0 / (w * w), acc);
                    Sa = Sa1;
                    Sb = Sb1;
                }
            };
            if (k >= kdeep)
                row(std::true_type{});
            else
                row(std::false_type{});
        }
    }
    if (o < n) partial[(int64_t)chunk * n + o] = acc;
}

// FP64 weighted row sums: 8-corner prism terms from node Psi, carrying the
// four corners of the previous column pair along j (four new Psi per prism).
__global__ __launch_bounds__(kBlock) void k_trace_f64(
    const double *__restrict__ xn, const double *__restrict__ yn, const double *__restrict__ zn,
    int nx, int ny, int nz, const double *__restrict__ wdepth, const double *__restrict__ ox,
    const double *__restrict__ oy, const double *__restrict__ oz, int64_t n,
    int64_t rows_per_chunk, int nchunk, double *__restrict__ partial) {
    const int chunk = (int)(blockIdx.x % nchunk);
    const int64_t o = (int64_t)(blockIdx.x / nchunk) * kBlock + threadIdx.x;
    const int64_t oc = o < n ? o : n - 1;
    const double xo = ox[oc], yo = oy[oc], zo = oz[oc];
    const int i0 = (int)(chunk * rows_per_chunk);
    const int i1 = (int)(i0 + rows_per_chunk < nx ? i0 + rows_per_chunk : nx);
    double acc = 0.0;
    for (int i = i0; i < i1; ++i) {
        const double xa = xn[i] - xo, xb = xn[i + 1] - xo;
        for (int k = 0; k < nz; ++k) {
            const double z1 = zn[k] - zo, z2 = zn[k + 1] - zo;
            double y = yn[0] - yo;
            // edge term e(x, y) = Psi(x, y, z2) - Psi(x, y, z1)
            double ea = psi_f64(xa, y, z2) - psi_f64(xa, y, z1);
            double eb = psi_f64(xb, y, z2) - psi_f64(xb, y, z1);
            for (int j = 0; j < ny; ++j) {
                y = yn[j + 1] - yo;
                const double ea1 = psi_f64(xa, y, z2) - psi_f64(xa, y, z1);
                const double eb1 = psi_f64(xb, y, z2) - psi_f64(xb, y, z1);
                const double g = (ea - eb) - (ea1 - eb1);
                const double w = wdepth[((int64_t)i * ny + j) * nz + k];
                acc = fma(g * g, 1.0 / (w * w), acc);
                ea = ea1;
                eb = eb1;
            }
        }
    }
    if (o < n) partial[(int64_t)chunk * n + o] = acc;
}

// ------------------------------------------------------------------ validation

__global__ void k_validate(const double *__restrict__ xn, int nx, const double *__restrict__ yn,
                           int ny, const double *__restrict__ zn, int nz,
                           const double *__restrict__ ox, const double *__restrict__ oy,
                           const double *__restrict__ oz, int64_t n, int *flags) {
    constexpr double kRange = 1.0e6;   // metres: |node - observation| limit of the FP32 terms
    const double x_lo = xn[0], x_hi = xn[nx], y_lo = yn[0], y_hi = yn[ny];
    const double z_top = zn[0], z_bot = zn[nz];
    int f = 0;
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < nx; i += stride)
        if (!(xn[i + 1] > xn[i]) || !isfinite(xn[i + 1] - xn[i])) f |= kBadMesh;
    for (int64_t i = tid; i < ny; i += stride)
        if (!(yn[i + 1] > yn[i]) || !isfinite(yn[i + 1] - yn[i])) f |= kBadMesh;
    for (int64_t i = tid; i < nz; i += stride)
        if (!(zn[i + 1] > zn[i]) || !isfinite(zn[i + 1] - zn[i])) f |= kBadMesh;
    for (int64_t i = tid; i < n; i += stride) {
        const double x = ox[i], y = oy[i], z = oz[i];
        if (!isfinite(x) || !isfinite(y) || !isfinite(z)) { f |= kBadObs; continue; }
        if (z > z_top) f |= kObsBelowTop;
        const double dx = fmax(fabs(x - x_lo), fabs(x_hi - x));
        const double dy = fmax(fabs(y - y_lo), fabs(y_hi - y));
        const double dz = z_bot - z;
        if (dx > kRange || dy > kRange || dz > kRange) f |= kOutOfRange;
    }
    if (f) atomicOr(flags, f);
}

__global__ void k_validate_positive(const double *__restrict__ w, int64_t len, int *flags) {
    int f = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x)
        if (!(w[i] > 0.0) || !isfinite(w[i])) f = kBadWeights;
    if (f) atomicOr(flags, f);
}

__global__ void k_validate_finite(const double *__restrict__ w, int64_t len, int *flags) {
    int f = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(w[i])) f = kBadValues;
    if (f) atomicOr(flags, f);
}

inline unsigned grid_for(int64_t len, int block = 256, int64_t cap = 8192) {
    int64_t g = ceil_div(len, block);
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

// ------------------------------------------------------------------ plans

// Enough equal-work waves that the drain at the end of a launch (8 waves
// per SIMD on 1024 SIMDs finish at different times) costs little: measured at
// the paper-scale workload, 16k -> 128k waves shortens the forward sweep by
// 2 %, and the adjoint (whose waves are longer) gains 3 % from 16k -> 57k and
// 4.6 % more from 57k -> 143k (0.7 % more at 286k, for twice the partial
// sums).  Chunk and part counts are a multiple of 8 (one residue class per
// XCD), capped so that every chunk keeps >= 8 node columns and every
// observation part >= 16 observations (64 for the FP64 node adjoint) and
// 2 GiB of partial sums (1.07 GB at paper scale).
#ifndef GRAV_TARGET_WAVES_FWD
#define GRAV_TARGET_WAVES_FWD 131072
#endif
#ifndef GRAV_TARGET_WAVES_ADJ
#define GRAV_TARGET_WAVES_ADJ 131072
#endif
static constexpr int64_t kTargetWavesFwd = GRAV_TARGET_WAVES_FWD;
static constexpr int64_t kTargetWavesAdj = GRAV_TARGET_WAVES_ADJ;
static constexpr int64_t kMinColsPerChunk = 8;
// At least 16 observations per part of the mixed adjoint: small surveys
// (about a thousand stations) then split into enough parts to fill the GPU
// (the 32 x 32 x 16 dyke problem's adjoint: 0.25 -> 0.10 ms).  The FP64
// node adjoint keeps 64 (it is the comparator path).
static constexpr int64_t kMinObsPerPart = 16;
static constexpr int64_t kMinObsPerPartNodes = 64;
#ifndef GRAV_MAX_PARTIAL_MIB
#define GRAV_MAX_PARTIAL_MIB 2048
#endif
static constexpr int64_t kMaxPartialBytes = int64_t(GRAV_MAX_PARTIAL_MIB) << 20;

static int64_t round8_capped(int64_t want, int64_t cap) {
    if (cap < 1) cap = 1;
    int64_t v = ceil_div(want, 8) * 8;
    if (v > cap) v = cap;
    if (v < 1) v = 1;
    return v;
}

ForwardPlan plan_forward(int64_t ncols, int64_t n, int64_t target_waves) {
    if (target_waves <= 0) target_waves = kTargetWavesFwd;
    ForwardPlan p;
    p.nblk_obs = ceil_div(n, kBlock);
    const int64_t waves_obs = ceil_div(n, 64);
    const int64_t nchunk = round8_capped(ceil_div(target_waves, waves_obs),
                                         ncols / kMinColsPerChunk);
    p.cols_per_chunk = ceil_div(ncols, nchunk);
    p.nchunk = (int)ceil_div(ncols, p.cols_per_chunk);
    return p;
}

ForwardPlan plan_trace(int nx, int64_t n) {
    // chunks over prism rows i (nx of them), one or more rows per chunk
    ForwardPlan p;
    p.nblk_obs = ceil_div(n, kBlock);
    const int64_t nchunk = round8_capped(ceil_div(kTargetWavesFwd, ceil_div(n, 64)), nx);
    p.cols_per_chunk = ceil_div(nx, nchunk);
    p.nchunk = (int)ceil_div(nx, p.cols_per_chunk);
    return p;
}

// Layer chunks of the mixed adjoint: the layers above the first deep layer and
// the deep ones are chunked separately (the split depends on the mesh, known
// on the device only), ceil(a / 16) + ceil(b / 16) <= ceil(nz / 16) + 1 chunks
// for a + b = nz; chunk indices past the two ranges are empty.
static int adjoint_layer_chunks(int nz) { return (int)ceil_div(nz, kAdjLayers) + 1; }

AdjointPlan plan_adjoint(int64_t ncols, int nz, int64_t n, int64_t target_waves,
                         int64_t max_partial_bytes) {
    if (target_waves <= 0) target_waves = kTargetWavesAdj;
    if (max_partial_bytes <= 0) max_partial_bytes = kMaxPartialBytes;
    AdjointPlan p;
    p.nblk_col = ceil_div(ncols, kBlock);
    p.nkc = adjoint_layer_chunks(nz);
    const int64_t waves = p.nblk_col * p.nkc * (kBlock / 64);
    int64_t cap = n / kMinObsPerPart;
    const int64_t mem_cap = max_partial_bytes / (ncols * nz * 8);
    if (mem_cap < cap) cap = mem_cap;
    const int64_t parts = round8_capped(ceil_div(target_waves, waves), cap);
    p.obs_per_part = ceil_div(n, parts);
    p.nparts = (int)ceil_div(n, p.obs_per_part);
    return p;
}

NodeAdjointPlan plan_adjoint_nodes(int64_t nnodes, int64_t n) {
    NodeAdjointPlan p;
    p.nblk_node = ceil_div(nnodes, kBlock);
    const int64_t waves = p.nblk_node * (kBlock / 64);
    int64_t cap = n / kMinObsPerPartNodes;
    const int64_t mem_cap = kMaxPartialBytes / (nnodes * 8);
    if (mem_cap < cap) cap = mem_cap;
    const int64_t parts = round8_capped(ceil_div(kTargetWavesAdj, waves), cap);
    p.obs_per_part = ceil_div(n, parts);
    p.nparts = (int)ceil_div(n, p.obs_per_part);
    return p;
}

// Upper bounds on the partial-sum buffers above over every survey of at most
// n observations, so that a workspace sized for n serves any smaller survey
// (the plans round counts up to a multiple of 8, which alone is not monotone
// in n).  A chunk count rounded up to a multiple of 8 is below T / w + 8 for
// w = ceil(n' / 64) >= n' / 64 waves, so chunks x n' < 64 T + 8 n'; part
// counts requested for n bound the (monotone) requests of every n' <= n.
int64_t forward_partials_bound(int64_t ncols, int64_t n) {
    int64_t cap = ncols / kMinColsPerChunk;
    if (cap < 1) cap = 1;
    const int64_t a = cap * n, b = 64 * kTargetWavesFwd + 8 * n;
    return a < b ? a : b;
}

int64_t trace_partials_bound(int nx, int64_t n) {
    const int64_t a = (int64_t)(nx < 1 ? 1 : nx) * n, b = 64 * kTargetWavesFwd + 8 * n;
    return a < b ? a : b;
}

int64_t adjoint_parts_bound(int64_t ncols, int nz, int64_t n) {
    const int64_t waves = ceil_div(ncols, kBlock) * adjoint_layer_chunks(nz) * (kBlock / 64);
    int64_t cap = n / kMinObsPerPart;
    const int64_t mem_cap = kMaxPartialBytes / (ncols * nz * 8);
    if (mem_cap < cap) cap = mem_cap;
    return round8_capped(ceil_div(kTargetWavesAdj, waves), cap);
}

int64_t node_adjoint_parts_bound(int64_t nnodes, int64_t n) {
    const int64_t waves = ceil_div(nnodes, kBlock) * (kBlock / 64);
    int64_t cap = n / kMinObsPerPartNodes;
    const int64_t mem_cap = kMaxPartialBytes / (nnodes * 8);
    if (mem_cap < cap) cap = mem_cap;
    return round8_capped(ceil_div(kTargetWavesAdj, waves), cap);
}

// ------------------------------------------------------------------ launchers

hipError_t launch_layer_thickness(const Mesh &g, float *hk, hipStream_t st) {
    k_layer_thickness<<<grid_for(g.nz), 256, 0, st>>>(g.zn, g.nz, hk);
    return hipGetLastError();
}

hipError_t launch_edge_weights(const Mesh &g, const double *m, double *w2, hipStream_t st) {
    k_edge_weights<<<grid_for(g.nsegs()), 256, 0, st>>>(m, g.nx, g.ny, g.nz, w2);
    return hipGetLastError();
}

hipError_t launch_node_weights(const Mesh &g, const double *m, double *wn, hipStream_t st) {
    k_node_weights<<<grid_for(g.nnodes()), 256, 0, st>>>(m, g.nx, g.ny, g.nz, wn);
    return hipGetLastError();
}

hipError_t launch_reduce_parts(const double *part, int nparts, int64_t len, double scale,
                               const double *add, double coef, double *out, hipStream_t st) {
    k_reduce_parts<<<grid_for(len), 256, 0, st>>>(part, nparts, len, scale, add, coef, out);
    return hipGetLastError();
}

hipError_t launch_adjoint_finish_edges(const Mesh &g, const double *U, double scale,
                                       const double *wdepth, const double *base, double *out,
                                       hipStream_t st) {
    k_adjoint_finish_edges<<<grid_for(g.ncells()), 256, 0, st>>>(U, g.nx, g.ny, g.nz, scale,
                                                                 wdepth, base, out);
    return hipGetLastError();
}

hipError_t launch_adjoint_finish_nodes(const Mesh &g, const double *P, double scale,
                                       const double *wdepth, const double *base, double *out,
                                       hipStream_t st) {
    k_adjoint_finish_nodes<<<grid_for(g.ncells()), 256, 0, st>>>(P, g.nx, g.ny, g.nz, scale,
                                                                 wdepth, base, out);
    return hipGetLastError();
}

hipError_t launch_forward_mixed(const Mesh &g, const Obs &o, const float *hk, const double *w2,
                                const ForwardPlan &p, double *partial, hipStream_t st) {
    const int64_t blocks = p.nblk_obs * p.nchunk;
    k_forward_mixed<<<dim3((unsigned)blocks), kBlock, 0, st>>>(
        g.xn, g.yn, g.zn, g.ny + 1, g.nz, hk, o.x, o.y, o.z, o.n, w2, g.ncols(), p.cols_per_chunk,
        p.nchunk, partial);
    return hipGetLastError();
}

hipError_t launch_forward_f64(const Mesh &g, const Obs &o, const double *wn,
                              const ForwardPlan &p, double *partial, hipStream_t st) {
    const int64_t blocks = p.nblk_obs * p.nchunk;
    k_forward_f64<<<dim3((unsigned)blocks), kBlock, 0, st>>>(
        g.xn, g.yn, g.zn, g.ny + 1, g.nz, o.x, o.y, o.z, o.n, wn, g.ncols(), p.cols_per_chunk,
        p.nchunk, partial);
    return hipGetLastError();
}

hipError_t launch_adjoint_mixed(const Mesh &g, const Obs &o, const float *hk, const double *v,
                                const AdjointPlan &p, double *upart, hipStream_t st) {
    const int64_t blocks = p.nblk_col * p.nkc * p.nparts;
    k_adjoint_mixed<<<dim3((unsigned)blocks), kBlock, 0, st>>>(
        g.xn, g.yn, g.zn, g.ny + 1, g.nz, hk, o.x, o.y, o.z, v, o.n, p.obs_per_part, p.nparts,
        g.ncols(), p.nkc, upart);
    return hipGetLastError();
}

hipError_t launch_adjoint_f64(const Mesh &g, const Obs &o, const double *v,
                              const NodeAdjointPlan &p, double *ppart, hipStream_t st) {
    const int64_t blocks = p.nblk_node * p.nparts;
    k_adjoint_f64<<<dim3((unsigned)blocks), kBlock, 0, st>>>(
        g.xn, g.yn, g.zn, g.ny + 1, g.nz, o.x, o.y, o.z, v, o.n, p.obs_per_part, p.nparts,
        g.nnodes(), ppart);
    return hipGetLastError();
}

hipError_t launch_trace_mixed(const Mesh &g, const Obs &o, const float *hk, const double *wdepth,
                              const ForwardPlan &p, double *partial, hipStream_t st) {
    const int64_t blocks = p.nblk_obs * p.nchunk;
    k_trace_mixed<<<dim3((unsigned)blocks), kBlock, 0, st>>>(
        g.xn, g.yn, g.zn, g.nx, g.ny, g.nz, hk, wdepth, o.x, o.y, o.z, o.n, p.cols_per_chunk,
        p.nchunk, partial);
    return hipGetLastError();
}

hipError_t launch_trace_f64(const Mesh &g, const Obs &o, const double *wdepth,
                            const ForwardPlan &p, double *partial, hipStream_t st) {
    const int64_t blocks = p.nblk_obs * p.nchunk;
    k_trace_f64<<<dim3((unsigned)blocks), kBlock, 0, st>>>(
        g.xn, g.yn, g.zn, g.nx, g.ny, g.nz, wdepth, o.x, o.y, o.z, o.n, p.cols_per_chunk,
        p.nchunk, partial);
    return hipGetLastError();
}

hipError_t launch_validate(const Mesh &g, const Obs &o, int *flags, hipStream_t st) {
    int64_t len = o.n;
    if (g.nx > len) len = g.nx;
    if (g.ny > len) len = g.ny;
    if (g.nz > len) len = g.nz;
    k_validate<<<grid_for(len, 256, 1024), 256, 0, st>>>(g.xn, g.nx, g.yn, g.ny, g.zn, g.nz, o.x,
                                                         o.y, o.z, o.n, flags);
    return hipGetLastError();
}

hipError_t launch_validate_positive(const double *w, int64_t len, int *flags, hipStream_t st) {
    k_validate_positive<<<grid_for(len, 256, 1024), 256, 0, st>>>(w, len, flags);
    return hipGetLastError();
}

hipError_t launch_validate_finite(const double *w, int64_t len, int *flags, hipStream_t st) {
    k_validate_finite<<<grid_for(len, 256, 1024), 256, 0, st>>>(w, len, flags);
    return hipGetLastError();
}

}  // namespace grav
