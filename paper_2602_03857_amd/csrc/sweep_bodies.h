// Per-block bodies of the mixed-precision sweeps, shared by the single-call
// kernels and by the server's batched multi-request kernels so that both run
// exactly the same arithmetic for a given request and launch plan.
#pragma once

#include "grav_internal.h"
#include "edge_math.h"

namespace grav {

// Depth below the observation of node c of a column, Z_c - z_o, as the FP32 sum
// of (Z_c - Z_0) from the layer table and ztop = Z_0 - z_o: both terms are
// non-negative FP64 differences rounded to FP32, so the sum has no
// cancellation (relative error below 2^-22), and every sweep forms the same
// value for the same node.
__device__ __forceinline__ float node_depth(const float *__restrict__ zrel, int c, float ztop) {
    return c == 0 ? ztop : zrel[c - 1] + ztop;
}

// Forward sweep, one block: observations oblk*kBlock + [0, kBlock) against node
// columns [chunk*cols_per_chunk, ...), writing partial[chunk*n + o] =
// sum over the chunk's segments of S * W2 (FP64 accumulation).
__device__ __forceinline__ void forward_mixed_block(
    const double *__restrict__ xn, const double *__restrict__ yn, const double *__restrict__ zn,
    int ny1, int nz, const float *__restrict__ hk, const double *__restrict__ ox,
    const double *__restrict__ oy, const double *__restrict__ oz, int64_t n,
    const double *__restrict__ w2, int64_t ncols, int64_t cols_per_chunk, int chunk, int64_t oblk,
    double *__restrict__ partial) {
    const int64_t o = oblk * kBlock + threadIdx.x;
    const int64_t oc = o < n ? o : n - 1;
    const double xo = ox[oc], yo = oy[oc], zo = oz[oc];
    const float ztop = static_cast<float>(zn[0] - zo);
    const int64_t c0 = (int64_t)chunk * cols_per_chunk;
    const int64_t c1 = c0 + cols_per_chunk < ncols ? c0 + cols_per_chunk : ncols;
    const int kdeep = reinterpret_cast<const int *>(hk + nz)[0];
    const float *__restrict__ zrel = hk + nz + 1;
    double acc = 0.0;
    int a = (int)(c0 / ny1), b = (int)(c0 - (int64_t)a * ny1);
    for (int64_t col = c0; col < c1; ++col) {
        const Column c = make_column(xn[a], yn[b], xo, yo);
        Node top = make_node(c, ztop);
        const double *__restrict__ w = w2 + col * nz;
        // The layer constants (edge weight, thickness, node depth) are
        // wave-uniform scalar loads.  Used as soon as they are loaded, each
        // layer would wait on a scalar-cache round trip; instead they run
        // through a two-deep pipeline: layer k's values were loaded while
        // layers k-2 and k-1 were computed (indices clamped at the last layer,
        // so no load leaves the column).
        int k = 0;
        double w_a = w[0], w_b = w[nz > 1 ? 1 : 0];
        float h_a = hk[0], z_a = zrel[0], h_b = hk[nz > 1 ? 1 : 0], z_b = zrel[nz > 1 ? 1 : 0];
#pragma unroll 16
        for (; k < kdeep; ++k) {
            const int kn = k + 2 < nz ? k + 2 : nz - 1;
            const double wc = w_a;
            const float hc = h_a, zc = z_a;
            w_a = w_b; h_a = h_b; z_a = z_b;
            w_b = w[kn]; h_b = hk[kn]; z_b = zrel[kn];
            const Node bot = make_node(c, zc + ztop);
            const float S = edge_segment<false>(c, top, bot, hc);
            acc = fma(static_cast<double>(S), wc, acc);
            top = bot;
        }
#pragma unroll 16
        for (; k < nz; ++k) {
            const int kn = k + 2 < nz ? k + 2 : nz - 1;
            const double wc = w_a;
            const float hc = h_a, zc = z_a;
            w_a = w_b; h_a = h_b; z_a = z_b;
            w_b = w[kn]; h_b = hk[kn]; z_b = zrel[kn];
            const Node bot = make_node(c, zc + ztop);
            const float S = edge_segment<true>(c, top, bot, hc);
            acc = fma(static_cast<double>(S), wc, acc);
            top = bot;
        }
        if (++b == ny1) { b = 0; ++a; }
    }
    if (o < n) partial[(int64_t)chunk * n + o] = acc;
}

// One observation's contribution to a lane's layer chunk of the adjoint:
// layers k0 .. k0 + cnt - 1 (cnt <= kAdjLayers; the guard on j < cnt is
// uniform across the block).
template <bool kDeep>
__device__ __forceinline__ void adjoint_obs(double X, double Y, const float *__restrict__ zrel,
                                            double zn0, int k0, int cnt,
                                            const float (&h)[kAdjLayers], double xo, double yo,
                                            double zo, double vo, double (&acc)[kAdjLayers]) {
    const Column c = make_column(X, Y, xo, yo);
    const float ztop = static_cast<float>(zn0 - zo);
    Node top = make_node(c, node_depth(zrel, k0, ztop));
#pragma unroll
    for (int j = 0; j < kAdjLayers; ++j) {
        if (j < cnt) {
            const Node bot = make_node(c, zrel[k0 + j] + ztop);
            const float S = edge_segment<kDeep>(c, top, bot, h[j]);
            acc[j] = fma(vo, static_cast<double>(S), acc[j]);
            top = bot;
        }
    }
}

// Adjoint sweep, one block: lanes own node columns colblk*kBlock + lane and
// layer chunk kc of nkc (nkc = ceil(nz / kAdjLayers) chunks of near-equal
// length, at most kAdjLayers layers each), observations of part `part`;
// writes upart[part][segment] = sum_{o in part} v_o S (FP64, one register
// pair per layer, no cross-lane reduction).
__device__ __forceinline__ void adjoint_mixed_block(
    const double *__restrict__ xn, const double *__restrict__ yn, const double *__restrict__ zn,
    int ny1, int nz, const float *__restrict__ hk, const double *__restrict__ ox,
    const double *__restrict__ oy, const double *__restrict__ oz, const double *__restrict__ v,
    int64_t n, int64_t obs_per_part, int64_t ncols, int nkc, int part, int kc, int64_t colblk,
    double *__restrict__ upart) {
    const int64_t col = colblk * kBlock + threadIdx.x;
    const int64_t colc = col < ncols ? col : ncols - 1;
    const int a = (int)(colc / ny1);
    const int b = (int)(colc - (int64_t)a * ny1);
    const double X = xn[a], Y = yn[b];
    const int k0 = (int)((int64_t)kc * nz / nkc);
    const int cnt = (int)((int64_t)(kc + 1) * nz / nkc) - k0;
    const float *__restrict__ zrel = hk + nz + 1;
    const double zn0 = zn[0];
    float h[kAdjLayers];
#pragma unroll
    for (int j = 0; j < kAdjLayers; ++j) h[j] = j < cnt ? hk[k0 + j] : 1.0f;
    double acc[kAdjLayers];
#pragma unroll
    for (int j = 0; j < kAdjLayers; ++j) acc[j] = 0.0;
    const int64_t o0 = (int64_t)part * obs_per_part;
    const int64_t o1 = o0 + obs_per_part < n ? o0 + obs_per_part : n;
    const bool deep = k0 >= reinterpret_cast<const int *>(hk + nz)[0];   // uniform per block
    if (deep) {
        for (int64_t o = o0; o < o1; ++o)
            adjoint_obs<true>(X, Y, zrel, zn0, k0, cnt, h, ox[o], oy[o], oz[o], v[o], acc);
    } else {
        for (int64_t o = o0; o < o1; ++o)
            adjoint_obs<false>(X, Y, zrel, zn0, k0, cnt, h, ox[o], oy[o], oz[o], v[o], acc);
    }
    if (col < ncols) {
        double *__restrict__ dst = upart + (int64_t)part * ncols * nz + col * nz + k0;
#pragma unroll
        for (int j = 0; j < kAdjLayers; ++j)
            if (j < cnt) dst[j] = acc[j];
    }
}

}  // namespace grav
