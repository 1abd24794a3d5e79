// Per-block bodies of the mixed-precision sweeps, shared by the single-call
// kernels and by the server's batched multi-request kernels so that both run
// exactly the same arithmetic for a given request and launch plan.
#pragma once

#include "grav_internal.h"
#include "edge_math.h"

namespace grav {

// A pointer the compiler sees as generic (read from memory, or made opaque)
// but which points to device global memory: casting it through the global
// address space lets the compiler use global loads and, for wave-uniform
// addresses, scalar loads instead of the flat path.
template <typename T>
__device__ __forceinline__ T *global_ptr(T *p) {
    return (T *)(__attribute__((address_space(1))) T *)(uintptr_t)p;
}

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
// sum over the chunk's segments of S * W2 (FP64 accumulation).  `lane` in
// [0, kBlock) is the calling thread's place in the block (threadIdx.x for a
// kBlock-thread block).
__device__ __forceinline__ void forward_mixed_block(
    const double *__restrict__ xn, const double *__restrict__ yn, const double *__restrict__ zn,
    int ny1, int nz, const float *__restrict__ hk, const double *__restrict__ ox,
    const double *__restrict__ oy, const double *__restrict__ oz, int64_t n,
    const double *__restrict__ w2, int64_t ncols, int64_t cols_per_chunk, int chunk, int64_t oblk,
    double *__restrict__ partial, int lane) {
    const int64_t o = oblk * kBlock + lane;
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
        // atan(u) of the first deep node, carried down the deep layers in FP64
        double A = k < nz ? static_cast<double>(fm::atan_ratio(c.xy, top.zR)) : 0.0;
#pragma unroll 16
        for (; k < nz; ++k) {
            const int kn = k + 2 < nz ? k + 2 : nz - 1;
            const double wc = w_a;
            const float hc = h_a, zc = z_a;
            w_a = w_b; h_a = h_b; z_a = z_b;
            w_b = w[kn]; h_b = hk[kn]; z_b = zrel[kn];
            const Node bot = make_node(c, zc + ztop);
            const float S = edge_segment_carry(c, top, bot, hc, A);
            acc = fma(static_cast<double>(S), wc, acc);
            top = bot;
        }
        if (++b == ny1) { b = 0; ++a; }
    }
    if (o < n) partial[(int64_t)chunk * n + o] = acc;
}

// One observation's contribution to a lane's layer chunk of the adjoint:
// layers k0 .. k0 + cnt - 1 (1 <= cnt <= kAdjLayers, uniform across the
// block), two layers per step.  The thickness and node depth of the next two
// layers are loaded while the current two compute (indices clamped to the
// chunk's last layer), so each step waits only on loads issued a step earlier;
// the two layers of a step share one guard and need no register copies
// between them.
static_assert(kAdjLayers % 2 == 0, "the adjoint steps two layers at a time");

template <bool kDeep>
__device__ __forceinline__ void adjoint_obs(double X, double Y, const float *__restrict__ zrel,
                                            const float *__restrict__ hk, double zn0, int k0,
                                            int cnt, double xo, double yo, double zo, double vo,
                                            double (&acc)[kAdjLayers]) {
    const Column c = make_column(X, Y, xo, yo);
    const float ztop = static_cast<float>(zn0 - zo);
    Node top = make_node(c, node_depth(zrel, k0, ztop));
    // deep chunks carry atan(u) down their (at most 16) layers in FP32
    float A = kDeep ? fm::atan_ratio(c.xy, top.zR) : 0.0f;
    const int kl = k0 + cnt - 1;
    float za = zrel[k0], zb = zrel[k0 + 1 <= kl ? k0 + 1 : kl];
    float ha = hk[k0], hb = hk[k0 + 1 <= kl ? k0 + 1 : kl];
#pragma unroll
    for (int j = 0; j < kAdjLayers; j += 2) {
        if (j < cnt) {
            const float z1 = za, z2 = zb, h1 = ha, h2 = hb;
            const int n1 = k0 + j + 2 <= kl ? k0 + j + 2 : kl;
            const int n2 = k0 + j + 3 <= kl ? k0 + j + 3 : kl;
            za = zrel[n1]; zb = zrel[n2]; ha = hk[n1]; hb = hk[n2];
            const Node b1 = make_node(c, z1 + ztop);
            const float S1 = kDeep ? edge_segment_carry(c, top, b1, h1, A)
                                   : edge_segment<false>(c, top, b1, h1);
            acc[j] = fma(vo, static_cast<double>(S1), acc[j]);
            if (j + 1 < cnt) {
                const Node b2 = make_node(c, z2 + ztop);
                const float S2 = kDeep ? edge_segment_carry(c, b1, b2, h2, A)
                                       : edge_segment<false>(c, b1, b2, h2);
                acc[j + 1] = fma(vo, static_cast<double>(S2), acc[j + 1]);
                top = b2;
            }
        }
    }
}

// The observation loop of one lane.  The layer count and the two table
// pointers pass through an empty asm statement once per observation: the
// compiler can no longer hoist the per-layer loads out of the loop, where they
// would hold 2 * kAdjLayers scalar registers and cut the waves per SIMD.
template <bool kDeep>
__device__ __forceinline__ void adjoint_obs_range(
    double X, double Y, const float *__restrict__ zrel, const float *__restrict__ hk, double zn0,
    int k0, int cnt, const double *__restrict__ ox, const double *__restrict__ oy,
    const double *__restrict__ oz, const double *__restrict__ v, int64_t o0, int64_t o1,
    double (&acc)[kAdjLayers]) {
    // the next observation's coordinates and weight are loaded while this
    // one's layers compute (index clamped at the part's last observation)
    if (o0 >= o1) return;
    double xq = ox[o0], yq = oy[o0], zq = oz[o0], vq = v[o0];
    for (int64_t o = o0; o < o1; ++o) {
        const double xo = xq, yo = yq, zo = zq, vo = vq;
        const int64_t on = o + 1 < o1 ? o + 1 : o;
        xq = ox[on];
        yq = oy[on];
        zq = oz[on];
        vq = v[on];
        int cnt_o = cnt;
        const float *zr_o = zrel, *hk_o = hk;
        asm volatile("" : "+s"(cnt_o), "+s"(zr_o), "+s"(hk_o));
        adjoint_obs<kDeep>(X, Y, global_ptr(zr_o), global_ptr(hk_o), zn0, k0, cnt_o, xo, yo, zo,
                           vo, acc);
    }
}

// Adjoint sweep, one block: lanes own node columns colblk*kBlock + lane and
// layer chunk kc of nkc (at most 16 consecutive layers, all above the first
// deep layer or all at or below it), observations of part `part`; writes
// upart[part][segment] = sum_{o in part} v_o S (FP64, one register pair per
// layer, no cross-lane reduction).  `lane` as in the forward block.
__device__ __forceinline__ void adjoint_mixed_block(
    const double *__restrict__ xn, const double *__restrict__ yn, const double *__restrict__ zn,
    int ny1, int nz, const float *__restrict__ hk, const double *__restrict__ ox,
    const double *__restrict__ oy, const double *__restrict__ oz, const double *__restrict__ v,
    int64_t n, int64_t obs_per_part, int64_t ncols, int nkc, int part, int kc, int64_t colblk,
    double *__restrict__ upart, int lane) {
    const int64_t col = colblk * kBlock + lane;
    const int64_t colc = col < ncols ? col : ncols - 1;
    int a, b;
    if (ncols <= 0x7fffffff) {   // 32-bit division when the column index fits
        const unsigned cu = (unsigned)colc;
        a = (int)(cu / (unsigned)ny1);
        b = (int)(cu - (unsigned)a * (unsigned)ny1);
    } else {
        a = (int)(colc / ny1);
        b = (int)(colc - (int64_t)a * ny1);
    }
    // Layer chunks: the layers above the first deep one (kdeep) and the deep
    // layers are chunked separately, ceil(len / kAdjLayers) balanced chunks each,
    // so that every deep layer takes the short formula; nkc (from plan_adjoint)
    // leaves room for both and chunks past them are empty.
    const int kdeep = reinterpret_cast<const int *>(hk + nz)[0];
    const int ng = (kdeep + kAdjLayers - 1) / kAdjLayers;
    const bool deep = kc >= ng;   // uniform per block
    const int lo = deep ? kdeep : 0, len = deep ? nz - kdeep : kdeep;
    const int idx = deep ? kc - ng : kc;
    const int nch = (len + kAdjLayers - 1) / kAdjLayers;
    if (idx >= nch) return;
    const int kq = len / nch, kr = len - kq * nch;
    const int k0 = lo + idx * kq + (idx < kr ? idx : kr);
    const int cnt = kq + (idx < kr ? 1 : 0);
    const double X = xn[a], Y = yn[b];
    const float *__restrict__ zrel = hk + nz + 1;
    const double zn0 = zn[0];
    double acc[kAdjLayers];
#pragma unroll
    for (int j = 0; j < kAdjLayers; ++j) acc[j] = 0.0;
    const int64_t o0 = (int64_t)part * obs_per_part;
    const int64_t o1 = o0 + obs_per_part < n ? o0 + obs_per_part : n;
    if (deep)
        adjoint_obs_range<true>(X, Y, zrel, hk, zn0, k0, cnt, ox, oy, oz, v, o0, o1, acc);
    else
        adjoint_obs_range<false>(X, Y, zrel, hk, zn0, k0, cnt, ox, oy, oz, v, o0, o1, acc);
    if (col < ncols) {
        double *__restrict__ dst = upart + (int64_t)part * ncols * nz + col * nz + k0;
#pragma unroll
        for (int j = 0; j < kAdjLayers; ++j)
            if (j < cnt) dst[j] = acc[j];
    }
}

}  // namespace grav
