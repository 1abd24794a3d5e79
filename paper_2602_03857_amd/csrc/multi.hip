// Multi-model forward D = G [m_1 ... m_K] (paper Eq. 6 applied to a block of
// K <= 64 density models): a dense contraction over prisms, so it runs on
// the matrix cores.
//
// Per workgroup: 64 observations x all 64 (padded) models and one chunk of
// consecutive kPBX x kPBY prism-column blocks; the layers are the outer loop,
// two per step, and the chunk's blocks the inner one.  One block step (two
// layers of one block):
//   1. VALU: edge-segment terms S of the block's vertical edges in both
//      layers for the 64 observations -> LDS.  Consecutive blocks along y
//      share an edge row, and the LDS rows form a ring, so a step evaluates
//      only the (kPBX+1) x kPBY new edges: 20 for the 16 prisms of a 4 x 4
//      block (1.25 per prism, five per wave), all 25 at the start of a chunk
//      or a block row.  Each edge takes three nodes for its two segments, and
//      the angle atan(u) of the middle node, evaluated for the upper segment,
//      is carried to the lower one by the addition formula of atan.
//   Then per layer of the step:
//   2. VALU: per prism G = S00 - S10 - S01 + S11 (the (x, y) vertex parity of
//      Eq. 1), split into bf16 hi = bf16(G), lo = bf16(G - hi) -> LDS in the
//      MFMA A-operand order (obs x prisms).
//   3. MFMA: four waves each own a 32 obs x 32 model block;
//      acc += A_hi B_hi + A_hi B_lo + A_lo B_hi with v_mfma_f32_32x32x16_bf16
//      (FP32 accumulation), 16 prisms per instruction, B = the models
//      pre-split into bf16 hi/lo and packed so that each lane loads its 8
//      operands with one 16-byte load, issued after step 2.
// Every kFlushBlocks layer steps and at the end of each pair of layers the
// FP32 accumulators are added into per-thread FP64 accumulators (some in
// registers, the rest in LDS), so FP32 sums at most 512 prism terms.  The
// GRAV_FP32_VALU variant keeps steps 1-2 (G in FP32) and contracts on the
// vector ALUs.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "api_internal.h"
#include "edge_math.h"

namespace grav {

namespace {

constexpr int kTileObs = 64;
#ifndef GRAV_MULTI_PBX
#define GRAV_MULTI_PBX 4
#endif
#ifndef GRAV_MULTI_PBY
#define GRAV_MULTI_PBY 4
#endif
constexpr int kPBX = GRAV_MULTI_PBX;                     // prism columns per block along x
constexpr int kPBY = GRAV_MULTI_PBY;                     // ... along y
constexpr int kEdgeX = kPBX + 1, kEdgeY = kPBY + 1;
constexpr int kPrismsPerStep = kPBX * kPBY;              // prisms per layer step
constexpr int kKSteps = kPrismsPerStep / 16;             // MFMA K = 16 per instruction
constexpr int kModels = 64;
static_assert(kPrismsPerStep % 16 == 0, "prisms per step must fill whole MFMA K blocks");
static_assert(kPBX % 4 == 0, "each of the four waves forms kPBX / 4 prism rows");
static_assert(kPBY == 4, "a prism row is stored as one 8-byte (bf16) or 16-byte (FP32) write");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Packed bf16 hi/lo models: index ((blk * nz + k) * 64 + j) * P + p, with
// P = kPrismsPerStep, blk = bi * nby + bj the prism-column block and
// p = ii * kPBY + jj inside it.
__global__ void k_pack_models_bf16(const float *__restrict__ models, int K, int nx, int ny, int nz,
                                   int nby, int64_t total, __bf16 *__restrict__ hi,
                                   __bf16 *__restrict__ lo) {
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(idx % kPrismsPerStep);
        const int j = (int)((idx / kPrismsPerStep) & 63);
        const int64_t rest = idx / (kPrismsPerStep * kModels);
        const int k = (int)(rest % nz);
        const int64_t blk = rest / nz;
        const int i = (int)(blk / nby) * kPBX + p / kPBY;
        const int jj = (int)(blk % nby) * kPBY + p % kPBY;
        float v = 0.0f;
        if (j < K && i < nx && jj < ny) v = models[(((int64_t)i * ny + jj) * nz + k) * K + j];
        const __bf16 h = static_cast<__bf16>(v);
        hi[idx] = h;
        lo[idx] = static_cast<__bf16>(v - static_cast<float>(h));
    }
}

// Packed FP32 models for the VALU path: ((blk * nz + k) * P + p) * 64 + j.
__global__ void k_pack_models_f32(const float *__restrict__ models, int K, int nx, int ny, int nz,
                                  int nby, int64_t total, float *__restrict__ out) {
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(idx & 63);
        const int p = (int)((idx >> 6) % kPrismsPerStep);
        const int64_t rest = idx / (kPrismsPerStep * kModels);
        const int k = (int)(rest % nz);
        const int64_t blk = rest / nz;
        const int i = (int)(blk / nby) * kPBX + p / kPBY;
        const int jj = (int)(blk % nby) * kPBY + p % kPBY;
        float v = 0.0f;
        if (j < K && i < nx && jj < ny) v = models[(((int64_t)i * ny + jj) * nz + k) * K + j];
        out[idx] = v;
    }
}

// FP64 accumulators per thread held in registers (the other 16 - n in LDS):
// as many as keep the block's LDS within a quarter of the CU's 160 KiB (four
// blocks of four waves per CU), the MFMA kernel holding less LDS than the
// VALU kernel's model tile.
#ifndef GRAV_MULTI_REG_ACC
#define GRAV_MULTI_REG_ACC 5
#endif
constexpr int kRegAccMfma = GRAV_MULTI_REG_ACC;
constexpr int kRegAccValu = 8;
static_assert(kRegAccMfma >= 1 && kRegAccMfma < 16, "at least one accumulator lives in LDS");

// Accumulator v of thread t (v is a compile-time index after unrolling).
template <int kRA>
__device__ __forceinline__ double &acc_ref(double (&r)[kRA], double (&lds)[16 - kRA][256], int v,
                                           int t) {
    return v < kRA ? r[v] : lds[v - kRA][t];
}

// The FP32 accumulators (MFMA or VALU) are added into the FP64 ones after
// this many layer steps of a block and at the end of every pair of layers, so
// an FP32 sum holds at most kFlushBlocks * kPrismsPerStep prism terms.
constexpr int kFlushBlocks = 32;

template <bool kMfma>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_forward_multi(
    const double *__restrict__ xn, const double *__restrict__ yn, const double *__restrict__ zn,
    int nx, int ny, int nz, const float *__restrict__ hk, const double *__restrict__ ox,
    const double *__restrict__ oy, const double *__restrict__ oz, int64_t n,
    const __bf16 *__restrict__ bhi, const __bf16 *__restrict__ blo,
    const float *__restrict__ b32, int nby, int64_t nblk, int64_t blocks_per_chunk, int nchunk,
    double *__restrict__ partial) {
    // edge terms of the current block step: [layer of the step][y slot][x
    // edge][observation]; the kEdgeY y slots form a ring, so the last edge row
    // of one block is the first of the next block along y without being copied
    // (slot indices stay below 2 kEdgeY, so one subtraction wraps them)
    static_assert(kPBY < kEdgeY, "a block's edge rows fit the ring");
    auto ring = [](int x) { return x >= kEdgeY ? x - kEdgeY : x; };
    __shared__ float sS[2][kEdgeY][kEdgeX][kTileObs];
    __shared__ __attribute__((aligned(16))) __bf16 sAhi[kTileObs][kPrismsPerStep];
    __shared__ __attribute__((aligned(16))) __bf16 sAlo[kTileObs][kPrismsPerStep];
    __shared__ __attribute__((aligned(16))) float sA32[kTileObs][kPrismsPerStep];
    __shared__ __attribute__((aligned(16))) float sB32[kPrismsPerStep][kModels];
    // per-thread FP64 accumulators: the first kRA in registers, the rest in
    // LDS (column t), which keeps the block's LDS small enough for four blocks
    // per CU
    constexpr int kRA = kMfma ? kRegAccMfma : kRegAccValu;
    __shared__ double sAcc[16 - kRA][256];
    double rAcc[kRA];

    const int chunk = (int)(blockIdx.x % nchunk);
    const int64_t tile = blockIdx.x / nchunk;
    const int t = threadIdx.x;
    const int lo_ = t & 63;          // observation within the tile (phases 1-2), lane (phase 3)
    // wave index 0..3, made wave-uniform for the compiler (readfirstlane), so
    // that the edge rows, prism rows and their bounds checks that depend on it
    // use scalar loads and branches instead of per-lane masks
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int64_t o = tile * kTileObs + lo_;
    const int64_t oc = o < n ? o : n - 1;
    const double xo = ox[oc], yo = oy[oc], zo = oz[oc];
    const int kdeep = reinterpret_cast<const int *>(hk + nz)[0];
    const int64_t b0 = (int64_t)chunk * blocks_per_chunk;
    const int64_t b1 = b0 + blocks_per_chunk < nblk ? b0 + blocks_per_chunk : nblk;
    const int bi0 = (int)(b0 / nby), bj0 = (int)(b0 - (int64_t)bi0 * nby);

    // phase-3 roles
    const int r0 = 32 * (wv & 1), c0 = 32 * (wv >> 1);
    f32x16 acc;
    float acc32[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        acc[v] = 0.0f;
        acc32[v] = 0.0f;
        acc_ref<kRA>(rAcc, sAcc, v, t) = 0.0;
    }
    auto flush = [&]() {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            if (kMfma) {
                acc_ref<kRA>(rAcc, sAcc, v, t) += static_cast<double>(acc[v]);
                acc[v] = 0.0f;
            } else {
                acc_ref<kRA>(rAcc, sAcc, v, t) += static_cast<double>(acc32[v]);
                acc32[v] = 0.0f;
            }
        }
    };

    // Layers outside (two per step), the chunk's prism-column blocks inside:
    // consecutive blocks along y share an edge row, so a block step evaluates
    // the kEdgeX x kPBY new edges only (4 x 4 block: 20 edges for 16 prisms,
    // 1.25 per prism, five per wave), and the full kEdgeX x kEdgeY at the
    // start of a chunk or of a block row.  Each edge is walked over the two
    // layers k, k + 1 of the step: three nodes instead of four, and the angle
    // atan(u) of the middle node, evaluated for layer k, is carried to the
    // bottom node by the addition formula (atan(u2) = atan(u1) + atan(delta),
    // u1 u2 >= 0), so the second segment needs no range-reduced atan of its
    // own.  The middle node lies at least one layer below the mesh top (z > 0).
    for (int k = 0; k < nz; k += 2) {
        const bool two = k + 1 < nz;    // uniform; the last step of an odd nz has one layer
        const float zt = static_cast<float>(zn[k] - zo);
        const float zm = static_cast<float>(zn[k + 1] - zo);
        const float zb = two ? static_cast<float>(zn[k + 2] - zo) : zm;
        const float h0 = hk[k];
        const float h1 = two ? hk[k + 1] : 0.0f;
        const bool deep0 = k >= kdeep, deep1 = k + 1 >= kdeep;   // uniform
        int slot0 = 0;                  // ring slot of the block's first edge row
        int nacc = 0;
        float cxr[kEdgeX];              // x offsets of the current block row's edges
        bool vx[kEdgeX];
        int bi = bi0, bj = bj0;         // block coordinates of blk, stepped along y
        for (int64_t blk = b0; blk < b1; ++blk) {
            const int i0 = bi * kPBX, j0 = bj * kPBY;
            const bool fresh = blk == b0 || bj == 0;
            if (fresh) {
                slot0 = 0;
#pragma unroll
                for (int ii = 0; ii < kEdgeX; ++ii) {
                    const int a = i0 + ii;
                    vx[ii] = a <= nx;
                    cxr[ii] = column_offset(xn[a <= nx ? a : nx], xo);
                }
            } else {
                slot0 = ring(slot0 + kPBY);
            }
            // phase 1: edge terms S of both layers for edge row q (y node
            // j0 + q) at the x edges ii with (ii mod 4) == wv, or at all of them
            auto edge_row = [&](auto d0, auto d1, int q, bool all_x) {
                constexpr bool kD0 = decltype(d0)::value, kD1 = decltype(d1)::value;
                const int b = j0 + q;
                const bool vy = b <= ny;
                const float cy = column_offset(yn[vy ? b : ny], yo);
                const int slot = ring(slot0 + q);
#pragma unroll
                for (int ii = 0; ii < kEdgeX; ++ii) {
                    if (all_x || (ii & 3) == wv) {
                        const Column col = column_from_xy(cxr[ii], cy);
                        const Node top = make_node(col, zt);
                        const Node mid = make_node(col, zm);
                        const Node bot = make_node(col, zb);
                        float lnY, lnX;
                        const float hz0 = h0 * (top.z + mid.z);
                        edge_logs<kD0>(col, top, mid, hz0, lnY, lnX);
                        const float A = fm::atan_ratio(col.xy, mid.zR);
                        const float atd0 = edge_atan_delta<kD0>(col, top, mid, hz0);
                        const float S0 = edge_assemble<kD0>(col, top, h0, A, atd0, lnY, lnX);
                        const float hz1 = h1 * (mid.z + bot.z);
                        edge_logs<kD1>(col, mid, bot, hz1, lnY, lnX);
                        const float atd1 = edge_atan_delta<kD1>(col, mid, bot, hz1);
                        const float S1 = edge_assemble<kD1>(col, mid, h1, A + atd1, atd1, lnY, lnX);
                        const bool valid = vx[ii] && vy;
                        sS[0][slot][ii][lo_] = valid ? S0 : 0.0f;
                        sS[1][slot][ii][lo_] = valid ? S1 : 0.0f;
                    }
                }
            };
            auto phase1 = [&](auto d0, auto d1) {
                // wave wv owns the new edge row q = wv + 1 (kPBY == 4 waves)
                edge_row(d0, d1, wv + 1, true);
                if (fresh) edge_row(d0, d1, 0, false);
            };
            if (deep0)
                phase1(std::true_type{}, std::true_type{});
            else if (deep1)
                phase1(std::false_type{}, std::true_type{});
            else
                phase1(std::false_type{}, std::false_type{});
            for (int L = 0; L < (two ? 2 : 1); ++L) {
                const int kl = k + L;
                // L = 0: the edge terms are complete; L = 1: every wave is
                // done reading layer k's prism terms before they are replaced
                __syncthreads();
                // phase 2: prism terms of prism rows ii = wv, wv + 4, ... (all
                // jj) for observation lo_.  A row's kPBY prisms are stored with
                // one vector write per array (scattered 2-byte writes to rows
                // 32 bytes apart conflict on the LDS banks).
#pragma unroll
                for (int r = 0; r < kPBX / 4; ++r) {
                    const int ii = wv + 4 * r;
                    __bf16 hi4[kPBY], lo4[kPBY];
                    float g4[kPBY];
#pragma unroll
                    for (int q = 0; q < kPBY; ++q) {
                        const int s0 = ring(slot0 + q), s1 = ring(slot0 + q + 1);
                        float G = (sS[L][s0][ii][lo_] - sS[L][s0][ii + 1][lo_]) -
                                  (sS[L][s1][ii][lo_] - sS[L][s1][ii + 1][lo_]);
                        G = (i0 + ii < nx && j0 + q < ny) ? G : 0.0f;
                        g4[q] = G;
                        hi4[q] = static_cast<__bf16>(G);
                        lo4[q] = static_cast<__bf16>(G - static_cast<float>(hi4[q]));
                    }
                    const int p0 = ii * kPBY;
                    if (kMfma) {
                        *reinterpret_cast<bf16x4 *>(&sAhi[lo_][p0]) = *reinterpret_cast<bf16x4 *>(hi4);
                        *reinterpret_cast<bf16x4 *>(&sAlo[lo_][p0]) = *reinterpret_cast<bf16x4 *>(lo4);
                    } else {
                        *reinterpret_cast<float4 *>(&sA32[lo_][p0]) = *reinterpret_cast<float4 *>(g4);
                    }
                }
                if (!kMfma) {
                    const float4 *src = reinterpret_cast<const float4 *>(
                        b32 + ((blk * nz + kl) * kPrismsPerStep) * kModels);
                    for (int q = t; q < kPrismsPerStep * kModels / 4; q += 256)
                        reinterpret_cast<float4 *>(&sB32[0][0])[q] = src[q];
                }
                // this layer's model operands: loaded here, after the edge and
                // prism terms, they wait at the barrier instead of holding
                // eight registers through phase 1
                bf16x8 bh[kKSteps], bl[kKSteps];
                if (kMfma) {
                    const int l = lo_;
                    const int64_t bo =
                        ((blk * nz + kl) * kModels + c0 + (l & 31)) * kPrismsPerStep + (l >> 5) * 8;
#pragma unroll
                    for (int kk = 0; kk < kKSteps; ++kk) {
                        bh[kk] = *reinterpret_cast<const bf16x8 *>(bhi + bo + 16 * kk);
                        bl[kk] = *reinterpret_cast<const bf16x8 *>(blo + bo + 16 * kk);
                    }
                }
                __syncthreads();
                // phase 3: contraction over the prisms of this layer step
                if (kMfma) {
                    const int l = lo_;
#pragma unroll
                    for (int kk = 0; kk < kKSteps; ++kk) {
                        const int kc = 16 * kk + (l >> 5) * 8;
                        const bf16x8 ahi = *reinterpret_cast<const bf16x8 *>(&sAhi[r0 + (l & 31)][kc]);
                        const bf16x8 alo = *reinterpret_cast<const bf16x8 *>(&sAlo[r0 + (l & 31)][kc]);
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, bh[kk], acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, bl[kk], acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bh[kk], acc, 0, 0, 0);
                    }
                } else {
#pragma unroll
                    for (int p = 0; p < kPrismsPerStep; ++p) {
                        const float gp = sA32[lo_][p];
#pragma unroll
                        for (int v = 0; v < 16; ++v) acc32[v] = fmaf(gp, sB32[p][wv * 16 + v], acc32[v]);
                    }
                }
                if (++nacc == kFlushBlocks) {
                    flush();
                    nacc = 0;
                }
            }
            if (++bj == nby) {
                bj = 0;
                ++bi;
            }
        }
        if (nacc > 0) flush();
    }

    if (kMfma) {
        const int l = lo_;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int row = r0 + 8 * (v >> 2) + 4 * (l >> 5) + (v & 3);
            const int64_t og = tile * kTileObs + row;
            if (og < n)
                partial[((int64_t)chunk * n + og) * kModels + c0 + (l & 31)] =
                    acc_ref<kRA>(rAcc, sAcc, v, t);
        }
    } else if (o < n) {
#pragma unroll
        for (int v = 0; v < 16; ++v)
            partial[((int64_t)chunk * n + o) * kModels + wv * 16 + v] = acc_ref<kRA>(rAcc, sAcc, v, t);
    }
}

// D[o*K + j] = gamma * sum_chunks partial[chunk][o][j]   (j < K), FP32 output
__global__ void k_reduce_multi(const double *__restrict__ partial, int nchunk, int64_t n, int K,
                               double scale, float *__restrict__ D) {
    const int64_t total = n * K;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = idx / K;
        const int j = (int)(idx % K);
        double s = 0.0;
        for (int c = 0; c < nchunk; ++c) s += partial[((int64_t)c * n + o) * kModels + j];
        D[idx] = static_cast<float>(scale * s);
    }
}

// hk[k] = Z_{k+1} - Z_k; hk[nz] (as int) = first layer of the deep run: every
// layer from it on has its top at least kDeepRatio thicknesses and
// kDeepMinDepth below the mesh top.
__global__ void k_layer_thickness_m(const double *__restrict__ zn, int nz, float *__restrict__ hk) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nz) hk[k] = static_cast<float>(zn[k + 1] - zn[k]);
    if (k == 0) {
        int kdeep = nz;
        while (kdeep > 0 && (zn[kdeep - 1] - zn[0]) >= kDeepRatio * (zn[kdeep] - zn[kdeep - 1]) &&
               (zn[kdeep - 1] - zn[0]) >= kDeepMinDepth)
            --kdeep;
        reinterpret_cast<int *>(hk + nz)[0] = kdeep;
    }
}

struct MultiPlan {
    int nbx, nby;
    int64_t nblk, ntile, blocks_per_chunk;
    int nchunk;
};

MultiPlan plan_multi(const Mesh &g, int64_t n) {
    MultiPlan p;
    p.nbx = (int)cdiv(g.nx, kPBX);
    p.nby = (int)cdiv(g.ny, kPBY);
    p.nblk = (int64_t)p.nbx * p.nby;
    p.ntile = cdiv(n, kTileObs);
    // a multiple of 8 chunks: block b works on chunk b mod nchunk and runs on
    // XCD b mod 8, so each XCD only ever reads its own chunks' packed models
    // and the tiles working on one chunk share them in that XCD's L2
    int64_t nchunk = cdiv(cdiv(4096, p.ntile), 8) * 8;
    if (nchunk > p.nblk) nchunk = p.nblk;
    if (nchunk < 1) nchunk = 1;
    p.blocks_per_chunk = cdiv(p.nblk, nchunk);
    p.nchunk = (int)cdiv(p.nblk, p.blocks_per_chunk);
    return p;
}

unsigned grid_cap(int64_t len) {
    int64_t gsz = cdiv(len, 256);
    if (gsz < 1) gsz = 1;
    if (gsz > 16384) gsz = 16384;
    return (unsigned)gsz;
}

}  // namespace

uint64_t multi_workspace_need(const Mesh &g, int64_t n, grav_prec prec, int K) {
    (void)K;
    const MultiPlan mp = plan_multi(g, n);
    Counter c;
    const size_t packed = (size_t)mp.nblk * g.nz * kModels * kPrismsPerStep;
    if (prec == GRAV_MIXED_BF16X3) {
        c.take<__bf16>(packed);
        c.take<__bf16>(packed);
    } else {
        c.take<float>(packed);
    }
    c.take<float>(g.nz + 1);
    // chunks x n for every survey of at most n observations: a chunk count
    // rounded up to a multiple of 8 is below 4096 / tiles + 8, and tiles >=
    // n / kTileObs, so chunks x n stays below 4096 kTileObs + 8 n
    int64_t cn = (mp.nblk > 0 ? mp.nblk : 1) * n;
    const int64_t cn_round = 4096 * (int64_t)kTileObs + 8 * n;
    if (cn_round < cn) cn = cn_round;
    c.take<double>((size_t)cn * kModels);
    return c.off;
}

}  // namespace grav

using namespace grav;

extern "C" int grav_forward_multi(grav_ctx *ctx, const grav_mesh *mesh, const grav_obs *obs,
                                  const float *models, int32_t K, float *D, grav_prec prec,
                                  grav_stream stream) {
    if (!ctx) return GRAV_EINVAL;
    ctx->err.clear();
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
    int rc = check_geometry_host(ctx, mesh, obs);
    if (rc) return rc;
    if (!models || !D) return fail(ctx, GRAV_EINVAL, "models or D is NULL");
    if (K < 1 || K > kModels) return fail(ctx, GRAV_EINVAL, "K must be in [1, 64]");
    if (prec != GRAV_MIXED_BF16X3 && prec != GRAV_FP32_VALU)
        return fail(ctx, GRAV_EINVAL, "precision must be GRAV_MIXED_BF16X3 or GRAV_FP32_VALU");
    const Mesh g{mesh->nx, mesh->ny, mesh->nz, mesh->xn, mesh->yn, mesh->zn};
    const Obs o{obs->n, obs->x, obs->y, obs->z};
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    rc = validate_on_device(ctx, g, o, st, {});
    if (rc) return rc;

    const MultiPlan mp = plan_multi(g, o.n);
    Arena ar = ctx_arena(ctx);
    const size_t packed = (size_t)mp.nblk * g.nz * kModels * kPrismsPerStep;
    __bf16 *bhi = nullptr, *blo = nullptr;
    float *b32 = nullptr;
    if (prec == GRAV_MIXED_BF16X3) {
        bhi = ar.take<__bf16>(packed);
        blo = ar.take<__bf16>(packed);
    } else {
        b32 = ar.take<float>(packed);
    }
    float *hk = ar.take<float>(g.nz + 1);
    double *part = ar.take<double>((size_t)mp.nchunk * o.n * kModels);
    if (ar.failed) return fail(ctx, GRAV_ENOMEM, "workspace too small for the multi-model forward");

    k_layer_thickness_m<<<(unsigned)cdiv(g.nz, 256), 256, 0, st>>>(g.zn, g.nz, hk);
    if (prec == GRAV_MIXED_BF16X3)
        k_pack_models_bf16<<<grid_cap((int64_t)packed), 256, 0, st>>>(models, K, g.nx, g.ny, g.nz,
                                                                     mp.nby, (int64_t)packed, bhi, blo);
    else
        k_pack_models_f32<<<grid_cap((int64_t)packed), 256, 0, st>>>(models, K, g.nx, g.ny, g.nz,
                                                                    mp.nby, (int64_t)packed, b32);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "pack models");
    const unsigned blocks = (unsigned)(mp.ntile * mp.nchunk);
    {
        KernelTimer kt(ctx, prec == GRAV_MIXED_BF16X3 ? "multi_bf16x3" : "multi_fp32", st);
        if (prec == GRAV_MIXED_BF16X3)
            k_forward_multi<true><<<blocks, 256, 0, st>>>(g.xn, g.yn, g.zn, g.nx, g.ny, g.nz, hk, o.x,
                                                          o.y, o.z, o.n, bhi, blo, nullptr, mp.nby,
                                                          mp.nblk, mp.blocks_per_chunk, mp.nchunk,
                                                          part);
        else
            k_forward_multi<false><<<blocks, 256, 0, st>>>(g.xn, g.yn, g.zn, g.nx, g.ny, g.nz, hk, o.x,
                                                           o.y, o.z, o.n, nullptr, nullptr, b32, mp.nby,
                                                           mp.nblk, mp.blocks_per_chunk, mp.nchunk,
                                                           part);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(ctx, e, "multi-model sweep");
    }
    k_reduce_multi<<<grid_cap(o.n * K), 256, 0, st>>>(part, mp.nchunk, o.n, K, GRAV_GAMMA, D);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "multi-model reduce");
    return GRAV_OK;
}
