// Internal interfaces of the gravity library: device-side descriptions of the
// problem, launch plans of the sweep kernels, and the launchers the C-ABI
// layer calls.  Nothing here is exported.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "grav.h"

namespace grav {

struct Mesh {
    int nx, ny, nz;
    const double *xn, *yn, *zn;
    int64_t ncells() const { return (int64_t)nx * ny * nz; }
    int64_t ncols() const { return (int64_t)(nx + 1) * (ny + 1); }   // vertical node columns
    int64_t nsegs() const { return ncols() * nz; }                   // vertical edge segments
    int64_t nnodes() const { return ncols() * (nz + 1); }
};

struct Obs {
    int64_t n;
    const double *x, *y, *z;
};

// Bump allocator over the context's workspace.  Every slice is 256-byte aligned.
struct Arena {
    char *base = nullptr;
    size_t size = 0;
    size_t off = 0;
    bool failed = false;
    template <typename T>
    T *take(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
        if (off + bytes > size) { failed = true; return nullptr; }
        T *p = reinterpret_cast<T *>(base + off);
        off += bytes;
        return p;
    }
};

// Byte counter with the same rounding as Arena (workspace queries).
struct Counter {
    size_t off = 0;
    template <typename T>
    void take(size_t count) { off += (count * sizeof(T) + 255) & ~size_t(255); }
};

// ---- launch plans -------------------------------------------------------

constexpr int kBlock = 128;          // threads per block of the sweeps (2 waves)
#ifndef GRAV_ADJ_LAYERS
#define GRAV_ADJ_LAYERS 16
#endif
constexpr int kAdjLayers = GRAV_ADJ_LAYERS;   // max layers per lane in the mixed adjoint sweep

// Layer table of the mixed sweeps (floats): [0, nz) the layer thicknesses
// h_k = Z_{k+1} - Z_k; [nz] (as an int) the first "deep" layer; [nz+1, 2nz+1)
// the node depths below the mesh top Z_{k+1} - Z_0.  Each entry is an FP64
// difference rounded once to FP32.
inline size_t layer_table_len(int nz) { return 2 * (size_t)nz + 1; }

// Forward sweep: lanes own observations; the mesh columns are split into
// `nchunk` contiguous chunks, one per block row, with partial sums per chunk.
struct ForwardPlan {
    int64_t nblk_obs;
    int nchunk;
    int64_t cols_per_chunk;
};

// Mixed adjoint sweep: lanes own (mesh column, layer chunk); observations are
// split into `nparts` parts, each producing its own partial U.
struct AdjointPlan {
    int64_t nblk_col;
    int nkc;                 // layer chunks per column
    int nparts;
    int64_t obs_per_part;
};

// FP64 adjoint sweep: lanes own mesh nodes; observation parts as above.
struct NodeAdjointPlan {
    int64_t nblk_node;
    int nparts;
    int64_t obs_per_part;
};

ForwardPlan plan_forward(int64_t ncols, int64_t n, int64_t target_waves = 0);   // 0 = default
// target_waves, max_partial_bytes: 0 = the single-call defaults
AdjointPlan plan_adjoint(int64_t ncols, int nz, int64_t n, int64_t target_waves = 0,
                         int64_t max_partial_bytes = 0);
NodeAdjointPlan plan_adjoint_nodes(int64_t nnodes, int64_t n);
ForwardPlan plan_trace(int nx, int64_t n);
// Workspace bounds: the largest partial buffers (doubles, or part counts) the
// plans above make for any survey of at most n observations.
int64_t forward_partials_bound(int64_t ncols, int64_t n);
int64_t trace_partials_bound(int nx, int64_t n);
int64_t adjoint_parts_bound(int64_t ncols, int nz, int64_t n);
int64_t node_adjoint_parts_bound(int64_t nnodes, int64_t n);

// ---- launchers (enqueue on `st`; return hipSuccess or the launch error) ---

hipError_t launch_layer_thickness(const Mesh &g, float *hk, hipStream_t st);
hipError_t launch_edge_weights(const Mesh &g, const double *m, double *w2, hipStream_t st);
hipError_t launch_node_weights(const Mesh &g, const double *m, double *wn, hipStream_t st);
hipError_t launch_forward_mixed(const Mesh &g, const Obs &o, const float *hk, const double *w2,
                                const ForwardPlan &p, double *partial, hipStream_t st);
hipError_t launch_forward_f64(const Mesh &g, const Obs &o, const double *wn,
                              const ForwardPlan &p, double *partial, hipStream_t st);
hipError_t launch_adjoint_mixed(const Mesh &g, const Obs &o, const float *hk, const double *v,
                                const AdjointPlan &p, double *upart, hipStream_t st);
hipError_t launch_adjoint_f64(const Mesh &g, const Obs &o, const double *v,
                              const NodeAdjointPlan &p, double *ppart, hipStream_t st);
// out[i] = scale * sum_p part[p*len + i] + coef * add[i]   (add may be null)
hipError_t launch_reduce_parts(const double *part, int nparts, int64_t len, double scale,
                               const double *add, double coef, double *out, hipStream_t st);
// out_cell = scale * cov_cell * sum_{p,q} (-1)^(p+q) U(edge p,q of the cell's column pair)
// where cov_cell = wdepth^-2 if wdepth != null, else 1; plus base[cell] if base != null.
hipError_t launch_adjoint_finish_edges(const Mesh &g, const double *U, double scale,
                                       const double *wdepth, const double *base, double *out,
                                       hipStream_t st);
hipError_t launch_adjoint_finish_nodes(const Mesh &g, const double *P, double scale,
                                       const double *wdepth, const double *base, double *out,
                                       hipStream_t st);
hipError_t launch_trace_mixed(const Mesh &g, const Obs &o, const float *hk, const double *wdepth,
                              const ForwardPlan &p, double *partial, hipStream_t st);
hipError_t launch_trace_f64(const Mesh &g, const Obs &o, const double *wdepth,
                            const ForwardPlan &p, double *partial, hipStream_t st);

// Validation: sets bits in *flags (device int, caller zeroes it).
enum : int {
    kBadMesh = 1, kBadObs = 2, kObsBelowTop = 4, kOutOfRange = 8, kBadWeights = 16, kBadValues = 32
};
hipError_t launch_validate(const Mesh &g, const Obs &o, int *flags, hipStream_t st);
hipError_t launch_validate_positive(const double *w, int64_t len, int *flags, hipStream_t st);
hipError_t launch_validate_finite(const double *w, int64_t len, int *flags, hipStream_t st);

// ---- vector kernels for CG ------------------------------------------------
constexpr int kDotBlocks = 512;
enum : int {
    kRR = 0, kPQ = 1, kRRNew = 2, kB2 = 3, kAlpha = 4, kBeta = 5, kRZ = 6,
    kYB = 7,                // restarted CG: y . (delta_d + r), i.e. -2 Q(y)
    kNumScalars = 8
};
enum : int {
    kFinishInit = 0, kFinishPQ = 1, kFinishRRNew = 2, kFinishPlain = 3,
    kFinishPQPrecond = 4,   // alpha = (r.z) / (p.Ap)
    kFinishRZNew = 5        // beta = (r'.z') / (r.z), then r.z <- r'.z'
};
hipError_t launch_dot(const double *a, const double *b, int64_t n, double *partials, hipStream_t st);
hipError_t launch_dot_finish(const double *partials, double *scal, int mode, int slot, hipStream_t st);
// y += alpha p ; r -= alpha q ; partial (r . r) into partials
hipError_t launch_cg_update_yr(double *y, double *r, const double *p, const double *q, int64_t n,
                               const double *scal, double *partials, hipStream_t st);
// Jacobi-preconditioned CG: dinv = 1 / (diag + lambda); z = dinv r, p = z,
// partial r.r and r.z (first iterate)
hipError_t launch_pcg_setup(const double *diag, double lambda, double *dinv, const double *r,
                            double *z, double *p, int64_t n, double *part_rr, double *part_rz,
                            hipStream_t st);
// y += alpha p ; r -= alpha q ; z = dinv r ; partial r.r and r.z
hipError_t launch_pcg_update_yrz(double *y, double *r, double *z, const double *p, const double *q,
                                 const double *dinv, int64_t n, const double *scal,
                                 double *part_rr, double *part_rz, hipStream_t st);
// p = r + beta p
hipError_t launch_cg_update_p(double *p, const double *r, int64_t n, const double *scal,
                              hipStream_t st);
// dst = a - b (b may be null: dst = a)
hipError_t launch_sub(const double *a, const double *b, double *dst, int64_t n, hipStream_t st);
hipError_t launch_fill(double *dst, double value, int64_t n, hipStream_t st);
// dst = ca a + cb b (dst may alias a or b)
hipError_t launch_lincomb(double *dst, double ca, const double *a, double cb, const double *b,
                          int64_t n, hipStream_t st);

}  // namespace grav
