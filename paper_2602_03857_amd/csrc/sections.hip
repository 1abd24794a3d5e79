// Regional inversion by adjoining sections (paper Section 4.5), with the
// residual separation of Section 2.2: a regional problem is divided into
// sections that adjoin along y, each section is inverted on its own
// (Eq. 10-11) from its own stations, the section models are placed into the
// regional mesh, and one trend surface per layer, fitted across the complete
// domain, is removed from the combined model.
//
// Everything runs on the device: station assignment and a stable compaction
// of each section's stations, gathers of the section surveys, data-trend
// removal (trend.hip), the section CG solves (solver.hip) and the copies of
// cell blocks between section and regional order.  The host only sequences
// the steps and reads back the per-section station counts.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "api_internal.h"

namespace grav {

namespace {

constexpr int kScanBlock = 1024;

struct SplitRows {
    int32_t j[kMaxSections + 1];
};

// sec[o] = number of interior section boundaries yn[j[s]] (s = 1 .. nsec-1)
// at or below y_o: a station on a boundary belongs to the section above it.
__global__ __launch_bounds__(256) void k_station_sections(const double *__restrict__ y, int64_t n,
                                                          const double *__restrict__ yn,
                                                          SplitRows split, int nsec,
                                                          int32_t *__restrict__ sec) {
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= n) return;
    const double yo = y[o];
    int s = 0;
    for (int b = 1; b < nsec; ++b) s += (yo >= yn[split.j[b]]) ? 1 : 0;
    sec[o] = s;
}

// Stable compaction of the stations of section s: idx[r] = o for the r-th
// station (in input order) with sec[o] == s; *count receives their number.
// One block walks the stations in tiles, with a block-wide exclusive scan of
// the membership flags per tile.
__global__ __launch_bounds__(kScanBlock) void k_compact_section(const int32_t *__restrict__ sec,
                                                                int64_t n, int s,
                                                                int64_t *__restrict__ idx,
                                                                int64_t *__restrict__ count) {
    __shared__ int wave_tot[kScanBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t base = 0;
    for (int64_t t0 = 0; t0 < n; t0 += kScanBlock) {
        const int64_t o = t0 + threadIdx.x;
        const bool f = o < n && sec[o] == s;
        const uint64_t mask = __ballot(f);
        const int below = __popcll(mask & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
        if (lane == 0) wave_tot[wave] = __popcll(mask);
        __syncthreads();
        int wave_off = 0, tile_tot = 0;
        for (int w = 0; w < kScanBlock / 64; ++w) {
            wave_off += (w < wave) ? wave_tot[w] : 0;
            tile_tot += wave_tot[w];
        }
        if (f) idx[base + wave_off + below] = o;
        base += tile_tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = base;
}

// xs[r] = x[idx[r]] etc. for the r-th station of a section.
__global__ __launch_bounds__(256) void k_gather_survey(
    const int64_t *__restrict__ idx, int64_t ns, const double *__restrict__ x,
    const double *__restrict__ y, const double *__restrict__ z, const double *__restrict__ d,
    double *__restrict__ xs, double *__restrict__ ys, double *__restrict__ zs,
    double *__restrict__ ds) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= ns) return;
    const int64_t o = idx[r];
    xs[r] = x[o];
    ys[r] = y[o];
    zs[r] = z[o];
    ds[r] = d[o];
}

// Cell blocks between meshes that share x and z nodes:
// dst[(i*ny_dst + jd0 + j)*nz + k] = src[(i*ny_src + js0 + j)*nz + k] for
// i < nx, j < nyc, k < nz.
__global__ __launch_bounds__(256) void k_copy_cell_block(const double *__restrict__ src,
                                                         int ny_src, int js0,
                                                         double *__restrict__ dst, int ny_dst,
                                                         int jd0, int nx, int nyc, int nz) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t per_i = (int64_t)nyc * nz;
    if (t >= (int64_t)nx * per_i) return;
    const int64_t i = t / per_i;
    const int64_t rem = t - i * per_i;   // (j, k) within the block, k fastest
    const int64_t j = rem / nz, k = rem - j * nz;
    dst[(i * ny_dst + jd0 + j) * nz + k] = src[(i * ny_src + js0 + j) * nz + k];
}

// Cell-centre coordinates of the horizontal cells, X/Y[i*ny + j].
__global__ __launch_bounds__(256) void k_cell_centres(const double *__restrict__ xn,
                                                      const double *__restrict__ yn, int nx,
                                                      int ny, double *__restrict__ X,
                                                      double *__restrict__ Y) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)nx * ny) return;
    const int i = (int)(t / ny), j = (int)(t - (int64_t)i * ny);
    X[t] = 0.5 * (xn[i] + xn[i + 1]);
    Y[t] = 0.5 * (yn[j] + yn[j + 1]);
}

// One layer k of a model in flat cell order <-> a horizontal vector.
__global__ __launch_bounds__(256) void k_layer_get(const double *__restrict__ m, int64_t ncol,
                                                   int nz, int k, double *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < ncol) out[t] = m[t * nz + k];
}
__global__ __launch_bounds__(256) void k_layer_put(const double *__restrict__ in, int64_t ncol,
                                                   int nz, int k, double *__restrict__ m) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < ncol) m[t * nz + k] = in[t];
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// Restores ctx->arena_skip when the workflow returns.
struct ArenaHold {
    grav_ctx *ctx;
    size_t saved;
    ArenaHold(grav_ctx *c, size_t bytes) : ctx(c), saved(c->arena_skip) { c->arena_skip += bytes; }
    ~ArenaHold() { ctx->arena_skip = saved; }
};

#define HIP_TRY(expr, where)                                       \
    do {                                                           \
        hipError_t _e = (expr);                                    \
        if (_e != hipSuccess) return hip_fail(ctx, _e, where);     \
    } while (0)

}  // namespace

// Workspace the workflow keeps for itself (the section solves and trend fits
// run in the rest): station sections and section order, one section survey
// and data vector, the domain residual, section weights and model, and the
// horizontal vectors of the model-trend fit.  Sizes are those of the whole
// problem, an upper bound for any section.
static void take_sections_head(Counter &c, const Mesh &g, int64_t n) {
    c.take<int32_t>(n);                     // sec
    c.take<int64_t>(n);                     // idx (all sections, in section order)
    c.take<int64_t>(kMaxSections);          // counts
    for (int i = 0; i < 5; ++i) c.take<double>(n);   // xs ys zs ds d_res
    c.take<double>(g.ncells());             // section weights
    c.take<double>(g.ncells());             // section model
    const int64_t ncol = (int64_t)g.nx * g.ny;
    for (int i = 0; i < 3; ++i) c.take<double>(ncol);   // X Y layer
}

// The section solves need at most the largest inversion workspace over every
// section width (1 .. ny cell rows) with all n stations: a narrower section
// can split its stations into more parts than a wider one, so the whole
// problem's own need is not a bound.
uint64_t sections_workspace_need(const Mesh &g, int64_t n, grav_prec prec) {
    Counter c;
    take_sections_head(c, g, n);
    size_t inner = trend_workspace_need();
    for (int nys = 1; nys <= g.ny; ++nys) {
        const size_t inv = workspace_need(g.nx, nys, g.nz, n, GRAV_OP_INVERT, prec, 0);
        if (inv > inner) inner = inv;
    }
    return c.off + inner;
}

int run_sections(grav_ctx *ctx, const Mesh &g, const Obs &o, const double *d_obs,
                 const double *wdepth, double lambda, const grav_cg_opts &cg,
                 const grav_section_opts &so, double *m_out, double *m_detr,
                 grav_cg_info *info, grav_prec prec, hipStream_t st) {
    const int nsec = so.nsec;
    const int64_t n = o.n, ncol = (int64_t)g.nx * g.ny;
    Arena ar = ctx_arena(ctx);
    int32_t *sec = ar.take<int32_t>(n);
    int64_t *idx = ar.take<int64_t>(n);
    int64_t *dcount = ar.take<int64_t>(kMaxSections);
    double *xs = ar.take<double>(n), *ys = ar.take<double>(n), *zs = ar.take<double>(n);
    double *ds = ar.take<double>(n), *dres = ar.take<double>(n);
    double *ws = ar.take<double>(g.ncells()), *msec = ar.take<double>(g.ncells());
    double *X = ar.take<double>(ncol), *Y = ar.take<double>(ncol), *L = ar.take<double>(ncol);
    if (ar.failed) return fail(ctx, GRAV_ENOMEM, "workspace too small for the section workflow");
    const ArenaHold hold(ctx, ar.off);

    // 1. stations -> sections, each section's stations in input order
    SplitRows split{};
    for (int s = 0; s <= nsec; ++s) split.j[s] = so.ysplit[s];
    k_station_sections<<<blocks_for(n), 256, 0, st>>>(o.y, n, g.yn, split, nsec, sec);
    HIP_TRY(hipGetLastError(), "station sections");
    std::vector<int64_t> count(nsec), offset(nsec + 1, 0);
    for (int s = 0; s < nsec; ++s) {
        k_compact_section<<<1, kScanBlock, 0, st>>>(sec, n, s, idx + offset[s], dcount + s);
        HIP_TRY(hipGetLastError(), "section compaction");
        HIP_TRY(hipMemcpyAsync(ctx->h_scal, dcount + s, sizeof(int64_t), hipMemcpyDeviceToHost, st),
                "section count");
        HIP_TRY(hipStreamSynchronize(st), "section count");
        std::memcpy(&count[s], ctx->h_scal, sizeof(int64_t));
        if (count[s] == 0)
            return fail(ctx, GRAV_EINVAL, "section " + std::to_string(s) + " holds no stations");
        offset[s + 1] = offset[s] + count[s];
    }

    const int64_t basis_d = so.data_degree == 2 ? 6 : 3, basis_m = so.model_degree == 2 ? 6 : 3;
    if (so.data_degree > 0) {
        const bool per_section = so.data_scope == GRAV_TREND_SECTION;
        for (int s = 0; s < (per_section ? nsec : 1); ++s)
            if ((per_section ? count[s] : n) < basis_d)
                return fail(ctx, GRAV_EINVAL, "fewer stations than the data trend surface needs");
    }
    if (m_detr && so.model_degree > 0 && ncol < basis_m)
        return fail(ctx, GRAV_EINVAL, "fewer horizontal cells than the model trend surface needs");

    // 2. residual separation over the whole survey, if asked for
    const double *d_src = d_obs;
    double coef[6], frame[3];
    if (so.data_degree > 0 && so.data_scope == GRAV_TREND_DOMAIN) {
        int rc = op_trend_surface(ctx, o.x, o.y, d_obs, n, so.data_degree, coef, frame, dres,
                                  nullptr, st);
        if (rc) return rc;
        d_src = dres;
    }

    // 3. each section: its survey, data residual, weights; CG solve; model
    //    block into the regional model
    bool noconv = false;
    for (int s = 0; s < nsec; ++s) {
        const int j0 = so.ysplit[s], j1 = so.ysplit[s + 1], nys = j1 - j0;
        const int64_t ns = count[s];
        k_gather_survey<<<blocks_for(ns), 256, 0, st>>>(idx + offset[s], ns, o.x, o.y, o.z, d_src,
                                                        xs, ys, zs, ds);
        HIP_TRY(hipGetLastError(), "section survey");
        if (so.data_degree > 0 && so.data_scope == GRAV_TREND_SECTION) {
            int rc = op_trend_surface(ctx, xs, ys, ds, ns, so.data_degree, coef, frame, ds, nullptr,
                                      st);
            if (rc) {
                ctx->err = "section " + std::to_string(s) + ": " + ctx->err;
                return rc;
            }
        }
        const int64_t cells_s = (int64_t)g.nx * nys * g.nz;
        k_copy_cell_block<<<blocks_for(cells_s), 256, 0, st>>>(wdepth, g.ny, j0, ws, nys, 0, g.nx,
                                                               nys, g.nz);
        HIP_TRY(hipGetLastError(), "section weights");
        const Mesh gs{g.nx, nys, g.nz, g.xn, g.yn + j0, g.zn};
        const Obs os{ns, xs, ys, zs};
        grav_cg_info is{};
        int rc = run_invert(ctx, gs, os, ds, ws, lambda, nullptr, cg, msec, nullptr, &is, prec, st);
        if (rc == GRAV_ENOCONV) {
            noconv = true;
        } else if (rc) {
            ctx->err = "section " + std::to_string(s) + ": " + ctx->err;
            return rc;
        }
        if (info) info[s] = is;
        k_copy_cell_block<<<blocks_for(cells_s), 256, 0, st>>>(msec, nys, 0, m_out, g.ny, j0, g.nx,
                                                               nys, g.nz);
        HIP_TRY(hipGetLastError(), "section model");
    }

    // 4. one trend surface per layer across the complete domain, removed
    //    from the combined model
    if (m_detr) {
        if (so.model_degree > 0) {
            k_cell_centres<<<blocks_for(ncol), 256, 0, st>>>(g.xn, g.yn, g.nx, g.ny, X, Y);
            HIP_TRY(hipGetLastError(), "cell centres");
            for (int k = 0; k < g.nz; ++k) {
                k_layer_get<<<blocks_for(ncol), 256, 0, st>>>(m_out, ncol, g.nz, k, L);
                HIP_TRY(hipGetLastError(), "layer");
                int rc = op_trend_surface(ctx, X, Y, L, ncol, so.model_degree, coef, frame, L,
                                          nullptr, st);
                if (rc) {
                    ctx->err = "model trend, layer " + std::to_string(k) + ": " + ctx->err;
                    return rc;
                }
                k_layer_put<<<blocks_for(ncol), 256, 0, st>>>(L, ncol, g.nz, k, m_detr);
                HIP_TRY(hipGetLastError(), "layer");
            }
        } else {
            HIP_TRY(hipMemcpyAsync(m_detr, m_out, g.ncells() * sizeof(double),
                                   hipMemcpyDeviceToDevice, st), "model copy");
        }
    }
    HIP_TRY(hipStreamSynchronize(st), "sections sync");
    if (noconv) {
        ctx->err = "a section's CG reached its iteration cap before tol";
        return GRAV_ENOCONV;
    }
    return GRAV_OK;
}

}  // namespace grav
