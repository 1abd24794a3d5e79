// C-ABI entry points of the gravity library (declared in include/grav.h):
// argument checks, device-side validation, workspace carving, and the
// composition of the sweep kernels into the forward, adjoint and data-space
// operators and the data-space CG inversion (paper Eq. 5-11).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "grav_internal.h"
#include "api_internal.h"

using namespace grav;

static thread_local std::string g_create_error;
extern "C" int grav_reset_timing(grav_ctx *ctx);

// ---------------------------------------------------------------- helpers

namespace grav {

void set_context_free_error(const std::string &msg) { g_create_error = msg; }

int fail(grav_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return code;
}

int hip_fail(grav_ctx *ctx, hipError_t e, const char *where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(ctx, GRAV_EDEVICE, m);
}

Arena ctx_arena(grav_ctx *ctx) {
    Arena a;
    const size_t head = kReserveBytes + ctx->arena_skip;
    a.base = ctx->ws + head;
    a.size = ctx->ws_bytes > head ? ctx->ws_bytes - head : 0;
    return a;
}

int check_geometry_host(grav_ctx *ctx, const grav_mesh *mesh, const grav_obs *obs) {
    if (!mesh || !obs) return fail(ctx, GRAV_EINVAL, "mesh or obs is NULL");
    if (mesh->nx <= 0 || mesh->ny <= 0 || mesh->nz <= 0)
        return fail(ctx, GRAV_EINVAL, "mesh dimensions must be positive");
    if (!mesh->xn || !mesh->yn || !mesh->zn) return fail(ctx, GRAV_EINVAL, "mesh node vector is NULL");
    if (obs->n <= 0) return fail(ctx, GRAV_EINVAL, "observation count must be positive");
    if (obs->n > (int64_t)1 << 31) return fail(ctx, GRAV_EINVAL, "more than 2^31 observations");
    if (!obs->x || !obs->y || !obs->z) return fail(ctx, GRAV_EINVAL, "observation vector is NULL");
    const int64_t segs = (int64_t)(mesh->nx + 1) * (mesh->ny + 1) * (mesh->nz + 1);
    if (segs > ((int64_t)1 << 40)) return fail(ctx, GRAV_EINVAL, "mesh too large");
    return GRAV_OK;
}

static const char *flag_text(int f) {
    if (f & kBadMesh) return "mesh node coordinates must be finite and strictly increasing";
    if (f & kBadObs) return "observation coordinates must be finite";
    if (f & kObsBelowTop) return "observation below the mesh top (z > zn[0])";
    if (f & kOutOfRange) return "node-observation distance above 1e6 m";
    if (f & kBadWeights) return "depth weights must be finite and > 0";
    if (f & kBadValues) return "input vector has non-finite values";
    return "invalid input";
}

int validate_on_device(grav_ctx *ctx, const Mesh &g, const Obs &o, hipStream_t st,
                       std::initializer_list<ArrayCheck> arrays) {
    if (!ctx->validate) return GRAV_OK;
    int *flags = reinterpret_cast<int *>(ctx->ws);
    hipError_t e = hipMemsetAsync(flags, 0, sizeof(int), st);
    if (e != hipSuccess) return hip_fail(ctx, e, "validate memset");
    e = launch_validate(g, o, flags, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "validate launch");
    for (const ArrayCheck &a : arrays) {
        if (!a.ptr) continue;
        e = a.positive ? launch_validate_positive(a.ptr, a.len, flags, st)
                       : launch_validate_finite(a.ptr, a.len, flags, st);
        if (e != hipSuccess) return hip_fail(ctx, e, "validate launch");
    }
    e = hipMemcpyAsync(ctx->h_flags, flags, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "validate copy");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(ctx, e, "validate sync");
    const int f = *ctx->h_flags;
    if (f) return fail(ctx, GRAV_EINVAL, flag_text(f));
    return GRAV_OK;
}

// ---------------------------------------------------------------- operators

#define HIP_TRY(expr, where)                                       \
    do {                                                           \
        hipError_t _e = (expr);                                    \
        if (_e != hipSuccess) return hip_fail(ctx, _e, where);     \
    } while (0)

// d = scale * sum_parts + coef * add
int op_forward(grav_ctx *ctx, Arena &ar, const Mesh &g, const Obs &o, const double *m, double *d,
               grav_prec prec, hipStream_t st, double scale, const double *add, double coef) {
    const ForwardPlan fp = plan_forward(g.ncols(), o.n);
    const size_t mark = ar.off;
    double *part = ar.take<double>((size_t)fp.nchunk * o.n);
    if (prec == GRAV_MIXED) {
        float *hk = ar.take<float>(layer_table_len(g.nz));
        double *w2 = ar.take<double>(g.nsegs());
        if (ar.failed) return fail(ctx, GRAV_ENOMEM, "workspace too small for the forward sweep");
        HIP_TRY(launch_layer_thickness(g, hk, st), "layer thickness");
        HIP_TRY(launch_edge_weights(g, m, w2, st), "edge weights");
        KernelTimer kt(ctx, "forward_mixed", st);
        HIP_TRY(launch_forward_mixed(g, o, hk, w2, fp, part, st), "forward sweep");
    } else {
        double *wn = ar.take<double>(g.nnodes());
        if (ar.failed) return fail(ctx, GRAV_ENOMEM, "workspace too small for the forward sweep");
        HIP_TRY(launch_node_weights(g, m, wn, st), "node weights");
        KernelTimer kt(ctx, "forward_f64", st);
        HIP_TRY(launch_forward_f64(g, o, wn, fp, part, st), "forward sweep");
    }
    HIP_TRY(launch_reduce_parts(part, fp.nchunk, o.n, scale, add, coef, d, st), "forward reduce");
    ar.off = mark;
    return GRAV_OK;
}

// out = base + scale * C * G^T v / gamma-free (scale carries gamma)
int op_adjoint(grav_ctx *ctx, Arena &ar, const Mesh &g, const Obs &o, const double *v, double *out,
               grav_prec prec, hipStream_t st, double scale, const double *wdepth,
               const double *base) {
    const size_t mark = ar.off;
    if (prec == GRAV_MIXED) {
        const AdjointPlan ap = plan_adjoint(g.ncols(), g.nz, o.n);
        float *hk = ar.take<float>(layer_table_len(g.nz));
        double *upart = ar.take<double>((size_t)ap.nparts * g.nsegs());
        double *U = ar.take<double>(g.nsegs());
        if (ar.failed) return fail(ctx, GRAV_ENOMEM, "workspace too small for the adjoint sweep");
        HIP_TRY(launch_layer_thickness(g, hk, st), "layer thickness");
        {
            KernelTimer kt(ctx, "adjoint_mixed", st);
            HIP_TRY(launch_adjoint_mixed(g, o, hk, v, ap, upart, st), "adjoint sweep");
        }
        HIP_TRY(launch_reduce_parts(upart, ap.nparts, g.nsegs(), 1.0, nullptr, 0.0, U, st),
                "adjoint reduce");
        HIP_TRY(launch_adjoint_finish_edges(g, U, scale, wdepth, base, out, st), "adjoint finish");
    } else {
        const NodeAdjointPlan ap = plan_adjoint_nodes(g.nnodes(), o.n);
        double *ppart = ar.take<double>((size_t)ap.nparts * g.nnodes());
        double *P = ar.take<double>(g.nnodes());
        if (ar.failed) return fail(ctx, GRAV_ENOMEM, "workspace too small for the adjoint sweep");
        {
            KernelTimer kt(ctx, "adjoint_f64", st);
            HIP_TRY(launch_adjoint_f64(g, o, v, ap, ppart, st), "adjoint sweep");
        }
        HIP_TRY(launch_reduce_parts(ppart, ap.nparts, g.nnodes(), 1.0, nullptr, 0.0, P, st),
                "adjoint reduce");
        HIP_TRY(launch_adjoint_finish_nodes(g, P, scale, wdepth, base, out, st), "adjoint finish");
    }
    ar.off = mark;
    return GRAV_OK;
}

// out = G C G^T v + lambda v
int op_dataspace(grav_ctx *ctx, Arena &ar, const Mesh &g, const Obs &o, const double *wdepth,
                 double lambda, const double *v, double *out, grav_prec prec, hipStream_t st) {
    const size_t mark = ar.off;
    double *t = ar.take<double>(g.ncells());
    if (ar.failed) return fail(ctx, GRAV_ENOMEM, "workspace too small for the data-space operator");
    int rc = op_adjoint(ctx, ar, g, o, v, t, prec, st, GRAV_GAMMA, wdepth, nullptr);
    if (rc) return rc;
    rc = op_forward(ctx, ar, g, o, t, out, prec, st, GRAV_GAMMA, v, lambda);
    if (rc) return rc;
    ar.off = mark;
    return GRAV_OK;
}

// diag (device, may be null) and the trace (host)
int op_trace(grav_ctx *ctx, Arena &ar, const Mesh &g, const Obs &o, const double *wdepth,
             double *trace, double *diag, grav_prec prec, hipStream_t st) {
    const size_t mark = ar.off;
    const ForwardPlan tp = plan_trace(g.nx, o.n);
    double *part = ar.take<double>((size_t)tp.nchunk * o.n);
    double *dg = diag ? diag : ar.take<double>(o.n);
    float *hk = ar.take<float>(layer_table_len(g.nz));
    if (ar.failed) return fail(ctx, GRAV_ENOMEM, "workspace too small for the trace sweep");
    if (prec == GRAV_MIXED) {
        HIP_TRY(launch_layer_thickness(g, hk, st), "layer thickness");
        KernelTimer kt(ctx, "trace_mixed", st);
        HIP_TRY(launch_trace_mixed(g, o, hk, wdepth, tp, part, st), "trace sweep");
    } else {
        KernelTimer kt(ctx, "trace_f64", st);
        HIP_TRY(launch_trace_f64(g, o, wdepth, tp, part, st), "trace sweep");
    }
    HIP_TRY(launch_reduce_parts(part, tp.nchunk, o.n, GRAV_GAMMA * GRAV_GAMMA, nullptr, 0.0, dg, st),
            "trace reduce");
    double *scal = ctx_scalars(ctx);
    double *dpart = ctx_dot_partials(ctx);
    HIP_TRY(launch_dot(dg, nullptr, o.n, dpart, st), "trace sum");
    HIP_TRY(launch_dot_finish(dpart, scal, kFinishPlain, kNumScalars - 1, st), "trace sum");
    HIP_TRY(hipMemcpyAsync(ctx->h_scal, scal, kNumScalars * sizeof(double), hipMemcpyDeviceToHost, st),
            "trace copy");
    HIP_TRY(hipStreamSynchronize(st), "trace sync");
    *trace = ctx->h_scal[kNumScalars - 1];
    ar.off = mark;
    return GRAV_OK;
}

}  // namespace grav

// ---------------------------------------------------------------- context

extern "C" void grav_ctx_opts_default(grav_ctx_opts *opts) {
    if (!opts) return;
    opts->device = 0;
    opts->validate = 1;
    opts->workspace_bytes = 0;
}

extern "C" int grav_ctx_create(grav_ctx **out, const grav_ctx_opts *opts_in) {
    if (!out) return GRAV_EINVAL;
    *out = nullptr;
    grav_ctx_opts opts;
    grav_ctx_opts_default(&opts);
    if (opts_in) opts = *opts_in;
    if (opts.workspace_bytes == 0) opts.workspace_bytes = (uint64_t)4 << 30;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) {
        g_create_error = "no HIP device available";
        return GRAV_EDEVICE;
    }
    if (opts.device < 0 || opts.device >= ndev) {
        g_create_error = "device ordinal out of range";
        return GRAV_EINVAL;
    }
    e = hipSetDevice(opts.device);
    if (e != hipSuccess) {
        g_create_error = std::string("hipSetDevice: ") + hipGetErrorString(e);
        return GRAV_EDEVICE;
    }
    grav_ctx *ctx = new grav_ctx();
    ctx->device = opts.device;
    ctx->validate = opts.validate != 0;
    ctx->ws_bytes = (size_t)opts.workspace_bytes + kReserveBytes;
    e = hipMalloc(reinterpret_cast<void **>(&ctx->ws), ctx->ws_bytes);
    if (e != hipSuccess) {
        g_create_error = std::string("workspace allocation: ") + hipGetErrorString(e);
        delete ctx;
        return GRAV_ENOMEM;
    }
    e = hipHostMalloc(reinterpret_cast<void **>(&ctx->h_pinned), 4096, hipHostMallocDefault);
    if (e != hipSuccess) {
        g_create_error = std::string("pinned allocation: ") + hipGetErrorString(e);
        (void)hipFree(ctx->ws);
        delete ctx;
        return GRAV_ENOMEM;
    }
    ctx->h_flags = reinterpret_cast<int *>(ctx->h_pinned);
    ctx->h_scal = reinterpret_cast<double *>(ctx->h_pinned + 256);
    *out = ctx;
    return GRAV_OK;
}

extern "C" void grav_ctx_destroy(grav_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    (void)grav_reset_timing(ctx);
    (void)hipFree(ctx->ws);
    (void)hipHostFree(ctx->h_pinned);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
}

extern "C" const char *grav_last_error(const grav_ctx *ctx) {
    if (!ctx) return g_create_error.c_str();
    return ctx->err.c_str();
}

extern "C" uint64_t grav_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, int64_t n, grav_op op,
                                         grav_prec prec, int32_t K) {
    if (op == GRAV_OP_TREND) return grav::trend_workspace_need();
    if (nx <= 0 || ny <= 0 || nz <= 0 || n <= 0) return 0;
    if (op == GRAV_OP_SECTIONS)
        return grav::sections_workspace_need(grav::Mesh{nx, ny, nz, nullptr, nullptr, nullptr}, n,
                                             prec);
    return grav::workspace_need(nx, ny, nz, n, op, prec, K);
}

// ---------------------------------------------------------------- operators

#define ENTER(ctx)                                          \
    if (!(ctx)) return GRAV_EINVAL;                         \
    (ctx)->err.clear();                                     \
    do {                                                    \
        hipError_t _e = hipSetDevice((ctx)->device);        \
        if (_e != hipSuccess) return hip_fail(ctx, _e, "hipSetDevice"); \
    } while (0)

static inline Mesh to_mesh(const grav_mesh *m) { return Mesh{m->nx, m->ny, m->nz, m->xn, m->yn, m->zn}; }
static inline Obs to_obs(const grav_obs *o) { return Obs{o->n, o->x, o->y, o->z}; }

extern "C" int grav_forward(grav_ctx *ctx, const grav_mesh *mesh, const grav_obs *obs,
                            const double *m, double *d, grav_prec prec, grav_stream stream) {
    ENTER(ctx);
    int rc = check_geometry_host(ctx, mesh, obs);
    if (rc) return rc;
    if (!m || !d) return fail(ctx, GRAV_EINVAL, "m or d is NULL");
    if (prec != GRAV_FP64 && prec != GRAV_MIXED) return fail(ctx, GRAV_EINVAL, "precision must be GRAV_FP64 or GRAV_MIXED");
    const Mesh g = to_mesh(mesh);
    const Obs o = to_obs(obs);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    rc = validate_on_device(ctx, g, o, st, {ArrayCheck{m, g.ncells(), false}});
    if (rc) return rc;
    Arena ar = ctx_arena(ctx);
    return op_forward(ctx, ar, g, o, m, d, prec, st, GRAV_GAMMA, nullptr, 0.0);
}

extern "C" int grav_adjoint(grav_ctx *ctx, const grav_mesh *mesh, const grav_obs *obs,
                            const double *v, double *gout, grav_prec prec, grav_stream stream) {
    ENTER(ctx);
    int rc = check_geometry_host(ctx, mesh, obs);
    if (rc) return rc;
    if (!v || !gout) return fail(ctx, GRAV_EINVAL, "v or g is NULL");
    if (prec != GRAV_FP64 && prec != GRAV_MIXED) return fail(ctx, GRAV_EINVAL, "precision must be GRAV_FP64 or GRAV_MIXED");
    const Mesh g = to_mesh(mesh);
    const Obs o = to_obs(obs);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    rc = validate_on_device(ctx, g, o, st, {ArrayCheck{v, o.n, false}});
    if (rc) return rc;
    Arena ar = ctx_arena(ctx);
    return op_adjoint(ctx, ar, g, o, v, gout, prec, st, GRAV_GAMMA, nullptr, nullptr);
}

extern "C" int grav_dataspace_apply(grav_ctx *ctx, const grav_mesh *mesh, const grav_obs *obs,
                                    const double *wdepth, double lambda, const double *v,
                                    double *out, grav_prec prec, grav_stream stream) {
    ENTER(ctx);
    int rc = check_geometry_host(ctx, mesh, obs);
    if (rc) return rc;
    if (!wdepth || !v || !out) return fail(ctx, GRAV_EINVAL, "wdepth, v or out is NULL");
    if (v == out) return fail(ctx, GRAV_EINVAL, "out may not alias v");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(ctx, GRAV_EINVAL, "lambda must be finite and >= 0");
    if (prec != GRAV_FP64 && prec != GRAV_MIXED) return fail(ctx, GRAV_EINVAL, "precision must be GRAV_FP64 or GRAV_MIXED");
    const Mesh g = to_mesh(mesh);
    const Obs o = to_obs(obs);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    rc = validate_on_device(ctx, g, o, st,
                            {ArrayCheck{wdepth, g.ncells(), true}, ArrayCheck{v, o.n, false}});
    if (rc) return rc;
    Arena ar = ctx_arena(ctx);
    return op_dataspace(ctx, ar, g, o, wdepth, lambda, v, out, prec, st);
}

extern "C" int grav_trace(grav_ctx *ctx, const grav_mesh *mesh, const grav_obs *obs,
                          const double *wdepth, double *trace, double *diag, grav_prec prec,
                          grav_stream stream) {
    ENTER(ctx);
    int rc = check_geometry_host(ctx, mesh, obs);
    if (rc) return rc;
    if (!wdepth || !trace) return fail(ctx, GRAV_EINVAL, "wdepth or trace is NULL");
    if (prec != GRAV_FP64 && prec != GRAV_MIXED) return fail(ctx, GRAV_EINVAL, "precision must be GRAV_FP64 or GRAV_MIXED");
    const Mesh g = to_mesh(mesh);
    const Obs o = to_obs(obs);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    rc = validate_on_device(ctx, g, o, st, {ArrayCheck{wdepth, g.ncells(), true}});
    if (rc) return rc;
    Arena ar = ctx_arena(ctx);
    return op_trace(ctx, ar, g, o, wdepth, trace, diag, prec, st);
}

extern "C" int grav_issue_rates(grav_ctx *ctx, double *rates, grav_stream stream) {
    ENTER(ctx);
    if (!rates) return fail(ctx, GRAV_EINVAL, "rates is NULL");
    return grav::op_issue_rates(ctx, rates, reinterpret_cast<hipStream_t>(stream));
}

extern "C" int grav_issue_pair_rates(grav_ctx *ctx, double *rates, grav_stream stream) {
    ENTER(ctx);
    if (!rates) return fail(ctx, GRAV_EINVAL, "rates is NULL");
    return grav::op_issue_pair_rates(ctx, rates, reinterpret_cast<hipStream_t>(stream));
}

extern "C" int grav_trend_surface(grav_ctx *ctx, const double *x, const double *y, const double *v,
                                  int64_t n, int32_t degree, double *coef, double *frame,
                                  double *resid, double *trend, grav_stream stream) {
    ENTER(ctx);
    if (!x || !y || !v || !coef || !frame) return fail(ctx, GRAV_EINVAL, "x, y, v, coef or frame is NULL");
    if (degree != 1 && degree != 2) return fail(ctx, GRAV_EINVAL, "degree must be 1 or 2");
    if (n < (degree == 2 ? 6 : 3)) return fail(ctx, GRAV_EINVAL, "fewer points than basis functions");
    return grav::op_trend_surface(ctx, x, y, v, n, degree, coef, frame, resid, trend,
                                  reinterpret_cast<hipStream_t>(stream));
}

extern "C" int grav_invert(grav_ctx *ctx, const grav_mesh *mesh, const grav_obs *obs,
                           const double *d_obs, const double *wdepth, double lambda,
                           const double *m_ref, const grav_cg_opts *cg, double *m_out,
                           double *d_pred, grav_cg_info *info, grav_prec prec,
                           grav_stream stream) {
    ENTER(ctx);
    int rc = check_geometry_host(ctx, mesh, obs);
    if (rc) return rc;
    if (!d_obs || !wdepth || !cg || !m_out) return fail(ctx, GRAV_EINVAL, "d_obs, wdepth, cg or m_out is NULL");
    if (!std::isfinite(lambda)) return fail(ctx, GRAV_EINVAL, "lambda must be finite");
    rc = check_cg_opts(ctx, cg);
    if (rc) return rc;
    if (prec != GRAV_FP64 && prec != GRAV_MIXED) return fail(ctx, GRAV_EINVAL, "precision must be GRAV_FP64 or GRAV_MIXED");
    const Mesh g = to_mesh(mesh);
    const Obs o = to_obs(obs);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    rc = validate_on_device(ctx, g, o, st,
                            {ArrayCheck{wdepth, g.ncells(), true}, ArrayCheck{d_obs, o.n, false},
                             ArrayCheck{m_ref, g.ncells(), false}, ArrayCheck{cg->y0, o.n, false}});
    if (rc) return rc;
    return grav::run_invert(ctx, g, o, d_obs, wdepth, lambda, m_ref, *cg, m_out, d_pred, info, prec, st);
}

extern "C" int grav_invert_sections(grav_ctx *ctx, const grav_mesh *mesh, const grav_obs *obs,
                                    const double *d_obs, const double *wdepth, double lambda,
                                    const grav_cg_opts *cg, const grav_section_opts *sec,
                                    double *m_out, double *m_detrended, grav_cg_info *info,
                                    grav_prec prec, grav_stream stream) {
    ENTER(ctx);
    int rc = check_geometry_host(ctx, mesh, obs);
    if (rc) return rc;
    if (!d_obs || !wdepth || !cg || !sec || !m_out)
        return fail(ctx, GRAV_EINVAL, "d_obs, wdepth, cg, sec or m_out is NULL");
    if (m_detrended == m_out) return fail(ctx, GRAV_EINVAL, "m_detrended may not alias m_out");
    if (!std::isfinite(lambda)) return fail(ctx, GRAV_EINVAL, "lambda must be finite");
    rc = check_cg_opts(ctx, cg);
    if (rc) return rc;
    if (cg->y0 || cg->y_out || cg->history_cap != 0)
        return fail(ctx, GRAV_EINVAL, "section inversions take no y0, y_out or history");
    if (sec->nsec < 1 || sec->nsec > kMaxSections || !sec->ysplit)
        return fail(ctx, GRAV_EINVAL, "nsec must be 1..64 with a ysplit array");
    if (sec->ysplit[0] != 0 || sec->ysplit[sec->nsec] != mesh->ny)
        return fail(ctx, GRAV_EINVAL, "ysplit must run from 0 to ny");
    for (int s = 0; s < sec->nsec; ++s)
        if (sec->ysplit[s + 1] <= sec->ysplit[s])
            return fail(ctx, GRAV_EINVAL, "ysplit must be strictly increasing");
    if (sec->data_degree < 0 || sec->data_degree > 2 || sec->model_degree < 0 || sec->model_degree > 2)
        return fail(ctx, GRAV_EINVAL, "trend degrees must be 0, 1 or 2");
    if (sec->data_scope != GRAV_TREND_SECTION && sec->data_scope != GRAV_TREND_DOMAIN)
        return fail(ctx, GRAV_EINVAL, "data_scope must be GRAV_TREND_SECTION or GRAV_TREND_DOMAIN");
    if (prec != GRAV_FP64 && prec != GRAV_MIXED) return fail(ctx, GRAV_EINVAL, "precision must be GRAV_FP64 or GRAV_MIXED");
    const Mesh g = to_mesh(mesh);
    const Obs o = to_obs(obs);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    rc = validate_on_device(ctx, g, o, st,
                            {ArrayCheck{wdepth, g.ncells(), true}, ArrayCheck{d_obs, o.n, false}});
    if (rc) return rc;
    return grav::run_sections(ctx, g, o, d_obs, wdepth, lambda, *cg, *sec, m_out, m_detrended,
                              info, prec, st);
}

namespace grav {

int check_cg_opts(grav_ctx *ctx, const grav_cg_opts *cg) {
    if (cg->restart < 0) return fail(ctx, GRAV_EINVAL, "restart must be >= 0");
    if (cg->history_cap < 0 || (cg->history_cap > 0 && !cg->history))
        return fail(ctx, GRAV_EINVAL, "history_cap must be >= 0, with a history array when > 0");
    if (cg->restart > 0) {
        if (cg->max_cycles < 1 || cg->max_halvings < 0 || !(cg->tol >= 0.0))
            return fail(ctx, GRAV_EINVAL, "restarted CG needs max_cycles >= 1, max_halvings >= 0, tol >= 0");
        if (cg->fixed_iters != 0 || cg->precond != 0)
            return fail(ctx, GRAV_EINVAL, "restarted CG needs fixed_iters = 0 and precond = 0");
    } else if (cg->fixed_iters <= 0 && (cg->max_iter < 1 || !(cg->tol >= 0.0))) {
        return fail(ctx, GRAV_EINVAL, "CG needs max_iter >= 1 and tol >= 0, or fixed_iters > 0");
    }
    if (cg->precond != 0 && cg->precond != 1)
        return fail(ctx, GRAV_EINVAL, "precond must be 0 (none) or 1 (Jacobi)");
    if (cg->graph != 0 && cg->graph != 1) return fail(ctx, GRAV_EINVAL, "graph must be 0 or 1");
    return GRAV_OK;
}

}  // namespace grav

// ---------------------------------------------------------------- timing

static const char *const kTimedKernels[] = {"forward_mixed", "forward_f64", "adjoint_mixed",
                                            "adjoint_f64", "trace_mixed", "trace_f64",
                                            "multi_bf16x3", "multi_fp32"};

namespace grav {

KernelTimer::KernelTimer(grav_ctx *ctx, const char *name, hipStream_t st)
    : ctx_(ctx), name_(name), st_(st) {
    if (!ctx_->timing) return;
    if (hipEventCreate(&start_) != hipSuccess) { start_ = nullptr; return; }
    if (hipEventRecord(start_, st_) != hipSuccess) {
        (void)hipEventDestroy(start_);
        start_ = nullptr;
    }
}

KernelTimer::~KernelTimer() {
    if (!start_) return;
    hipEvent_t stop = nullptr;
    if (hipEventCreate(&stop) != hipSuccess || hipEventRecord(stop, st_) != hipSuccess) {
        (void)hipEventDestroy(start_);
        if (stop) (void)hipEventDestroy(stop);
        return;
    }
    ctx_->pending[name_].emplace_back(start_, stop);
}

}  // namespace grav

static bool known_kernel(const char *k) {
    for (const char *n : kTimedKernels)
        if (std::strcmp(n, k) == 0) return true;
    return false;
}

extern "C" int grav_set_timing(grav_ctx *ctx, int32_t enable) {
    if (!ctx) return GRAV_EINVAL;
    ctx->timing = enable != 0;
    return GRAV_OK;
}

extern "C" int grav_kernel_time(grav_ctx *ctx, const char *kernel, double *total_ms,
                                int64_t *launches) {
    if (!ctx || !kernel || !total_ms || !launches) return GRAV_EINVAL;
    if (!known_kernel(kernel)) return fail(ctx, GRAV_EINVAL, "unknown kernel name");
    auto &tot = ctx->totals[kernel];
    auto it = ctx->pending.find(kernel);
    if (it != ctx->pending.end()) {
        for (auto &ev : it->second) {
            hipError_t e = hipEventSynchronize(ev.second);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.first, ev.second);
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
            if (e != hipSuccess) return hip_fail(ctx, e, "kernel timing");
            tot.first += ms;
            tot.second += 1;
        }
        it->second.clear();
    }
    *total_ms = tot.first;
    *launches = tot.second;
    return GRAV_OK;
}

extern "C" int grav_reset_timing(grav_ctx *ctx) {
    if (!ctx) return GRAV_EINVAL;
    for (auto &kv : ctx->pending)
        for (auto &ev : kv.second) {
            (void)hipEventSynchronize(ev.second);
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
    ctx->pending.clear();
    ctx->totals.clear();
    return GRAV_OK;
}
