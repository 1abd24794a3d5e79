/*
 * grav.h - matrix-free prism-gravity operators for AMD Instinct MI355X (gfx950).
 *
 * The library evaluates the closed-form vertical attraction of rectangular
 * prisms (paper Section 2.1, Eq. 1-3), superposed over a prism mesh (Eq. 4-6),
 * without ever forming the sensitivity matrix G, and the data-space inversion
 * built on it (Section 2.2, Eq. 7-11).
 *
 * ---------------------------------------------------------------------------
 * Conventions shared by every entry point
 * ---------------------------------------------------------------------------
 * Geometry.  A rectilinear mesh is given by its node coordinate vectors
 *   xn[0..nx], yn[0..ny], zn[0..nz] (metres, strictly increasing), z positive
 *   DOWN, zn[0] = mesh top.  Cell (i, j, k) is the prism
 *   [xn[i],xn[i+1]] x [yn[j],yn[j+1]] x [zn[k],zn[k+1]].  Flat cell index
 *   (i*ny + j)*nz + k (C order, z fastest); M = nx*ny*nz cells.
 * Observations.  n points (x[o], y[o], z[o]), z down; a point at height h
 *   above the mesh top has z = zn[0] - h.  PRECONDITION: z[o] <= zn[0] (no
 *   observation below the mesh top); the closed form used on the GPU assumes
 *   it, and validation rejects violations with GRAV_EINVAL.
 * Units.  Density contrast in kg/m^3, gravity in m/s^2 (1 mGal = 1e-5 m/s^2).
 *   The constant gamma (GRAV_GAMMA) is applied in FP64.
 * Sign.  gz > 0 means a downward pull: positive density below an observation
 *   gives positive data (Eq. 1 with corner-minus-observation coordinates and
 *   vertex parity (-1)^(p+q+r), vertex 1 = smaller coordinate).
 * Memory.  EVERY array argument is a caller-owned DEVICE pointer on the
 *   context's device (e.g. a torch tensor's data_ptr()).  The library never
 *   frees or retains them past the completion of the work it enqueues; it
 *   writes only the documented outputs.  Scalars marked "host" are host
 *   memory.
 * Streams.  Work is enqueued on `stream` (a hipStream_t; NULL = the null
 *   stream) in order.  With validation on (grav_ctx_opts.validate != 0, the
 *   default) each public call first checks its arguments on the device and
 *   waits for that check on `stream`, so the call returns only after all work
 *   previously enqueued on `stream` has finished; with validation off the
 *   operator calls are fully asynchronous and the caller guarantees the
 *   preconditions.
 * Workspace.  A context owns one device workspace allocated at creation; the
 *   operator calls allocate nothing.  One context serves one call at a time:
 *   calls that may overlap (different streams or threads) need separate
 *   contexts.  grav_workspace_bytes() tells how much a call needs.
 * Errors.  Every call returns a grav_status; no exception crosses the ABI.
 *   On an error return nothing has been written to the outputs unless stated.
 *   grav_last_error(ctx) gives a human-readable reason.
 * Determinism.  No atomics are used in any reduction; results are bitwise
 *   reproducible for the same inputs, precision and device.
 */
#ifndef GRAV_H
#define GRAV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GRAV_GAMMA 6.674e-11   /* gravitational constant used by the workloads, SI */

typedef enum {
    GRAV_OK = 0,
    GRAV_EINVAL = 1,    /* bad argument: null pointer, size <= 0, non-increasing nodes,
                           observation below the mesh top, non-finite input,
                           coordinates out of range, lambda < 0 where not allowed */
    GRAV_ENOMEM = 2,    /* context workspace (or device memory at creation) too small */
    GRAV_EDEVICE = 3,   /* HIP runtime error; grav_last_error() has the text */
    GRAV_ENOCONV = 4,   /* positive warning: CG stopped at max_iter before reaching tol;
                           all outputs are valid */
    GRAV_EBUSY = 5,     /* server: request not finished yet / queue full */
    GRAV_ECANCELED = 6  /* server: the request was cancelled; its outputs are unspecified */
} grav_status;

typedef enum {
    GRAV_FP64 = 0,          /* plain path: every corner term Psi(node - obs) in FP64 */
    GRAV_MIXED = 1,         /* FP32 edge-segment terms from FP64 coordinate differences,
                               FP64 alternating sums, accumulation and CG dot products.
                               Accurate to 1e-5 relative for stations over and around
                               the mesh (tested to half its width beyond it).  Far
                               outside it (distance R >> mesh width L) the edge terms
                               cancel by about (R/L)^2, and a result is only good to
                               16 eps32 x the sum of the magnitudes of its terms:
                               use GRAV_FP64 for such stations. */
    GRAV_MIXED_BF16X3 = 2,  /* multi-model only: FP32 G tiles split into bf16 hi+lo,
                               3-product split-BF16 MFMA, FP32 accumulation */
    GRAV_FP32_VALU = 3      /* multi-model only: the same FP32 G tiles contracted on the
                               FP32 vector ALUs (comparison path) */
} grav_prec;

typedef void *grav_stream;   /* a hipStream_t */

/* Rectilinear prism mesh: node vectors are device pointers of nx+1, ny+1, nz+1
 * doubles, strictly increasing, z down. */
typedef struct {
    int32_t nx, ny, nz;
    const double *xn, *yn, *zn;
} grav_mesh;

/* Observation points: three device vectors of n doubles, z down. */
typedef struct {
    int64_t n;
    const double *x, *y, *z;
} grav_obs;

typedef struct {
    int32_t device;            /* HIP device ordinal */
    int32_t validate;          /* 1 (default) = check arguments on every call, 0 = trust them */
    uint64_t workspace_bytes;  /* device workspace owned by the context; 0 = 4 GiB */
} grav_ctx_opts;

typedef struct grav_ctx grav_ctx;

/* Operation codes for grav_workspace_bytes(). */
typedef enum {
    GRAV_OP_FORWARD = 0, GRAV_OP_ADJOINT = 1, GRAV_OP_DATASPACE = 2, GRAV_OP_TRACE = 3,
    GRAV_OP_INVERT = 4, GRAV_OP_FORWARD_MULTI = 5, GRAV_OP_TREND = 6, GRAV_OP_SECTIONS = 7
} grav_op;

/* Fill `opts` with the defaults (device 0, validate 1, 4 GiB workspace). */
void grav_ctx_opts_default(grav_ctx_opts *opts);

/* Create a context on opts->device (NULL opts = defaults) and allocate its
 * workspace.  *ctx receives the handle (NULL on failure).
 * Errors: GRAV_EINVAL (ctx NULL), GRAV_ENOMEM (allocation failed),
 * GRAV_EDEVICE (no such device / HIP failure). */
int grav_ctx_create(grav_ctx **ctx, const grav_ctx_opts *opts);

/* Release the context and its workspace (waits for the device to finish the
 * context's work).  NULL is ignored. */
void grav_ctx_destroy(grav_ctx *ctx);

/* Text of the last error on this context ("" if none).  Owned by the context,
 * valid until the next call on it.  NULL ctx: the last error of grav_ctx_create or
 * grav_forward_static on the calling thread. */
const char *grav_last_error(const grav_ctx *ctx);

/* Device workspace bytes that `op` needs for this shape and precision (K =
 * models for GRAV_OP_FORWARD_MULTI, ignored otherwise; GRAV_OP_TREND ignores
 * nx, ny, nz, n and prec).  Host-only; 0 means the shape or combination is
 * invalid.  The figure for n observations also covers every survey of fewer
 * observations on the same mesh. */
uint64_t grav_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, int64_t n, grav_op op,
                              grav_prec prec, int32_t K);

/* Forward product d = G m (paper Eq. 5-6; G from Eq. 1-3).
 *   m : M doubles (density contrast, flat cell order), d : n doubles (output, m/s^2).
 *   prec : GRAV_FP64 or GRAV_MIXED.
 * Errors: GRAV_EINVAL, GRAV_ENOMEM, GRAV_EDEVICE. */
int grav_forward(grav_ctx *ctx, const grav_mesh *mesh, const grav_obs *obs, const double *m,
                 double *d, grav_prec prec, grav_stream stream);

/* Adjoint product g = G^T v (the transpose of the forward operator, which the
 * data-space solution of Eq. 10-11 applies).
 *   v : n doubles, g : M doubles (output).  prec : GRAV_FP64 or GRAV_MIXED. */
int grav_adjoint(grav_ctx *ctx, const grav_mesh *mesh, const grav_obs *obs, const double *v,
                 double *g, grav_prec prec, grav_stream stream);

/* Data-space operator of Eq. 10-11: out = G C G^T v + lambda v with
 * W_m = C = diag(wdepth^-2) (depth weights w, Li-Oldenburg) and W_d = lambda I.
 *   wdepth : M doubles (> 0), lambda >= 0, v and out : n doubles (out may not
 *   alias v).  prec : GRAV_FP64 or GRAV_MIXED. */
int grav_dataspace_apply(grav_ctx *ctx, const grav_mesh *mesh, const grav_obs *obs,
                         const double *wdepth, double lambda, const double *v, double *out,
                         grav_prec prec, grav_stream stream);

/* trace(G C G^T) = sum_o sum_k C_k G_ok^2 with C = diag(wdepth^-2), written to
 * *trace (HOST pointer; the call waits for the result).  It sets the scale of
 * the data-space covariance W_d = delta I of Section 2.2 (a diagonal term with
 * one uniform value, which the paper does not give): grav_invert's
 * lambda < 0 rule is delta = 1e-2 trace / n.  Optional `diag`
 * (device, n doubles, may be NULL) receives the per-observation terms
 * sum_k C_k G_ok^2, i.e. the diagonal of G C G^T.  prec : GRAV_MIXED or GRAV_FP64. */
int grav_trace(grav_ctx *ctx, const grav_mesh *mesh, const grav_obs *obs, const double *wdepth,
               double *trace, double *diag, grav_prec prec, grav_stream stream);

/* Conjugate-gradient options for grav_invert. */
typedef struct {
    double tol;          /* stop when ||delta_d - A y||_2 / ||delta_d||_2 <= tol (recursive residual) */
    int32_t max_iter;    /* iteration cap (>= 1) */
    int32_t fixed_iters; /* > 0: run exactly this many iterations, no residual checks */
    int32_t precond;     /* 0: plain CG; 1: Jacobi-preconditioned CG with
                            M = diag(G C G^T) + lambda I (the trace sweep's
                            per-observation terms; grav_invert only, the
                            server requires 0) */
    /* Restarted CG, the solver policy of Section 2.2 (bounded inner CG runs
     * inside bounded outer model updates, with step backtracking).  With
     * restart > 0: each cycle restarts CG from the current y with the true
     * residual r = delta_d - A y and p = r and runs at most `restart`
     * iterations (leaving early once the recursive residual meets tol); after
     * the cycle the true residual is formed and, while the cycle raised
     * Q(y) = y^T A y / 2 - y^T delta_d, its step is halved (at most
     * `max_halvings` times); the solve stops when the true relative residual
     * meets tol or after `max_cycles` cycles.  max_iter and fixed_iters are
     * then unused (fixed_iters must be 0) and precond must be 0.
     * grav_invert only: the server requires restart = 0. */
    int32_t restart;      /* 0: plain (or Jacobi) CG as above; > 0: inner iteration cap */
    int32_t max_cycles;   /* restarted CG: outer cycle cap (>= 1) */
    int32_t max_halvings; /* restarted CG: step halvings per cycle (>= 0; 0 = no backtracking) */
    /* Misfit log: if history is non-NULL (HOST array of history_cap doubles),
     * entry k receives ||r_k|| / ||delta_d|| (the recursive residual) after
     * CG iteration k+1, over all cycles in order, for the first history_cap
     * iterations; later entries are untouched.  Not written with
     * fixed_iters > 0 (that mode reads no residual until the end).
     * grav_invert only: the server requires history_cap = 0. */
    int32_t history_cap;
    double *history;
    /* Warm start / resume: y0 (DEVICE, n doubles, or NULL = start from 0) is
     * the initial data-space iterate; residuals stay relative to
     * ||delta_d||.  y_out (DEVICE, n doubles, or NULL) receives the final
     * iterate, so a solve stopped at max_iter can be resumed later with it as
     * y0.  grav_invert only: the server requires both NULL. */
    const double *y0;
    double *y_out;
    /* 1: each plain or Jacobi CG iteration (the operator, dot products and
     * vector updates, up to the convergence check) is captured once per solve
     * into a HIP graph and replayed on `stream`: the same kernels with the
     * same arguments, fewer launches.  Ignored with restart > 0 or with kernel
     * timing on.  0: the kernels are launched one by one.  The server ignores
     * it. */
    int32_t graph;
} grav_cg_opts;

typedef struct {
    int32_t iters;       /* iterations performed */
    double relres;       /* final ||r|| / ||delta_d|| */
    double lambda_used;  /* lambda actually used */
    double trace;        /* trace(G C G^T) if it was computed (lambda < 0 or precond), else 0 */
    int32_t cycles;      /* restarted CG: outer cycles run (else 1) */
    int32_t halvings;    /* restarted CG: step halvings applied in total (else 0) */
} grav_cg_info;

/* Data-space inversion (paper Eq. 10-11): delta_d = d_obs - G m_ref;
 * solve (G C G^T + lambda I) y = delta_d by CG from y = 0; m = m_ref + C G^T y.
 *   d_obs : n doubles; wdepth : M doubles (> 0); lambda < 0 selects
 *   lambda = 1e-2 * trace(G C G^T) / n; m_ref : M doubles or NULL (= 0);
 *   m_out : M doubles (output); d_pred : n doubles (output G m_out) or NULL;
 *   info : HOST pointer or NULL.  The call waits for completion.
 * With cg->restart > 0 the solve follows the restarted policy described at
 * grav_cg_opts; info->iters then counts inner iterations over all cycles.
 * Returns GRAV_OK, GRAV_ENOCONV (iteration or cycle cap reached, outputs
 * valid), or an error. */
int grav_invert(grav_ctx *ctx, const grav_mesh *mesh, const grav_obs *obs, const double *d_obs,
                const double *wdepth, double lambda, const double *m_ref,
                const grav_cg_opts *cg, double *m_out, double *d_pred, grav_cg_info *info,
                grav_prec prec, grav_stream stream);

/* Regional-residual separation (the second-degree trend-surface removal of
 * the field workflow, Section 2.2; one surface over the whole domain also
 * joins sections inverted separately, Section 4.5): least-squares fit
 *   T(x, y) = sum_j coef[j] phi_j(u, w),  u = (x - x0) / L,  w = (y - y0) / L,
 *   phi = (1, u, w, u^2, u w, w^2) for degree 2, (1, u, w) for degree 1,
 * (x0, y0) the centre of the points' bounding box and L half its larger side
 * (1 for a single point).
 *   x, y, v : n doubles (DEVICE): station coordinates and values;
 *   coef : HOST, 6 doubles (output; entries past the degree's basis are 0);
 *   frame : HOST, 3 doubles (output) {x0, y0, L};
 *   resid : DEVICE, n doubles (output v - T) or NULL; may alias v;
 *   trend : DEVICE, n doubles (output T) or NULL.
 * The call waits for completion.  Errors: GRAV_EINVAL (NULL argument,
 * degree not 1 or 2, n below the basis size, a non-finite input, points that
 * do not determine the surface), GRAV_ENOMEM (workspace under
 * grav_workspace_bytes(.., GRAV_OP_TREND, ..)), GRAV_EDEVICE. */
int grav_trend_surface(grav_ctx *ctx, const double *x, const double *y, const double *v,
                       int64_t n, int32_t degree, double *coef, double *frame, double *resid,
                       double *trend, grav_stream stream);

/* Regional inversion by adjoining sections (Section 4.5, with the trend
 * separation of Section 2.2).  A regional problem too large to invert at once
 * is divided into sections that adjoin along y; each is inverted on its own
 * (grav_invert's data-space CG, Eq. 10-11, reference model 0) from its own
 * stations; the section models are placed into the regional mesh; then one
 * trend surface per layer, fitted across the complete domain, is removed from
 * the combined model to even out the steps the separate inversions leave at
 * the section boundaries.
 *   Section s spans mesh node rows ysplit[s] .. ysplit[s+1] of y (cells
 *   ysplit[s] .. ysplit[s+1]-1) and owns the stations with
 *   yn[ysplit[s]] <= y < yn[ysplit[s+1]]; stations below yn[ysplit[1]] belong
 *   to section 0 and those at or above yn[ysplit[nsec-1]] to the last one.
 *   data_degree (0 = none, 1, 2): the data minus its least-squares trend
 *   surface (grav_trend_surface) is inverted, the surface fitted per section
 *   (GRAV_TREND_SECTION: each section processed like a survey of its own) or
 *   once over all stations (GRAV_TREND_DOMAIN).
 *   model_degree (0, 1, 2): per layer k, the surface fitted to the combined
 *   model's layer values at the cell centres (x, y) is subtracted.
 *   lambda < 0: each section uses 1e-2 trace(G_s C_s G_s^T) / n_s. */
typedef enum { GRAV_TREND_SECTION = 0, GRAV_TREND_DOMAIN = 1 } grav_trend_scope;

typedef struct {
    int32_t nsec;            /* 1 .. 64 sections */
    const int32_t *ysplit;   /* HOST, nsec + 1 node indices: 0 = ysplit[0] < ... < ysplit[nsec] = ny */
    int32_t data_degree;     /* 0, 1 or 2 */
    int32_t data_scope;      /* grav_trend_scope */
    int32_t model_degree;    /* 0, 1 or 2 */
} grav_section_opts;

/*   d_obs : n doubles; wdepth : M doubles (> 0); cg : as for grav_invert,
 *   without y0, y_out or history (they must be NULL / 0);
 *   m_out : M doubles (output): the combined model;
 *   m_detrended : M doubles (output) or NULL: m_out minus its per-layer trend
 *   (a copy of m_out when model_degree = 0); may not alias m_out;
 *   info : HOST array of nsec entries or NULL: each section's CG summary.
 *   The call waits for completion.
 * Returns GRAV_OK, GRAV_ENOCONV (a section reached its iteration cap; all
 * outputs valid), or an error (after which m_out and m_detrended may hold the
 * sections finished before it): GRAV_EINVAL also for a section without
 * stations, fewer stations (or horizontal cells) than a trend surface needs,
 * or points that do not determine it; GRAV_ENOMEM below
 * grav_workspace_bytes(.., GRAV_OP_SECTIONS, ..), which bounds every split
 * of that mesh and survey. */
int grav_invert_sections(grav_ctx *ctx, const grav_mesh *mesh, const grav_obs *obs,
                         const double *d_obs, const double *wdepth, double lambda,
                         const grav_cg_opts *cg, const grav_section_opts *sec, double *m_out,
                         double *m_detrended, grav_cg_info *info, grav_prec prec,
                         grav_stream stream);

/* Multi-model forward D = G [m_1 ... m_K] (Eq. 6 for a block of models, a
 * dense contraction over prisms).
 *   models : M x K floats, model index fastest (models[k*K + j]);
 *   D : n x K floats (output), model index fastest; 1 <= K <= 64.
 *   prec : GRAV_MIXED_BF16X3 (MFMA) or GRAV_FP32_VALU. */
int grav_forward_multi(grav_ctx *ctx, const grav_mesh *mesh, const grav_obs *obs,
                       const float *models, int32_t K, float *D, grav_prec prec,
                       grav_stream stream);

/* Size of the library's static device scratch buffer (bytes, per device). */
#define GRAV_STATIC_SCRATCH_BYTES ((uint64_t)128 << 20)

/* Forward product d = G m without a context or any device allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same operator,
 * arguments, launch plan and kernels as grav_forward, so the result is
 * bitwise that of grav_forward for the same inputs and precision.
 *   Runs on the calling thread's current HIP device.  Its scratch memory is a
 *   static device array of GRAV_STATIC_SCRATCH_BYTES that the library holds
 *   on every device it runs on until the process ends; the call allocates and
 *   frees nothing (no hipMalloc/hipFree, no allocating library call).
 *   Problems whose forward workspace (grav_workspace_bytes(.., GRAV_OP_FORWARD,
 *   ..) plus 16 KiB) exceeds it are rejected with GRAV_ENOMEM before any work
 *   is enqueued (the paper-scale 178,797 x 3,307,500 forward needs 101 MiB).
 *   validate != 0: the arguments are checked on the device first and the call
 *   waits for that check on `stream` (as with a validating context); 0: the
 *   call is fully asynchronous and the caller guarantees the preconditions.
 *   All calls on one device share that device's buffer and leave their
 *   intermediate values in it: calls that may overlap in time on one device
 *   (different streams or threads) race and must be serialised by the caller.
 * Errors: GRAV_EINVAL, GRAV_ENOMEM (problem too large for the buffer),
 * GRAV_EDEVICE; grav_last_error(NULL) gives the reason (per thread). */
int grav_forward_static(const grav_mesh *mesh, const grav_obs *obs, const double *m, double *d,
                        grav_prec prec, int32_t validate, grav_stream stream);


/* ---------------------------------------------------------------------------
 * Serving: continuous batching of forward and inversion requests on one GPU
 * (GRAV_MIXED precision).  A worker thread owns a device memory pool of
 * `budget_bytes`; queued requests are admitted while their state (O(N + M)
 * per request: partial sums, CG vectors) fits in the pool: inversions in
 * arrival order while fewer than `max_active` are in flight, forward requests
 * (one step each) in arrival order on `max_active` slots of their own, passing
 * inversions that wait only for an inversion slot (never one that waits for
 * pool memory, so no request starves).  Every scheduling step issues one
 * persistent launch per sweep type: a grid of as many waves as the GPU holds
 * drains the tiles of all active requests (longest tiles first) from a
 * device counter, so each active inversion advances one CG iteration per step
 * and requests that arrive meanwhile join at the next step.  A request's launch
 * plan depends only on its own shape, so its result is bitwise the same alone
 * and in any mix.  A forward request is bitwise the same as grav_forward
 * (GRAV_MIXED).  An inversion's sweeps split the work into fewer observation
 * parts (adjoint) and column chunks (forward) than grav_invert's do once a
 * problem is larger than a few thousand observations or a few thousand node
 * columns (a batched launch fills the GPU with every request's waves), so it
 * agrees with grav_invert to rounding there and bitwise below that.
 * Requests may be submitted from any thread.
 * ------------------------------------------------------------------------ */
typedef struct grav_server grav_server;

typedef enum { GRAV_REQ_FORWARD = 0, GRAV_REQ_INVERT = 1 } grav_req_kind;

typedef struct {
    int32_t device;         /* HIP device ordinal */
    int32_t max_active;     /* inversions in flight at once, and as many forward
                               requests; 0 = 64 (max 256) */
    uint64_t budget_bytes;  /* device memory for request state; 0 = 16 GiB */
} grav_server_opts;

/* One request.  All arrays are caller-owned DEVICE pointers that must stay
 * valid and unmodified until the request is reported done.
 *   FORWARD: m (M) -> d (n), d = G m.
 *   INVERT : d_obs (n), wdepth (M, > 0), lambda (< 0 = 1e-2 trace/n), cg
 *            options -> m_out (M) = C G^T y, y the CG solution of
 *            (G C G^T + lambda I) y = d_obs (reference model 0).
 * `stream` is the stream on which the caller produced the inputs (NULL = the
 * null stream).  grav_server_submit makes the server wait for all work
 * enqueued on it before the call, so inputs still being written
 * asynchronously on that stream are complete before the server reads them;
 * inputs written on any other stream must be complete before submit.
 * Outputs are complete and visible once the request is reported done. */
typedef struct {
    int32_t kind;            /* grav_req_kind */
    grav_mesh mesh;
    grav_obs obs;
    const double *m;
    double *d;
    const double *d_obs;
    const double *wdepth;
    double lambda;
    grav_cg_opts cg;
    double *m_out;
    grav_stream stream;
} grav_request;

typedef struct {
    int32_t status;          /* GRAV_OK, GRAV_ENOCONV (max_iter reached), GRAV_ECANCELED
                                or an error */
    int32_t iters;           /* CG iterations (inversions) */
    double relres;           /* final relative residual (inversions) */
    double lambda_used;      /* (inversions) */
    double queue_ms;         /* submit -> admitted */
    double run_ms;           /* admitted -> done (device work finished) */
    uint64_t state_bytes;    /* pool bytes the request held */
} grav_request_info;

/* Create a server (allocates its pool, starts its worker thread).
 * Errors: GRAV_EINVAL, GRAV_ENOMEM, GRAV_EDEVICE. */
int grav_server_create(grav_server **srv, const grav_server_opts *opts);

/* Queue a request; *ticket identifies it.  The request is checked on the
 * device before it is queued (same rules as grav_forward / grav_invert).
 * Errors: GRAV_EINVAL (bad request), GRAV_ENOMEM (its state alone exceeds the
 * pool), GRAV_EDEVICE. */
int grav_server_submit(grav_server *srv, const grav_request *req, uint64_t *ticket);

/* *done = 1 when the request has finished (outputs written and visible);
 * then `info` (nullable) is filled and the ticket is retired.  Returns
 * GRAV_OK, or GRAV_EINVAL for an unknown/retired ticket. */
int grav_server_poll(grav_server *srv, uint64_t ticket, int32_t *done, grav_request_info *info);

/* Block until the request has finished; fills `info` (nullable), retires the
 * ticket, returns its status. */
int grav_server_wait(grav_server *srv, uint64_t ticket, grav_request_info *info);

/* Cancel a request.  A queued request is dropped at once; a request in
 * flight stops after the scheduling step under way.  Either way it then
 * reports done with status GRAV_ECANCELED (its outputs are unspecified) and
 * is retired by grav_server_poll or grav_server_wait as usual.  A request
 * that has already finished keeps its result.  Returns GRAV_OK, or
 * GRAV_EINVAL for an unknown/retired ticket. */
int grav_server_cancel(grav_server *srv, uint64_t ticket);

/* Finish all admitted and queued requests, stop the worker, free the pool. */
void grav_server_destroy(grav_server *srv);

/* ---------------------------------------------------------------------------
 * Diagnostics: per-kernel timing.  With timing enabled, the library records a
 * pair of HIP events on the call's stream around every launch of its sweep
 * kernels ("forward_mixed", "forward_f64", "adjoint_mixed", "adjoint_f64",
 * "trace_mixed", "trace_f64", "multi_bf16x3", "multi_fp32").
 * grav_kernel_time() waits for the recorded events of `kernel` and returns the
 * summed duration (HOST *total_ms) and launch count (HOST *launches) since the
 * last reset.  Errors: GRAV_EINVAL (null ctx/out, unknown kernel name). */
int grav_set_timing(grav_ctx *ctx, int32_t enable);

/* Diagnostics: sustained issue rates of the instruction classes the sweeps
 * are built from, measured on the context's device with eight independent
 * dependency chains per lane and eight waves per SIMD.  rates (HOST, 6
 * doubles) receives chain steps per second summed over lanes for:
 *   [0] FP32 FMA, [1] v_log_f32 + FP32 add, [2] v_rcp_f32 + FP32 add,
 *   [3] v_sqrt_f32 + FP32 add, [4] FP64 FMA, [5] FP32 add.
 * A transcendental's cost in FP32-FMA issue slots is
 * rates[0]/rates[i] - rates[0]/rates[5].
 * Runs about 20 ms of device work; waits for it.
 * Errors: GRAV_EINVAL (null ctx/rates), GRAV_ENOMEM, GRAV_EDEVICE. */
int grav_issue_rates(grav_ctx *ctx, double *rates, grav_stream stream);

/* Diagnostics: issue rates of pairs of instruction classes, measured like
 * grav_issue_rates.  rates (HOST, 5 doubles) receives chain steps per second
 * summed over lanes; in [0]-[3] half of the chains are FP32 FMA and half of
 * the other class:
 *   [0] v_log_f32 + add chains on alternating waves (even waves FMA, odd
 *       waves the other class), [1] the same two classes interleaved in every
 *       wave, [2] v_cmp + v_cndmask + add chains on alternating waves,
 *   [3] interleaved, [4] the compare-and-select chains alone.
 * With r_a, r_b the single-class rates (grav_issue_rates, or [4]), the two
 * halves run one after the other would reach 2 / (1/r_a + 1/r_b); a higher
 * rate is work issued together.
 * Errors: GRAV_EINVAL (null ctx/rates), GRAV_ENOMEM, GRAV_EDEVICE. */
int grav_issue_pair_rates(grav_ctx *ctx, double *rates, grav_stream stream);
int grav_kernel_time(grav_ctx *ctx, const char *kernel, double *total_ms, int64_t *launches);
int grav_reset_timing(grav_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* GRAV_H */
