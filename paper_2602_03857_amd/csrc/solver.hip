// Data-space inversion (paper Section 2.2, Eq. 10-11) with conjugate
// gradients on the N x N system (G C G^T + lambda I) y = delta_d, the
// operator applied matrix-free by the sweeps, all vectors and scalars on the
// device.  Also the workspace sizing shared by every entry point.
#include <hip/hip_runtime.h>

#include <rocprofiler-sdk-roctx/roctx.h>

#include <cmath>

#include "api_internal.h"

namespace grav {

// A named range (rocprofv3 --marker-trace) for the lifetime of the object.
struct RoctxRange {
    explicit RoctxRange(const char *name) { roctxRangePushA(name); }
    ~RoctxRange() { roctxRangePop(); }
    RoctxRange(const RoctxRange &) = delete;
    RoctxRange &operator=(const RoctxRange &) = delete;
};

#define HIP_TRY(expr, where)                                       \
    do {                                                           \
        hipError_t _e = (expr);                                    \
        if (_e != hipSuccess) return hip_fail(ctx, _e, where);     \
    } while (0)

// A HIP graph and its executable, destroyed with the object.
struct IterGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    IterGraph() = default;
    IterGraph(const IterGraph &) = delete;
    IterGraph &operator=(const IterGraph &) = delete;
    ~IterGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

static int read_scalars(grav_ctx *ctx, hipStream_t st) {
    HIP_TRY(hipMemcpyAsync(ctx->h_scal, ctx_scalars(ctx), kNumScalars * sizeof(double),
                           hipMemcpyDeviceToHost, st), "scalar copy");
    HIP_TRY(hipStreamSynchronize(st), "scalar sync");
    return GRAV_OK;
}

// Restarted CG (the solver policy of Section 2.2).  On entry y holds the
// initial iterate (0 or a warm start), r = dd - A y its residual and scal[kB2]
// the squared norm of dd (= delta_d).  Each cycle
// restarts from the true residual; after a cycle the true residual r = dd - A y
// is formed and, while Q(y) = -(y . (dd + r)) / 2 rose above the previous
// cycle's value, the step is halved.  The residual is affine in y, so the
// halved iterate's residual is the mean of the two residuals and needs no
// operator application.
struct SolveStats {
    int iters = 0, cycles = 0, halvings = 0;
    double relres = 0.0;
    bool converged = false;
};

static int restarted_cg(grav_ctx *ctx, Arena &ar, const Mesh &g, const Obs &o, const double *wdepth,
                        double lambda, grav_prec prec, hipStream_t st, const grav_cg_opts &cg,
                        const double *dd, double *y, double *r, double *p, double *q, double *yold,
                        double *rold, double b2, SolveStats *out) {
    const int64_t n = o.n;
    double *scal = ctx_scalars(ctx);
    double *dpart = ctx_dot_partials(ctx);
    double *dpart2 = ctx_dot_partials2(ctx);
    SolveStats s;
    s.relres = b2 > 0.0 ? 1.0 : 0.0;
    s.converged = b2 == 0.0;
    double rr = b2;         // r . r of the current (true) residual
    double q_prev = 0.0;    // Q of the iterate the cycle starts from
    // Q(y) and r.r of the current y, r
    auto objective = [&](double *q_val) -> int {
        HIP_TRY(launch_lincomb(q, 1.0, dd, 1.0, r, n, st), "lincomb");
        HIP_TRY(launch_dot(y, q, n, dpart, st), "dot");
        HIP_TRY(launch_dot_finish(dpart, scal, kFinishPlain, kYB, st), "dot");
        HIP_TRY(launch_dot(r, r, n, dpart2, st), "dot");
        HIP_TRY(launch_dot_finish(dpart2, scal, kFinishPlain, kRR, st), "dot");
        int rc = read_scalars(ctx, st);
        if (rc) return rc;
        *q_val = -0.5 * ctx->h_scal[kYB];
        rr = ctx->h_scal[kRR];
        return GRAV_OK;
    };
    if (!s.converged) {
        int rc = objective(&q_prev);            // Q(0) = 0 and r.r = b2 without a warm start
        if (rc) return rc;
        s.relres = std::sqrt(rr / b2);
        s.converged = s.relres <= cg.tol;
    }
    while (s.cycles < cg.max_cycles && !s.converged) {
        ++s.cycles;
        HIP_TRY(launch_sub(y, nullptr, yold, n, st), "copy");
        HIP_TRY(launch_sub(r, nullptr, rold, n, st), "copy");
        HIP_TRY(launch_sub(r, nullptr, p, n, st), "copy");
        for (int j = 0; j < cg.restart && std::sqrt(rr / b2) > cg.tol; ++j) {
            const RoctxRange range("grav cg iteration");
            int rc = op_dataspace(ctx, ar, g, o, wdepth, lambda, p, q, prec, st);
            if (rc) return rc;
            HIP_TRY(launch_dot(p, q, n, dpart, st), "dot");
            HIP_TRY(launch_dot_finish(dpart, scal, kFinishPQ, 0, st), "dot");
            HIP_TRY(launch_cg_update_yr(y, r, p, q, n, scal, dpart, st), "cg update");
            HIP_TRY(launch_dot_finish(dpart, scal, kFinishRRNew, 0, st), "dot");
            rc = read_scalars(ctx, st);
            if (rc) return rc;
            rr = ctx->h_scal[kRR];
            if (s.iters < cg.history_cap && cg.history) cg.history[s.iters] = std::sqrt(rr / b2);
            ++s.iters;
            HIP_TRY(launch_cg_update_p(p, r, n, scal, st), "cg update");
        }
        // true residual r = dd - A y
        int rc = op_dataspace(ctx, ar, g, o, wdepth, lambda, y, q, prec, st);
        if (rc) return rc;
        HIP_TRY(launch_sub(dd, q, r, n, st), "residual");
        double q_new = 0.0;
        rc = objective(&q_new);
        if (rc) return rc;
        for (int h = 0; h < cg.max_halvings && q_new > q_prev; ++h) {
            HIP_TRY(launch_lincomb(y, 0.5, y, 0.5, yold, n, st), "halve");
            HIP_TRY(launch_lincomb(r, 0.5, r, 0.5, rold, n, st), "halve");
            rc = objective(&q_new);
            if (rc) return rc;
            ++s.halvings;
        }
        q_prev = q_new;
        s.relres = std::sqrt(rr / b2);
        s.converged = s.relres <= cg.tol;
    }
    *out = s;
    return GRAV_OK;
}

int run_invert(grav_ctx *ctx, const Mesh &g, const Obs &o, const double *d_obs,
               const double *wdepth, double lambda, const double *m_ref, const grav_cg_opts &cg,
               double *m_out, double *d_pred, grav_cg_info *info, grav_prec prec, hipStream_t st) {
    Arena ar = ctx_arena(ctx);
    const int64_t n = o.n;
    double *y = ar.take<double>(n);
    double *r = ar.take<double>(n);
    double *p = ar.take<double>(n);
    double *q = ar.take<double>(n);
    const bool pc = cg.precond == 1;            // Jacobi preconditioner
    double *z = pc ? ar.take<double>(n) : nullptr;
    double *dinv = pc ? ar.take<double>(n) : nullptr;
    const bool restarted = cg.restart > 0;      // delta_d, y and r of the cycle start
    double *dd = restarted ? ar.take<double>(n) : nullptr;
    double *yold = restarted ? ar.take<double>(n) : nullptr;
    double *rold = restarted ? ar.take<double>(n) : nullptr;
    if (ar.failed) return fail(ctx, GRAV_ENOMEM, "workspace too small for the CG vectors");
    double *scal = ctx_scalars(ctx);
    double *dpart = ctx_dot_partials(ctx);
    double *dpart2 = ctx_dot_partials2(ctx);

    double trace = 0.0;
    if (lambda < 0.0 || pc) {   // lambda = 1e-2 * trace(G C G^T) / n; diag(G C G^T) for M
        int rc = op_trace(ctx, ar, g, o, wdepth, &trace, dinv, prec, st);
        if (rc) return rc;
        if (lambda < 0.0) lambda = 1e-2 * trace / (double)n;
    }

    // r = delta_d = d_obs - G m_ref ; ||delta_d||^2 -> scal[kB2] (and kRR)
    if (m_ref) {
        int rc = op_forward(ctx, ar, g, o, m_ref, r, prec, st, -GRAV_GAMMA, d_obs, 1.0);
        if (rc) return rc;
    } else {
        HIP_TRY(launch_sub(d_obs, nullptr, r, n, st), "copy");
    }
    HIP_TRY(launch_dot(r, r, n, dpart, st), "dot");
    HIP_TRY(launch_dot_finish(dpart, scal, kFinishInit, 0, st), "dot");
    if (restarted) HIP_TRY(launch_sub(r, nullptr, dd, n, st), "copy");
    // y = y0 (warm start: r = delta_d - A y0) or 0
    if (cg.y0) {
        HIP_TRY(launch_sub(cg.y0, nullptr, y, n, st), "copy");
        int rc = op_dataspace(ctx, ar, g, o, wdepth, lambda, y, q, prec, st);
        if (rc) return rc;
        HIP_TRY(launch_lincomb(r, 1.0, r, -1.0, q, n, st), "residual");
    } else {
        HIP_TRY(launch_fill(y, 0.0, n, st), "fill");
    }
    // p = r (or M^-1 r); r.r (and r.z) of the starting residual
    if (pc) {
        HIP_TRY(launch_pcg_setup(dinv, lambda, dinv, r, z, p, n, dpart, dpart2, st), "pcg setup");
        HIP_TRY(launch_dot_finish(dpart, scal, kFinishPlain, kRR, st), "dot");
        HIP_TRY(launch_dot_finish(dpart2, scal, kFinishPlain, kRZ, st), "dot");
    } else {
        HIP_TRY(launch_sub(r, nullptr, p, n, st), "copy");
        if (cg.y0) {
            HIP_TRY(launch_dot(r, r, n, dpart, st), "dot");
            HIP_TRY(launch_dot_finish(dpart, scal, kFinishPlain, kRR, st), "dot");
        }
    }
    int rc = read_scalars(ctx, st);
    if (rc) return rc;
    const double b2 = ctx->h_scal[kB2];
    if (b2 == 0.0 && cg.y0) HIP_TRY(launch_fill(y, 0.0, n, st), "fill");   // delta_d = 0: y = 0

    const bool fixed = !restarted && cg.fixed_iters > 0;
    const int iters_cap = restarted ? 0 : fixed ? cg.fixed_iters : cg.max_iter;
    int it = 0, cycles = 1, halvings = 0;
    double relres = b2 > 0.0 ? std::sqrt(ctx->h_scal[kRR] / b2) : 0.0;
    bool converged = b2 == 0.0 || (!fixed && relres <= cg.tol);
    if (restarted) {
        SolveStats ss;
        rc = restarted_cg(ctx, ar, g, o, wdepth, lambda, prec, st, cg, dd, y, r, p, q, yold, rold,
                          b2, &ss);
        if (rc) return rc;
        it = ss.iters;
        cycles = ss.cycles;
        halvings = ss.halvings;
        relres = ss.relres;
        converged = ss.converged;
    }
    // One iteration up to its convergence check: q = A p, alpha, y, r (z) and
    // the new residual norm, all on the device.
    auto iteration = [&](hipStream_t s) -> int {
        int irc = op_dataspace(ctx, ar, g, o, wdepth, lambda, p, q, prec, s);
        if (irc) return irc;
        HIP_TRY(launch_dot(p, q, n, dpart, s), "dot");
        if (pc) {
            HIP_TRY(launch_dot_finish(dpart, scal, kFinishPQPrecond, 0, s), "dot");
            HIP_TRY(launch_pcg_update_yrz(y, r, z, p, q, dinv, n, scal, dpart, dpart2, s), "pcg update");
            HIP_TRY(launch_dot_finish(dpart, scal, kFinishPlain, kRR, s), "dot");
            HIP_TRY(launch_dot_finish(dpart2, scal, kFinishRZNew, 0, s), "dot");
        } else {
            HIP_TRY(launch_dot_finish(dpart, scal, kFinishPQ, 0, s), "dot");
            HIP_TRY(launch_cg_update_yr(y, r, p, q, n, scal, dpart, s), "cg update");
            HIP_TRY(launch_dot_finish(dpart, scal, kFinishRRNew, 0, s), "dot");
        }
        return GRAV_OK;
    };
    // cg.graph: the iteration's launches are captured once, on a stream of the
    // context (the caller's stream may be the null stream, which cannot be
    // captured), and replayed on the caller's stream; they take the same
    // pointers every iteration.  Not with kernel timing on (its events would
    // be captured too).
    IterGraph ig;
    const bool graph = cg.graph != 0 && !restarted && !ctx->timing && it < iters_cap && !converged;
    if (graph) {
        if (!ctx->cap_stream)
            HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking), "capture stream");
        HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
        const int crc = iteration(ctx->cap_stream);
        const hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &ig.graph);
        if (crc) return crc;
        HIP_TRY(ce, "end capture");
        HIP_TRY(hipGraphInstantiate(&ig.exec, ig.graph, nullptr, nullptr, 0), "graph instantiate");
    }
    for (it = restarted ? it : 0; it < iters_cap && !converged;) {
        const RoctxRange range("grav cg iteration");
        if (graph) {
            HIP_TRY(hipGraphLaunch(ig.exec, st), "graph launch");
        } else {
            rc = iteration(st);
            if (rc) return rc;
        }
        ++it;
        if (!fixed) {
            rc = read_scalars(ctx, st);
            if (rc) return rc;
            relres = std::sqrt(ctx->h_scal[kRR] / b2);
            if (it - 1 < cg.history_cap && cg.history) cg.history[it - 1] = relres;
            if (relres <= cg.tol) { converged = true; break; }
        }
        HIP_TRY(launch_cg_update_p(p, pc ? z : r, n, scal, st), "cg update");
    }
    if (fixed && b2 > 0.0) {
        rc = read_scalars(ctx, st);
        if (rc) return rc;
        relres = std::sqrt(ctx->h_scal[kRR] / b2);
    }

    if (cg.y_out) HIP_TRY(launch_sub(y, nullptr, cg.y_out, n, st), "copy");
    // m = m_ref + C G^T y ; optional predicted data
    rc = op_adjoint(ctx, ar, g, o, y, m_out, prec, st, GRAV_GAMMA, wdepth, m_ref);
    if (rc) return rc;
    if (d_pred) {
        rc = op_forward(ctx, ar, g, o, m_out, d_pred, prec, st, GRAV_GAMMA, nullptr, 0.0);
        if (rc) return rc;
    }
    HIP_TRY(hipStreamSynchronize(st), "final sync");
    if (info) {
        info->iters = it;
        info->relres = relres;
        info->lambda_used = lambda;
        info->trace = trace;
        info->cycles = cycles;
        info->halvings = halvings;
    }
    if (!fixed && !converged) {
        ctx->err = restarted ? "restarted CG reached max_cycles before tol"
                             : "CG reached max_iter before tol";
        return GRAV_ENOCONV;
    }
    return GRAV_OK;
}

// ------------------------------------------------------------------ sizing

static size_t need_forward(const Mesh &g, int64_t n, grav_prec prec) {
    Counter c;
    c.take<double>((size_t)forward_partials_bound(g.ncols(), n));
    if (prec == GRAV_MIXED) {
        c.take<float>(layer_table_len(g.nz));
        c.take<double>(g.nsegs());
    } else {
        c.take<double>(g.nnodes());
    }
    return c.off;
}

static size_t need_adjoint(const Mesh &g, int64_t n, grav_prec prec) {
    Counter c;
    if (prec == GRAV_MIXED) {
        c.take<float>(layer_table_len(g.nz));
        c.take<double>((size_t)adjoint_parts_bound(g.ncols(), g.nz, n) * g.nsegs());
        c.take<double>(g.nsegs());
    } else {
        c.take<double>((size_t)node_adjoint_parts_bound(g.nnodes(), n) * g.nnodes());
        c.take<double>(g.nnodes());
    }
    return c.off;
}

static size_t need_trace(const Mesh &g, int64_t n) {
    Counter c;
    c.take<double>((size_t)trace_partials_bound(g.nx, n));
    c.take<double>(n);
    c.take<float>(layer_table_len(g.nz));
    return c.off;
}

static size_t need_dataspace(const Mesh &g, int64_t n, grav_prec prec) {
    Counter c;
    c.take<double>(g.ncells());
    const size_t a = need_adjoint(g, n, prec), f = need_forward(g, n, prec);
    return c.off + (a > f ? a : f);
}

uint64_t workspace_need(int nx, int ny, int nz, int64_t n, grav_op op, grav_prec prec, int K) {
    const Mesh g{nx, ny, nz, nullptr, nullptr, nullptr};
    switch (op) {
        case GRAV_OP_FORWARD:
            return need_forward(g, n, prec);
        case GRAV_OP_ADJOINT:
            return need_adjoint(g, n, prec);
        case GRAV_OP_DATASPACE:
            return need_dataspace(g, n, prec);
        case GRAV_OP_TRACE:
            return need_trace(g, n);
        case GRAV_OP_INVERT: {
            Counter c;
            for (int i = 0; i < 7; ++i) c.take<double>(n);   // CG vectors (restarted: 7)
            size_t inner = need_dataspace(g, n, prec);
            const size_t t = need_trace(g, n);
            if (t > inner) inner = t;
            return c.off + inner;
        }
        case GRAV_OP_FORWARD_MULTI:
            return multi_workspace_need(g, n, prec, K);
    }
    return 0;
}

}  // namespace grav
