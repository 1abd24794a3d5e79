// Context layout and the operator compositions shared by the C-ABI files.
#pragma once

#include <hip/hip_runtime.h>

#include <initializer_list>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "grav_internal.h"

struct grav_ctx {
    int device = 0;
    bool validate = true;
    char *ws = nullptr;          // device workspace; the first kReserveBytes hold flags,
    size_t ws_bytes = 0;         // CG scalars and dot-product partials
    char *h_pinned = nullptr;    // pinned host staging (flags, scalars)
    int *h_flags = nullptr;
    double *h_scal = nullptr;
    std::string err;
    size_t arena_skip = 0;  // bytes at the arena's head held by an enclosing workflow
    bool timing = false;    // record events around sweep launches
    hipStream_t cap_stream = nullptr;   // for capturing CG iterations into a graph (lazily created)
    std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::map<std::string, std::pair<double, int64_t>> totals;
};

namespace grav {

// Reserved head of the workspace: [0,256) flags, [256,512) scalars,
// [512, 512 + 16*kDotBlocks) two arrays of dot partials.
constexpr size_t kReserveBytes = 16384;

inline double *ctx_scalars(grav_ctx *ctx) { return reinterpret_cast<double *>(ctx->ws + 256); }
inline double *ctx_dot_partials(grav_ctx *ctx) { return reinterpret_cast<double *>(ctx->ws + 512); }
inline double *ctx_dot_partials2(grav_ctx *ctx) {
    return reinterpret_cast<double *>(ctx->ws + 512 + 8 * kDotBlocks);
}

struct ArrayCheck {
    const double *ptr;
    int64_t len;
    bool positive;   // true: finite and > 0; false: finite
};

int fail(grav_ctx *ctx, int code, const std::string &msg);
// Error text of the calls that take no context (grav_last_error(NULL)), per thread.
void set_context_free_error(const std::string &msg);
int hip_fail(grav_ctx *ctx, hipError_t e, const char *where);
Arena ctx_arena(grav_ctx *ctx);
int check_geometry_host(grav_ctx *ctx, const grav_mesh *mesh, const grav_obs *obs);
int validate_on_device(grav_ctx *ctx, const Mesh &g, const Obs &o, hipStream_t st,
                       std::initializer_list<ArrayCheck> arrays);

int op_forward(grav_ctx *ctx, Arena &ar, const Mesh &g, const Obs &o, const double *m, double *d,
               grav_prec prec, hipStream_t st, double scale, const double *add, double coef);
int op_adjoint(grav_ctx *ctx, Arena &ar, const Mesh &g, const Obs &o, const double *v, double *out,
               grav_prec prec, hipStream_t st, double scale, const double *wdepth,
               const double *base);
int op_dataspace(grav_ctx *ctx, Arena &ar, const Mesh &g, const Obs &o, const double *wdepth,
                 double lambda, const double *v, double *out, grav_prec prec, hipStream_t st);
int op_trend_surface(grav_ctx *ctx, const double *x, const double *y, const double *v, int64_t n,
                     int degree, double *coef, double *frame, double *resid, double *trend,
                     hipStream_t st);
uint64_t trend_workspace_need();
int op_issue_rates(grav_ctx *ctx, double *rates, hipStream_t st);
int op_issue_pair_rates(grav_ctx *ctx, double *rates, hipStream_t st);
int op_trace(grav_ctx *ctx, Arena &ar, const Mesh &g, const Obs &o, const double *wdepth,
             double *trace, double *diag, grav_prec prec, hipStream_t st);
constexpr int kMaxSections = 64;
int check_cg_opts(grav_ctx *ctx, const grav_cg_opts *cg);
uint64_t sections_workspace_need(const Mesh &g, int64_t n, grav_prec prec);
int run_sections(grav_ctx *ctx, const Mesh &g, const Obs &o, const double *d_obs,
                 const double *wdepth, double lambda, const grav_cg_opts &cg,
                 const grav_section_opts &so, double *m_out, double *m_detr,
                 grav_cg_info *info, grav_prec prec, hipStream_t st);
int run_invert(grav_ctx *ctx, const Mesh &g, const Obs &o, const double *d_obs,
               const double *wdepth, double lambda, const double *m_ref, const grav_cg_opts &cg,
               double *m_out, double *d_pred, grav_cg_info *info, grav_prec prec, hipStream_t st);

// Records a start event now and an end event when it goes out of scope (both
// on `st`), if timing is enabled on the context.
class KernelTimer {
  public:
    KernelTimer(grav_ctx *ctx, const char *name, hipStream_t st);
    ~KernelTimer();
  private:
    grav_ctx *ctx_;
    const char *name_;
    hipStream_t st_;
    hipEvent_t start_ = nullptr;
};

uint64_t workspace_need(int nx, int ny, int nz, int64_t n, grav_op op, grav_prec prec, int K);
uint64_t multi_workspace_need(const Mesh &g, int64_t n, grav_prec prec, int K);

}  // namespace grav
