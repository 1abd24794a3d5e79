// Continuous-batching server for forward and inversion requests (declared in
// include/grav.h).  One worker thread per server runs scheduling steps:
//
//   admit   queued requests while their state fits in the device pool:
//           inversions in arrival order while fewer than max_active are in
//           flight; forward requests (one step each) in arrival order on
//           their own max_active slots, passing inversions that wait only
//           for an inversion slot (never one that waits for pool memory);
//   init    per newly admitted request: layer thicknesses, W2(m) (forward) or
//           trace -> lambda, r = p = d_obs, y = 0, r.r (inversion);
//   sweep A one batched adjoint launch over every inversion in CG
//           (v = p) or in its final step (v = y);
//   post A  per request: reduce U, finish (x C, gamma) -> t and W2(t), or m_out;
//   sweep F one batched forward launch over every new forward
//           request and every inversion in CG;
//   post F  per request: d = gamma sum (forward) or the CG update
//           q = gamma sum + lambda p, alpha, y, r, beta, p;
//   sync    one copy of the CG scalar table, then the host advances each
//           request (converged / max_iter -> final step; final -> done).
//
// A batched sweep is a persistent launch: a grid of as many waves as fit on
// the GPU at once drains the tiles (virtual blocks, taken half a tile per wave)
// of every request from one device counter.  A tile finds its request in a
// table of per-request jobs
// (each with its own plan and buffers, tiles numbered consecutively) and runs
// the same per-block body as the single-call kernels, so a request's
// arithmetic does not depend on what it is batched with or which block runs
// it.  The table lists the requests by decreasing tile cost, so the longest
// tiles are taken first and the last ones to finish are the shortest.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "api_internal.h"
#include "sweep_bodies.h"
#include "admission.h"
#include "pool_allocator.h"

using namespace grav;

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kMaxActiveCap = 256;
constexpr int kSlotScalars = 16;     // per active request in the device scalar table
constexpr int kLambdaSlot = 6;       // lambda used by the request
constexpr int kTraceSlot = 7;        // trace(G C G^T) when computed
// Adjoint plan of a served request: the batched launch mixes the waves of
// every active request, so each request needs fewer observation parts than a
// single call to fill the GPU, and its partial sums stay small in the pool.
constexpr int64_t kServerTargetWavesAdj = 32768;
constexpr int64_t kServerMaxPartialBytes = int64_t(512) << 20;
// Forward plan of an inversion's CG iterations, for the same reason: fewer
// column chunks, so the per-iteration reduction of the chunk partial sums
// reads less.  A forward request keeps the single-call plan, so that its
// result is bitwise that of grav_forward.
constexpr int64_t kServerTargetWavesFwdCG = 16384;

struct FwdJob {
    const double *xn, *yn, *zn, *ox, *oy, *oz, *w2;
    const float *hk;
    double *partial;
    int64_t n, ncols, cols_per_chunk, block_begin;
    int32_t ny1, nz, nchunk, pad;
};

struct AdjJob {
    const double *xn, *yn, *zn, *ox, *oy, *oz, *v;
    const float *hk;
    double *upart;
    int64_t n, obs_per_part, ncols, block_begin;
    int32_t ny1, nz, nparts, nkc;
};

// Pointers read from a job table are generic pointers to the compiler, so
// loads through them would go through the flat path in vector registers; they
// all point to device global memory and pass through global_ptr().

template <typename Job>
__device__ __forceinline__ int find_job(const Job *__restrict__ jobs, int njobs, int64_t vb) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].block_begin <= vb) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Persistent launches drain half tiles: a tile is a kBlock-lane block of the
// single-call plan, and each wave (one 64-thread block) takes the next half
// tile from a device counter (one atomic add by lane 0, made wave-uniform with
// readfirstlane) and runs its 64 lanes of that block's body, with no barrier
// and no shared memory.  The counter only grows, so every wave leaves its
// loop once the counter has passed the number of half tiles.
__device__ __forceinline__ uint32_t next_half_tile(uint32_t *next) {
    uint32_t v = 0;
    if (threadIdx.x == 0) v = atomicAdd(next, 1u);
    return __builtin_amdgcn_readfirstlane(v);
}

constexpr int kHalves = kBlock / 64;   // waves per tile

__global__ __launch_bounds__(64) void k_forward_batched(const FwdJob *__restrict__ jobs, int njobs,
                                                        uint32_t halves, uint32_t *__restrict__ next) {
    for (uint32_t hv = next_half_tile(next); hv < halves; hv = next_half_tile(next)) {
        const int64_t vb = hv / kHalves;
        const int lane = (int)(hv % kHalves) * 64 + (int)threadIdx.x;
        const FwdJob &j = jobs[find_job(jobs, njobs, vb)];
        const int64_t local = vb - j.block_begin;
        forward_mixed_block(global_ptr(j.xn), global_ptr(j.yn), global_ptr(j.zn), j.ny1, j.nz,
                            global_ptr(j.hk), global_ptr(j.ox), global_ptr(j.oy), global_ptr(j.oz), j.n,
                            global_ptr(j.w2), j.ncols, j.cols_per_chunk, (int)(local % j.nchunk),
                            local / j.nchunk, global_ptr(j.partial), lane);
    }
}

// Bounded to 8 waves per SIMD like the single-call adjoint sweep.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(8, 8)))
void k_adjoint_batched(const AdjJob *__restrict__ jobs, int njobs, uint32_t halves,
                       uint32_t *__restrict__ next) {
    for (uint32_t hv = next_half_tile(next); hv < halves; hv = next_half_tile(next)) {
        const int64_t vb = hv / kHalves;
        const int lane = (int)(hv % kHalves) * 64 + (int)threadIdx.x;
        const AdjJob &j = jobs[find_job(jobs, njobs, vb)];
        int64_t local = vb - j.block_begin;
        const int part = (int)(local % j.nparts);
        local /= j.nparts;
        const int kc = (int)(local % j.nkc);
        local /= j.nkc;
        adjoint_mixed_block(global_ptr(j.xn), global_ptr(j.yn), global_ptr(j.zn), j.ny1, j.nz,
                            global_ptr(j.hk), global_ptr(j.ox), global_ptr(j.oy), global_ptr(j.oz),
                            global_ptr(j.v), j.n, j.obs_per_part, j.ncols, j.nkc, part, kc, local,
                            global_ptr(j.upart), lane);
    }
}

// scal[kLambdaSlot] = lambda >= 0 ? lambda : 1e-2 * scal[kTraceSlot] / n
__global__ void k_set_lambda(double *scal, double lambda, int64_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        scal[kLambdaSlot] = lambda >= 0.0 ? lambda : 1e-2 * scal[kTraceSlot] / (double)n;
}

// out = scale * sum_p part[p][i] + (*coef) * add[i]
__global__ void k_reduce_parts_dcoef(const double *__restrict__ part, int nparts, int64_t len,
                                     double scale, const double *__restrict__ add,
                                     const double *__restrict__ coef, double *__restrict__ out) {
    const double c = *coef;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int p = 0; p < nparts; ++p) acc += part[(int64_t)p * len + i];
        out[i] = fma(c, add[i], scale * acc);
    }
}

unsigned grid_of(int64_t len) {
    int64_t g = (len + 255) / 256;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (unsigned)g;
}

enum class Phase { Queued, Init, CG, Final, Done };

struct Request {
    uint64_t ticket = 0;
    grav_request r{};
    Mesh g{};
    Obs o{};
    Phase phase = Phase::Queued;
    size_t off = 0, bytes = 0;
    int slot = -1;
    ForwardPlan fp{};
    AdjointPlan ap{};
    ForwardPlan tp{};
    float *hk = nullptr;
    double *w2 = nullptr, *fpart = nullptr, *upart = nullptr, *U = nullptr, *t = nullptr;
    double *y = nullptr, *res = nullptr, *p = nullptr, *q = nullptr, *tpart = nullptr,
           *diag = nullptr, *dpart = nullptr;
    int iters = 0;
    double relres = 0.0, lambda = 0.0;
    int status = GRAV_OK;
    bool finished = false;   // worker-private: the last step completed it
    bool done = false;       // published under the server mutex after release
    bool cancel = false;     // set under the server mutex by grav_server_cancel
    Clock::time_point t_submit, t_admit, t_done;
};

// Device bytes of a request's state, and (optionally) the carving of it.
size_t request_layout(Request &q, char *base) {
    Arena ar;
    ar.base = base;
    ar.size = base ? q.bytes : ~size_t(0) >> 1;
    const Mesh &g = q.g;
    const int64_t n = q.o.n;
    q.fp = plan_forward(g.ncols(), n, q.r.kind == GRAV_REQ_INVERT ? kServerTargetWavesFwdCG : 0);
    q.hk = ar.take<float>(layer_table_len(g.nz));
    q.w2 = ar.take<double>(g.nsegs());
    q.fpart = ar.take<double>((size_t)q.fp.nchunk * n);
    if (q.r.kind == GRAV_REQ_INVERT) {
        q.ap = plan_adjoint(g.ncols(), g.nz, n, kServerTargetWavesAdj, kServerMaxPartialBytes);
        q.tp = plan_trace(g.nx, n);
        q.upart = ar.take<double>((size_t)q.ap.nparts * g.nsegs());
        q.U = ar.take<double>(g.nsegs());
        q.t = ar.take<double>(g.ncells());
        q.y = ar.take<double>(n);
        q.res = ar.take<double>(n);
        q.p = ar.take<double>(n);
        q.q = ar.take<double>(n);
        q.diag = ar.take<double>(n);
        q.dpart = ar.take<double>(kDotBlocks);
        if (q.r.lambda < 0.0) q.tpart = ar.take<double>((size_t)q.tp.nchunk * n);
    }
    return ar.off;
}

}  // namespace

struct grav_server {
    int device = 0;
    int max_active = 64;
    hipStream_t stream = nullptr;    // worker stream
    hipStream_t vstream = nullptr;   // submit-time validation stream
    hipEvent_t vevent = nullptr;     // marks the end of a submitter's input work
    char *pool = nullptr;
    size_t pool_bytes = 0;
    PoolAllocator *alloc = nullptr;
    // Slots: [0, max_active) inversions, [max_active, 2 max_active) forwards.
    double *scal_dev = nullptr;      // [2 max_active][kSlotScalars]
    double *scal_host = nullptr;     // pinned mirror
    FwdJob *fjobs_dev = nullptr, *fjobs_host = nullptr;   // 2 max_active entries
    AdjJob *ajobs_dev = nullptr, *ajobs_host = nullptr;   // max_active entries
    uint32_t *tile_next = nullptr;                        // [0] adjoint, [1] forward half-tile counter
    unsigned fwd_grid = 1, adj_grid = 1;                  // resident waves of the persistent sweeps
    std::vector<int> free_inv_slots, free_fwd_slots;
    grav_ctx *vctx = nullptr;        // validation of submitted requests
    std::mutex vmu;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::vector<Request *> active;
    std::unordered_map<uint64_t, Request *> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;

    void run();
    int step(std::vector<Request *> &reqs);
    double *slot_scal(const Request *q) const { return scal_dev + (size_t)q->slot * kSlotScalars; }
};

namespace {

#define STEP_TRY(expr)                          \
    do {                                        \
        hipError_t _e = (expr);                 \
        if (_e != hipSuccess) return (int)_e;   \
    } while (0)

}  // namespace

// Enqueue one scheduling step for `reqs` (all admitted, not done) and wait for it.
int grav_server::step(std::vector<Request *> &reqs) {
    hipStream_t st = stream;
    // ---- init of newly admitted requests
    for (Request *q : reqs) {
        if (q->phase != Phase::Init) continue;
        const Mesh &g = q->g;
        STEP_TRY(launch_layer_thickness(g, q->hk, st));
        if (q->r.kind == GRAV_REQ_FORWARD) {
            STEP_TRY(launch_edge_weights(g, q->r.m, q->w2, st));
            continue;
        }
        double *scal = slot_scal(q);
        if (q->r.lambda < 0.0) {
            STEP_TRY(launch_trace_mixed(g, q->o, q->hk, q->r.wdepth, q->tp, q->tpart, st));
            STEP_TRY(launch_reduce_parts(q->tpart, q->tp.nchunk, q->o.n, GRAV_GAMMA * GRAV_GAMMA,
                                         nullptr, 0.0, q->diag, st));
            STEP_TRY(launch_dot(q->diag, nullptr, q->o.n, q->dpart, st));
            STEP_TRY(launch_dot_finish(q->dpart, scal, kFinishPlain, kTraceSlot, st));
        }
        k_set_lambda<<<1, 1, 0, st>>>(scal, q->r.lambda, q->o.n);
        STEP_TRY(hipGetLastError());
        STEP_TRY(launch_sub(q->r.d_obs, nullptr, q->res, q->o.n, st));
        STEP_TRY(launch_sub(q->r.d_obs, nullptr, q->p, q->o.n, st));
        STEP_TRY(launch_fill(q->y, 0.0, q->o.n, st));
        STEP_TRY(launch_dot(q->res, q->res, q->o.n, q->dpart, st));
        STEP_TRY(launch_dot_finish(q->dpart, scal, kFinishInit, 0, st));
        q->phase = Phase::CG;
    }
    // ---- batched adjoint sweep (requests by decreasing tile cost: observations
    // per part x layers per chunk, taken as ceil(nz / ceil(nz / 16)); the plan
    // has one chunk index more for the split at the first deep layer, which is
    // known on the device only)
    std::vector<Request *> order;
    for (Request *q : reqs)
        if (q->phase == Phase::CG || q->phase == Phase::Final) order.push_back(q);
    auto adj_tile_cost = [](const Request *q) {
        const int nch = q->ap.nkc - 1;
        return q->ap.obs_per_part * (int64_t)((q->g.nz + nch - 1) / nch);
    };
    std::stable_sort(order.begin(), order.end(), [&](const Request *a, const Request *b) {
        return adj_tile_cost(a) > adj_tile_cost(b);
    });
    int na = 0;
    int64_t atotal = 0;
    for (Request *q : order) {
        AdjJob &j = ajobs_host[na++];
        j = AdjJob{q->g.xn, q->g.yn, q->g.zn, q->o.x, q->o.y, q->o.z,
                   q->phase == Phase::CG ? q->p : q->y, q->hk, q->upart, q->o.n, q->ap.obs_per_part,
                   q->g.ncols(), atotal, q->g.ny + 1, q->g.nz, q->ap.nparts, q->ap.nkc};
        atotal += q->ap.nblk_col * q->ap.nkc * q->ap.nparts;
    }
    if (na) {
        STEP_TRY(hipMemcpyAsync(ajobs_dev, ajobs_host, na * sizeof(AdjJob), hipMemcpyHostToDevice, st));
        if (atotal * kHalves > INT32_MAX) return (int)hipErrorInvalidValue;
        STEP_TRY(hipMemsetAsync(tile_next, 0, sizeof(uint32_t), st));
        const unsigned grid = (unsigned)std::min<int64_t>(atotal * kHalves, adj_grid);
        k_adjoint_batched<<<grid, 64, 0, st>>>(ajobs_dev, na, (uint32_t)(atotal * kHalves), tile_next);
        STEP_TRY(hipGetLastError());
    }
    for (Request *q : reqs) {
        if (q->phase != Phase::CG && q->phase != Phase::Final) continue;
        const Mesh &g = q->g;
        STEP_TRY(launch_reduce_parts(q->upart, q->ap.nparts, g.nsegs(), 1.0, nullptr, 0.0, q->U, st));
        if (q->phase == Phase::CG) {
            STEP_TRY(launch_adjoint_finish_edges(g, q->U, GRAV_GAMMA, q->r.wdepth, nullptr, q->t, st));
            STEP_TRY(launch_edge_weights(g, q->t, q->w2, st));
        } else {
            STEP_TRY(launch_adjoint_finish_edges(g, q->U, GRAV_GAMMA, q->r.wdepth, nullptr, q->r.m_out, st));
        }
    }
    // ---- batched forward sweep (requests by decreasing tile cost: node
    // columns per chunk x layers)
    order.clear();
    for (Request *q : reqs) {
        const bool fwd = q->r.kind == GRAV_REQ_FORWARD && q->phase == Phase::Init;
        if (fwd || q->phase == Phase::CG) order.push_back(q);
    }
    auto fwd_tile_cost = [](const Request *q) { return q->fp.cols_per_chunk * (int64_t)q->g.nz; };
    std::stable_sort(order.begin(), order.end(), [&](const Request *a, const Request *b) {
        return fwd_tile_cost(a) > fwd_tile_cost(b);
    });
    int nf = 0;
    int64_t ftotal = 0;
    for (Request *q : order) {
        FwdJob &j = fjobs_host[nf++];
        j = FwdJob{q->g.xn, q->g.yn, q->g.zn, q->o.x, q->o.y, q->o.z, q->w2, q->hk, q->fpart, q->o.n,
                   q->g.ncols(), q->fp.cols_per_chunk, ftotal, q->g.ny + 1, q->g.nz, q->fp.nchunk, 0};
        ftotal += q->fp.nblk_obs * q->fp.nchunk;
    }
    if (nf) {
        STEP_TRY(hipMemcpyAsync(fjobs_dev, fjobs_host, nf * sizeof(FwdJob), hipMemcpyHostToDevice, st));
        if (ftotal * kHalves > INT32_MAX) return (int)hipErrorInvalidValue;
        STEP_TRY(hipMemsetAsync(tile_next + 1, 0, sizeof(uint32_t), st));
        const unsigned grid = (unsigned)std::min<int64_t>(ftotal * kHalves, fwd_grid);
        k_forward_batched<<<grid, 64, 0, st>>>(fjobs_dev, nf, (uint32_t)(ftotal * kHalves), tile_next + 1);
        STEP_TRY(hipGetLastError());
    }
    for (Request *q : reqs) {
        const int64_t n = q->o.n;
        if (q->r.kind == GRAV_REQ_FORWARD && q->phase == Phase::Init) {
            STEP_TRY(launch_reduce_parts(q->fpart, q->fp.nchunk, n, GRAV_GAMMA, nullptr, 0.0, q->r.d, st));
        } else if (q->phase == Phase::CG) {
            double *scal = slot_scal(q);
            k_reduce_parts_dcoef<<<grid_of(n), 256, 0, st>>>(q->fpart, q->fp.nchunk, n, GRAV_GAMMA, q->p,
                                                            scal + kLambdaSlot, q->q);
            STEP_TRY(hipGetLastError());
            STEP_TRY(launch_dot(q->p, q->q, n, q->dpart, st));
            STEP_TRY(launch_dot_finish(q->dpart, scal, kFinishPQ, 0, st));
            STEP_TRY(launch_cg_update_yr(q->y, q->res, q->p, q->q, n, scal, q->dpart, st));
            STEP_TRY(launch_dot_finish(q->dpart, scal, kFinishRRNew, 0, st));
            STEP_TRY(launch_cg_update_p(q->p, q->res, n, scal, st));
        }
    }
    STEP_TRY(hipMemcpyAsync(scal_host, scal_dev, (size_t)max_active * kSlotScalars * sizeof(double),
                            hipMemcpyDeviceToHost, st));
    STEP_TRY(hipStreamSynchronize(st));
    // ---- advance the state machines
    const Clock::time_point now = Clock::now();
    for (Request *q : reqs) {
        if (q->r.kind == GRAV_REQ_FORWARD || q->phase == Phase::Final) {
            q->phase = Phase::Done;
            q->finished = true;
            q->t_done = now;
            continue;
        }
        const double *hs = scal_host + (size_t)q->slot * kSlotScalars;
        q->iters += 1;
        q->lambda = hs[kLambdaSlot];
        q->relres = hs[kB2] > 0.0 ? std::sqrt(hs[kRR] / hs[kB2]) : 0.0;
        const grav_cg_opts &cg = q->r.cg;
        const bool fixed = cg.fixed_iters > 0;
        const int cap = fixed ? cg.fixed_iters : cg.max_iter;
        const bool conv = !fixed && q->relres <= cg.tol;
        if (conv || q->iters >= cap || hs[kB2] == 0.0) {
            q->phase = Phase::Final;
            if (!fixed && !conv && hs[kB2] != 0.0) q->status = GRAV_ENOCONV;
        }
    }
    return 0;
}

void grav_server::run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        cv_work.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
        if (stop && queue.empty() && active.empty()) break;
        // admission (policy at the top of this file and in admission.h)
        admission_pass(
            queue, [](Request *q) { return q->r.kind == GRAV_REQ_FORWARD; },
            [&](bool fwd) { return !(fwd ? free_fwd_slots : free_inv_slots).empty(); },
            [&](Request *q) { return alloc->alloc(q->bytes, &q->off); },
            [&](Request *q, bool fwd) {
                std::vector<int> &slots = fwd ? free_fwd_slots : free_inv_slots;
                q->slot = slots.back();
                slots.pop_back();
                request_layout(*q, pool + q->off);
                q->phase = Phase::Init;
                q->t_admit = Clock::now();
                active.push_back(q);
            });
        if (active.empty()) continue;   // head of queue cannot fit: nothing else can run
        std::vector<Request *> work = active;
        lk.unlock();
        roctxRangePushA("grav server step");
        const int err = step(work);
        roctxRangePop();
        lk.lock();
        if (err) {
            // kernels enqueued before the failure may still be writing the
            // requests' outputs and pool ranges: let them finish before the
            // requests are reported done and their memory is reused
            (void)hipStreamSynchronize(stream);
            for (Request *q : work) {
                q->status = GRAV_EDEVICE;
                q->phase = Phase::Done;
                q->finished = true;
                q->t_done = Clock::now();
            }
        }
        std::vector<Request *> still;
        for (Request *q : active) {
            if (q->cancel && !q->finished) {
                q->finished = true;
                q->phase = Phase::Done;
                q->status = GRAV_ECANCELED;
                q->t_done = Clock::now();
            }
            if (q->finished) {
                alloc->release(q->off, q->bytes);
                (q->r.kind == GRAV_REQ_FORWARD ? free_fwd_slots : free_inv_slots).push_back(q->slot);
                q->done = true;
            } else {
                still.push_back(q);
            }
        }
        const bool any_done = still.size() != active.size();
        active.swap(still);
        if (any_done) cv_done.notify_all();
    }
}

// ---------------------------------------------------------------- C ABI

static void fill_info(const Request *q, grav_request_info *info) {
    if (!info) return;
    info->status = q->status;
    info->iters = q->iters;
    info->relres = q->relres;
    info->lambda_used = q->lambda;
    info->queue_ms = std::chrono::duration<double, std::milli>(q->t_admit - q->t_submit).count();
    info->run_ms = std::chrono::duration<double, std::milli>(q->t_done - q->t_admit).count();
    info->state_bytes = q->bytes;
}

extern "C" int grav_server_create(grav_server **out, const grav_server_opts *opts_in) {
    if (!out) return GRAV_EINVAL;
    *out = nullptr;
    grav_server_opts opts{0, 0, 0};
    if (opts_in) opts = *opts_in;
    if (opts.max_active <= 0) opts.max_active = 64;
    if (opts.max_active > kMaxActiveCap) return GRAV_EINVAL;
    if (opts.budget_bytes == 0) opts.budget_bytes = (uint64_t)16 << 30;
    grav_ctx_opts co;
    grav_ctx_opts_default(&co);
    co.device = opts.device;
    co.workspace_bytes = 1 << 20;
    grav_ctx *vctx = nullptr;
    int rc = grav_ctx_create(&vctx, &co);
    if (rc) return rc;
    grav_server *s = new grav_server();
    s->device = opts.device;
    s->max_active = opts.max_active;
    s->vctx = vctx;
    s->pool_bytes = opts.budget_bytes;
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->vstream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->vevent, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&s->pool), s->pool_bytes);
    const size_t nslots = 2 * (size_t)s->max_active;
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&s->scal_dev), nslots * kSlotScalars * sizeof(double));
    if (e == hipSuccess)
        e = hipMemset(s->scal_dev, 0, nslots * kSlotScalars * sizeof(double));
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&s->scal_host), nslots * kSlotScalars * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&s->fjobs_dev), nslots * sizeof(FwdJob));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&s->ajobs_dev), (size_t)s->max_active * sizeof(AdjJob));
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&s->fjobs_host), nslots * sizeof(FwdJob), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&s->ajobs_host), (size_t)s->max_active * sizeof(AdjJob), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&s->tile_next), 2 * sizeof(uint32_t));
    if (e == hipSuccess) {
        // persistent grids: every wave resident at once
        int ncu = 0, bf = 0, ba = 0;
        e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, s->device);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bf, k_forward_batched, 64, 0);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&ba, k_adjoint_batched, 64, 0);
        if (e == hipSuccess) {
            s->fwd_grid = (unsigned)std::max(1, ncu * bf);
            s->adj_grid = (unsigned)std::max(1, ncu * ba);
        }
    }
    if (e != hipSuccess) {
        const bool oom = e == hipErrorOutOfMemory;
        if (s->pool) (void)hipFree(s->pool);
        if (s->scal_dev) (void)hipFree(s->scal_dev);
        if (s->scal_host) (void)hipHostFree(s->scal_host);
        if (s->fjobs_dev) (void)hipFree(s->fjobs_dev);
        if (s->ajobs_dev) (void)hipFree(s->ajobs_dev);
        if (s->fjobs_host) (void)hipHostFree(s->fjobs_host);
        if (s->ajobs_host) (void)hipHostFree(s->ajobs_host);
        if (s->tile_next) (void)hipFree(s->tile_next);
        if (s->stream) (void)hipStreamDestroy(s->stream);
        if (s->vstream) (void)hipStreamDestroy(s->vstream);
        if (s->vevent) (void)hipEventDestroy(s->vevent);
        grav_ctx_destroy(vctx);
        delete s;
        return oom ? GRAV_ENOMEM : GRAV_EDEVICE;
    }
    s->alloc = new PoolAllocator(s->pool_bytes);
    for (int i = s->max_active - 1; i >= 0; --i) s->free_inv_slots.push_back(i);
    for (int i = 2 * s->max_active - 1; i >= s->max_active; --i) s->free_fwd_slots.push_back(i);
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return GRAV_OK;
}

extern "C" int grav_server_submit(grav_server *s, const grav_request *req, uint64_t *ticket) {
    if (!s || !req || !ticket) return GRAV_EINVAL;
    Request *q = new Request();
    q->r = *req;
    q->t_submit = Clock::now();
    int rc = GRAV_OK;
    {
        std::lock_guard<std::mutex> vl(s->vmu);
        grav_ctx *v = s->vctx;
        // Order the validation (and with it every later read: validation
        // waits for its stream) after the submitter's work on req->stream.
        (void)hipSetDevice(s->device);
        hipError_t ee = hipEventRecord(s->vevent, reinterpret_cast<hipStream_t>(req->stream));
        if (ee == hipSuccess) ee = hipStreamWaitEvent(s->vstream, s->vevent, 0);
        rc = ee == hipSuccess ? check_geometry_host(v, &req->mesh, &req->obs) : GRAV_EDEVICE;
        const Mesh g{req->mesh.nx, req->mesh.ny, req->mesh.nz, req->mesh.xn, req->mesh.yn, req->mesh.zn};
        const Obs o{req->obs.n, req->obs.x, req->obs.y, req->obs.z};
        if (!rc) {
            if (req->kind == GRAV_REQ_FORWARD) {
                if (!req->m || !req->d) rc = GRAV_EINVAL;
                else rc = validate_on_device(v, g, o, s->vstream, {ArrayCheck{req->m, g.ncells(), false}});
            } else if (req->kind == GRAV_REQ_INVERT) {
                const grav_cg_opts &cg = req->cg;
                if (!req->d_obs || !req->wdepth || !req->m_out || !std::isfinite(req->lambda) ||
                    (cg.fixed_iters <= 0 && (cg.max_iter < 1 || !(cg.tol >= 0.0))) ||
                    cg.precond != 0 || cg.restart != 0 || cg.history_cap != 0 || cg.y0 ||
                    cg.y_out)
                    rc = GRAV_EINVAL;
                else
                    rc = validate_on_device(v, g, o, s->vstream,
                                            {ArrayCheck{req->wdepth, g.ncells(), true},
                                             ArrayCheck{req->d_obs, o.n, false}});
            } else {
                rc = GRAV_EINVAL;
            }
        }
        if (!rc) {
            q->g = g;
            q->o = o;
            q->bytes = request_layout(*q, nullptr);
            if (q->bytes > s->pool_bytes) rc = GRAV_ENOMEM;
        }
    }
    if (rc) {
        delete q;
        return rc;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    q->ticket = s->next_ticket++;
    s->all[q->ticket] = q;
    s->queue.push_back(q);
    *ticket = q->ticket;
    s->cv_work.notify_one();
    return GRAV_OK;
}

extern "C" int grav_server_poll(grav_server *s, uint64_t ticket, int32_t *done,
                                grav_request_info *info) {
    if (!s || !done) return GRAV_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return GRAV_EINVAL;
    Request *q = it->second;
    *done = q->done ? 1 : 0;
    if (q->done) {
        fill_info(q, info);
        s->all.erase(it);
        delete q;
    }
    return GRAV_OK;
}

extern "C" int grav_server_wait(grav_server *s, uint64_t ticket, grav_request_info *info) {
    if (!s) return GRAV_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return GRAV_EINVAL;
    Request *q = it->second;
    s->cv_done.wait(lk, [&] { return q->done; });
    const int status = q->status;
    fill_info(q, info);
    s->all.erase(ticket);
    delete q;
    return status;
}

extern "C" int grav_server_cancel(grav_server *s, uint64_t ticket) {
    if (!s) return GRAV_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return GRAV_EINVAL;
    Request *q = it->second;
    if (q->done) return GRAV_OK;
    auto qi = std::find(s->queue.begin(), s->queue.end(), q);
    if (qi != s->queue.end()) {            // not admitted: nothing on the device
        s->queue.erase(qi);
        q->status = GRAV_ECANCELED;
        q->phase = Phase::Done;
        q->finished = true;
        q->t_admit = q->t_done = Clock::now();
        q->done = true;
        s->cv_done.notify_all();
    } else {
        q->cancel = true;                  // the worker stops it after the current step
    }
    return GRAV_OK;
}

extern "C" void grav_server_destroy(grav_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto &kv : s->all) delete kv.second;
    (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(s->stream);
    (void)hipFree(s->pool);
    (void)hipFree(s->scal_dev);
    (void)hipHostFree(s->scal_host);
    (void)hipFree(s->fjobs_dev);
    (void)hipFree(s->ajobs_dev);
    (void)hipHostFree(s->fjobs_host);
    (void)hipHostFree(s->ajobs_host);
    (void)hipFree(s->tile_next);
    (void)hipStreamDestroy(s->stream);
    (void)hipStreamDestroy(s->vstream);
    (void)hipEventDestroy(s->vevent);
    grav_ctx_destroy(s->vctx);
    delete s->alloc;
    delete s;
}
