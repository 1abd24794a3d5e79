// grav_forward_static: the forward product d = G m without a context, on a
// fixed device buffer that the library holds for the life of the process,
// for callers that may not allocate device memory.
//
// The buffer is the file-scope array `scratch` below.  Its name in host code
// stands for the symbol, not for a device address: the address is looked up
// once per device with hipGetSymbolAddress (with that device current) and
// only that address is handed to kernels.  The call then runs exactly the
// operator of grav_forward (same validation kernels, launch plan and sweep
// kernels), carved out of that address instead of a context's workspace.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "grav_internal.h"
#include "api_internal.h"

using namespace grav;

static __device__ __align__(256) char scratch[GRAV_STATIC_SCRATCH_BYTES];

namespace {

constexpr size_t kStaticScratchBytes = GRAV_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

std::mutex g_lock;
void *g_scratch_addr[kMaxDevices] = {};

int static_fail(int code, const std::string &msg) {
    set_context_free_error(msg);
    return code;
}

// Device address of this device's copy of `scratch` (looked up on the first
// call on the device, with the device current).
int scratch_address(int dev, char **out) {
    std::lock_guard<std::mutex> guard(g_lock);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return static_fail(GRAV_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                                 hipGetErrorString(e));
        g_scratch_addr[dev] = p;
    }
    *out = static_cast<char *>(g_scratch_addr[dev]);
    return GRAV_OK;
}

}  // namespace

extern "C" int grav_forward_static(const grav_mesh *mesh, const grav_obs *obs, const double *m,
                                   double *d, grav_prec prec, int32_t validate,
                                   grav_stream stream) {
    set_context_free_error("");
    // A stack context: no workspace of its own, pageable host staging for the
    // validation flag; its error text is copied out before it goes away.
    int h_flags = 0;
    grav_ctx tmp;
    tmp.validate = validate != 0;
    tmp.h_flags = &h_flags;
    int rc = check_geometry_host(&tmp, mesh, obs);
    if (rc) return static_fail(rc, tmp.err);
    if (!m || !d) return static_fail(GRAV_EINVAL, "m or d is NULL");
    if (prec != GRAV_FP64 && prec != GRAV_MIXED)
        return static_fail(GRAV_EINVAL, "precision must be GRAV_FP64 or GRAV_MIXED");
    const uint64_t need = (uint64_t)kReserveBytes +
                          workspace_need(mesh->nx, mesh->ny, mesh->nz, obs->n, GRAV_OP_FORWARD,
                                         prec, 0);
    if (need > kStaticScratchBytes)
        return static_fail(GRAV_ENOMEM, "problem needs " + std::to_string(need) +
                                            " bytes of device scratch; the static buffer holds " +
                                            std::to_string(kStaticScratchBytes));
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return static_fail(GRAV_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return static_fail(GRAV_EDEVICE, "device ordinal above 63");
    rc = scratch_address(dev, &tmp.ws);
    if (rc) return rc;
    tmp.device = dev;
    tmp.ws_bytes = kStaticScratchBytes;
    const Mesh g{mesh->nx, mesh->ny, mesh->nz, mesh->xn, mesh->yn, mesh->zn};
    const Obs o{obs->n, obs->x, obs->y, obs->z};
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    rc = validate_on_device(&tmp, g, o, st, {ArrayCheck{m, g.ncells(), false}});
    if (rc) return static_fail(rc, tmp.err);
    Arena ar = ctx_arena(&tmp);
    rc = op_forward(&tmp, ar, g, o, m, d, prec, st, GRAV_GAMMA, nullptr, 0.0);
    if (rc) return static_fail(rc, tmp.err);
    return GRAV_OK;
}
