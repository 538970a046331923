// odp_hj_solve_noalloc: odp_hj_solve for callers that cannot allocate.
//
// The workspace is `scratch`, a file-scope device array of kScratchBytes
// that every GPU the library runs on holds until the process ends.  Host
// code never passes the array's name to a kernel or a copy (in host code it
// names a host-side stand-in): the device address comes from
// hipGetSymbolAddress, once per device, on the first call made with that
// device current.  The call allocates nothing: no device or pinned memory,
// no events, no graphs (its stepping is launched eagerly); the plan's upload
// is a plain copy from pageable host memory, which the runtime performs
// synchronously.  Calls on one GPU share its array, which keeps the last
// call's contents: calls that overlap on one GPU (other host threads, or
// streams that run concurrently) race on it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "plan.h"
#include "runtime.h"

namespace odp {

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's `scratch`.
int scratch_address(unsigned char **out) {
    int dev = 0, rc;
    if ((rc = check_hip(hipGetDevice(&dev), "device"))) return rc;
    if (dev < 0 || dev >= kMaxDevices) return set_error(ODP_EUNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if ((rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address"))) return rc;
        if (!p) return set_error(ODP_EHIP, "scratch address is null");
        g_scratch_ptr[dev] = (unsigned char *)p;
    }
    *out = g_scratch_ptr[dev];
    return ODP_OK;
}

}  // namespace

}  // namespace odp

using namespace odp;

extern "C" {

int odp_hj_solve_noalloc(const odp_grid *grid, const odp_dynamics *dyn, const void *V0_dev,
                         const void *V_init_dev, const double *tau, int ntau, const odp_solve_opts *opts,
                         void *V_out_dev, void *V_all_dev, odp_solve_stats *stats) {
    if (!grid) return set_error(ODP_EINVAL, "grid is NULL");
    int rc;
    if ((rc = validate_opts(opts)) || (rc = validate_dyn(grid, dyn)) || (rc = validate_tau(tau, ntau))) return rc;
    if (!V0_dev || !V_out_dev) return set_error(ODP_EINVAL, "V0 and V_out are required");
    if (V_out_dev == V0_dev || V_out_dev == V_init_dev)
        return set_error(ODP_EINVAL, "V_out may not alias V0 or V_init");
    if (V_out_dev == opts->target_dev || V_out_dev == opts->obstacle_dev)
        return set_error(ODP_EINVAL, "V_out may not alias the target or obstacle array");
    if (opts->set_slices > 1 && opts->set_slices != ntau)
        return set_error(ODP_EINVAL, "set_slices must be 0, 1 or ntau");
    if (opts->save_all && !V_all_dev) return set_error(ODP_EINVAL, "save_all needs V_all");
    // eager stepping and the default tiling (a graph or the tuner's timing
    // runs would allocate)
    odp_solve_opts o = *opts;
    o.graph = 2;
    if (o.tile_chunk == ODP_TILE_AUTOTUNE) o.tile_chunk = 0;
    hipStream_t st = (hipStream_t)o.stream;

    Plan p;
    PlanItem it;
    it.g = grid;
    it.dyn = *dyn;
    it.V0 = V0_dev;
    it.Vinit = V_init_dev;
    it.A = V_out_dev;
    it.tau.assign(tau, tau + ntau);
    std::vector<PlanItem> items{it};
    plan_build(p, std::move(items), o, o.tile_chunk);
    if (p.total > kScratchBytes)
        return set_error(ODP_ENOMEM, "odp_hj_solve_noalloc: this solve needs " + std::to_string(p.total) +
                                         " bytes of workspace, over the " + std::to_string(kScratchBytes) +
                                         "-byte scratch array");
    unsigned char *base = nullptr;
    if ((rc = scratch_address(&base))) return rc;
    if ((rc = plan_prologue(p, base, st, true))) return rc;
    if (o.save_all) {
        const size_t bytes = size_t(grid->npts) * (o.precision == 32 ? 4 : 8);
        const void *src = V_init_dev ? V_init_dev : V0_dev;
        if ((rc = check_hip(hipMemcpyAsync(V_all_dev, src, bytes, hipMemcpyDeviceToDevice, st), "save start")))
            return rc;
    }
    if ((rc = plan_steps(p, base, st, o.save_all ? V_all_dev : nullptr))) return rc;
    if (stats) return plan_stats(p, base, 0.0, stats, st);
    return ODP_OK;
}

}  // extern "C"
